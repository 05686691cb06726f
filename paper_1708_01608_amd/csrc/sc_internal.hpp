// sc_internal.hpp -- host-side declarations shared by the translation units of libsc.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "sc.h"

namespace sc {

// Records the calling thread's error message (returned by sc_last_error) and returns code.
int set_error(int code, const std::string& msg);

// Arguments of the fused step kernel.
struct StepArgs {
    int nx, ny, nz;
    int planes;        // planes (z in 3D, rows y in 2D) marched by one block
    int64_t N;
    float tau, omega, G, rho_ref;
    double taud, omegad, Gd, rho_refd;
    // modified Shan-Chen barrier: owner id per node (null: barrier off) and psi(rho_liquid),
    // which a node sees where a neighbour belongs to a different, un-merged bubble
    const uint16_t* owner;
    float psi_l;
    double psi_ld;
    // gravity: body force (rho - rho0) g added to the Shan-Chen force (grav = 0: off)
    int grav;
    float g[3], rho0;
    double gd[3], rho0d;
};

struct StepShape {
    int tile_x, tile_y, tile_z;  // tile_y is 1 in 2D; tile_z = planes per block
    int variant;                 // 1: plain marching kernel, 2: software-pipelined (3D only)
};

// storage codes as in sc.h: 0 F32, 1 F16, 2 BF16
size_t storage_bytes(int storage);

// --- step kernels (sc_step.hip) ------------------------------------------------------------
bool step_shape_supported(int q, const StepShape& s);
bool step_combo_supported(int storage, int compute);
hipError_t launch_step(int q, int storage, int compute, const void* src, void* dst,
                       const StepArgs& a, const StepShape& s, hipStream_t st);
// --- two-component kernels (sc_step2c.hip) ---------------------------------------------------
// Two-component step (FP32 unshifted storage, FP64 arithmetic): one fused marching kernel per
// step (both densities over the tile and its ring in LDS, the cross forces, the common velocity,
// both collisions with streaming).  Shapes: tile_x, tile_y, planes = tile_z, variant 1 or 3
// (non-temporal stores); in D3Q19 also 4 or 5 (one component per wave; 5 non-temporal).
struct Step2cArgs {
    int nx, ny, nz;
    int planes;  // set by launch_step2c from the shape
    int64_t N;
    double tau_l, tau_v, Gx;
    double ref_l, ref_v;  // storage shifts of the two components (0 with FP32 storage)
};
bool step2c_shape_supported(int q, const StepShape& s);
// FP32 storage runs FP64 arithmetic, FP16 / BF16 storage FP32 arithmetic.
hipError_t launch_step2c(int q, int storage, const void* src_l, const void* src_v, void* dst_l,
                         void* dst_v, const Step2cArgs& a, const StepShape& s, hipStream_t st);
// Reported fields of the mixture: rho_l, rho_v (FP32) and the barycentric velocity; dens holds
// [2][N] FP64 densities afterwards.
hipError_t launch_fields2c(int q, int storage, const void* f_l, const void* f_v, double* dens,
                           float* rho_l, float* rho_v, float* u, const Step2cArgs& a,
                           hipStream_t st);

// Barrier fix-up of the listed frontier nodes after a step (same src/dst as that step).
hipError_t launch_barrier_fix(int q, int storage, int compute, const void* src, void* dst,
                              const StepArgs& a, const uint32_t* list, int count, hipStream_t st);

// --- state kernels (sc_step.hip) -----------------------------------------------------------
struct InitArgs {
    int nx, ny, nz;
    int64_t N;
    double rho, amp, rho_ref;
    uint64_t seed;
};
hipError_t launch_init(int q, int storage, void* f, const InitArgs& a, hipStream_t st);
// Paint a ball of radius R around c (minimal image), rho = rho_gas + amp (2U - 1), u = 0.
hipError_t launch_paint(int q, int storage, void* f, const InitArgs& a, const double c[3],
                        double R, hipStream_t st);
hipError_t launch_set_eq(int q, int storage, void* f, const InitArgs& a, const double* rho_d,
                         const double* u_d, hipStream_t st);
hipError_t launch_get_f(int q, int storage, const void* f, double* out_d, const InitArgs& a,
                        hipStream_t st);
hipError_t launch_set_f(int q, int storage, void* f, const double* in_d, const InitArgs& a,
                        hipStream_t st);

// --- field / test kernels (sc_test.hip) ----------------------------------------------------
struct FieldArgs {
    int nx, ny, nz;
    int64_t N;
    float G;
    float rho_ref;
    double Gd, rho_ref_d, theta;
    const uint16_t* owner;  // barrier owner field for the force in the fields (null: off)
    double psi_ld;
    int grav;               // gravity body force (rho - rho0) g in the reported velocity
    double gd[3], rho0d;
    // two-component mode: the gas component's populations (null: one component) and the cross
    // interaction; pressures then follow p = (rho_l + rho_v)/3 + (Gx/3) rho_l rho_v
    const void* f2;
    double Gx;
    double rho_ref2;  // storage shift of the gas component
};
hipError_t launch_psi(int q, int storage, const void* f, double* psi, const FieldArgs& a,
                      hipStream_t st);
hipError_t launch_fields(int q, int storage, const void* f, const double* psi, float* rho,
                         float* u, const FieldArgs& a, hipStream_t st);
hipError_t launch_pressure(int q, int storage, const void* f, double* p, const FieldArgs& a,
                           hipStream_t st);
hipError_t launch_laplacian(int q, const double* p, double* lap, const FieldArgs& a,
                            hipStream_t st);
// FP64 totals (M, Jx, Jy, Jz) into out_d[4] (device); partials holds >= totals_blocks() * 4.
int totals_blocks(int64_t N);
hipError_t launch_totals(int q, int storage, const void* f, double* partials, double* out_d,
                         const FieldArgs& a, hipStream_t st);

// Labelling: parent[N] (uint32, 0xffffffff = liquid), labels[N] (1 + root, 0 = liquid).
// Gas mask (as launch_mask_from_rho) and the FP64 totals (as launch_totals, into out_d[4]) from
// one sweep of the populations.
hipError_t launch_mask_totals(int q, int storage, const void* f, uint32_t* parent,
                              double* partials, double* out_d, const FieldArgs& a, hipStream_t st);
hipError_t launch_mask_from_rho(int q, int storage, const void* f, uint32_t* parent,
                                const FieldArgs& a, hipStream_t st);
hipError_t launch_mask_from_bytes(const uint8_t* mask_d, uint32_t* parent, int64_t N,
                                  hipStream_t st);
// Union-find of the mask in parent (tile-local in LDS, then the links between tiles); with
// zero_counter, the counter of the flatten that follows is set to zero.
hipError_t launch_union(int q, uint32_t* parent, uint32_t* zero_counter, const FieldArgs& a,
                        hipStream_t st);
hipError_t launch_flatten(uint32_t* parent, uint32_t* labels, uint32_t* ncomp_d, int64_t N,
                          hipStream_t st);

// Bubble statistics and the merge test.
hipError_t launch_gather_labels(const uint32_t* labels, const int64_t* nodes_d, uint32_t* out_d,
                                int n, int64_t N, hipStream_t st);
hipError_t launch_set_slots(int32_t* slot_of_root, const uint32_t* labels_of_bubbles_d, int nb,
                            int clear, hipStream_t st);
hipError_t launch_stats(const uint32_t* labels, const int32_t* slot_of_root,
                        const int32_t* anchors_d /*[nb][3]*/, unsigned long long* count_d,
                        unsigned long long* sums_d /*[nb][3]*/, const FieldArgs& a,
                        hipStream_t st);
// Fed gas nodes in node order; block_counts holds gas_list_scratch_words() words of scratch.
int gas_list_scratch_words();
hipError_t launch_gas_list(const uint32_t* labels, const int32_t* slot_of_root,
                           const int32_t* feed_d /*[nb]: 1 if the bubble is fed*/,
                           uint32_t* list_node, int32_t* list_slot, unsigned int* count_d,
                           unsigned int* block_counts, int64_t N, hipStream_t st);

struct MergePair {
    double cen_a[3];
    double dv[3];
    uint32_t label_a, label_b;
    int32_t T;
    int32_t pad;
};
struct MergeResult {
    int32_t fired;
    int32_t film_len;
    int64_t film_node;
    double lap_p;
    double rho_film;
};

// Bubble table of a test pass, built on the device so that the pass needs one synchronization:
// the label at every nucleus node, the distinct nonzero labels in ascending order (the bubbles),
// the lead (smallest) nucleus of each with its node's coordinates (the centroid anchor), the slot
// of each bubble's root in slot_of_root, and zeroed statistics for k_stats.  One buffer of
// bubble_tab_bytes(n) bytes holds every table; head[0] = nb, head[1] = candidate pairs found.
constexpr int kStatStride = 16;
struct BubbleTab {
    int32_t* head;
    uint32_t* comp;             // [n]
    uint32_t* distinct;         // [n], nb used
    int32_t* lead;              // [n]
    int32_t* first;             // [n] scratch: 1 for the smallest nucleus of each label
    int32_t* anchors;           // [3n]
    // bubble b's node count at count[b * kStatStride] and its centroid sums at
    // sums[b * kStatStride + c] (sums = count + 1): one 128-byte line per bubble, since every
    // wave of a bubble's gas nodes adds to them atomically and atomics to one line serialize
    unsigned long long* count;
    unsigned long long* sums;
    double* cen;                // [3n]
    double* rad;                // [n]
};
size_t bubble_tab_bytes(int n);
BubbleTab bubble_tab_view(void* base, int n);
// prev: the table of the previous pass (same buffer, its own nucleus count): its bubbles' slots
// are cleared first.
hipError_t launch_bubble_table(const uint32_t* labels, const int64_t* nuc_node, int n,
                               const BubbleTab& prev, const BubbleTab& t, int32_t* slot_of_root,
                               const FieldArgs& a, hipStream_t st);
// Candidate pairs of the merge test: FP64 centroids and radii formed as the host forms them,
// then every pair a < b of different merge groups (group[k]: representative of nucleus k) within
// radius_a + radius_b + film_max + 1e-6 (a superset of the host's exact test), compacted into
// pairs[] with the bubble indices in ab[2k], ab[2k + 1] (order unspecified); head[1] = the number
// found, which may exceed cap (then the first cap are written).
hipError_t launch_pairs(const BubbleTab& t, const int32_t* group, int dim, int film_max,
                        MergePair* pairs, int32_t* ab, int cap, const FieldArgs& a,
                        hipStream_t st);
// Everything a test pass reads back, gathered by one kernel into pinned host memory (dst_*,
// device-accessible addresses of it): one write over the bus instead of a copy per table.
struct StageOut {
    const double* tot;          // [4] (and [4] gas-component totals when tot2 != nullptr)
    const double* tot2;
    const int32_t* head;        // [16]
    const uint32_t* comp;       // [n]
    const unsigned long long* count;  // [n]
    const unsigned long long* sums;   // [3n]
    const double* owed;         // [ledger_nb]
    const MergePair* pairs;     // [npairs]
    const int32_t* ab;          // [2 npairs]
    const MergeResult* res;     // [npairs]
    double* dst_tot;            // [8]
    int32_t* dst_head;
    uint32_t* dst_comp;
    unsigned long long* dst_count;
    unsigned long long* dst_sums;
    double* dst_owed;
    MergePair* dst_pairs;
    int32_t* dst_ab;
    MergeResult* dst_res;
    int n, ledger_nb, npairs;
};
hipError_t launch_stage_out(const StageOut& o, hipStream_t st);

// The tail of a test pass in one block: with do_pairs, the candidate pairs (as launch_pairs)
// and their merge test; then the read-back (as launch_stage_out).
hipError_t launch_pass_tail(int q, int storage, const BubbleTab& t, const int32_t* group,
                            int film_max, MergePair* pairs, int32_t* ab, MergeResult* res,
                            int cap, int do_pairs, const StageOut& o, const void* f,
                            const uint32_t* labels, const FieldArgs& a, hipStream_t st);
// k_merge over the first min(*count_d, cap) pairs.
hipError_t launch_merge_counted(int q, int storage, const void* f, const uint32_t* labels,
                                const MergePair* pairs_d, MergeResult* res_d, int cap,
                                const int32_t* count_d, int film_max, const FieldArgs& a,
                                hipStream_t st);

// Film geometry of a bubble pair (h and the line count behind R_d): lines parallel to the
// centroid segment, at offsets i n1 + j n2 (i^2 + j^2 <= K^2), walked like the merge test.
struct FilmArgs {
    double cen[3], dv[3], n1[3], n2[3];
    uint32_t label_a, label_b;
    int32_t T, K, dim, film_max;
};
struct FilmOut {
    unsigned int count;  // lines crossing a film of 1..film_max liquid nodes
    int32_t pad;
    double h;            // centre-line thickness (rho = theta crossings), -1 if no film there
};
hipError_t launch_film(int q, int storage, const void* f, const uint32_t* labels,
                       const FilmArgs& g, FilmOut* out_d, const FieldArgs& a, hipStream_t st);

// Blowing-agent source for one step: f_i(x) += w_i * T_b / n_b on the listed gas nodes, with
// T_b = owed[b] + dm[b]; the stored values' exact gain closes the ledger (owed[b] = T_b - gain).
// Device tables of nb bubble slots; gain (2^-40 fixed point) is zero between steps.
// Bubble b's gain sits at gain[b * kLedgerGainStride]: one 128-byte line per bubble, since every
// wave of a bubble's gas nodes adds to it atomically and atomics to one line serialize.
constexpr int kLedgerGainStride = 16;
struct SourceLedger {
    const double* dm;          // this step's release of each bubble's nuclei
    const double* nodes;       // n_b, gas nodes listed for the bubble
    double* owed;              // mass released earlier that the storage has not taken yet
    unsigned long long* gain;  // sum of this step's gains in 2^-40 units (two's complement),
                               // at stride kLedgerGainStride
    int nb;
    uint64_t key;              // stochastic-rounding stream (16-bit storage)
};
hipError_t launch_source(int q, int storage, void* f, const uint32_t* list_node,
                         const int32_t* list_slot, int64_t count, const SourceLedger& led,
                         int64_t t, const FieldArgs& a, hipStream_t st);

// Barrier owner field: seed = owner id of each gas node's bubble (ids_d[slot], 0 elsewhere;
// nb == 0 writes zeros and reads neither table), then one corona layer per grow call.
hipError_t launch_owner_seed(const uint32_t* labels, const int32_t* slot_of_root,
                             const uint16_t* ids_d, int nb, uint16_t* owner, int64_t N,
                             hipStream_t st);
hipError_t launch_owner_grow(int q, const uint16_t* in, uint16_t* out, const FieldArgs& a,
                             hipStream_t st);
// Frontier nodes (owned, with a lattice neighbour of a different owner) appended to list.
hipError_t launch_frontier_list(int q, const uint16_t* owner, uint32_t* list,
                                unsigned int* count_d, const FieldArgs& a, hipStream_t st);

hipError_t launch_fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t st);
hipError_t launch_fill_u64(unsigned long long* p, unsigned long long v, int64_t n,
                           hipStream_t st);

}  // namespace sc
