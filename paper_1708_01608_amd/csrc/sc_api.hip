// sc_api.hip -- runtime and C ABI of libsc (see include/sc.h).
//
// Host side: parameter validation, device buffers, the time-step loop, and the bubble registry
// (nuclei, FP64 agent budgets, merge and topological events).  All per-node work runs in the
// HIP kernels of sc_step.hip, sc_step2c.hip and sc_test.hip; the host touches only per-bubble
// tables.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "sc_internal.hpp"

using namespace sc;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg)
{
    g_err = msg;
    return code;
}

struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
};

struct ProfRec {
    hipEvent_t a, b;
    int cls;
    int launches = 1;  // kernel launches between a and b (a K-step graph records K)
};

}  // namespace

int sc::set_error(int code, const std::string& msg) { return fail(code, msg); }

struct sc_sim {
    sc_params p;
    sc_allocator alloc;
    bool has_alloc = false;
    int q = 9, d = 2;
    int64_t N = 0;
    double theta = 0.0, rho_ref = 0.0;
    double rho_ref_v = 0.0;  // storage shift of the gas component (0 when the liquid's is 0)
    double pass_tot[4] = {0.0, 0.0, 0.0, 0.0};  // test-pass totals (target of a queued copy)
    hipStream_t stream = nullptr;
    bool own_stream = false;
    size_t es = 4;
    int compute = SC_COMPUTE_F64;
    void* f[2] = {nullptr, nullptr};
    int cur = 0;
    StepShape shape{};
    int64_t t = 0;
    int latched = 0;

    // scratch buffers (allocated on first use)
    DevBuf parent, labels, labels2, slots, psi, rho_out, u_out, p_out, lap_out, partials, small,
        tmp64, mask8, nodes, list_node, list_slot, list_scan, add_tab, pair_buf, res_buf, bub_tab;
    bool slots_ready = false;

    // modified Shan-Chen barrier: owner id per node (uint16, fixed address for the step
    // kernel), a second buffer for the corona layers, and the owner id of each bubble slot
    DevBuf owner, owner2, owner_ids, frontier;
    double psi_l = 0.0;
    int frontier_count = 0;  // frontier nodes the barrier fix-up re-steps after each step

    // gravity: buoyancy reference density (the mean density when rho_buoyancy <= 0)
    bool grav = false;
    double rho0 = 0.0;

    // two-component mode: the gas component's populations (same layout and cur as f) and the
    // FP64 densities of both components that the reported fields are formed from
    bool two = false;
    void* fv[2] = {nullptr, nullptr};
    DevBuf dens2;
    double tau_v = 1.0;

    // nuclei (Sec. 3.1) and agent budgets (Sec. 3)
    std::vector<double> cen, rad, rem, budget0;
    double rate = 0.0;
    std::vector<int64_t> nuc_node;
    std::vector<uint32_t> comp;
    std::vector<int> merge_parent, topo_parent;

    // last test pass
    std::vector<sc_bubble> bub;
    std::vector<std::vector<int>> bub_nuclei;
    bool have_labels = false;
    int64_t list_count = 0;

    // source schedule: add_host[s * nb + b], the mass bubble b's nuclei release at step s of the
    // current chunk
    std::vector<double> add_host;
    std::vector<double> rem_host;  // rem after each step of the chunk, [s * n + k]
    std::vector<char> step_active;
    int chunk_len = 0, chunk_pos = 0;

    // source ledger: released agent mass the storage has not taken yet.  On the device per
    // bubble slot of the last pass (owed, node count, gain: ledger_nb slots, slot b led
    // by nucleus ledger_lead[b]); on the host per nucleus for mass whose bubble is not fed
    DevBuf ledger;
    int ledger_nb = 0;
    std::vector<int> ledger_lead;
    std::vector<double> owed_nuc;
    uint64_t sr_key = 0;

    // the test pass on the device: bubble table, statistics and candidate pairs (btab, the
    // nucleus nodes in `nodes`, pairs in pair_buf / res_buf / pair_ab), read back through pinned
    // host memory (stage, stage_n nuclei; the merge groups are staged there too) with one
    // synchronization
    DevBuf btab, pair_ab;
    int btab_n = 0;  // nucleus count the table in btab is laid out for (its last pass)
    int pair_cap = 0;
    bool group_dirty = true;
    char* stage = nullptr;      // host address
    char* stage_dev = nullptr;  // the same memory as the device addresses it
    int stage_n = -1;

    // K-step blocks of a launch-bound box as HIP graphs: one executable per starting buffer
    // parity, valid while the captured arguments (graph_key) stay the same
    bool graphs = true;
    hipGraphExec_t graph_exec[2] = {nullptr, nullptr};
    std::vector<char> graph_key[2];
    // and the device part of the test pass that follows such a block (per parity)
    hipGraphExec_t pass_exec[2] = {nullptr, nullptr};
    std::vector<char> pass_key[2];

    std::vector<sc_merge_event> events;
    std::vector<sc_topo_event> topo;

    bool prof = false;
    std::vector<ProfRec> recs;
    std::vector<hipEvent_t> pool;
};

namespace {

void* dev_alloc(sc_sim* s, size_t bytes)
{
    if (bytes == 0) bytes = 256;
    if (s->has_alloc) return s->alloc.alloc(bytes, s->alloc.user);
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return p;
}

void dev_free(sc_sim* s, void* p)
{
    if (!p) return;
    if (s->has_alloc)
        s->alloc.free(p, s->alloc.user);
    else
        (void)hipFree(p);
}

int device_fail(sc_sim* s, hipError_t e, const char* what)
{
    s->latched = SC_E_DEVICE;
    return fail(SC_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIPX(call)                                                                               \
    do {                                                                                         \
        hipError_t e_ = (call);                                                                  \
        if (e_ != hipSuccess) return device_fail(s, e_, #call);                                  \
    } while (0)

int ensure(sc_sim* s, DevBuf& b, size_t bytes)
{
    if (b.bytes >= bytes && b.p) return SC_OK;
    if (b.p) {
        // the stream may still use the old buffer
        HIPX(hipStreamSynchronize(s->stream));
        dev_free(s, b.p);
        b.p = nullptr;
        b.bytes = 0;
    }
    b.p = dev_alloc(s, bytes);
    if (!b.p) return fail(SC_E_NOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed");
    b.bytes = bytes;
    return SC_OK;
}

#define TRY(expr)                                                                                \
    do {                                                                                         \
        int rc_ = (expr);                                                                        \
        if (rc_ != SC_OK) return rc_;                                                            \
    } while (0)

int check_usable(sc_sim* s)
{
    if (!s) return fail(SC_E_INVAL, "NULL simulation handle");
    if (s->latched)
        return fail(SC_E_STATE, "simulation latched by an earlier error (" +
                                    std::to_string(s->latched) + ")");
    return SC_OK;
}

FieldArgs field_args(const sc_sim* s)
{
    FieldArgs a;
    std::memset(&a, 0, sizeof(a));  // padding included: the graph cache compares the bytes
    a.nx = s->p.nx; a.ny = s->p.ny; a.nz = s->p.nz;
    a.N = s->N;
    a.G = (float)s->p.G;
    a.rho_ref = (float)s->rho_ref;
    a.Gd = s->p.G;
    a.rho_ref_d = s->rho_ref;
    a.theta = s->theta;
    a.owner = s->p.barrier ? (const uint16_t*)s->owner.p : nullptr;
    a.psi_ld = s->psi_l;
    a.grav = s->grav ? 1 : 0;
    for (int c = 0; c < 3; ++c) a.gd[c] = s->p.gravity[c];
    a.rho0d = s->rho0;
    a.f2 = s->two ? s->fv[s->cur] : nullptr;
    a.Gx = s->p.G_cross;
    a.rho_ref2 = s->rho_ref_v;
    return a;
}

Step2cArgs step2c_args(const sc_sim* s)
{
    Step2cArgs a;
    std::memset(&a, 0, sizeof(a));  // padding included: the graph cache compares the bytes
    a.nx = s->p.nx; a.ny = s->p.ny; a.nz = s->p.nz;
    a.N = s->N;
    a.planes = s->shape.tile_z;
    a.tau_l = s->p.tau;
    a.tau_v = s->tau_v;
    a.Gx = s->p.G_cross;
    a.ref_l = s->rho_ref;
    a.ref_v = s->rho_ref_v;
    return a;
}

StepArgs step_args(const sc_sim* s)
{
    StepArgs a;
    std::memset(&a, 0, sizeof(a));  // padding included: the graph cache compares the bytes
    a.nx = s->p.nx; a.ny = s->p.ny; a.nz = s->p.nz;
    a.planes = s->shape.tile_z;
    a.N = s->N;
    a.tau = (float)s->p.tau;
    a.omega = (float)(1.0 / s->p.tau);
    a.G = (float)s->p.G;
    a.rho_ref = (float)s->rho_ref;
    a.taud = s->p.tau;
    a.omegad = 1.0 / s->p.tau;
    a.Gd = s->p.G;
    a.rho_refd = s->rho_ref;
    a.owner = s->p.barrier ? (const uint16_t*)s->owner.p : nullptr;
    a.psi_l = (float)s->psi_l;
    a.psi_ld = s->psi_l;
    a.grav = s->grav ? 1 : 0;
    for (int c = 0; c < 3; ++c) {
        a.gd[c] = s->p.gravity[c];
        a.g[c] = (float)s->p.gravity[c];
    }
    a.rho0d = s->rho0;
    a.rho0 = (float)s->rho0;
    return a;
}

InitArgs init_args(const sc_sim* s, double rho)
{
    InitArgs a;
    a.nx = s->p.nx; a.ny = s->p.ny; a.nz = s->p.nz;
    a.N = s->N;
    a.rho = rho;
    a.amp = s->p.noise_amp;
    a.rho_ref = s->rho_ref;
    a.seed = s->p.noise_seed;
    return a;
}

// Arguments of the gas component's state kernels: its own storage shift.
InitArgs init_args_gas(const sc_sim* s, double rho)
{
    InitArgs a = init_args(s, rho);
    a.amp = 0.0;
    a.rho_ref = s->rho_ref_v;
    return a;
}

StepShape default_shape(const sc_params& p)
{
    StepShape sh;
    sh.variant = 1;
    if (p.lattice == SC_D2Q9) {
        sh.tile_x = p.nx >= 256 ? 256 : (p.nx >= 128 ? 128 : 64);
        sh.tile_y = 1;
        const int64_t tiles = (p.nx + sh.tile_x - 1) / sh.tile_x;
        int64_t planes = (tiles * p.ny + 2047) / 2048;  // about 2048 blocks
        sh.tile_z = (int)std::max<int64_t>(4, std::min<int64_t>(64, planes));
    } else {
        sh.tile_x = 32;
        sh.tile_y = 8;
        sh.tile_z = 16;
    }
    return sh;
}

// Shapes chosen by sc_autotune, per (lattice, nx, ny, nz, storage, compute, components), for
// this process.
using TuneKey = std::tuple<int, int, int, int, int, int, int>;
std::mutex g_tune_mu;
std::map<TuneKey, StepShape> g_tuned;

TuneKey tune_key(const sc_params& p, int compute)
{
    return TuneKey{p.lattice, p.nx, p.ny, p.nz, p.storage, compute, p.components};
}

std::vector<StepShape> tune_candidates(int q)
{
    std::vector<StepShape> c;
    if (q == SC_D2Q9) {
        for (int tx : {64, 128, 256, 512})
            for (int tz : {1, 2, 4, 8, 16, 32, 64})
                for (int v : {1, 3}) c.push_back(StepShape{tx, 1, tz, v});
    } else {
        const int tiles[][2] = {{32, 8}, {64, 4}, {64, 8}, {128, 4}, {128, 8}, {256, 4}};
        for (auto& t : tiles)
            for (int tz : {16, 32, 64, 128, 256, 512})
                for (int v : {1, 2, 3}) c.push_back(StepShape{t[0], t[1], tz, v});
    }
    return c;
}

std::vector<StepShape> tune_candidates_2c(int q)
{
    std::vector<StepShape> c;
    if (q == SC_D2Q9) {
        for (int tx : {64, 128, 256, 512})
            for (int tz : {2, 4, 8, 16, 32, 64})
                for (int v : {1, 3}) c.push_back(StepShape{tx, 1, tz, v});
    } else {
        const int tiles[][2] = {{32, 4}, {32, 8}, {64, 4}, {64, 8}, {128, 4}};
        for (auto& t : tiles)
            for (int tz : {16, 32, 64})
                for (int v : {1, 3, 4, 5}) c.push_back(StepShape{t[0], t[1], tz, v});
    }
    return c;
}

// Explicit tile and variant from the parameters, defaults filling the fields left at zero.
StepShape shape_from_params(const sc_params& p)
{
    StepShape sh = default_shape(p);
    if (p.tile_x) sh.tile_x = p.tile_x;
    if (p.tile_y) sh.tile_y = p.tile_y;
    if (p.lattice == SC_D2Q9) sh.tile_y = 1;
    if (p.tile_z) sh.tile_z = p.tile_z;
    if (p.step_variant) sh.variant = p.step_variant;
    return sh;
}

int prof_begin(sc_sim* s, int cls, hipEvent_t* out_b)
{
    *out_b = nullptr;
    if (!s->prof) return SC_OK;
    ProfRec r;
    r.cls = cls;
    for (hipEvent_t* e : {&r.a, &r.b}) {
        if (!s->pool.empty()) {
            *e = s->pool.back();
            s->pool.pop_back();
        } else {
            // timing only: no system-scope fence (cache writeback) at each record, which
            // would cost every profiled launch several microseconds
            HIPX(hipEventCreateWithFlags(e, hipEventDisableSystemFence));
        }
    }
    HIPX(hipEventRecord(r.a, s->stream));
    s->recs.push_back(r);
    *out_b = r.b;
    return SC_OK;
}

int prof_end(sc_sim* s, hipEvent_t b)
{
    if (!s->prof || !b) return SC_OK;
    HIPX(hipEventRecord(b, s->stream));
    return SC_OK;
}

// ---- FP64 bookkeeping of the registry (identical arithmetic to the method statement) ---------
int uf_find(std::vector<int>& parent, int k)
{
    while (parent[k] != k) k = parent[k];
    return k;
}

double min_image(double d, int n) { return d - n * std::floor(d / n + 0.5); }

int64_t nearest_node(const sc_sim* s, const double* c)
{
    auto wrapi = [](int a, int n) {
        int r = a % n;
        return r < 0 ? r + n : r;
    };
    const int x = wrapi((int)std::floor(c[0] + 0.5), s->p.nx);
    const int y = wrapi((int)std::floor(c[1] + 0.5), s->p.ny);
    const int z = (s->d == 3) ? wrapi((int)std::floor(c[2] + 0.5), s->p.nz) : 0;
    return (int64_t)x + (int64_t)s->p.nx * ((int64_t)y + (int64_t)s->p.ny * z);
}

// Source schedule for the next `len` steps: bubbles frozen, budgets spent in nucleus order.
void build_schedule(sc_sim* s, int len)
{
#pragma clang fp contract(off)
    const int nb = (int)s->bub.size();
    const int n = (int)s->rem.size();
    s->chunk_len = len;
    s->chunk_pos = 0;
    s->add_host.assign((size_t)len * std::max(nb, 1), 0.0);
    s->rem_host.assign((size_t)len * std::max(n, 1), 0.0);
    s->step_active.assign((size_t)len, 0);
    std::vector<double> rem = s->rem;
    for (int st = 0; st < len; ++st) {
        if (s->rate > 0.0) {
            for (int b = 0; b < nb; ++b) {
                double dm = 0.0;
                for (int k : s->bub_nuclei[b]) {
                    const double dk = rem[k] < s->rate ? rem[k] : s->rate;
                    dm += dk;
                    rem[k] -= dk;
                }
                s->add_host[(size_t)st * nb + b] = dm;
                if (dm != 0.0) s->step_active[st] = 1;
            }
        }
        for (int k = 0; k < n; ++k) s->rem_host[(size_t)st * n + k] = rem[k];
    }
}

int upload_schedule(sc_sim* s)
{
    const int nb = (int)s->bub.size();
    if (nb == 0 || s->chunk_len == 0 || !(s->rate > 0.0)) return SC_OK;
    const size_t bytes = sizeof(double) * (size_t)s->chunk_len * nb;
    TRY(ensure(s, s->add_tab, bytes));
    HIPX(hipMemcpyAsync(s->add_tab.p, s->add_host.data(), bytes, hipMemcpyHostToDevice,
                        s->stream));
    HIPX(hipStreamSynchronize(s->stream));
    return SC_OK;
}

// Ledger slots of this pass's bubbles: a fed bubble takes over what its nuclei are owed; an
// unfed one leaves it with them.  Device layout: owed[nb], nodes[nb], then gain (zero) with one
// 128-byte line per bubble.
int ledger_setup(sc_sim* s, const std::vector<int32_t>& feed)
{
#pragma clang fp contract(off)
    const int nb = (int)s->bub.size();
    s->ledger_nb = nb;
    s->ledger_lead.assign((size_t)nb, -1);
    if (nb == 0) return SC_OK;
    std::vector<double> host((size_t)(2 + kLedgerGainStride) * nb, 0.0);
    for (int b = 0; b < nb; ++b) {
        s->ledger_lead[b] = s->bub[b].nucleus;
        host[(size_t)nb + b] = (double)s->bub[b].n;
        if (!feed[b]) continue;
        double o = 0.0;
        for (int k : s->bub_nuclei[b]) {
            o += s->owed_nuc[k];
            s->owed_nuc[k] = 0.0;
        }
        host[b] = o;
    }
    TRY(ensure(s, s->ledger, sizeof(double) * host.size()));
    HIPX(hipMemcpyAsync(s->ledger.p, host.data(), sizeof(double) * host.size(),
                        hipMemcpyHostToDevice, s->stream));
    HIPX(hipStreamSynchronize(s->stream));  // the staging vector lives on the host stack
    return SC_OK;
}

SourceLedger ledger_view(sc_sim* s, int step_in_chunk)
{
    const int nb = s->ledger_nb;
    SourceLedger led;
    led.dm = (const double*)s->add_tab.p + (size_t)step_in_chunk * nb;
    led.owed = (double*)s->ledger.p;
    led.nodes = led.owed + nb;
    led.gain = (unsigned long long*)(led.owed + 2 * (size_t)nb);
    led.nb = nb;
    led.key = s->sr_key;
    return led;
}

int schedule_chunk_len(const sc_sim* s)
{
    return s->p.test_every > 0 ? s->p.test_every : 1024;
}

// ---- test pass (Fig. 1 step 7; Sec. 3.1 eta_m) ------------------------------------------------
// With tot_host (and no caller mask) the FP64 totals come from the same sweep of populations as
// the mask; the gas component's, with two components, are added from a sweep of its own.  With
// defer, the totals' copy is only queued: the caller synchronizes the stream and adds the gas
// component's totals itself.
int gas_totals_add(sc_sim* s, double out[4]);
int gas_totals_queue(sc_sim* s);
int totals_now(sc_sim* s, double out[4]);

int label_current(sc_sim* s, uint32_t* labels_d, uint32_t* ncomp_host, const uint8_t* mask_host,
                  double* tot_host = nullptr, bool defer = false, bool copy_tot = true)
{
    const FieldArgs fa = field_args(s);
    TRY(ensure(s, s->parent, sizeof(uint32_t) * (size_t)s->N));
    TRY(ensure(s, s->small, 4096));
    double* out_d = (double*)s->small.p;
    if (tot_host && !mask_host) {
        TRY(ensure(s, s->partials, sizeof(double) * 4 * (size_t)totals_blocks(s->N)));
        HIPX(launch_mask_totals(s->q, s->p.storage, s->f[s->cur], (uint32_t*)s->parent.p,
                                (double*)s->partials.p, out_d, fa, s->stream));
    } else if (mask_host) {
        TRY(ensure(s, s->mask8, (size_t)s->N));
        HIPX(hipMemcpyAsync(s->mask8.p, mask_host, (size_t)s->N, hipMemcpyHostToDevice,
                            s->stream));
        HIPX(launch_mask_from_bytes((const uint8_t*)s->mask8.p, (uint32_t*)s->parent.p, s->N,
                                    s->stream));
    } else {
        HIPX(launch_mask_from_rho(s->q, s->p.storage, s->f[s->cur], (uint32_t*)s->parent.p, fa,
                                  s->stream));
    }
    uint32_t* ncomp_d = (uint32_t*)((char*)s->small.p + 64);
    HIPX(launch_union(s->q, (uint32_t*)s->parent.p, ncomp_d, fa, s->stream));
    HIPX(launch_flatten((uint32_t*)s->parent.p, labels_d, ncomp_d, s->N, s->stream));
    if (ncomp_host)
        HIPX(hipMemcpyAsync(ncomp_host, ncomp_d, sizeof(uint32_t), hipMemcpyDeviceToHost,
                            s->stream));
    if (tot_host && !mask_host && copy_tot)
        HIPX(hipMemcpyAsync(tot_host, out_d, 4 * sizeof(double), hipMemcpyDeviceToHost,
                            s->stream));
    if (ncomp_host || (tot_host && !defer)) HIPX(hipStreamSynchronize(s->stream));
    if (tot_host && !mask_host && s->two && !defer) TRY(gas_totals_add(s, tot_host));
    if (tot_host && mask_host) TRY(totals_now(s, tot_host));
    return SC_OK;
}

int totals_now(sc_sim* s, double out[4])
{
    const FieldArgs fa = field_args(s);
    TRY(ensure(s, s->partials, sizeof(double) * 4 * (size_t)totals_blocks(s->N)));
    TRY(ensure(s, s->small, 4096));
    double* out_d = (double*)s->small.p;
    HIPX(launch_totals(s->q, s->p.storage, s->f[s->cur], (double*)s->partials.p, out_d, fa,
                       s->stream));
    HIPX(hipMemcpyAsync(out, out_d, 4 * sizeof(double), hipMemcpyDeviceToHost, s->stream));
    HIPX(hipStreamSynchronize(s->stream));
    if (s->two) TRY(gas_totals_add(s, out));  // the mixture's totals: both components
    return SC_OK;
}

// The gas component's FP64 totals, queued into the device slot small + 64 bytes (read back by the
// test pass's stage-out kernel).
int gas_totals_queue(sc_sim* s)
{
    FieldArgs fg = field_args(s);
    fg.rho_ref_d = s->rho_ref_v;
    fg.rho_ref = (float)s->rho_ref_v;
    TRY(ensure(s, s->partials, sizeof(double) * 4 * (size_t)totals_blocks(s->N)));
    TRY(ensure(s, s->small, 4096));
    double* out_d = (double*)s->small.p + 8;
    HIPX(launch_totals(s->q, s->p.storage, s->fv[s->cur], (double*)s->partials.p, out_d, fg,
                       s->stream));
    return SC_OK;
}

int gas_totals_add(sc_sim* s, double out[4])
{
    FieldArgs fg = field_args(s);
    fg.rho_ref_d = s->rho_ref_v;
    fg.rho_ref = (float)s->rho_ref_v;
    TRY(ensure(s, s->partials, sizeof(double) * 4 * (size_t)totals_blocks(s->N)));
    TRY(ensure(s, s->small, 4096));
    double* out_d = (double*)s->small.p;
    double gas[4];
    HIPX(launch_totals(s->q, s->p.storage, s->fv[s->cur], (double*)s->partials.p, out_d, fg,
                       s->stream));
    HIPX(hipMemcpyAsync(gas, out_d, 4 * sizeof(double), hipMemcpyDeviceToHost, s->stream));
    HIPX(hipStreamSynchronize(s->stream));
    for (int c = 0; c < 4; ++c) out[c] += gas[c];
    return SC_OK;
}

// Owner field of the barrier after this pass's merges (Sec. 3.1, Fig. 1 steps 3-6): every
// bubble's gas nodes carry 1 + the smallest nucleus index of the criterion-merged groups of its
// nuclei, then `corona` layers grow into the liquid, a free node taking the smallest id among
// its lattice neighbours.  The layers alternate between two buffers and the seed goes to the one
// that makes the last layer land in s->owner, whose address the kernels keep.  Then the frontier
// nodes (owned, next to another bubble's node: the only ones whose force the barrier changes)
// are listed for the fix-up that follows every step until the next pass.
int build_owner(sc_sim* s, int nb)
{
    const FieldArgs fa = field_args(s);
    const int r = s->p.corona;
    uint16_t* bufs[2] = {(uint16_t*)s->owner.p, (uint16_t*)s->owner2.p};
    int cur = r % 2;
    const uint16_t* ids_d = nullptr;
    if (nb > 0) {
        std::vector<uint16_t> ids((size_t)nb);
        for (int b = 0; b < nb; ++b) {
            int m = -1;
            for (int k : s->bub_nuclei[b]) {
                const int g = uf_find(s->merge_parent, k);
                if (m < 0 || g < m) m = g;
            }
            ids[b] = (uint16_t)(1 + m);
        }
        TRY(ensure(s, s->owner_ids, sizeof(uint16_t) * (size_t)nb));
        HIPX(hipMemcpyAsync(s->owner_ids.p, ids.data(), sizeof(uint16_t) * nb,
                            hipMemcpyHostToDevice, s->stream));
        HIPX(hipStreamSynchronize(s->stream));  // ids lives on the host stack
        ids_d = (const uint16_t*)s->owner_ids.p;
    }
    HIPX(launch_owner_seed((const uint32_t*)s->labels.p, nb > 0 ? (const int32_t*)s->slots.p : nullptr,
                           ids_d, nb, bufs[cur], s->N, s->stream));
    for (int k = 0; k < r; ++k) {
        HIPX(launch_owner_grow(s->q, bufs[cur], bufs[cur ^ 1], fa, s->stream));
        cur ^= 1;
    }
    s->frontier_count = 0;
    if (nb < 2) return SC_OK;  // one bubble or none: no node can see another bubble
    TRY(ensure(s, s->frontier, sizeof(uint32_t) * (size_t)s->N));
    TRY(ensure(s, s->small, 4096));
    unsigned int* cnt_d = (unsigned int*)((char*)s->small.p + 192);
    HIPX(launch_fill_i32((int32_t*)cnt_d, 0, 1, s->stream));
    HIPX(launch_frontier_list(s->q, (const uint16_t*)s->owner.p, (uint32_t*)s->frontier.p, cnt_d,
                              fa, s->stream));
    unsigned int got = 0;
    HIPX(hipMemcpyAsync(&got, cnt_d, sizeof(got), hipMemcpyDeviceToHost, s->stream));
    HIPX(hipStreamSynchronize(s->stream));
    s->frontier_count = (int)got;
    return SC_OK;
}

// Buoyancy reference: the given density, or the mean density M/N of the box as it stands (at
// creation and again when nuclei are seeded).
int set_rho0(sc_sim* s)
{
    if (s->p.rho_buoyancy > 0.0) {
        s->rho0 = s->p.rho_buoyancy;
        return SC_OK;
    }
    double tot[4];
    TRY(totals_now(s, tot));
    s->rho0 = tot[0] / (double)s->N;
    return SC_OK;
}

// Pinned host memory the test pass reads back into: the FP64 totals (both components), the
// bubble table's head, the nucleus labels, the statistics, the ledger of the last pass, the first
// kStagePairs candidate pairs with their merge results, and the merge groups it uploads.
constexpr int kStagePairs = 64;
struct Stage {
    double* tot;        // [8]: liquid (or only) component, then the gas component
    int32_t* head;      // [16]
    uint32_t* comp;     // [n]
    unsigned long long* count;  // [n]
    unsigned long long* sums;   // [3n]
    double* owed;       // [n]
    MergePair* pairs;   // [kStagePairs]
    int32_t* ab;        // [2 kStagePairs]
    MergeResult* res;   // [kStagePairs]
    int32_t* group;     // [n]
};

size_t stage_bytes(int n)
{
    const size_t m = (size_t)(n > 0 ? n : 1);
    auto al = [](size_t b) { return (b + 63) & ~size_t(63); };
    return al(64) + al(64) + al(4 * m) + al(8 * m) + al(24 * m) + al(8 * m) +
           al(sizeof(MergePair) * kStagePairs) + al(8 * kStagePairs) +
           al(sizeof(MergeResult) * kStagePairs) + al(4 * m);
}

Stage stage_view(char* p, int n)
{
    const size_t m = (size_t)(n > 0 ? n : 1);
    auto al = [](size_t b) { return (b + 63) & ~size_t(63); };
    Stage st;
    st.tot = (double*)p; p += al(64);
    st.head = (int32_t*)p; p += al(64);
    st.comp = (uint32_t*)p; p += al(4 * m);
    st.count = (unsigned long long*)p; p += al(8 * m);
    st.sums = (unsigned long long*)p; p += al(24 * m);
    st.owed = (double*)p; p += al(8 * m);
    st.pairs = (MergePair*)p; p += al(sizeof(MergePair) * kStagePairs);
    st.ab = (int32_t*)p; p += al(8 * kStagePairs);
    st.res = (MergeResult*)p; p += al(sizeof(MergeResult) * kStagePairs);
    st.group = (int32_t*)p;
    return st;
}

int ensure_stage(sc_sim* s, int n)
{
    if (s->stage && s->stage_n >= n) return SC_OK;
    if (s->stage) {
        HIPX(hipStreamSynchronize(s->stream));
        (void)hipHostFree(s->stage);
        s->stage = nullptr;
    }
    void* p = nullptr;
    if (hipHostMalloc(&p, stage_bytes(n), hipHostMallocDefault) != hipSuccess || !p) {
        (void)hipGetLastError();
        return fail(SC_E_NOMEM, "pinned host staging of the test pass");
    }
    void* d = nullptr;
    if (hipHostGetDevicePointer(&d, p, 0) != hipSuccess || !d) {
        (void)hipGetLastError();
        (void)hipHostFree(p);
        return fail(SC_E_DEVICE, "device address of the pinned staging");
    }
    s->stage = (char*)p;
    s->stage_dev = (char*)d;
    s->stage_n = n;
    s->group_dirty = true;
    return SC_OK;
}

// The test pass in three parts.  pass_prepare allocates what the pass needs and stages the merge
// groups; pass_enqueue queues every kernel and copy up to the pass's one synchronization (no
// allocation, no host read of device data, so it can be captured in a graph); pass_finish
// synchronizes and runs the host registry on what came back.
int pass_prepare(sc_sim* s, bool with_criterion)
{
    const int n = (int)s->rad.size();
    TRY(ensure_stage(s, n));
    TRY(ensure(s, s->labels, sizeof(uint32_t) * (size_t)s->N));
    TRY(ensure(s, s->parent, sizeof(uint32_t) * (size_t)s->N));
    TRY(ensure(s, s->small, 4096));
    TRY(ensure(s, s->partials, sizeof(double) * 4 * (size_t)totals_blocks(s->N)));
    if (n > 0) {
        if (!s->slots_ready) {
            TRY(ensure(s, s->slots, sizeof(int32_t) * (size_t)s->N));
            HIPX(launch_fill_i32((int32_t*)s->slots.p, -1, s->N, s->stream));
            s->slots_ready = true;
        }
        if (!s->btab.p || s->btab.bytes < bubble_tab_bytes(n)) {
            // a new table buffer: the old table's bubbles leave the slot map now, and the new
            // head starts at zero bubbles
            if (s->btab.p) {
                const BubbleTab old = bubble_tab_view(s->btab.p, s->btab_n);
                HIPX(launch_bubble_table((const uint32_t*)s->labels.p, (const int64_t*)s->nodes.p,
                                         0, old, old, (int32_t*)s->slots.p, field_args(s),
                                         s->stream));
                HIPX(hipStreamSynchronize(s->stream));
            }
            TRY(ensure(s, s->btab, bubble_tab_bytes(n)));
            HIPX(launch_fill_i32((int32_t*)s->btab.p, 0, 16, s->stream));
            s->btab_n = n;
        }
        if (with_criterion && n >= 2) {
            const Stage st = stage_view(s->stage, n);
            if (s->group_dirty) {
                for (int k = 0; k < n; ++k) st.group[k] = uf_find(s->merge_parent, k);
                s->group_dirty = false;
            }
            const int cap = std::max(kStagePairs, s->pair_cap);
            TRY(ensure(s, s->pair_buf, sizeof(MergePair) * (size_t)cap));
            TRY(ensure(s, s->res_buf, sizeof(MergeResult) * (size_t)cap));
            TRY(ensure(s, s->pair_ab, sizeof(int32_t) * 2 * (size_t)cap));
        }
    }
    return SC_OK;
}

int pass_enqueue(sc_sim* s, bool with_criterion)
{
    const FieldArgs fa = field_args(s);
    const int n = (int)s->rad.size();
    const Stage st = stage_view(s->stage, n);

    const Stage sd = stage_view(s->stage_dev, n);  // the staging as the device addresses it
    StageOut o{};
    o.dst_tot = sd.tot; o.dst_head = sd.head; o.dst_comp = sd.comp; o.dst_count = sd.count;
    o.dst_sums = sd.sums; o.dst_owed = sd.owed; o.dst_pairs = sd.pairs; o.dst_ab = sd.ab;
    o.dst_res = sd.res;

    // 1. gas mask, labels and FP64 totals
    TRY(label_current(s, (uint32_t*)s->labels.p, nullptr, nullptr, st.tot, true, false));
    o.tot = (const double*)s->small.p;
    if (s->two) {
        TRY(gas_totals_queue(s));
        o.tot2 = (const double*)s->small.p + 8;
    }

    // 2. on the device: nucleus labels, the bubble table, statistics and, with the criterion,
    // the candidate pairs' merge test; then the read-back (one block does the tail)
    BubbleTab t{};
    bool do_pairs = false;
    int pair_cap = 0;
    if (n > 0) {
        t = bubble_tab_view(s->btab.p, n);
        const BubbleTab prev = bubble_tab_view(s->btab.p, s->btab_n);
        HIPX(launch_bubble_table((const uint32_t*)s->labels.p, (const int64_t*)s->nodes.p, n,
                                 prev, t, (int32_t*)s->slots.p, fa, s->stream));
        HIPX(launch_stats((const uint32_t*)s->labels.p, (const int32_t*)s->slots.p, t.anchors,
                          t.count, t.sums, fa, s->stream));
        if (with_criterion && n >= 2) {
            do_pairs = true;
            pair_cap = std::max(kStagePairs, s->pair_cap);
            o.pairs = (const MergePair*)s->pair_buf.p;
            o.ab = (const int32_t*)s->pair_ab.p;
            o.res = (const MergeResult*)s->res_buf.p;
            o.npairs = kStagePairs;
        }
        o.head = t.head;
        o.comp = t.comp;
        o.count = t.count;
        o.sums = t.sums;
        o.n = n;
    }
    // the source ledger of the last pass's bubbles, handed back to the nuclei that led them
    o.owed = (const double*)s->ledger.p;
    o.ledger_nb = s->ledger_nb;
    // the merge groups are read where the host staged them (pinned memory)
    HIPX(launch_pass_tail(s->q, s->p.storage, t, sd.group, s->p.film_max,
                          (MergePair*)s->pair_buf.p, (int32_t*)s->pair_ab.p,
                          (MergeResult*)s->res_buf.p, pair_cap, do_pairs ? 1 : 0, o,
                          s->f[s->cur], (const uint32_t*)s->labels.p, fa, s->stream));
    return SC_OK;
}

int pass_finish(sc_sim* s, bool with_criterion)
{
#pragma clang fp contract(off)
    const FieldArgs fa = field_args(s);
    const int n = (int)s->rad.size();
    const Stage st = stage_view(s->stage, n);
    const int ledger_nb = s->ledger_nb;
    int pair_cap = (with_criterion && n >= 2) ? std::max(kStagePairs, s->pair_cap) : 0;
    const BubbleTab t = n > 0 ? bubble_tab_view(s->btab.p, n) : BubbleTab{};
    s->have_labels = true;
    HIPX(hipStreamSynchronize(s->stream));

    for (int b = 0; b < ledger_nb; ++b)
        if (st.owed[b] != 0.0) s->owed_nuc[(size_t)s->ledger_lead[b]] += st.owed[b];
    s->ledger_nb = 0;
    double tot[4];
    for (int c = 0; c < 4; ++c) tot[c] = st.tot[c] + (s->two ? st.tot[4 + c] : 0.0);
    for (int c = 0; c < 4; ++c) s->pass_tot[c] = tot[c];
    const bool finite = std::isfinite(tot[0]) && std::isfinite(tot[1]) &&
                        std::isfinite(tot[2]) && std::isfinite(tot[3]);

    // 3. the host's registry from the nucleus labels: bubbles = distinct nonzero labels held by
    // nuclei, ascending, each led by its smallest nucleus (the device table follows the same
    // rules; its statistics are read by bubble index)
    s->comp.assign(st.comp, st.comp + n);
    std::vector<uint32_t> distinct;
    for (int k = 0; k < n; ++k)
        if (s->comp[k]) distinct.push_back(s->comp[k]);
    std::sort(distinct.begin(), distinct.end());
    distinct.erase(std::unique(distinct.begin(), distinct.end()), distinct.end());
    const int nb = (int)distinct.size();
    if (n > 0 && st.head[0] != nb) {
        s->latched = SC_E_STATE;
        return fail(SC_E_STATE, "device bubble table disagrees with the nucleus labels");
    }
    s->bub.assign((size_t)nb, sc_bubble{});
    s->bub_nuclei.assign((size_t)nb, std::vector<int>());
    for (int b = 0; b < nb; ++b) {
        s->bub[b].label = distinct[b];
        s->bub[b].nucleus = -1;
    }
    for (int k = 0; k < n; ++k) {
        if (!s->comp[k]) continue;
        const int b = (int)(std::lower_bound(distinct.begin(), distinct.end(), s->comp[k]) -
                            distinct.begin());
        if (s->bub[b].nucleus < 0) s->bub[b].nucleus = k;
        s->bub[b].n_nuclei++;
        s->bub_nuclei[b].push_back(k);
    }
    for (int b = 0; b < nb; ++b) {
        sc_bubble& B = s->bub[b];
        const int64_t a0 = s->nuc_node[B.nucleus];
        const int64_t anchor[3] = {a0 % s->p.nx, (a0 / s->p.nx) % s->p.ny,
                                   a0 / ((int64_t)s->p.nx * s->p.ny)};
        B.n = (int64_t)st.count[b];
        for (int c = 0; c < 3; ++c)
            B.centroid[c] = (double)anchor[c] + (double)(int64_t)st.sums[3 * b + c] / (double)B.n;
        if (s->d == 2) {
            B.centroid[2] = 0.0;
            B.radius = std::sqrt((double)B.n / M_PI);
        } else {
            B.radius = std::cbrt(3.0 * (double)B.n / (4.0 * M_PI));
        }
    }

    // 4. gas-node list of the bubbles the source feeds until the next pass
    s->list_count = 0;
    if (nb > 0) {
        std::vector<int32_t> feed((size_t)nb, 0);
        int64_t cap = 0;
        if (s->rate > 0.0) {
            for (int b = 0; b < nb; ++b) {
                for (int k : s->bub_nuclei[b])
                    if (s->rem[k] > 0.0) feed[b] = 1;
                if (feed[b]) cap += s->bub[b].n;
            }
        }
        if (cap > 0) {
            TRY(ensure(s, s->bub_tab, sizeof(int32_t) * (size_t)nb));
            HIPX(hipMemcpyAsync(s->bub_tab.p, feed.data(), sizeof(int32_t) * nb,
                                hipMemcpyHostToDevice, s->stream));
            TRY(ensure(s, s->list_node, sizeof(uint32_t) * (size_t)cap));
            TRY(ensure(s, s->list_slot, sizeof(int32_t) * (size_t)cap));
            TRY(ensure(s, s->small, 4096));
            unsigned int* cnt_d = (unsigned int*)((char*)s->small.p + 128);
            HIPX(launch_fill_i32((int32_t*)cnt_d, 0, 1, s->stream));
            TRY(ensure(s, s->list_scan, sizeof(uint32_t) * (size_t)gas_list_scratch_words()));
            HIPX(launch_gas_list((const uint32_t*)s->labels.p, (const int32_t*)s->slots.p,
                                 (const int32_t*)s->bub_tab.p, (uint32_t*)s->list_node.p,
                                 (int32_t*)s->list_slot.p, cnt_d, (unsigned int*)s->list_scan.p,
                                 s->N, s->stream));
            unsigned int got = 0;
            HIPX(hipMemcpyAsync(&got, cnt_d, sizeof(got), hipMemcpyDeviceToHost, s->stream));
            HIPX(hipStreamSynchronize(s->stream));
            s->list_count = got;
        }
        if (s->rate > 0.0) TRY(ledger_setup(s, feed));
    }

    // 5. topological merges: nuclei of one component join one group (smallest index leads)
    for (int b = 0; b < nb; ++b) {
        const int k0 = s->bub[b].nucleus;
        for (int k : s->bub_nuclei[b]) {
            if (k == k0) continue;
            const int ra = uf_find(s->topo_parent, k0), rb = uf_find(s->topo_parent, k);
            if (ra == rb) continue;
            sc_topo_event te;
            te.step = s->t;
            te.nucleus_a = std::min(ra, rb);
            te.nucleus_b = std::max(ra, rb);
            s->topo.push_back(te);
            s->topo_parent[te.nucleus_b] = te.nucleus_a;
        }
    }

    // 6. merge criterion on candidate pairs (pairs in label order, state of the pass start).
    // The host forms the pairs exactly as before; the device has already walked every film of
    // a superset of them, and each pair's result is taken from there after checking that the
    // device formed the identical pair (centroid, offset and sample count).
    if (with_criterion && nb >= 2) {
        int found = st.head[1];
        const MergePair* dev_pairs = st.pairs;
        const int32_t* dev_ab = st.ab;
        const MergeResult* dev_res = st.res;
        std::vector<MergePair> more_pairs;
        std::vector<int32_t> more_ab;
        std::vector<MergeResult> more_res;
        if (found > pair_cap) {  // grow the buffers and walk them all again on the device
            s->pair_cap = found;
            pair_cap = found;
            TRY(ensure(s, s->pair_buf, sizeof(MergePair) * (size_t)pair_cap));
            TRY(ensure(s, s->res_buf, sizeof(MergeResult) * (size_t)pair_cap));
            TRY(ensure(s, s->pair_ab, sizeof(int32_t) * 2 * (size_t)pair_cap));
            HIPX(launch_fill_i32(t.head + 1, 0, 1, s->stream));  // the pair count starts over
            HIPX(launch_pairs(t, stage_view(s->stage_dev, n).group, s->d, s->p.film_max,
                              (MergePair*)s->pair_buf.p, (int32_t*)s->pair_ab.p, pair_cap, fa,
                              s->stream));
            HIPX(launch_merge_counted(s->q, s->p.storage, s->f[s->cur],
                                      (const uint32_t*)s->labels.p,
                                      (const MergePair*)s->pair_buf.p,
                                      (MergeResult*)s->res_buf.p, pair_cap, t.head + 1,
                                      s->p.film_max, fa, s->stream));
        }
        if (found > kStagePairs) {
            more_pairs.resize((size_t)found);
            more_ab.resize(2 * (size_t)found);
            more_res.resize((size_t)found);
            HIPX(hipMemcpyAsync(more_pairs.data(), s->pair_buf.p, sizeof(MergePair) * found,
                                hipMemcpyDeviceToHost, s->stream));
            HIPX(hipMemcpyAsync(more_ab.data(), s->pair_ab.p, sizeof(int32_t) * 2 * found,
                                hipMemcpyDeviceToHost, s->stream));
            HIPX(hipMemcpyAsync(more_res.data(), s->res_buf.p, sizeof(MergeResult) * found,
                                hipMemcpyDeviceToHost, s->stream));
            HIPX(hipStreamSynchronize(s->stream));
            dev_pairs = more_pairs.data();
            dev_ab = more_ab.data();
            dev_res = more_res.data();
        }
        std::map<std::pair<int, int>, int> at;
        for (int k = 0; k < found; ++k) at[{dev_ab[2 * k], dev_ab[2 * k + 1]}] = k;
        std::vector<std::pair<int, int>> fired;
        for (int a = 0; a < nb; ++a) {
            for (int b = a + 1; b < nb; ++b) {
                const sc_bubble& A = s->bub[a];
                const sc_bubble& B = s->bub[b];
                if (uf_find(s->merge_parent, A.nucleus) == uf_find(s->merge_parent, B.nucleus))
                    continue;
                double dv[3];
                dv[0] = min_image(B.centroid[0] - A.centroid[0], s->p.nx);
                dv[1] = min_image(B.centroid[1] - A.centroid[1], s->p.ny);
                dv[2] = (s->d == 3) ? min_image(B.centroid[2] - A.centroid[2], s->p.nz) : 0.0;
                const double dist = std::sqrt(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
                if (dist > A.radius + B.radius + (double)s->p.film_max) continue;
                const int T = (int)std::ceil(dist);
                if (T <= 0) continue;
                const auto it = at.find({a, b});
                bool same = it != at.end();
                if (same) {
                    const MergePair& dp = dev_pairs[it->second];
                    same = dp.T == T && dp.label_a == A.label && dp.label_b == B.label;
                    for (int c = 0; c < 3; ++c)
                        same = same && dp.cen_a[c] == A.centroid[c] && dp.dv[c] == dv[c];
                }
                if (!same) {
                    s->latched = SC_E_STATE;
                    return fail(SC_E_STATE, "device merge pair differs from the registry's");
                }
                const MergeResult& r = dev_res[it->second];
                if (!r.fired) continue;
                sc_merge_event e;
                std::memset(&e, 0, sizeof(e));
                e.step = s->t;
                e.nucleus_a = A.nucleus;
                e.nucleus_b = B.nucleus;
                e.label_a = A.label;
                e.label_b = B.label;
                e.film_node = r.film_node;
                e.film_len = r.film_len;
                e.lap_p = r.lap_p;
                e.rho_film = r.rho_film;
                s->events.push_back(e);
                fired.emplace_back(A.nucleus, B.nucleus);
            }
        }
        // eta_m: 1 -> 0, applied after every pair was tested
        for (auto& pr : fired) {
            const int ra = uf_find(s->merge_parent, pr.first);
            const int rb = uf_find(s->merge_parent, pr.second);
            if (ra == rb) continue;
            if (ra < rb) s->merge_parent[rb] = ra; else s->merge_parent[ra] = rb;
            s->group_dirty = true;
        }
    }

    if (s->p.barrier) TRY(build_owner(s, nb));
    // (the slot map keeps this pass's bubbles until the next pass's bubble table clears them)
    if (n > 0) s->btab_n = n;

    build_schedule(s, schedule_chunk_len(s));
    if (s->rate > 0.0) TRY(upload_schedule(s));
    if (!finite) {
        s->latched = SC_E_NUMERIC;
        return fail(SC_E_NUMERIC, "non-finite FP64 total at step " + std::to_string(s->t));
    }
    return SC_OK;
}

int test_pass(sc_sim* s, bool with_criterion)
{
    hipEvent_t pe;
    TRY(prof_begin(s, SC_KERNEL_TEST, &pe));
    TRY(pass_prepare(s, with_criterion));
    TRY(pass_enqueue(s, with_criterion));
    const int rc = pass_finish(s, with_criterion);
    TRY(prof_end(s, pe));
    return rc;
}

int validate(const sc_params* p)
{
    if (!p) return fail(SC_E_INVAL, "NULL parameters");
    if (p->abi_version != SC_ABI_VERSION) return fail(SC_E_INVAL, "abi_version mismatch");
    if (p->lattice != SC_D2Q9 && p->lattice != SC_D3Q19) return fail(SC_E_INVAL, "lattice must be 9 or 19");
    if (p->nx < 4 || p->ny < 4) return fail(SC_E_INVAL, "nx and ny must be >= 4");
    if (p->lattice == SC_D2Q9 && p->nz != 1) return fail(SC_E_INVAL, "D2Q9 needs nz == 1");
    if (p->lattice == SC_D3Q19 && p->nz < 4) return fail(SC_E_INVAL, "D3Q19 needs nz >= 4");
    const double N = (double)p->nx * p->ny * p->nz;
    if (N > 2147483000.0) return fail(SC_E_INVAL, "box larger than 2^31 nodes");
    if (!(p->tau > 0.5) || !std::isfinite(p->tau)) return fail(SC_E_INVAL, "tau must be > 0.5");
    if (!std::isfinite(p->G)) return fail(SC_E_INVAL, "G must be finite");
    if (!(p->rho_liquid > 0.0) || !std::isfinite(p->rho_liquid)) return fail(SC_E_INVAL, "rho_liquid must be > 0");
    if (!(p->rho_gas > 0.0) || !std::isfinite(p->rho_gas)) return fail(SC_E_INVAL, "rho_gas must be > 0");
    if (!(p->noise_amp >= 0.0) || !std::isfinite(p->noise_amp)) return fail(SC_E_INVAL, "noise_amp must be >= 0");
    if (!std::isfinite(p->gas_threshold)) return fail(SC_E_INVAL, "gas_threshold must be finite");
    if (p->test_every < 0) return fail(SC_E_INVAL, "test_every must be >= 0");
    if (p->film_max < 1) return fail(SC_E_INVAL, "film_max must be >= 1");
    if (p->storage < SC_STORE_F32 || p->storage > SC_STORE_BF16) return fail(SC_E_INVAL, "unknown storage");
    // the step kernels address a population array with 32-bit byte offsets
    if (N * (double)storage_bytes(p->storage) > 4294967296.0)
        return fail(SC_E_INVAL, "box too large: nodes x bytes per stored value must be <= 2^32");
    if (p->compute < SC_COMPUTE_AUTO || p->compute > SC_COMPUTE_F64) return fail(SC_E_INVAL, "unknown compute type");
    if (p->compute == SC_COMPUTE_F64 && p->storage != SC_STORE_F32)
        return fail(SC_E_UNSUPPORTED, "FP64 arithmetic is offered on FP32 storage only");
    if (!std::isfinite(p->rho_ref)) return fail(SC_E_INVAL, "rho_ref must be finite");
    if (p->barrier != 0 && p->barrier != 1) return fail(SC_E_INVAL, "barrier must be 0 or 1");
    if (p->barrier && (p->corona < 0 || p->corona > 64))
        return fail(SC_E_INVAL, "corona must be in [0, 64]");
    if (p->barrier && p->storage != SC_STORE_F32 && p->compute == SC_COMPUTE_F64)
        return fail(SC_E_UNSUPPORTED, "the barrier on 16-bit storage runs FP32 arithmetic");
    if (p->components != 1 && p->components != 2) return fail(SC_E_INVAL, "components must be 1 or 2");
    if (p->components == 2) {
        if (!std::isfinite(p->G_cross)) return fail(SC_E_INVAL, "G_cross must be finite");
        if (!(p->rho_vapour > 0.0) || !(p->rho_dissolved > 0.0) || !std::isfinite(p->rho_vapour) ||
            !std::isfinite(p->rho_dissolved))
            return fail(SC_E_INVAL, "rho_vapour and rho_dissolved must be > 0");
        if (p->tau_vapour > 0.0 && !(p->tau_vapour > 0.5))
            return fail(SC_E_INVAL, "tau_vapour must be > 0.5 (or <= 0 for tau)");
        if (p->storage == SC_STORE_F32 && p->compute == SC_COMPUTE_F32)
            return fail(SC_E_UNSUPPORTED, "two components on FP32 storage run FP64 arithmetic");
        if (p->storage != SC_STORE_F32 && p->compute == SC_COMPUTE_F64)
            return fail(SC_E_UNSUPPORTED, "two components on 16-bit storage run FP32 arithmetic");
        if (p->barrier) return fail(SC_E_UNSUPPORTED, "no barrier with two components");
        if (p->gravity[0] != 0.0 || p->gravity[1] != 0.0 || p->gravity[2] != 0.0)
            return fail(SC_E_UNSUPPORTED, "no gravity with two components");
    }
    for (int c = 0; c < 3; ++c)
        if (!std::isfinite(p->gravity[c])) return fail(SC_E_INVAL, "gravity must be finite");
    if (!std::isfinite(p->rho_buoyancy)) return fail(SC_E_INVAL, "rho_buoyancy must be finite");
    {
        const bool g_on = p->gravity[0] != 0.0 || p->gravity[1] != 0.0 ||
                          (p->lattice == SC_D3Q19 && p->gravity[2] != 0.0);
        if (g_on && p->step_variant == 2)
            return fail(SC_E_UNSUPPORTED, "gravity has no software-pipelined kernel");
    }
    if (p->allocator && (!p->allocator->alloc || !p->allocator->free))
        return fail(SC_E_INVAL, "allocator needs alloc and free");
    if (p->tile_x || p->tile_y || p->tile_z || p->step_variant) {
        StepShape sh = shape_from_params(*p);
        const bool ok = p->components == 2 ? step2c_shape_supported(p->lattice, sh)
                                           : step_shape_supported(p->lattice, sh);
        if (!ok) return fail(SC_E_INVAL, "unsupported step tile");
    }
    return SC_OK;
}

void release(sc_sim* s)
{
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    for (DevBuf* b : {&s->parent, &s->labels, &s->labels2, &s->slots, &s->psi, &s->rho_out,
                      &s->u_out, &s->p_out, &s->lap_out, &s->partials, &s->small, &s->tmp64,
                      &s->mask8, &s->nodes, &s->list_node, &s->list_slot, &s->add_tab,
                      &s->pair_buf, &s->res_buf, &s->bub_tab, &s->owner, &s->owner2,
                      &s->owner_ids, &s->frontier, &s->ledger, &s->list_scan, &s->btab,
                      &s->pair_ab})
        dev_free(s, b->p);
    if (s->stage) (void)hipHostFree(s->stage);
    dev_free(s, s->f[0]);
    dev_free(s, s->f[1]);
    dev_free(s, s->fv[0]);
    dev_free(s, s->fv[1]);
    dev_free(s, s->dens2.p);
    for (auto& r : s->recs) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    for (auto e : s->pool) (void)hipEventDestroy(e);
    for (auto& g : s->graph_exec)
        if (g) (void)hipGraphExecDestroy(g);
    for (auto& g : s->pass_exec)
        if (g) (void)hipGraphExecDestroy(g);
    if (s->own_stream && s->stream) (void)hipStreamDestroy(s->stream);
}

}  // namespace

// ==============================================================================================
// C ABI
// ==============================================================================================
extern "C" {

uint32_t sc_abi_version(void) { return SC_ABI_VERSION; }

const char* sc_last_error(void) { return g_err.c_str(); }

int sc_params_init(sc_params* p)
{
    if (!p) return fail(SC_E_INVAL, "NULL parameters");
    std::memset(p, 0, sizeof(*p));
    p->abi_version = SC_ABI_VERSION;
    p->lattice = SC_D2Q9;
    p->nx = 128; p->ny = 128; p->nz = 1;
    p->tau = 1.0; p->G = -5.0;
    p->rho_liquid = 1.93; p->rho_gas = 0.16;
    p->noise_amp = 1e-3; p->noise_seed = 1;
    p->gas_threshold = 0.0;
    p->test_every = 10;
    p->film_max = 8;
    p->storage = SC_STORE_F32;
    p->rho_ref = -1.0;
    p->barrier = 0;
    p->corona = 3;
    p->components = 1;
    p->G_cross = 1.5;
    p->tau_vapour = 0.0;
    p->rho_vapour = 1.0;
    p->rho_dissolved = 0.05;
    return SC_OK;
}

int sc_create(const sc_params* p, sc_sim** out)
{
    if (!out) return fail(SC_E_INVAL, "NULL output handle");
    TRY(validate(p));
    sc_sim* s = new sc_sim();
    s->p = *p;
    if (p->allocator) {
        s->alloc = *p->allocator;
        s->has_alloc = true;
    }
    s->q = p->lattice;
    s->d = p->lattice == SC_D2Q9 ? 2 : 3;
    s->N = (int64_t)p->nx * p->ny * p->nz;
    s->theta = p->gas_threshold > 0.0 ? p->gas_threshold : 0.5 * (p->rho_liquid + p->rho_gas);
    s->rho_ref = p->rho_ref >= 0.0 ? p->rho_ref : (p->storage == SC_STORE_F32 ? 0.0 : p->rho_liquid);
    s->es = storage_bytes(p->storage);
    s->compute = p->compute != SC_COMPUTE_AUTO
                     ? p->compute
                     : (p->storage == SC_STORE_F32 ? SC_COMPUTE_F64 : SC_COMPUTE_F32);
    s->shape = shape_from_params(*p);
    if (!(p->tile_x || p->tile_y || p->tile_z || p->step_variant)) {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tuned.find(tune_key(*p, s->compute));
        if (it != g_tuned.end()) s->shape = it->second;
    }
    s->grav = p->gravity[0] != 0.0 || p->gravity[1] != 0.0 ||
              (p->lattice == SC_D3Q19 && p->gravity[2] != 0.0);
    if (p->lattice == SC_D2Q9) s->p.gravity[2] = 0.0;
    // a tuned pipelined shape runs as the plain non-temporal variant of the gravity kernels
    if (s->grav && s->shape.variant == 2) s->shape.variant = 3;
    s->psi_l = 1.0 - std::exp(-p->rho_liquid);
    if (p->stream) {
        s->stream = (hipStream_t)p->stream;
    } else {
        if (hipStreamCreate(&s->stream) != hipSuccess) {
            (void)hipGetLastError();
            delete s;
            return fail(SC_E_DEVICE, "hipStreamCreate failed");
        }
        s->own_stream = true;
    }
    const size_t bytes = (size_t)s->q * (size_t)s->N * s->es;
    s->f[0] = dev_alloc(s, bytes);
    s->f[1] = dev_alloc(s, bytes);
    if (!s->f[0] || !s->f[1]) {
        release(s);
        delete s;
        return fail(SC_E_NOMEM, "population buffers (" + std::to_string(2 * bytes) + " bytes)");
    }
    if (p->barrier) {
        const size_t ob = sizeof(uint16_t) * (size_t)s->N;
        if (ensure(s, s->owner, ob) != SC_OK || ensure(s, s->owner2, ob) != SC_OK) {
            release(s);
            delete s;
            return fail(SC_E_NOMEM, "owner field");
        }
    }
    s->two = p->components == 2;
    if (s->two) {
        s->tau_v = p->tau_vapour > 0.0 ? p->tau_vapour : p->tau;
        // shifted liquid storage shifts the gas component by its bulk (dissolved) density
        s->rho_ref_v = s->rho_ref != 0.0 ? p->rho_dissolved : 0.0;
        s->fv[0] = dev_alloc(s, bytes);
        s->fv[1] = dev_alloc(s, bytes);
        if (!s->fv[0] || !s->fv[1] || ensure(s, s->dens2, sizeof(double) * 2 * (size_t)s->N) != SC_OK) {
            release(s);
            delete s;
            return fail(SC_E_NOMEM, "gas component buffers");
        }
    }
    hipError_t e = launch_init(s->q, p->storage, s->f[0], init_args(s, p->rho_liquid), s->stream);
    if (e == hipSuccess && s->two) {  // the liquid holds rho_dissolved of the gas component
        e = launch_init(s->q, p->storage, s->fv[0], init_args_gas(s, p->rho_dissolved), s->stream);
    }
    if (e == hipSuccess && p->barrier)
        e = launch_owner_seed(nullptr, nullptr, nullptr, 0, (uint16_t*)s->owner.p, s->N, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) {
        std::string m = std::string("initial fill: ") + hipGetErrorString(e);
        release(s);
        delete s;
        return fail(SC_E_DEVICE, m);
    }
    if (s->grav) {
        const int rc = set_rho0(s);
        if (rc != SC_OK) {
            release(s);
            delete s;
            return rc;
        }
    }
    *out = s;
    return SC_OK;
}

int sc_destroy(sc_sim* s)
{
    if (!s) return fail(SC_E_INVAL, "NULL simulation handle");
    release(s);
    delete s;
    return SC_OK;
}

int sc_seed_nuclei(sc_sim* s, int32_t n, const double* centre, const double* radius,
                   const double* budget, double rate)
{
    TRY(check_usable(s));
    if (n < 0) return fail(SC_E_INVAL, "n must be >= 0");
    if (n > 0 && (!centre || !radius || !budget)) return fail(SC_E_INVAL, "NULL nucleus arrays");
    if (!(rate >= 0.0) || !std::isfinite(rate)) return fail(SC_E_INVAL, "rate must be finite and >= 0");
    if (s->p.barrier && n > 65534) return fail(SC_E_INVAL, "the barrier's 16-bit owner ids allow 65534 nuclei");
    for (int k = 0; k < n; ++k) {
        for (int c = 0; c < 3; ++c)
            if (!std::isfinite(centre[3 * k + c])) return fail(SC_E_INVAL, "non-finite centre");
        if (!std::isfinite(radius[k])) return fail(SC_E_INVAL, "non-finite radius");
        if (!(budget[k] >= 0.0) || !std::isfinite(budget[k])) return fail(SC_E_INVAL, "budget must be finite and >= 0");
    }
    s->cen.assign((size_t)3 * n, 0.0);
    s->rad.assign((size_t)n, 0.0);
    s->rem.assign((size_t)n, 0.0);
    s->budget0.assign((size_t)n, 0.0);
    s->owed_nuc.assign((size_t)n, 0.0);
    s->ledger_nb = 0;
    s->sr_key = s->p.noise_seed ^ 0x736f757263652d31ull;  // stochastic rounding of the source
    s->nuc_node.assign((size_t)n, 0);
    s->merge_parent.resize((size_t)n);
    s->topo_parent.resize((size_t)n);
    s->rate = rate;
    for (int k = 0; k < n; ++k) {
        for (int c = 0; c < 3; ++c) s->cen[3 * k + c] = centre[3 * k + c];
        if (s->d == 2) s->cen[3 * k + 2] = 0.0;
        s->rad[k] = radius[k];
        s->rem[k] = budget[k];
        s->budget0[k] = budget[k];
        s->nuc_node[k] = nearest_node(s, &s->cen[3 * k]);
        s->merge_parent[k] = k;
        s->topo_parent[k] = k;
    }
    // the nucleus nodes live on the device for the test passes' bubble table
    s->group_dirty = true;
    if (n > 0) {
        TRY(ensure(s, s->nodes, sizeof(int64_t) * (size_t)n));
        HIPX(hipMemcpyAsync(s->nodes.p, s->nuc_node.data(), sizeof(int64_t) * n,
                            hipMemcpyHostToDevice, s->stream));
        HIPX(hipStreamSynchronize(s->stream));
    }
    const InitArgs ia = init_args(s, s->p.rho_gas);
    const InitArgs va = init_args_gas(s, s->p.rho_vapour);  // bubbles hold the gas component
    for (int k = 0; k < n; ++k) {
        if (s->rad[k] < 0.0) continue;
        HIPX(launch_paint(s->q, s->p.storage, s->f[s->cur], ia, &s->cen[3 * k], s->rad[k],
                          s->stream));
        if (s->two)
            HIPX(launch_paint(s->q, s->p.storage, s->fv[s->cur], va, &s->cen[3 * k], s->rad[k],
                              s->stream));
    }
    if (s->grav) TRY(set_rho0(s));
    return test_pass(s, false);
}

// The step launches of one time step (the fused step, and the barrier fix-up if any frontier).
static int launch_one_step(sc_sim* s, const StepArgs& a, int c)
{
    if (s->two)
        HIPX(launch_step2c(s->q, s->p.storage, s->f[c], s->fv[c], s->f[c ^ 1], s->fv[c ^ 1],
                           step2c_args(s), s->shape, s->stream));
    else
        HIPX(launch_step(s->q, s->p.storage, s->compute, s->f[c], s->f[c ^ 1], a, s->shape,
                         s->stream));
    if (s->p.barrier && s->frontier_count > 0)
        HIPX(launch_barrier_fix(s->q, s->p.storage, s->compute, s->f[c], s->f[c ^ 1], a,
                                (const uint32_t*)s->frontier.p, s->frontier_count, s->stream));
    return SC_OK;
}

// A K-step block runs as one graph when its launches are the same every block: a box small
// enough that launching dominates (N <= 2^22 nodes), no barrier fix-up, and no source launch in
// the block.  The block starts right after a test pass (t % K == 0, schedule position 0).
static bool block_graph_ok(const sc_sim* s, int K, int left)
{
    if (!s->graphs || K <= 0 || left < K || s->t % K != 0 || s->N > ((int64_t)1 << 22))
        return false;
    if (s->p.barrier && s->frontier_count > 0) return false;
    if (s->chunk_pos != 0 || s->chunk_len < K) return false;
    if (s->list_count > 0)
        for (int k = 0; k < K; ++k)
            if (s->step_active[(size_t)k]) return false;
    return true;
}

// Launches the K-step block from buffer parity s->cur, capturing it first if its arguments
// changed since the last capture.
static int run_block_graph(sc_sim* s, const StepArgs& a, int K)
{
    const int c0 = s->cur;
    std::vector<char> key(sizeof(StepArgs) + sizeof(Step2cArgs) + sizeof(StepShape) +
                          6 * sizeof(void*) + sizeof(int));
    {
        char* k = key.data();
        const Step2cArgs a2 = step2c_args(s);
        const void* ptrs[6] = {s->f[0], s->f[1], s->fv[0], s->fv[1], (void*)s->stream,
                           s->frontier.p};
        std::memcpy(k, &a, sizeof(a)); k += sizeof(a);
        std::memcpy(k, &a2, sizeof(a2)); k += sizeof(a2);
        std::memcpy(k, &s->shape, sizeof(s->shape)); k += sizeof(s->shape);
        std::memcpy(k, ptrs, sizeof(ptrs)); k += sizeof(ptrs);
        std::memcpy(k, &K, sizeof(K));
    }
    if (!s->graph_exec[c0] || s->graph_key[c0] != key) {
        if (s->graph_exec[c0]) {
            HIPX(hipGraphExecDestroy(s->graph_exec[c0]));
            s->graph_exec[c0] = nullptr;
        }
        HIPX(hipStreamBeginCapture(s->stream, hipStreamCaptureModeThreadLocal));
        int rc = SC_OK;
        int c = c0;
        for (int k = 0; k < K && rc == SC_OK; ++k, c ^= 1) rc = launch_one_step(s, a, c);
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(s->stream, &g);
        if (rc != SC_OK) {
            if (g) (void)hipGraphDestroy(g);
            return rc;
        }
        if (e != hipSuccess) return device_fail(s, e, "hipStreamEndCapture");
        const hipError_t ei = hipGraphInstantiate(&s->graph_exec[c0], g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ei != hipSuccess) {
            s->graph_exec[c0] = nullptr;
            return device_fail(s, ei, "hipGraphInstantiate");
        }
        s->graph_key[c0] = key;
    }
    hipEvent_t pe;
    TRY(prof_begin(s, SC_KERNEL_STEP, &pe));
    if (s->prof) s->recs.back().launches = K;
    HIPX(hipGraphLaunch(s->graph_exec[c0], s->stream));
    TRY(prof_end(s, pe));
    return SC_OK;
}

// The device part of the test pass after a graph-run block, itself as a graph: captured from
// pass_enqueue and valid while the buffers and arguments it captured stay the same.
static int run_pass_graph(sc_sim* s)
{
    const int c0 = s->cur;
    const FieldArgs fa = field_args(s);
    const int n = (int)s->rad.size();
    const int meta[7] = {n, s->pair_cap, s->two ? 1 : 0, c0, s->p.film_max, s->d, s->btab_n};
    const void* ptrs[16] = {s->labels.p, s->parent.p, s->small.p, s->partials.p, s->slots.p,
                            s->btab.p, (void*)s->stage_dev, s->pair_buf.p, s->res_buf.p, s->pair_ab.p,
                            s->nodes.p, (void*)s->stage, s->f[c0], s->fv[c0],
                            (void*)s->stream, nullptr};
    std::vector<char> key(sizeof(fa) + sizeof(meta) + sizeof(ptrs));
    std::memcpy(key.data(), &fa, sizeof(fa));
    std::memcpy(key.data() + sizeof(fa), meta, sizeof(meta));
    std::memcpy(key.data() + sizeof(fa) + sizeof(meta), ptrs, sizeof(ptrs));
    if (!s->pass_exec[c0] || s->pass_key[c0] != key) {
        if (s->pass_exec[c0]) {
            HIPX(hipGraphExecDestroy(s->pass_exec[c0]));
            s->pass_exec[c0] = nullptr;
        }
        HIPX(hipStreamBeginCapture(s->stream, hipStreamCaptureModeThreadLocal));
        const int rc = pass_enqueue(s, true);
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(s->stream, &g);
        if (rc != SC_OK) {
            if (g) (void)hipGraphDestroy(g);
            return rc;
        }
        if (e != hipSuccess) return device_fail(s, e, "hipStreamEndCapture");
        const hipError_t ei = hipGraphInstantiate(&s->pass_exec[c0], g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ei != hipSuccess) {
            s->pass_exec[c0] = nullptr;
            return device_fail(s, ei, "hipGraphInstantiate");
        }
        s->pass_key[c0] = key;
    }
    HIPX(hipGraphLaunch(s->pass_exec[c0], s->stream));
    return SC_OK;
}

int sc_step_graphs(sc_sim* s, int32_t enable)
{
    TRY(check_usable(s));
    s->graphs = enable != 0;
    return SC_OK;
}

int sc_step(sc_sim* s, int32_t nsteps)
{
    TRY(check_usable(s));
    if (nsteps < 0) return fail(SC_E_INVAL, "nsteps must be >= 0");
    const StepArgs a = step_args(s);
    const FieldArgs fa = field_args(s);
    const int K = s->p.test_every;
    for (int it = 0; it < nsteps; ++it) {
        if (block_graph_ok(s, K, nsteps - it)) {
            // a whole K-step block without source launches: one graph, then the bookkeeping
            // the per-step loop below does, and the test pass
            TRY(run_block_graph(s, a, K));
            if (K & 1) s->cur ^= 1;
            for (int k = 0; k < K; ++k) {
                if (!s->rem.empty() && s->chunk_len > 0) {
                    const size_t n = s->rem.size();
                    std::copy(s->rem_host.begin() + s->chunk_pos * n,
                              s->rem_host.begin() + (s->chunk_pos + 1) * n, s->rem.begin());
                }
                s->chunk_pos++;
                s->t += 1;
            }
            it += K - 1;
            // the pass's device part as a graph too, unless a ledger is to be read back
            hipEvent_t pe;
            TRY(prof_begin(s, SC_KERNEL_TEST, &pe));
            TRY(pass_prepare(s, true));
            if (s->ledger_nb == 0)
                TRY(run_pass_graph(s));
            else
                TRY(pass_enqueue(s, true));
            const int rc = pass_finish(s, true);
            TRY(prof_end(s, pe));
            TRY(rc);
            continue;
        }
        hipEvent_t pe;
        TRY(prof_begin(s, SC_KERNEL_STEP, &pe));
        TRY(launch_one_step(s, a, s->cur));
        TRY(prof_end(s, pe));
        s->cur ^= 1;
        // blowing-agent source after streaming
        if (s->chunk_pos >= s->chunk_len) {
            build_schedule(s, schedule_chunk_len(s));
            TRY(upload_schedule(s));
        }
        const int nb = (int)s->bub.size();
        if (s->step_active.size() && s->step_active[s->chunk_pos] && s->list_count > 0) {
            TRY(prof_begin(s, SC_KERNEL_SOURCE, &pe));
            // the agent's gas goes to the gas component when there is one
            if (s->ledger_nb != nb) return fail(SC_E_STATE, "source ledger out of step");
            HIPX(launch_source(s->q, s->p.storage, s->two ? s->fv[s->cur] : s->f[s->cur],
                               (const uint32_t*)s->list_node.p,
                               (const int32_t*)s->list_slot.p, s->list_count,
                               ledger_view(s, s->chunk_pos), s->t, fa, s->stream));
            TRY(prof_end(s, pe));
        }
        if (!s->rem.empty() && s->chunk_len > 0) {
            const size_t n = s->rem.size();
            std::copy(s->rem_host.begin() + s->chunk_pos * n,
                      s->rem_host.begin() + (s->chunk_pos + 1) * n, s->rem.begin());
        }
        s->chunk_pos++;
        s->t += 1;
        if (K > 0 && s->t % K == 0) TRY(test_pass(s, true));
    }
    HIPX(hipStreamSynchronize(s->stream));
    return SC_OK;
}

// Reported fields into device buffers rho_d[N] and u_d[d][N] (either may be NULL), queued on
// the sim's stream: the liquid density and the mixture's barycentric velocity with two
// components, rho and (j + F/2)/rho with one.
static int fields_to_device(sc_sim* s, float* rho_d, float* u_d)
{
    if (!rho_d && !u_d) return SC_OK;
    if (s->two) {
        HIPX(launch_fields2c(s->q, s->p.storage, s->f[s->cur], s->fv[s->cur],
                             (double*)s->dens2.p, rho_d, nullptr, u_d, step2c_args(s), s->stream));
        return SC_OK;
    }
    const FieldArgs fa = field_args(s);
    TRY(ensure(s, s->psi, sizeof(double) * (size_t)s->N));
    HIPX(launch_psi(s->q, s->p.storage, s->f[s->cur], (double*)s->psi.p, fa, s->stream));
    HIPX(launch_fields(s->q, s->p.storage, s->f[s->cur], (const double*)s->psi.p, rho_d, u_d, fa,
                       s->stream));
    return SC_OK;
}

// A caller's device buffer of `bytes` bytes: memory of the sim's device whose allocation covers
// [p, p + bytes).  A host pointer or one of another device is rejected before any kernel sees it.
static int check_device_buffer(const void* p, size_t bytes, const char* what)
{
    hipPointerAttribute_t at;
    if (hipPointerGetAttributes(&at, p) != hipSuccess) {
        (void)hipGetLastError();
        return fail(SC_E_INVAL, std::string(what) + " is not device memory");
    }
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        return fail(SC_E_DEVICE, "hipGetDevice failed");
    }
    if (at.type != hipMemoryTypeDevice || at.device != dev)
        return fail(SC_E_INVAL, std::string(what) + " is not memory of the sim's device");
    hipDeviceptr_t base = nullptr;
    size_t size = 0;
    if (hipMemGetAddressRange(&base, &size, (hipDeviceptr_t)p) != hipSuccess) {
        (void)hipGetLastError();
        return fail(SC_E_INVAL, std::string(what) + ": no allocation range");
    }
    if ((const char*)p + bytes > (const char*)base + size)
        return fail(SC_E_INVAL, std::string(what) + " is smaller than the fields it must hold");
    return SC_OK;
}

// Two output ranges [a, a + na) and [b, b + nb) of one call must not overlap: the kernels read
// neighbours of what they write (the Laplacian reads p around the node whose lap it stores), so
// overlapping outputs would race.
static int check_disjoint(const void* a, size_t na, const void* b, size_t nb, const char* what)
{
    if (!a || !b) return SC_OK;
    const char* pa = (const char*)a;
    const char* pb = (const char*)b;
    if (pa < pb + nb && pb < pa + na) return fail(SC_E_INVAL, std::string(what) + " overlap");
    return SC_OK;
}

int sc_fields(sc_sim* s, float* rho, float* u, double* totals)
{
    TRY(check_usable(s));
    if (rho || u) {
        if (rho) TRY(ensure(s, s->rho_out, sizeof(float) * (size_t)s->N));
        if (u) TRY(ensure(s, s->u_out, sizeof(float) * (size_t)s->N * s->d));
        TRY(fields_to_device(s, rho ? (float*)s->rho_out.p : nullptr,
                             u ? (float*)s->u_out.p : nullptr));
        if (rho)
            HIPX(hipMemcpyAsync(rho, s->rho_out.p, sizeof(float) * (size_t)s->N,
                                hipMemcpyDeviceToHost, s->stream));
        if (u)
            HIPX(hipMemcpyAsync(u, s->u_out.p, sizeof(float) * (size_t)s->N * s->d,
                                hipMemcpyDeviceToHost, s->stream));
        HIPX(hipStreamSynchronize(s->stream));
    }
    if (totals) TRY(totals_now(s, totals));
    return SC_OK;
}

int sc_fields_device(sc_sim* s, float* rho_dev, float* u_dev)
{
    TRY(check_usable(s));
    if (rho_dev) TRY(check_device_buffer(rho_dev, sizeof(float) * (size_t)s->N, "rho"));
    if (u_dev) TRY(check_device_buffer(u_dev, sizeof(float) * (size_t)s->N * s->d, "u"));
    TRY(check_disjoint(rho_dev, sizeof(float) * (size_t)s->N, u_dev,
                       sizeof(float) * (size_t)s->N * s->d, "rho and u"));
    TRY(fields_to_device(s, rho_dev, u_dev));
    HIPX(hipStreamSynchronize(s->stream));
    return SC_OK;
}

int sc_laplacian_p(sc_sim* s, double* p, double* lap)
{
    TRY(check_usable(s));
    if (!p && !lap) return SC_OK;
    const FieldArgs fa = field_args(s);
    TRY(ensure(s, s->p_out, sizeof(double) * (size_t)s->N));
    HIPX(launch_pressure(s->q, s->p.storage, s->f[s->cur], (double*)s->p_out.p, fa, s->stream));
    if (lap) {
        TRY(ensure(s, s->lap_out, sizeof(double) * (size_t)s->N));
        HIPX(launch_laplacian(s->q, (const double*)s->p_out.p, (double*)s->lap_out.p, fa,
                              s->stream));
        HIPX(hipMemcpyAsync(lap, s->lap_out.p, sizeof(double) * (size_t)s->N,
                            hipMemcpyDeviceToHost, s->stream));
    }
    if (p)
        HIPX(hipMemcpyAsync(p, s->p_out.p, sizeof(double) * (size_t)s->N, hipMemcpyDeviceToHost,
                            s->stream));
    HIPX(hipStreamSynchronize(s->stream));
    return SC_OK;
}

int sc_laplacian_p_device(sc_sim* s, double* p_dev, double* lap_dev)
{
    TRY(check_usable(s));
    if (!p_dev && !lap_dev) return SC_OK;
    if (p_dev) TRY(check_device_buffer(p_dev, sizeof(double) * (size_t)s->N, "p"));
    if (lap_dev) TRY(check_device_buffer(lap_dev, sizeof(double) * (size_t)s->N, "lap"));
    TRY(check_disjoint(p_dev, sizeof(double) * (size_t)s->N, lap_dev,
                       sizeof(double) * (size_t)s->N, "p and lap"));
    const FieldArgs fa = field_args(s);
    double* p_d = p_dev;
    if (!p_d) {  // the Laplacian alone still needs p
        TRY(ensure(s, s->p_out, sizeof(double) * (size_t)s->N));
        p_d = (double*)s->p_out.p;
    }
    HIPX(launch_pressure(s->q, s->p.storage, s->f[s->cur], p_d, fa, s->stream));
    if (lap_dev) HIPX(launch_laplacian(s->q, p_d, lap_dev, fa, s->stream));
    HIPX(hipStreamSynchronize(s->stream));
    return SC_OK;
}

int sc_label_bubbles(sc_sim* s, const uint8_t* mask, uint32_t* labels, int64_t* ncomp)
{
    TRY(check_usable(s));
    TRY(ensure(s, s->labels2, sizeof(uint32_t) * (size_t)s->N));
    uint32_t nc = 0;
    TRY(label_current(s, (uint32_t*)s->labels2.p, &nc, mask));
    if (labels)
        HIPX(hipMemcpyAsync(labels, s->labels2.p, sizeof(uint32_t) * (size_t)s->N,
                            hipMemcpyDeviceToHost, s->stream));
    HIPX(hipStreamSynchronize(s->stream));
    if (ncomp) *ncomp = nc;
    return SC_OK;
}

// ---- allocation-free labelling -----------------------------------------------------------------
// The union-find parent array and the component counter of sc_label_bubbles_noalloc live in a
// file-scope device array: every GPU the library runs on holds its own copy from the time the
// code object is loaded until the process ends.  Host code never passes `scratch` itself (in host
// code the name is a stand-in, not a device address): its device address is looked up once per
// device and kept in scratch_dev.
constexpr int64_t kScratchMaxNodes = 16777216;  // 256^3 nodes: 64 MiB of parents
constexpr int64_t kScratchWords = kScratchMaxNodes + 64;
static __device__ __align__(256) uint32_t scratch[kScratchWords];

namespace {
constexpr int kMaxDevices = 64;
std::mutex scratch_mu;
uint32_t* scratch_dev[kMaxDevices] = {};

int scratch_of_current_device(uint32_t** out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        return fail(SC_E_DEVICE, "hipGetDevice failed");
    }
    if (dev < 0 || dev >= kMaxDevices) return fail(SC_E_DEVICE, "device index out of range");
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_dev[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return fail(SC_E_DEVICE, std::string("hipGetSymbolAddress(scratch) failed: ") +
                                         hipGetErrorString(e));
        }
        scratch_dev[dev] = (uint32_t*)p;
    }
    *out = scratch_dev[dev];
    return SC_OK;
}
}  // namespace

int sc_label_bubbles_noalloc(sc_sim* s, const uint8_t* mask_dev, uint32_t* labels_dev,
                             int64_t* ncomp)
{
    TRY(check_usable(s));
    if (!labels_dev) return fail(SC_E_INVAL, "NULL labels");
    if (s->N > kScratchMaxNodes)
        return fail(SC_E_INVAL, "box of " + std::to_string(s->N) + " nodes exceeds the " +
                                    std::to_string(kScratchMaxNodes) +
                                    "-node scratch of the allocation-free labelling");
    TRY(check_device_buffer(labels_dev, sizeof(uint32_t) * (size_t)s->N, "labels"));
    if (mask_dev) TRY(check_device_buffer(mask_dev, (size_t)s->N, "mask"));
    uint32_t* base = nullptr;
    TRY(scratch_of_current_device(&base));
    uint32_t* parent = base;
    uint32_t* ncomp_d = base + kScratchMaxNodes;  // 256-byte aligned: kScratchMaxNodes * 4
    const FieldArgs fa = field_args(s);
    // every parent entry below N is written by the mask kernel; the counter is cleared by the
    // union kernel (the array keeps the previous call's contents)
    if (mask_dev)
        HIPX(launch_mask_from_bytes(mask_dev, parent, s->N, s->stream));
    else
        HIPX(launch_mask_from_rho(s->q, s->p.storage, s->f[s->cur], parent, fa, s->stream));
    HIPX(launch_union(s->q, parent, ncomp_d, fa, s->stream));
    HIPX(launch_flatten(parent, labels_dev, ncomp_d, s->N, s->stream));
    uint32_t nc = 0;
    HIPX(hipMemcpyAsync(&nc, ncomp_d, sizeof(nc), hipMemcpyDeviceToHost, s->stream));
    HIPX(hipStreamSynchronize(s->stream));
    if (ncomp) *ncomp = nc;
    return SC_OK;
}

int sc_merge_events(sc_sim* s, sc_merge_event* out, int32_t cap, int32_t* n_total)
{
    if (!s) return fail(SC_E_INVAL, "NULL simulation handle");
    if (cap < 0 || (cap > 0 && !out)) return fail(SC_E_INVAL, "bad output buffer");
    const int n = (int)s->events.size();
    for (int k = 0; k < n && k < cap; ++k) out[k] = s->events[k];
    if (n_total) *n_total = n;
    return SC_OK;
}

int sc_topo_events(sc_sim* s, sc_topo_event* out, int32_t cap, int32_t* n_total)
{
    if (!s) return fail(SC_E_INVAL, "NULL simulation handle");
    if (cap < 0 || (cap > 0 && !out)) return fail(SC_E_INVAL, "bad output buffer");
    const int n = (int)s->topo.size();
    for (int k = 0; k < n && k < cap; ++k) out[k] = s->topo[k];
    if (n_total) *n_total = n;
    return SC_OK;
}

int sc_bubbles(sc_sim* s, sc_bubble* out, int32_t cap, int32_t* n_total)
{
    if (!s) return fail(SC_E_INVAL, "NULL simulation handle");
    if (cap < 0 || (cap > 0 && !out)) return fail(SC_E_INVAL, "bad output buffer");
    const int n = (int)s->bub.size();
    for (int k = 0; k < n && k < cap; ++k) out[k] = s->bub[k];
    if (n_total) *n_total = n;
    return SC_OK;
}

int sc_last_labels(sc_sim* s, uint32_t* labels)
{
    TRY(check_usable(s));
    if (!labels) return fail(SC_E_INVAL, "NULL labels");
    if (!s->have_labels) return fail(SC_E_STATE, "no test pass has run yet");
    HIPX(hipMemcpyAsync(labels, s->labels.p, sizeof(uint32_t) * (size_t)s->N,
                        hipMemcpyDeviceToHost, s->stream));
    HIPX(hipStreamSynchronize(s->stream));
    return SC_OK;
}

int sc_film_geometry(sc_sim* s, int32_t nucleus_a, int32_t nucleus_b, double* h,
                     double* r_disc, int32_t* n_lines)
{
#pragma clang fp contract(off)
    TRY(check_usable(s));
    if (!h || !r_disc || !n_lines) return fail(SC_E_INVAL, "NULL output");
    const int n = (int)s->rad.size();
    if (nucleus_a < 0 || nucleus_b < 0 || nucleus_a >= n || nucleus_b >= n)
        return fail(SC_E_INVAL, "nucleus index out of range");
    if (!s->have_labels) return fail(SC_E_STATE, "no test pass has run");
    const uint32_t la = s->comp[nucleus_a], lb = s->comp[nucleus_b];
    if (la == 0 || lb == 0 || la == lb)
        return fail(SC_E_STATE, "the nuclei are not in two distinct bubbles");
    const sc_bubble* A = nullptr;
    const sc_bubble* B = nullptr;
    for (const sc_bubble& b : s->bub) {
        if (b.label == la) A = &b;
        if (b.label == lb) B = &b;
    }
    if (!A || !B) return fail(SC_E_STATE, "bubble not found");
    FilmArgs g;
    double dv[3];
    dv[0] = min_image(B->centroid[0] - A->centroid[0], s->p.nx);
    dv[1] = min_image(B->centroid[1] - A->centroid[1], s->p.ny);
    dv[2] = (s->d == 3) ? min_image(B->centroid[2] - A->centroid[2], s->p.nz) : 0.0;
    const double dist = std::sqrt(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
    const int T = (int)std::ceil(dist);
    if (T <= 0) return fail(SC_E_STATE, "coincident centroids");
    // unit axis and an orthonormal basis of the perpendicular plane (2D: one vector)
    const double u[3] = {dv[0] / dist, dv[1] / dist, dv[2] / dist};
    double n1[3], n2[3] = {0.0, 0.0, 0.0};
    if (s->d == 2) {
        n1[0] = -u[1]; n1[1] = u[0]; n1[2] = 0.0;
    } else {
        double c[3] = {u[1], -u[0], 0.0};  // u x z, or u x x when that is short
        if (c[0] * c[0] + c[1] * c[1] < 0.25) { c[0] = 0.0; c[1] = u[2]; c[2] = -u[1]; }
        const double cl = std::sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
        for (int k = 0; k < 3; ++k) n1[k] = c[k] / cl;
        n2[0] = u[1] * n1[2] - u[2] * n1[1];
        n2[1] = u[2] * n1[0] - u[0] * n1[2];
        n2[2] = u[0] * n1[1] - u[1] * n1[0];
    }
    for (int k = 0; k < 3; ++k) {
        g.cen[k] = A->centroid[k];
        g.dv[k] = dv[k];
        g.n1[k] = n1[k];
        g.n2[k] = n2[k];
    }
    g.label_a = la;
    g.label_b = lb;
    g.T = T;
    g.K = (int)std::floor(std::min(A->radius, B->radius));
    g.dim = s->d;
    g.film_max = s->p.film_max;
    TRY(ensure(s, s->small, 4096));
    FilmOut* out_d = (FilmOut*)((char*)s->small.p + 256);
    FilmOut init{0u, 0, -1.0};
    HIPX(hipMemcpyAsync(out_d, &init, sizeof(init), hipMemcpyHostToDevice, s->stream));
    HIPX(launch_film(s->q, s->p.storage, s->f[s->cur], (const uint32_t*)s->labels.p, g, out_d,
                     field_args(s), s->stream));
    FilmOut res;
    HIPX(hipMemcpyAsync(&res, out_d, sizeof(res), hipMemcpyDeviceToHost, s->stream));
    HIPX(hipStreamSynchronize(s->stream));
    *n_lines = (int32_t)res.count;
    *h = res.h;
    *r_disc = s->d == 2 ? 0.5 * (double)res.count : std::sqrt((double)res.count / M_PI);
    return SC_OK;
}

int sc_gas_density(sc_sim* s, float* rho_v)
{
    TRY(check_usable(s));
    if (!rho_v) return fail(SC_E_INVAL, "NULL output");
    if (!s->two) {
        std::memset(rho_v, 0, sizeof(float) * (size_t)s->N);
        return SC_OK;
    }
    TRY(ensure(s, s->rho_out, sizeof(float) * (size_t)s->N));
    HIPX(launch_fields2c(s->q, s->p.storage, s->f[s->cur], s->fv[s->cur],
                         (double*)s->dens2.p, nullptr, (float*)s->rho_out.p, nullptr,
                         step2c_args(s), s->stream));
    HIPX(hipMemcpyAsync(rho_v, s->rho_out.p, sizeof(float) * (size_t)s->N, hipMemcpyDeviceToHost,
                        s->stream));
    HIPX(hipStreamSynchronize(s->stream));
    return SC_OK;
}

int sc_set_gas_equilibrium(sc_sim* s, const double* rho_v)
{
    TRY(check_usable(s));
    if (!s->two) return fail(SC_E_STATE, "no gas component (components = 1)");
    if (!rho_v) return fail(SC_E_INVAL, "NULL density");
    for (int64_t n = 0; n < s->N; ++n)
        if (!(rho_v[n] > 0.0) || !std::isfinite(rho_v[n])) return fail(SC_E_INVAL, "rho_v must be finite and > 0");
    TRY(ensure(s, s->tmp64, sizeof(double) * (size_t)s->N * 4));
    double* rd = (double*)s->tmp64.p;
    HIPX(hipMemcpyAsync(rd, rho_v, sizeof(double) * (size_t)s->N, hipMemcpyHostToDevice,
                        s->stream));
    HIPX(launch_set_eq(s->q, s->p.storage, s->fv[s->cur], init_args_gas(s, 0.0), rd, nullptr,
                       s->stream));
    HIPX(hipStreamSynchronize(s->stream));
    return SC_OK;
}

int sc_buoyancy_density(sc_sim* s, double* rho0)
{
    TRY(check_usable(s));
    if (!rho0) return fail(SC_E_INVAL, "NULL output");
    *rho0 = s->rho0;
    return SC_OK;
}

int sc_owner(sc_sim* s, uint16_t* owner)
{
    TRY(check_usable(s));
    if (!owner) return fail(SC_E_INVAL, "NULL owner array");
    if (!s->p.barrier) {
        std::memset(owner, 0, sizeof(uint16_t) * (size_t)s->N);
        return SC_OK;
    }
    HIPX(hipMemcpyAsync(owner, s->owner.p, sizeof(uint16_t) * (size_t)s->N, hipMemcpyDeviceToHost,
                        s->stream));
    HIPX(hipStreamSynchronize(s->stream));
    return SC_OK;
}

int sc_nuclei(sc_sim* s, uint32_t* comp, double* remaining)
{
    if (!s) return fail(SC_E_INVAL, "NULL simulation handle");
    for (size_t k = 0; k < s->rem.size(); ++k) {
        if (comp) comp[k] = k < s->comp.size() ? s->comp[k] : 0u;
        if (remaining) remaining[k] = s->rem[k];
    }
    return SC_OK;
}

int sc_source_ledger(sc_sim* s, double* released, double* undelivered)
{
#pragma clang fp contract(off)
    TRY(check_usable(s));
    if (released) {
        double r = 0.0;
        for (size_t k = 0; k < s->rem.size(); ++k) r += s->budget0[k] - s->rem[k];
        *released = r;
    }
    if (undelivered) {
        double o = 0.0;
        for (double v : s->owed_nuc) o += v;
        if (s->ledger_nb > 0) {
            std::vector<double> owed((size_t)s->ledger_nb);
            HIPX(hipMemcpyAsync(owed.data(), s->ledger.p, sizeof(double) * owed.size(),
                                hipMemcpyDeviceToHost, s->stream));
            HIPX(hipStreamSynchronize(s->stream));
            for (double v : owed) o += v;
        }
        *undelivered = o;
    }
    return SC_OK;
}

int sc_time(sc_sim* s, int64_t* step)
{
    if (!s || !step) return fail(SC_E_INVAL, "NULL argument");
    *step = s->t;
    return SC_OK;
}

int sc_lattice(int32_t lattice, int32_t* e, double* w)
{
    static const int e9[9][3] = {{0, 0, 0}, {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0},
                                 {1, 1, 0}, {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0}};
    static const int e19[19][3] = {{0, 0, 0},  {1, 0, 0},   {-1, 0, 0}, {0, 1, 0},  {0, -1, 0},
                                   {0, 0, 1},  {0, 0, -1},  {1, 1, 0},  {-1, -1, 0}, {1, -1, 0},
                                   {-1, 1, 0}, {1, 0, 1},   {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
                                   {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
    if (lattice != SC_D2Q9 && lattice != SC_D3Q19) return fail(SC_E_INVAL, "lattice must be 9 or 19");
    const int q = lattice;
    for (int i = 0; i < q; ++i) {
        const int* v = q == 9 ? e9[i] : e19[i];
        const int m = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
        if (e)
            for (int c = 0; c < 3; ++c) e[3 * i + c] = v[c];
        if (w) {
            if (q == 9) w[i] = m == 0 ? 4.0 / 9.0 : (m == 1 ? 1.0 / 9.0 : 1.0 / 36.0);
            else w[i] = m == 0 ? 1.0 / 3.0 : (m == 1 ? 1.0 / 18.0 : 1.0 / 36.0);
        }
    }
    return SC_OK;
}

int sc_get_populations(sc_sim* s, double* f)
{
    TRY(check_usable(s));
    if (!f) return fail(SC_E_INVAL, "NULL output");
    const size_t bytes = sizeof(double) * (size_t)s->q * (size_t)s->N;
    TRY(ensure(s, s->tmp64, bytes));
    HIPX(launch_get_f(s->q, s->p.storage, s->f[s->cur], (double*)s->tmp64.p, init_args(s, 0.0),
                      s->stream));
    HIPX(hipMemcpyAsync(f, s->tmp64.p, bytes, hipMemcpyDeviceToHost, s->stream));
    HIPX(hipStreamSynchronize(s->stream));
    return SC_OK;
}

int sc_set_populations(sc_sim* s, const double* f)
{
    TRY(check_usable(s));
    if (!f) return fail(SC_E_INVAL, "NULL input");
    const size_t bytes = sizeof(double) * (size_t)s->q * (size_t)s->N;
    TRY(ensure(s, s->tmp64, bytes));
    HIPX(hipMemcpyAsync(s->tmp64.p, f, bytes, hipMemcpyHostToDevice, s->stream));
    HIPX(launch_set_f(s->q, s->p.storage, s->f[s->cur], (const double*)s->tmp64.p,
                      init_args(s, 0.0), s->stream));
    HIPX(hipStreamSynchronize(s->stream));
    return SC_OK;
}

// The gas component's populations, [q][N] FP64 as for the liquid (checkpoints of the mixture).
int sc_get_gas_populations(sc_sim* s, double* f)
{
    TRY(check_usable(s));
    if (!s->two) return fail(SC_E_STATE, "no gas component (components = 1)");
    if (!f) return fail(SC_E_INVAL, "NULL output");
    const size_t bytes = sizeof(double) * (size_t)s->q * (size_t)s->N;
    TRY(ensure(s, s->tmp64, bytes));
    HIPX(launch_get_f(s->q, s->p.storage, s->fv[s->cur], (double*)s->tmp64.p,
                      init_args_gas(s, 0.0), s->stream));
    HIPX(hipMemcpyAsync(f, s->tmp64.p, bytes, hipMemcpyDeviceToHost, s->stream));
    HIPX(hipStreamSynchronize(s->stream));
    return SC_OK;
}

int sc_set_gas_populations(sc_sim* s, const double* f)
{
    TRY(check_usable(s));
    if (!s->two) return fail(SC_E_STATE, "no gas component (components = 1)");
    if (!f) return fail(SC_E_INVAL, "NULL input");
    const size_t bytes = sizeof(double) * (size_t)s->q * (size_t)s->N;
    TRY(ensure(s, s->tmp64, bytes));
    HIPX(hipMemcpyAsync(s->tmp64.p, f, bytes, hipMemcpyHostToDevice, s->stream));
    HIPX(launch_set_f(s->q, s->p.storage, s->fv[s->cur], (const double*)s->tmp64.p,
                      init_args_gas(s, 0.0), s->stream));
    HIPX(hipStreamSynchronize(s->stream));
    return SC_OK;
}

int sc_set_equilibrium(sc_sim* s, const double* rho, const double* u)
{
    TRY(check_usable(s));
    if (!rho) return fail(SC_E_INVAL, "NULL rho");
    for (int64_t n = 0; n < s->N; ++n)
        if (!(rho[n] > 0.0) || !std::isfinite(rho[n])) return fail(SC_E_INVAL, "rho must be finite and > 0");
    const size_t nb_rho = sizeof(double) * (size_t)s->N;
    const size_t bytes = nb_rho * (1 + (u ? s->d : 0));
    TRY(ensure(s, s->tmp64, bytes));
    HIPX(hipMemcpyAsync(s->tmp64.p, rho, nb_rho, hipMemcpyHostToDevice, s->stream));
    if (u)
        HIPX(hipMemcpyAsync((char*)s->tmp64.p + nb_rho, u, nb_rho * s->d, hipMemcpyHostToDevice,
                            s->stream));
    HIPX(launch_set_eq(s->q, s->p.storage, s->f[s->cur], init_args(s, 0.0),
                       (const double*)s->tmp64.p,
                       u ? (const double*)((char*)s->tmp64.p + nb_rho) : nullptr, s->stream));
    HIPX(hipStreamSynchronize(s->stream));
    return SC_OK;
}

int sc_test_pass(sc_sim* s)
{
    TRY(check_usable(s));
    return test_pass(s, true);
}

int sc_profile(sc_sim* s, int32_t enable)
{
    TRY(check_usable(s));
    HIPX(hipStreamSynchronize(s->stream));
    for (auto& r : s->recs) {
        s->pool.push_back(r.a);
        s->pool.push_back(r.b);
    }
    s->recs.clear();
    s->prof = enable != 0;
    return SC_OK;
}

int sc_profile_read(sc_sim* s, int32_t cls, double* ms, int64_t* launches)
{
    TRY(check_usable(s));
    HIPX(hipStreamSynchronize(s->stream));
    double tot = 0.0;
    int64_t cnt = 0;
    for (auto& r : s->recs) {
        if (r.cls != cls) continue;
        float e = 0.0f;
        HIPX(hipEventElapsedTime(&e, r.a, r.b));
        tot += e;
        cnt += r.launches;
    }
    if (ms) *ms = tot;
    if (launches) *launches = cnt;
    return SC_OK;
}

int sc_autotune(sc_sim* s, int32_t trials, sc_tune_entry* out, int32_t cap, int32_t* n_out)
{
    TRY(check_usable(s));
    if (trials < 1 || cap < 0 || (cap > 0 && !out)) return fail(SC_E_INVAL, "bad autotune arguments");
    StepArgs a = step_args(s);
    const Step2cArgs a2 = step2c_args(s);
    const std::vector<StepShape> cand = s->two ? tune_candidates_2c(s->q) : tune_candidates(s->q);
    // one step current -> spare buffers (the state itself is left as it is)
    auto launch = [&](const StepShape& sh) {
        if (s->two)
            return launch_step2c(s->q, s->p.storage, s->f[s->cur], s->fv[s->cur],
                                 s->f[s->cur ^ 1], s->fv[s->cur ^ 1], a2, sh, s->stream);
        a.planes = sh.tile_z;
        return launch_step(s->q, s->p.storage, s->compute, s->f[s->cur], s->f[s->cur ^ 1], a, sh,
                           s->stream);
    };
    hipEvent_t e0, e1;
    HIPX(hipEventCreate(&e0));
    HIPX(hipEventCreate(&e1));
    double best = 1e300;
    StepShape best_shape = s->shape;
    int k = 0;
    int rc = SC_OK;
    for (const StepShape& sh : cand) {
        if (!(s->two ? step2c_shape_supported(s->q, sh) : step_shape_supported(s->q, sh))) continue;
        if (s->grav && sh.variant == 2) continue;  // no pipelined gravity kernel
        // one untimed launch, then `trials` timed launches
        hipError_t e = launch(sh);
        if (e == hipSuccess) e = hipEventRecord(e0, s->stream);
        for (int r = 0; r < trials && e == hipSuccess; ++r) e = launch(sh);
        if (e == hipSuccess) e = hipEventRecord(e1, s->stream);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess) {
            rc = device_fail(s, e, "autotune trial");
            break;
        }
        const double us = 1e3 * ms / trials;
        if (k < cap) out[k] = sc_tune_entry{sh.tile_x, sh.tile_y, sh.tile_z, sh.variant, us};
        ++k;
        if (us < best) {
            best = us;
            best_shape = sh;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != SC_OK) return rc;
    s->shape = best_shape;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tuned[tune_key(s->p, s->compute)] = best_shape;
    }
    if (n_out) *n_out = k;
    return SC_OK;
}

int sc_compute_type(sc_sim* s, int32_t* compute)
{
    if (!s || !compute) return fail(SC_E_INVAL, "NULL argument");
    *compute = s->compute;
    return SC_OK;
}

int sc_step_config(sc_sim* s, int32_t* tx, int32_t* ty, int32_t* tz, int32_t* variant)
{
    if (!s) return fail(SC_E_INVAL, "NULL simulation handle");
    if (tx) *tx = s->shape.tile_x;
    if (ty) *ty = s->shape.tile_y;
    if (tz) *tz = s->shape.tile_z;
    if (variant) *variant = s->shape.variant;
    return SC_OK;
}

}  // extern "C"
