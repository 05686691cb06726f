/*
 * sc.h -- C ABI of the MI355X (gfx950) Shan-Chen bubble growth / merging library (libsc.so).
 *
 * Paper: Barzegari, Bayani, Mirbagheri, "A criterion for bubble merging in liquid metal:
 * computational and experimental study" (arXiv 1708.01608).  The calls follow its problem
 * statement: nucleation sites with a blowing agent decomposed at them and liquid elsewhere
 * (Sec. 3.1), a Shan-Chen pseudopotential step per time step (Sec. 3.1, Fig. 1 step 6), gas added
 * to every bubble until the agent is spent (Sec. 3), new bubble sizes (Fig. 1 step 7), and the
 * film-rupture switch decided by the second derivative of pressure (Sec. 3.1 eta_m, Sec. 4).
 *
 * Conventions for every call:
 *  - Lattice units; periodic box nx * ny * nz, linear node index idx = x + nx * (y + ny * z), x
 *    fastest.  D2Q9 needs nz == 1; every axis is >= 4 nodes.
 *  - Host arrays passed in are borrowed for the duration of the call; output pointers that are
 *    NULL skip that output.  Calls are synchronous: they return after the work on the
 *    simulation's stream has completed.  One thread at a time per sc_sim.
 *  - Every call returns an sc_status.  SC_E_INVAL leaves the state unchanged.  After
 *    SC_E_DEVICE (a HIP error) or SC_E_NUMERIC (a non-finite FP64 total) the handle is latched:
 *    every later call except sc_destroy returns SC_E_STATE.  sc_last_error() gives the message
 *    of the calling thread's last failure.
 *  - The library owns the sc_sim, its device memory (obtained through sc_params.allocator, or
 *    hipMalloc when NULL) and its stream when it created one.
 */
#ifndef SC_H
#define SC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SC_ABI_VERSION 2u

typedef enum sc_status {
    SC_OK = 0,
    SC_E_INVAL = -1,       /* invalid argument; nothing changed */
    SC_E_NOMEM = -2,       /* device allocation failed */
    SC_E_DEVICE = -3,      /* a HIP call failed (handle latched) */
    SC_E_STATE = -4,       /* handle latched by an earlier failure, or call out of order */
    SC_E_NUMERIC = -5,     /* a global FP64 total was not finite (handle latched) */
    SC_E_UNSUPPORTED = -6  /* valid request the library does not provide */
} sc_status;

enum { SC_D2Q9 = 9, SC_D3Q19 = 19 };

/* Population storage.  Populations are stored as deviations f_i - w_i rho_ref (the paper leaves
 * precision open; the shift keeps the stored magnitudes small where the density is near
 * rho_ref). */
enum { SC_STORE_F32 = 0, SC_STORE_F16 = 1, SC_STORE_BF16 = 2 };

/* Arithmetic of the step kernel.  AUTO: FP64 on FP32 storage, FP32 on 16-bit storage.  FP64
 * arithmetic is offered on FP32 storage only (SC_E_UNSUPPORTED otherwise). */
enum { SC_COMPUTE_AUTO = 0, SC_COMPUTE_F32 = 1, SC_COMPUTE_F64 = 2 };

/* Device memory callbacks (PyTorch's caching allocator from Python, or any C allocator).
 * alloc returns NULL on failure; free receives exactly what alloc returned. */
typedef struct sc_allocator {
    void* (*alloc)(size_t bytes, void* user);
    void (*free)(void* ptr, void* user);
    void* user;
} sc_allocator;

typedef struct sc_params {
    uint32_t abi_version;      /* must equal SC_ABI_VERSION */
    int32_t lattice;           /* SC_D2Q9 or SC_D3Q19 */
    int32_t nx, ny, nz;        /* periodic box; nz == 1 for D2Q9; nx ny nz times the bytes of
                                  one stored value (4 for F32, 2 for F16/BF16) must be <= 2^32
                                  (e.g. 1024^3 on F32): kernels use 32-bit byte offsets */
    double tau;                /* BGK relaxation time, > 0.5 */
    double G;                  /* Shan-Chen strength (Sec. 3.1); G < 0 attracts */
    double rho_liquid;         /* fill density of every node (Sec. 3.1 "liquid") */
    double rho_gas;            /* density painted inside nuclei */
    double noise_amp;          /* additive U[-amp, amp] density noise on every node */
    uint64_t noise_seed;       /* SplitMix64 seed of the noise: U = (idx+1)-th output of the stream */
    double gas_threshold;      /* gas iff rho < threshold; <= 0 selects (rho_liquid + rho_gas)/2 */
    int32_t test_every;        /* K: labelling + merge test after every K-th step; 0 = never */
    int32_t film_max;          /* longest liquid run (nodes) still tested as a film; >= 1 */
    int32_t storage;           /* SC_STORE_F32 / F16 / BF16 */
    int32_t compute;           /* SC_COMPUTE_AUTO / F32 / F64 */
    double rho_ref;            /* storage shift; < 0 selects 0 for F32 and rho_liquid for 16-bit */
    void* stream;              /* hipStream_t to run on; NULL: the library creates one */
    const sc_allocator* allocator; /* NULL: hipMalloc / hipFree */
    int32_t tile_x, tile_y, tile_z; /* step-kernel tile; 0 selects the tuned default */
    int32_t step_variant;      /* 0 default, 1 plain marching, 2 software-pipelined (D3Q19),
                                  3 plain with non-temporal population stores; with two
                                  components also 4 and 5 (D3Q19, one component per wave) */
    /* Modified Shan-Chen barrier (Sec. 3.1, Fig. 1 steps 3-6: each bubble on its own lattice,
     * meeting the others only through the liquid until the criterion flips eta_m).  barrier = 1:
     * every bubble owns its gas nodes and `corona` liquid layers around them (grown by lattice
     * neighbours, ties to the smaller id); in the force a neighbour owned by a different bubble
     * that the criterion has not merged with the node's contributes psi(rho_liquid) instead of
     * its own psi.  Owners are rebuilt at every test pass after its merges; only the nodes next
     * to another bubble's node are affected, and they are re-stepped by a fix-up kernel after
     * every step.  Any storage (16-bit storage with FP32 arithmetic; FP64 arithmetic there is
     * SC_E_UNSUPPORTED); at most 65534 nuclei. */
    int32_t barrier;           /* 0 off (default), 1 on */
    int32_t corona;            /* liquid layers a bubble owns, 0..64 (default 3) */
    /* Gravity for drainage studies (the paper's runs leave it out): a body force
     * (rho - rho0) g is added to the Shan-Chen force of every node, in the step and in the
     * reported velocity.  rho0 = rho_buoyancy if > 0, else the mean density of the box, taken at
     * sc_create and again at sc_seed_nuclei (no net force on the periodic box).  Any storage;
     * SC_E_UNSUPPORTED with step_variant 2; gravity[2] is ignored in 2D. */
    double gravity[3];         /* g in lattice units; all zero (default) = off */
    double rho_buoyancy;       /* rho0; <= 0 selects the mean density */
    /* Two components (Sec. 3: the agent's gas raises bubble volume; Sec. 3.1: two simulations
     * run together for the two-phase model): a liquid and a gas component (Shan-Doolen mixture,
     * psi = rho; force on component a: -G_cross rho_a(x) sum_i w_i rho_b(x + e_i) e_i; common
     * velocity u' = sum_a (j_a/tau_a) / sum_a (rho_a/tau_a); equilibria at u' + tau_a F_a/rho_a).
     * rho_liquid / rho_gas / gas_threshold, labels, bubbles and the film walk refer to the liquid
     * component (G is not used); the gas component fills the box with rho_dissolved and painted
     * nuclei with rho_vapour; the blowing agent feeds the gas component; the criterion's EOS is
     * p = (rho_l + rho_v)/3 + (G_cross/3) rho_l rho_v; totals sum both components; sc_fields
     * reports the liquid density and the mixture's barycentric velocity
     * (j_l + j_v + (F_l + F_v)/2) / (rho_l + rho_v); population access concerns the liquid.
     * FP32 storage runs FP64 arithmetic, FP16 / BF16 storage FP32 arithmetic (the other
     * pairings: SC_E_UNSUPPORTED); when the liquid's populations are shifted (rho_ref != 0, the
     * default with 16-bit storage) the gas component's are shifted by w_i rho_dissolved.  No
     * barrier, no gravity (SC_E_UNSUPPORTED).  The step is one fused kernel for both components; its tiles
     * are D2Q9 tile_x in {64, 128, 256, 512}, D3Q19 (tile_x, tile_y) in {(32,4), (32,8), (64,4),
     * (64,8), (128,4)}, any tile_z >= 1 planes, step_variant 1 or 3 (both components per
     * thread; 3: non-temporal stores) or, in D3Q19, 4 or 5 (one component per wave, the node's
     * two threads meeting in LDS; 5: non-temporal stores); SC_E_INVAL otherwise. */
    int32_t components;        /* 1 (default) or 2 */
    int32_t reserved2;
    double G_cross;            /* cross interaction, > 0 repels (default 1.5) */
    double tau_vapour;         /* BGK time of the gas component; <= 0 selects tau */
    double rho_vapour;         /* gas component in painted nuclei (default 1.0) */
    double rho_dissolved;      /* gas component elsewhere at creation (default 0.05) */
} sc_params;

/* One firing of the merge criterion (Sec. 3.1 eta_m: 1 -> 0; Sec. 4 film rupture). */
typedef struct sc_merge_event {
    int64_t step;              /* time step of the test pass that fired */
    int32_t nucleus_a;         /* smallest nucleus index of each bubble (stable bubble ids) */
    int32_t nucleus_b;
    uint32_t label_a;          /* component labels at that pass, label_a < label_b */
    uint32_t label_b;
    int64_t film_node;         /* linear index of the film-centre node c* */
    int32_t film_len;          /* liquid nodes on the film run */
    int32_t reserved;
    double lap_p;              /* FP64 lattice Laplacian of p at c* (fired: >= 0) */
    double rho_film;           /* FP64 density at c* */
} sc_merge_event;

/* Two nucleus groups found in one gas component for the first time (topological merge). */
typedef struct sc_topo_event {
    int64_t step;
    int32_t nucleus_a;         /* group representatives (smallest nucleus index), a < b */
    int32_t nucleus_b;
} sc_topo_event;

/* Statistics of one bubble at the last test pass (Fig. 1 step 7, "new bubbles' size"). */
typedef struct sc_bubble {
    uint32_t label;            /* 1 + smallest linear index of the component */
    int32_t nucleus;           /* smallest nucleus index in the bubble */
    int64_t n;                 /* gas node count */
    double centroid[3];        /* anchor node + mean integer minimal-image offset */
    double radius;             /* sqrt(n/pi) (2D) or cbrt(3n/(4 pi)) (3D) */
    int32_t n_nuclei;
    int32_t reserved;
} sc_bubble;

/* Kernel classes for sc_profile_read. */
enum { SC_KERNEL_STEP = 0, SC_KERNEL_SOURCE = 1, SC_KERNEL_TEST = 2 };

uint32_t sc_abi_version(void);
const char* sc_last_error(void);

/* Fills *p with the defaults (abi_version set, D2Q9 128x128, tau 1, G -5, densities 1.93 / 0.16,
 * noise 1e-3 seed 1, K = 10, film_max = 8, FP32 storage, automatic compute type).
 * SC_E_INVAL if p is NULL. */
int sc_params_init(sc_params* p);

/* Sec. 3.1: every node is liquid, rho = rho_liquid + amp (2U - 1), f = f_eq(rho, 0).
 * Errors: SC_E_INVAL (bad parameters, *out untouched), SC_E_NOMEM, SC_E_DEVICE. */
int sc_create(const sc_params* p, struct sc_sim** out);
int sc_destroy(struct sc_sim* sim);

/* Sec. 3.1: nucleation sites and the blowing agent decomposed at them.  centre is [n][3] (z
 * ignored in 2D); nodes whose minimal-image distance to a centre is <= its radius become gas,
 * rho = rho_gas + amp (2U - 1), f = f_eq(rho, 0) (a negative radius registers the nucleus
 * without painting); budget[k] is the agent mass of nucleus k; rate is the mass each nucleus
 * gives per step while its budget lasts (Sec. 3).  Replaces any earlier nuclei and runs a test
 * pass (labels and bubble statistics, no merge criterion) at the current step.
 * Errors: SC_E_INVAL (n < 0, NULL arrays with n > 0, rate < 0, non-finite values). */
int sc_seed_nuclei(struct sc_sim* sim, int32_t n, const double* centre, const double* radius,
                   const double* budget, double rate);

/* Advances nsteps time steps (Fig. 1): pseudopotential, Shan-Chen force, forced BGK collision and
 * pull streaming in one fused kernel; then the blowing-agent source on the gas nodes of every
 * bubble; after every K-th step a test pass (gas labelling, bubble statistics, merge criterion,
 * FP64 totals).  nsteps >= 0.  SC_E_NUMERIC if a total is not finite. */
int sc_step(struct sc_sim* sim, int32_t nsteps);

/* K-step blocks as HIP graphs (Fig. 1 steps 1-6 repeated between two test passes): on a box of at
 * most 2^22 nodes, a block of test_every steps that launches no source and no barrier fix-up runs
 * as one captured graph (kernel launches only), the same kernels with the same arguments as the
 * launches one by one, so the results are identical.  enable = 0 launches step by step.  On by
 * default.  Errors: SC_E_INVAL (NULL sim), SC_E_STATE. */
int sc_step_graphs(struct sc_sim* sim, int32_t enable);

/* Fig. 1 steps 8-9 (the lattices merged to post-process the output; Sec. 3.1 model): rho[N] and
 * u[d][N] = (j + F/2)/rho (FP32; F with the body force when gravity is on; the mixture reports
 * its barycentric velocity), totals = (M, Jx, Jy, Jz) summed in FP64 over the post-streaming
 * populations in a fixed order.  Host arrays, caller-owned; any of the three may be NULL.
 * Errors: SC_E_INVAL (NULL sim), SC_E_STATE (after a device or numeric error), SC_E_DEVICE. */
int sc_fields(struct sc_sim* sim, float* rho, float* u, double* totals);

/* The same rho and u, written into the caller's device memory (rho_dev: N floats, u_dev: d x N
 * floats, SoA; either may be NULL) on the sim's stream; returns after the stream work completes.
 * The buffers stay the caller's.  A pointer that is not memory of the sim's device, or whose
 * allocation ends before the fields do, is SC_E_INVAL before any kernel runs.  (An allocator that
 * sub-allocates, as torch's does, reports its whole segment: the caller must size sub-buffers.
 * Memory whose allocation range HIP cannot report, such as virtual-memory mappings, is refused.) */
int sc_fields_device(struct sc_sim* sim, float* rho_dev, float* u_dev);

/* Sec. 3.1 EOS and the criterion's operator, in FP64: p = rho/3 + (G/6) psi^2 and
 * lap[x] = 6 sum_{i != 0} w_i (p(x + e_i) - p(x)). */
int sc_laplacian_p(struct sc_sim* sim, double* p, double* lap);

/* The same p and lap written into the caller's device memory (N doubles each; either may be
 * NULL), with the buffer checks of sc_fields_device. */
int sc_laplacian_p_device(struct sc_sim* sim, double* p_dev, double* lap_dev);

/* Fig. 1 step 7 (the new bubbles' size comes from the gas phase separated from the fluid, steps
 * 2 and 7): canonical labels of a gas mask: label = 1 + smallest linear index of the component,
 * 0 for liquid; connectivity = the lattice neighbours (8 in 2D, 18 in 3D), periodic.  mask[N]
 * (host, nonzero = gas) or NULL for rho < gas_threshold on the current state; labels[N] (host,
 * caller-owned).  *ncomp receives the component count.  Does not change the bubble registry.
 * Errors: SC_E_INVAL (NULL sim or labels), SC_E_STATE, SC_E_DEVICE. */
int sc_label_bubbles(struct sc_sim* sim, const uint8_t* mask, uint32_t* labels, int64_t* ncomp);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): sc_label_bubbles on device memory with no allocation.
 * mask_dev: N bytes of the sim's device (nonzero = gas) or NULL for rho < gas_threshold on the
 * current state; labels_dev: N uint32 of the sim's device, written with the same canonical labels
 * as sc_label_bubbles; *ncomp (host, may be NULL) the component count.  The union-find parents and
 * the counter live in a static device array of 16,777,216 + 64 uint32 (64 MiB) that each GPU the
 * library runs on holds until the process ends; a box of more than 16,777,216 nodes is SC_E_INVAL.
 * Every call on one GPU shares that array, so calls that overlap in time on one GPU (from two host
 * threads, or on two streams) race; calls in sequence are independent.  Buffers that are not
 * memory of the sim's device, or too small, are SC_E_INVAL before any kernel runs.  Returns after
 * the sim's stream has finished the work.  Errors: SC_E_INVAL, SC_E_STATE, SC_E_DEVICE. */
int sc_label_bubbles_noalloc(struct sc_sim* sim, const uint8_t* mask_dev, uint32_t* labels_dev,
                             int64_t* ncomp);

/* Registry of the last test pass and of all passes so far.  *n_total receives the full count;
 * at most cap entries are copied. */
int sc_merge_events(struct sc_sim* sim, sc_merge_event* out, int32_t cap, int32_t* n_total);
int sc_topo_events(struct sc_sim* sim, sc_topo_event* out, int32_t cap, int32_t* n_total);
int sc_bubbles(struct sc_sim* sim, sc_bubble* out, int32_t cap, int32_t* n_total);
int sc_last_labels(struct sc_sim* sim, uint32_t* labels);
/* comp[n]: label of each nucleus's node at the last pass (0: not gas); remaining[n]: budgets. */
int sc_nuclei(struct sc_sim* sim, uint32_t* comp, double* remaining);
/* Sec. 3 (gas added to every bubble each step until the agent is spent): the agent's mass
 * ledger, FP64.  *released = sum_k (budget_k - remaining_k), the mass the nuclei have given up;
 * *undelivered = the part of it the populations have not taken yet.  Each step the source adds
 * to a fed bubble what it is owed (earlier remainder plus this step's release) and books the
 * exact gain of the stored values, so released - undelivered is the mass the populations
 * gained from the source.  With FP16/BF16 storage the source rounds stochastically, so the
 * remainder stays about one step's release; with FP32 it is the rounding residue.  A bubble that
 * is no longer fed (budgets spent, or its nuclei no longer gas) keeps its remainder undelivered.
 * Either pointer may be NULL.  Errors: SC_E_INVAL (NULL sim), SC_E_STATE, SC_E_DEVICE. */
int sc_source_ledger(struct sc_sim* sim, double* released, double* undelivered);
/* owner[N] (host, caller-owned): the barrier's owner field as of the last test pass; 0 = no
 * bubble, else 1 + the smallest nucleus index of the criterion-merged group that owns the node.
 * All zero when the barrier is off.  Errors: SC_E_INVAL (NULL), SC_E_STATE, SC_E_DEVICE. */
int sc_owner(struct sc_sim* sim, uint16_t* owner);
/* Film geometry of the bubbles holding nuclei a and b at the last test pass (Sec. 3: the film
 * as a disc of radius R_d and thickness h between two interfaces; Fig. 3: h_c and R_d at
 * rupture).  Lines parallel to the centroid segment, shifted by integer multiples of an
 * orthonormal basis of the perpendicular plane up to the smaller bubble radius (2D: one basis
 * vector, the segment's normal; 3D: u x z, or u x x when u is nearly along z, and u x n1), are
 * walked like the merge test's centre line.  *n_lines = the lines crossing a film of
 * 1..film_max liquid nodes free of other labels; *r_disc = n_lines / 2 (2D) or
 * sqrt(n_lines / pi) (3D); *h = distance between the rho = theta crossings on the centre line,
 * linear in arc length between node centres, -1 if the centre line crosses no film.
 * Errors: SC_E_INVAL (bad index, NULL), SC_E_STATE (no pass yet; nuclei not in two distinct
 * bubbles), SC_E_DEVICE. */
int sc_film_geometry(struct sc_sim* sim, int32_t nucleus_a, int32_t nucleus_b, double* h,
                     double* r_disc, int32_t* n_lines);
/* rho_v[N] (host): density of the gas component (FP64 arithmetic, FP32 out); zeros with one
 * component.  Errors: SC_E_INVAL (NULL), SC_E_STATE, SC_E_DEVICE. */
int sc_gas_density(struct sc_sim* sim, float* rho_v);
/* Gas component at rest with density rho_v[N] (> 0); two components only (SC_E_STATE). */
int sc_set_gas_equilibrium(struct sc_sim* sim, const double* rho_v);
/* *rho0: the buoyancy reference density in use (0 when gravity is off).  Errors: SC_E_INVAL. */
int sc_buoyancy_density(struct sc_sim* sim, double* rho0);
int sc_time(struct sc_sim* sim, int64_t* step);

/* State access for tests and checkpoints.  f is [q][N] FP64 post-streaming populations f_i(x, t)
 * (velocity order: the lattice order of the library, see sc_lattice); set_equilibrium writes
 * f = f_eq(rho, u) with u [d][N] or NULL.  Bubble registry and step count are unchanged. */
int sc_lattice(int32_t lattice, int32_t* e /*[q][3]*/, double* w /*[q]*/);
int sc_get_populations(struct sc_sim* sim, double* f);
int sc_set_populations(struct sc_sim* sim, const double* f);
int sc_set_equilibrium(struct sc_sim* sim, const double* rho, const double* u);
/* The same [q][N] FP64 access to the gas component's populations (two components only,
 * otherwise SC_E_STATE), so a mixture can be saved and restored whole. */
int sc_get_gas_populations(struct sc_sim* sim, double* f);
int sc_set_gas_populations(struct sc_sim* sim, const double* f);
/* Runs a test pass now, with the merge criterion.  */
int sc_test_pass(struct sc_sim* sim);

/* Per-kernel-class timing with HIP events on the simulation's stream: enable != 0 starts
 * recording (and clears the counters); sc_profile_read returns the summed kernel time in ms and
 * the launch count of one class since then. */
int sc_profile(struct sc_sim* sim, int32_t enable);
int sc_profile_read(struct sc_sim* sim, int32_t kernel_class, double* ms, int64_t* launches);

/* Autotuner of the step kernel.  Times every candidate (tile_x, tile_y, tile_z, variant) on the
 * current state with HIP events -- each trial launch reads the current populations and writes the
 * spare buffer, so the simulation is unchanged -- and keeps the fastest for this handle.  The
 * choice is remembered for later handles of the same lattice, box, storage, compute type and
 * component count in this process (two components tune their own fused kernel's shapes).  trials >= 1 launches per candidate; out[cap] (may be NULL) receives the timings
 * in candidate order, *n_out the candidate count. */
typedef struct sc_tune_entry {
    int32_t tile_x, tile_y, tile_z, variant;
    double us_per_launch;
} sc_tune_entry;
int sc_autotune(struct sc_sim* sim, int32_t trials, sc_tune_entry* out, int32_t cap,
                int32_t* n_out);

/* Tile shape and compute type chosen for the step kernel (after tuning or from sc_params). */
int sc_step_config(struct sc_sim* sim, int32_t* tile_x, int32_t* tile_y, int32_t* tile_z,
                   int32_t* variant);
int sc_compute_type(struct sc_sim* sim, int32_t* compute);

/* ---- batch of independent two-bubble D2Q9 boxes (Sec. 4 two-bubble merging, Fig. 3 sizes) ----
 * Every box is filled with liquid plus noise and two gas balls as sc_create + sc_seed_nuclei
 * would (no blowing-agent source), then stepped, with a test pass every test_every steps, until
 * the merge criterion fires, the two nuclei share one gas component, or max_steps.  All boxes run
 * in one persistent kernel launch (captured once in a HIP graph) fed by a work queue; storage is
 * FP32, arithmetic FP64 (AUTO/F64) or FP32. */
typedef struct sc_batch_instance {
    int32_t nx, ny;            /* 4 <= nx <= 256, ny >= 4, periodic */
    double tau, G;
    double rho_liquid, rho_gas, noise_amp;
    uint64_t noise_seed;
    double gas_threshold;      /* <= 0: (rho_liquid + rho_gas)/2 */
    double centre[2][3];       /* the two nuclei (z ignored) */
    double radius[2];
} sc_batch_instance;

typedef struct sc_batch_result {
    int64_t merge_step;        /* step of the criterion firing, -1 if none */
    int64_t topo_step;         /* first test step with both nuclei in one component, -1 if none */
    int64_t steps_run;
    int64_t film_node;         /* c* of the firing (-1 if none) */
    int32_t film_len;
    int32_t status;            /* SC_OK, or SC_E_NUMERIC if a total was not finite */
    double lap_p, rho_film;
    double totals[3];          /* FP64 mass and momentum at the last test pass */
} sc_batch_result;

/* Copies the instance table; allocates [2][9][N] FP32 populations and N labels per box.
 * Errors: SC_E_INVAL (a box outside the limits above), SC_E_NOMEM, SC_E_DEVICE. */
int sc_batch_create(int32_t n, const sc_batch_instance* inst, int32_t test_every,
                    int32_t film_max, int32_t max_steps, int32_t compute, void* stream,
                    const sc_allocator* allocator, struct sc_batch** out);
/* Runs every box from its initial state (repeatable); results[n] may be NULL; *kernel_ms gets
 * the HIP-event time of the launch.  Synchronous. */
int sc_batch_run(struct sc_batch* b, sc_batch_result* results, double* kernel_ms);
/* Autotuner of the batch: runs every box for trial_steps with each candidate number of rows a
 * thread carries per iteration of the box step (1, 2, 4), keeps the fastest.  ms[3] (may be
 * NULL) receives the three timings.  The next sc_batch_run starts from the initial state. */
int sc_batch_tune(struct sc_batch* b, int32_t trial_steps, int32_t* rows_per_thread, double* ms);
/* FP32 density of box k after the last run (FP64 sums of the stored populations). */
int sc_batch_fields(struct sc_batch* b, int32_t k, float* rho);
int sc_batch_destroy(struct sc_batch* b);

/* HBM bandwidth probe: best-of-reps GB/s of a float4 copy (read + write) and of a float4
 * read-only pass over `bytes` (>= 1 MiB) of freshly allocated device memory; the measured
 * ceiling that the step kernel's bandwidth is compared with.  Uses the null stream. */
int sc_hbm_probe(size_t bytes, int32_t reps, double* copy_GBps, double* read_GBps);

/* The D3Q19 step's memory pattern without its arithmetic (pull streaming, Fig. 1 step 1): for
 * an nx x ny x nz box of `storage` (SC_STORE_F32 / F16 / BF16) elements, 19 arrays of
 * populations, every population of every node read from its upstream neighbour (periodic) and
 * written with non-temporal stores, on freshly allocated device memory (2 x 19 N elements,
 * freed on return; the null stream).  flat_GBps: one node per thread; march_GBps: blocks of
 * tile_x * tile_y (<= 1024) threads, each a tile_x x tile_y tile marching tile_z planes in
 * the step kernel's block order.  Best of `reps` timed launches after one untimed, as read +
 * written bytes per second.  SC_E_INVAL for a bad box (nx <= 2^30, ny, nz <= 65535; N
 * elements of at most 2^32 bytes per direction), tile, storage or reps; SC_E_DEVICE or the
 * allocation's error otherwise. */
int sc_pattern_probe(int32_t nx, int32_t ny, int32_t nz, int32_t storage, int32_t tile_x,
                     int32_t tile_y, int32_t tile_z, int32_t reps, double* flat_GBps,
                     double* march_GBps);

typedef struct sc_sim sc_sim;
typedef struct sc_batch sc_batch;

#ifdef __cplusplus
}
#endif
#endif
