/*
 * sc_oracle.h -- FP64 CPU oracle of the Shan-Chen bubble growth / merging time step.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes or calls this code;
 * only the test suite, the smoke check and the benchmark's CPU-baseline leg load it.  It shares
 * no source, header, table or helper with the HIP library: the lattice velocity sets are
 * enumerated here from their definition, and the random field is produced here from the
 * published SplitMix64 definition.
 *
 * Paper: Barzegari, Bayani, Mirbagheri, "A criterion for bubble merging in liquid metal:
 * computational and experimental study" (arXiv 1708.01608).
 *   Sec. 3      gas added to each bubble by a virtual blowing agent until the agent is spent;
 *               merging by film rupture, decided by the sign change of the pressure Laplacian.
 *   Sec. 3.1    random nucleation sites, liquid elsewhere; Shan-Chen pseudopotential model with
 *               EOS p0 = rho cs^2 + 0.166 G psi^2 and psi(rho) = 1 - exp(-rho); merge switch
 *               eta_m from the second derivative of pressure across the film.
 *   Sec. 4      pressure profile along the line between two bubbles (Fig. 2); rupture when the
 *               second derivative of pressure vanishes.
 *   Fig. 1      step order: init, stream/collide with interaction, new bubble sizes, merge, output.
 *
 * Everything the paper leaves open (lattice, forcing scheme, force sign and weights, noise,
 * labelling connectivity, film walk, ...) follows one stated reading per point; the readings
 * are listed with the design notes of the repository.
 *
 * Pins: every function below is checked by the test suite against something other than
 * itself (closed forms, conservation laws, brute force, the coexistence and Laplace laws, the
 * spinodal sign rule of the criterion).  The merge and topological steps a run produces are
 * pinned by the lattice's symmetries (a translated or rotated box gives the same run moved
 * with it) and by film-thickness ordering; their values themselves have no reference, because
 * the paper prints no merge time or film profile, and are compared GPU against oracle.
 */
#ifndef SC_ORACLE_H
#define SC_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct orc_sim orc_sim;

/* One merge-criterion firing (Sec. 3.1 eta_m switch, Sec. 4 film rupture). */
typedef struct {
    int64_t step;        /* time step of the test pass that fired */
    int32_t nucleus_a;   /* smallest nucleus index of bubble a */
    int32_t nucleus_b;   /* smallest nucleus index of bubble b */
    uint32_t label_a;    /* component labels at that pass (label_a < label_b) */
    uint32_t label_b;
    int64_t film_node;   /* linear index of the film-centre node c* */
    int32_t film_len;    /* number of liquid nodes on the film run */
    int32_t pad;
    double lap_p;        /* lattice Laplacian of p at c* (>= 0 fired) */
    double rho_film;     /* density at c* */
} orc_event;

/* Two nucleus groups found in one gas component for the first time (topological merge). */
typedef struct {
    int64_t step;
    int32_t nucleus_a;   /* group representative (smallest nucleus index), a < b */
    int32_t nucleus_b;
} orc_topo_event;

/* Per-bubble statistics of the last test pass. */
typedef struct {
    uint32_t label;      /* 1 + smallest linear index of the component */
    int32_t nucleus;     /* smallest nucleus index in the bubble (the anchor nucleus) */
    int64_t n;           /* gas node count n_b */
    double centroid[3];  /* anchor + mean minimal-image integer offset */
    double radius;       /* sqrt(n/pi) in 2D, cbrt(3n/(4 pi)) in 3D */
    int32_t n_nuclei;
    int32_t pad;
} orc_bubble;

/* q = 9 (D2Q9, nz must be 1) or 19 (D3Q19).  Fills rho = rho_l + amp (2U - 1) on every node and
 * f = f_eq(rho, 0).  theta <= 0 selects (rho_l + rho_g)/2.  K = test cadence (0: seed pass only).
 * Returns NULL on invalid arguments or allocation failure. */
orc_sim* orc_create(int q, int nx, int ny, int nz, double tau, double G, double rho_l,
                    double rho_g, double amp, uint64_t seed, double theta, int K, int film_max);
void orc_destroy(orc_sim* s);

/* Paint nuclei (rho = rho_g + amp (2U - 1), f = f_eq(rho, 0) where the minimal-image distance to
 * a centre is <= its radius; a negative radius registers the nucleus without painting), set
 * budgets, run the test pass at the current step (labels and statistics, no criterion).
 * centre is [n][3] (z ignored in 2D).  Returns 0, or -5 if the totals are not finite. */
int orc_seed_nuclei(orc_sim* s, int n, const double* centre, const double* radius,
                    const double* budget, double rate);

/* Modified Shan-Chen barrier (Sec. 3.1, Fig. 1 steps 3-6): with on != 0 every bubble owns its
 * gas nodes and `corona` liquid layers around them, and in the force a neighbour owned by a
 * different bubble not merged by the criterion contributes psi(rho_l) instead of its own psi.
 * The owner field is rebuilt now and at the end of every test pass (after that pass's merges).
 * Returns 0, or -1 if corona < 0. */
int orc_set_barrier(orc_sim* s, int on, int corona);
/* owner[N]: 0 = nobody, else 1 + the smallest nucleus index of the owning merged group. */
int orc_owner(const orc_sim* s, int32_t* owner);

/* Two components (a liquid and a gas, so that the blowing agent's gas grows the bubbles):
 * Shan-Doolen mixture with psi = rho, the force on component a being
 * -Gx rho_a(x) sum_i w_i rho_b(x + e_i) e_i, a common velocity
 * u' = sum_a (j_a / tau_a) / sum_a (rho_a / tau_a), equilibria at u' + tau_a F_a / rho_a.  The
 * liquid component keeps the existing populations (rho_l, rho_g, theta and labels refer to it;
 * G is not used); the gas component fills the box with rho_dissolved and painted nuclei with
 * rho_vapour; the blowing agent feeds the gas component; the criterion uses
 * p = (rho_l + rho_v)/3 + (Gx/3) rho_l rho_v; fields report the liquid density and the mixture's
 * barycentric velocity (j_l + j_v + (F_l + F_v)/2) / (rho_l + rho_v); totals sum both components.
 * Call before seeding.  Returns 0, -1 (bad parameters) or -2 (no memory). */
int orc_set_two_component(orc_sim* s, double Gx, double tau_v, double rho_vapour,
                          double rho_dissolved);
/* Gas component at rest with density rho_v[N] (two-component mode only; else returns -1). */
int orc_set_gas_equilibrium(orc_sim* s, const double* rho_v);
/* rho_v[N]: density of the gas component (zeros with one component). */
void orc_gas_density(const orc_sim* s, double* rho_v);

/* Gravity (drainage; the paper's runs leave it out): a body force (rho - rho0) g is added to the
 * Shan-Chen force of every node, in the collision and in the reported velocity.  g is [3] (z
 * ignored in 2D).  rho0 <= 0 selects the mean density of the box, taken now and again when
 * nuclei are seeded, which makes the net body force zero.  Returns 0, or -1 if not finite. */
int orc_set_gravity(orc_sim* s, const double* g, double rho0);
/* The buoyancy reference density in use. */
double orc_rho0(const orc_sim* s);

/* Advance nsteps time steps (collide-stream, source, test pass every K steps).
 * Returns 0, or -5 once a total is not finite. */
int orc_step(orc_sim* s, int nsteps);

/* rho[N], u[d][N] = (j + F/2)/rho, totals[4] = (M, Jx, Jy, Jz); any pointer may be NULL. */
void orc_fields(const orc_sim* s, double* rho, double* u, double* totals);
/* p[N] = rho/3 + (G/6) psi^2 and lap[N] = 6 sum_i w_i (p(x+e_i) - p(x)); NULL skips. */
void orc_laplacian_p(const orc_sim* s, double* p, double* lap);
/* F[d][N], the Shan-Chen force on the current state (with the barrier when it is on; the
 * mixture's total F_l + F_v in two-component mode). */
void orc_force(const orc_sim* s, double* F);

/* Canonical periodic labelling of a mask: label = 1 + smallest linear index of the component,
 * 0 where mask == 0; connectivity = the q-1 lattice neighbours.  Returns the component count. */
int64_t orc_label_mask(int q, int nx, int ny, int nz, const uint8_t* mask, uint32_t* labels);

/* State access (tests and checkpoints).  f is [q][N], post-streaming populations f_i(x, t). */
void orc_get_f(const orc_sim* s, double* f);
void orc_set_f(orc_sim* s, const double* f);
/* f = f_eq(rho, u) on every node; u is [d][N] or NULL (zero velocity). */
void orc_set_equilibrium(orc_sim* s, const double* rho, const double* u);
/* Run a test pass now (as at seeding); returns 0 or -5. */
int orc_test_pass(orc_sim* s);

/* Film geometry of the pair of bubbles holding nuclei a and b at the last test pass (Sec. 3:
 * the film as a disc of radius R_d and thickness h; Fig. 3).  Lines parallel to the centroid
 * segment, shifted by integer multiples of an orthonormal basis of the perpendicular plane up to
 * the smaller bubble radius, are walked like the merge test's centre line; *n_lines counts those
 * that cross a film of 1..film_max liquid nodes between the two bubbles, *r_disc = n_lines/2
 * (2D) or sqrt(n_lines/pi) (3D).  *h = distance between the rho = theta crossings on the centre
 * line (linear in arc length), -1 if that line crosses no film.  Returns 0, -1 (bad nucleus)
 * or -4 (the nuclei are not in two distinct bubbles). */
int orc_film_geometry(const orc_sim* s, int nucleus_a, int nucleus_b, double* h, double* r_disc,
                      int* n_lines);

int64_t orc_time(const orc_sim* s);
int64_t orc_num_nodes(const orc_sim* s);
int orc_labels(const orc_sim* s, uint32_t* labels);                  /* last test pass */
int orc_bubbles(const orc_sim* s, orc_bubble* out, int cap);         /* returns count */
int orc_events(const orc_sim* s, orc_event* out, int cap);           /* returns count */
int orc_topo_events(const orc_sim* s, orc_topo_event* out, int cap); /* returns count */
/* comp[n] = label of each nucleus's node at the last pass (0 = not gas), rem[n] = budgets left. */
int orc_nuclei(const orc_sim* s, uint32_t* comp, double* rem);

/* Pieces exposed for the pins. */
void orc_lattice(int q, int* e /*[q][3]*/, double* w /*[q]*/);
void orc_feq(int q, double rho, const double* u /*[3]*/, double* out /*[q]*/);
double orc_uniform(uint64_t seed, uint64_t idx);  /* U(seed, idx) in [0, 1) */
uint64_t orc_splitmix64(uint64_t seed, uint64_t k); /* k-th output (k >= 1) of the stream */
int orc_num_threads(void);                            /* OpenMP threads the oracle uses */

#ifdef __cplusplus
}
#endif
#endif
