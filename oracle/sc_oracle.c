/*
 * sc_oracle.c -- FP64 CPU oracle (test infrastructure only; see sc_oracle.h).
 *
 * Plain loops in double precision, in the order the method states them.  OpenMP is used only
 * over lattice nodes that are independent within one phase; every reduction runs serially in
 * index order, so results do not depend on the thread count.
 */
#include "sc_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* ------------------------------------------------------------------------------------------ */
/* Lattice velocity sets, enumerated from their definition.                                   */
/* D2Q9: every e in {-1,0,1}^2; w = 4/9 (|e|^2=0), 1/9 (|e|^2=1), 1/36 (|e|^2=2).             */
/* D3Q19: every e in {-1,0,1}^3 with |e|^2 <= 2; w = 1/3, 1/18, 1/36 by |e|^2.                */
/* The isotropy sum_i w_i e_i e_i = (1/3) I that these weights give is what turns the         */
/* Shan-Chen force into the EOS p0 = rho cs^2 + (G cs^2/2) psi^2 with cs^2 = 1/3 (Sec. 3.1).  */
/* ------------------------------------------------------------------------------------------ */
typedef struct {
    int q, d;
    int e[19][3];
    double w[19];
} lattice;

static int lattice_make(lattice* L, int q)
{
    int n = 0;
    memset(L, 0, sizeof(*L));
    if (q == 9) {
        L->q = 9; L->d = 2;
        for (int ey = -1; ey <= 1; ++ey)
            for (int ex = -1; ex <= 1; ++ex) {
                int m = ex * ex + ey * ey;
                L->e[n][0] = ex; L->e[n][1] = ey; L->e[n][2] = 0;
                L->w[n] = (m == 0) ? 4.0 / 9.0 : (m == 1) ? 1.0 / 9.0 : 1.0 / 36.0;
                ++n;
            }
    } else if (q == 19) {
        L->q = 19; L->d = 3;
        for (int ez = -1; ez <= 1; ++ez)
            for (int ey = -1; ey <= 1; ++ey)
                for (int ex = -1; ex <= 1; ++ex) {
                    int m = ex * ex + ey * ey + ez * ez;
                    if (m > 2) continue;
                    L->e[n][0] = ex; L->e[n][1] = ey; L->e[n][2] = ez;
                    L->w[n] = (m == 0) ? 1.0 / 3.0 : (m == 1) ? 1.0 / 18.0 : 1.0 / 36.0;
                    ++n;
                }
    } else {
        return -1;
    }
    return (n == q) ? 0 : -1;
}

void orc_lattice(int q, int* e, double* w)
{
    lattice L;
    if (lattice_make(&L, q) != 0) return;
    for (int i = 0; i < q; ++i) {
        for (int a = 0; a < 3; ++a) e[3 * i + a] = L.e[i][a];
        w[i] = L.w[i];
    }
}

/* Second-order equilibrium of the BGK model (textbook form, cs^2 = 1/3):
 * f_i^eq = w_i rho [1 + e.u/cs^2 + (e.u)^2/(2 cs^4) - u.u/(2 cs^2)]. */
static double feq_one(const lattice* L, int i, double rho, const double u[3])
{
    const double cs2 = 1.0 / 3.0;
    double eu = L->e[i][0] * u[0] + L->e[i][1] * u[1] + L->e[i][2] * u[2];
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    return L->w[i] * rho * (1.0 + eu / cs2 + (eu * eu) / (2.0 * cs2 * cs2) - uu / (2.0 * cs2));
}

void orc_feq(int q, double rho, const double* u, double* out)
{
    lattice L;
    if (lattice_make(&L, q) != 0) return;
    for (int i = 0; i < q; ++i) out[i] = feq_one(&L, i, rho, u);
}

/* ------------------------------------------------------------------------------------------ */
/* SplitMix64 (Steele, Lea, Flood, "Fast splittable pseudorandom number generators", OOPSLA    */
/* 2014, with the 64-bit finaliser constants of its public reference implementation).  The    */
/* stream seeded with s has state s + k*gamma before the k-th output is mixed, so the k-th     */
/* output is a pure function of (s, k): every lattice node draws its own value independently.  */
/* ------------------------------------------------------------------------------------------ */
uint64_t orc_splitmix64(uint64_t seed, uint64_t k)
{
    uint64_t z = seed + k * 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* U(seed, idx): top 53 bits of the (idx+1)-th output, scaled to [0, 1). */
double orc_uniform(uint64_t seed, uint64_t idx)
{
    return (double)(orc_splitmix64(seed, idx + 1) >> 11) * (1.0 / 9007199254740992.0);
}

/* ------------------------------------------------------------------------------------------ */
/* Simulation state                                                                            */
/* ------------------------------------------------------------------------------------------ */
struct orc_sim {
    lattice L;
    int nx, ny, nz;
    int64_t N;
    double tau, G, rho_l, rho_g, amp, theta;
    uint64_t seed;
    int K, film_max;
    double* f;   /* [q][N] post-streaming populations f_i(x, t) */
    double* fn;  /* second buffer */
    int64_t t;
    int numeric_error;

    /* nuclei (Sec. 3.1: nucleation sites and the blowing agent decomposed at them) */
    int n_nuc;
    double* cen;      /* [n][3] */
    double* rad;
    double* rem;      /* agent mass left per nucleus */
    double rate;      /* q: mass per step per nucleus while its budget lasts */
    int64_t* nuc_node;
    uint32_t* comp;   /* label at the nucleus node, last pass */
    int* merge_parent; /* criterion-merged nucleus groups (eta_m flipped to 0) */
    int* topo_parent;  /* nucleus groups that have shared a component */

    /* modified Shan-Chen barrier (Sec. 3.1, Fig. 1 steps 3-6): off unless orc_set_barrier */
    int barrier;       /* 1: bubbles interact only through the liquid until eta_m flips */
    int corona;        /* liquid layers a bubble owns around its gas */
    double psi_l;      /* psi(rho_l): what a bubble sees where another bubble's lattice is */
    int32_t* owner;    /* [N] owner id of each node (0: nobody), rebuilt at every test pass */

    /* two components (liquid, gas; off unless orc_set_two_component): Shan-Doolen mixture with
     * psi = rho and a cross interaction Gx; fv/fvn are the gas component's populations */
    int ncomp;
    double Gx, tau_v, rho_vap, rho_dis;
    double* fv;
    double* fvn;

    /* gravity (drainage, Sec. 3; off unless orc_set_gravity): body force (rho - rho0) g */
    double g[3];
    double rho0;       /* buoyancy reference density */
    int rho0_auto;     /* rho0 = mean density, taken now and again at the seed pass */

    /* last test pass */
    uint32_t* labels;  /* [N] */
    int nb;
    orc_bubble* bub;
    int* bub_of_label; /* [N+1]: bubble index of a label, -1 if none */

    orc_event* ev; int nev, cap_ev;
    orc_topo_event* tev; int ntev, cap_tev;
};

static int64_t node_index(const orc_sim* s, int x, int y, int z)
{
    return (int64_t)x + (int64_t)s->nx * ((int64_t)y + (int64_t)s->ny * z);
}

static void node_coords(const orc_sim* s, int64_t idx, int c[3])
{
    c[0] = (int)(idx % s->nx);
    c[1] = (int)((idx / s->nx) % s->ny);
    c[2] = (int)(idx / ((int64_t)s->nx * s->ny));
}

static int wrap(int a, int n)
{
    int r = a % n;
    return r < 0 ? r + n : r;
}

/* Periodic neighbour x + e_i (all axes periodic). */
static int64_t neighbour(const orc_sim* s, int64_t idx, int i)
{
    int c[3];
    node_coords(s, idx, c);
    return node_index(s, wrap(c[0] + s->L.e[i][0], s->nx), wrap(c[1] + s->L.e[i][1], s->ny),
                      wrap(c[2] + s->L.e[i][2], s->nz));
}

/* psi(rho) = 1 - exp(-rho) (Sec. 3.1, reference density 1). */
static double psi_of(double rho) { return 1.0 - exp(-rho); }

/* Bulk pressure p = rho cs^2 + (G cs^2 / 2) psi^2 = rho/3 + (G/6) psi^2 (Sec. 3.1; the printed
 * 0.166 is G cs^2/2 = G/6 truncated). */
static double pressure_of(double rho, double G)
{
    double ps = psi_of(rho);
    return rho / 3.0 + (G / 6.0) * ps * ps;
}

static double node_density(const orc_sim* s, const double* f, int64_t x)
{
    double r = 0.0;
    for (int i = 0; i < s->L.q; ++i) r += f[(int64_t)i * s->N + x];
    return r;
}

static void node_momentum(const orc_sim* s, const double* f, int64_t x, double j[3])
{
    j[0] = j[1] = j[2] = 0.0;
    for (int i = 0; i < s->L.q; ++i) {
        double fi = f[(int64_t)i * s->N + x];
        for (int a = 0; a < 3; ++a) j[a] += fi * s->L.e[i][a];
    }
}

/* Shan-Chen interaction force F(x) = -G psi(x) sum_{i != 0} w_i psi(x + e_i) e_i (Sec. 3.1,
 * ref. [5]).  The minus sign makes G < 0 attractive and reproduces p0 of Sec. 3.1. */
static void sc_force(const orc_sim* s, const double* psi, int64_t x, double F[3])
{
    double acc[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < s->L.q; ++i) {
        if (s->L.e[i][0] == 0 && s->L.e[i][1] == 0 && s->L.e[i][2] == 0) continue;
        int64_t y = neighbour(s, x, i);
        double pn = psi[y];
        /* Barrier: each bubble lives on its own lattice and meets the others only through the
         * liquid (Sec. 3.1), so a neighbour held by a different, un-merged bubble is seen as
         * bulk liquid. */
        if (s->barrier && s->owner[x] != 0 && s->owner[y] != 0 && s->owner[x] != s->owner[y])
            pn = s->psi_l;
        for (int a = 0; a < 3; ++a) acc[a] += s->L.w[i] * pn * s->L.e[i][a];
    }
    for (int a = 0; a < 3; ++a) F[a] = -s->G * psi[x] * acc[a];
}

static void psi_field(const orc_sim* s, double* psi)
{
    int64_t N = s->N;
#pragma omp parallel for schedule(static)
    for (int64_t x = 0; x < N; ++x) psi[x] = psi_of(node_density(s, s->f, x));
}

/* ------------------------------------------------------------------------------------------ */
/* Creation and nucleus painting (Sec. 3.1 first paragraph).                                   */
/* ------------------------------------------------------------------------------------------ */
orc_sim* orc_create(int q, int nx, int ny, int nz, double tau, double G, double rho_l,
                    double rho_g, double amp, uint64_t seed, double theta, int K, int film_max)
{
    lattice L;
    if (lattice_make(&L, q) != 0) return NULL;
    if (nx < 4 || ny < 4 || nz < 1) return NULL;
    if (q == 9 && nz != 1) return NULL;
    if (q == 19 && nz < 4) return NULL;
    if (!(tau > 0.5) || K < 0 || film_max < 1) return NULL;
    orc_sim* s = (orc_sim*)calloc(1, sizeof(orc_sim));
    if (!s) return NULL;
    s->L = L;
    s->nx = nx; s->ny = ny; s->nz = nz;
    s->N = (int64_t)nx * ny * nz;
    s->tau = tau; s->G = G; s->rho_l = rho_l; s->rho_g = rho_g; s->amp = amp; s->seed = seed;
    s->theta = (theta > 0.0) ? theta : 0.5 * (rho_l + rho_g);
    s->K = K; s->film_max = film_max;
    s->f = (double*)malloc(sizeof(double) * (size_t)q * (size_t)s->N);
    s->fn = (double*)malloc(sizeof(double) * (size_t)q * (size_t)s->N);
    s->labels = (uint32_t*)calloc((size_t)s->N, sizeof(uint32_t));
    s->owner = (int32_t*)calloc((size_t)s->N, sizeof(int32_t));
    s->psi_l = psi_of(rho_l);
    s->bub_of_label = (int*)malloc(sizeof(int) * (size_t)(s->N + 1));
    if (!s->f || !s->fn || !s->labels || !s->owner || !s->bub_of_label) { orc_destroy(s); return NULL; }
    for (int64_t l = 0; l <= s->N; ++l) s->bub_of_label[l] = -1;

    /* rho(x) = rho_l + amp (2U - 1) on every node; f = f_eq(rho, 0). */
    const double zero[3] = {0.0, 0.0, 0.0};
    int64_t N = s->N;
#pragma omp parallel for schedule(static)
    for (int64_t x = 0; x < N; ++x) {
        double rho = rho_l + amp * (2.0 * orc_uniform(seed, (uint64_t)x) - 1.0);
        for (int i = 0; i < q; ++i) s->f[(int64_t)i * N + x] = feq_one(&s->L, i, rho, zero);
    }
    return s;
}

void orc_destroy(orc_sim* s)
{
    if (!s) return;
    free(s->f); free(s->fn); free(s->fv); free(s->fvn); free(s->labels); free(s->owner);
    free(s->bub_of_label); free(s->bub);
    free(s->cen); free(s->rad); free(s->rem); free(s->nuc_node); free(s->comp);
    free(s->merge_parent); free(s->topo_parent); free(s->ev); free(s->tev);
    free(s);
}

/* Minimal-image difference of a real coordinate: d - n floor(d/n + 1/2). */
static double min_image(double d, int n) { return d - n * floor(d / n + 0.5); }

/* Integer minimal image into [-floor(n/2), n - 1 - floor(n/2)]. */
static int64_t min_image_int(int64_t d, int n)
{
    int64_t h = n / 2;
    int64_t r = (d + h) % n;
    if (r < 0) r += n;
    return r - h;
}

/* Node nearest to a point: floor(c + 1/2) per axis, wrapped. */
static int64_t nearest_node(const orc_sim* s, const double c[3])
{
    int x = wrap((int)floor(c[0] + 0.5), s->nx);
    int y = wrap((int)floor(c[1] + 0.5), s->ny);
    int z = (s->L.d == 3) ? wrap((int)floor(c[2] + 0.5), s->nz) : 0;
    return node_index(s, x, y, z);
}

static int test_pass(orc_sim* s, int with_criterion);

static double mean_density(const orc_sim* s)
{
    double M = 0.0;
    for (int64_t x = 0; x < s->N; ++x) M += node_density(s, s->f, x);
    return M / (double)s->N;
}

int orc_set_gravity(orc_sim* s, const double* g, double rho0)
{
    for (int a = 0; a < 3; ++a) {
        if (!isfinite(g[a])) return -1;
        s->g[a] = (a < s->L.d) ? g[a] : 0.0;
    }
    if (!isfinite(rho0)) return -1;
    s->rho0_auto = rho0 <= 0.0;
    s->rho0 = s->rho0_auto ? mean_density(s) : rho0;
    return 0;
}

int orc_seed_nuclei(orc_sim* s, int n, const double* centre, const double* radius,
                    const double* budget, double rate)
{
    if (n < 0 || (n > 0 && (!centre || !radius || !budget)) || rate < 0.0) return -1;
    free(s->cen); free(s->rad); free(s->rem); free(s->nuc_node); free(s->comp);
    free(s->merge_parent); free(s->topo_parent);
    s->n_nuc = n;
    size_t m = n > 0 ? (size_t)n : 1;
    s->cen = (double*)calloc(3 * m, sizeof(double));
    s->rad = (double*)calloc(m, sizeof(double));
    s->rem = (double*)calloc(m, sizeof(double));
    s->nuc_node = (int64_t*)calloc(m, sizeof(int64_t));
    s->comp = (uint32_t*)calloc(m, sizeof(uint32_t));
    s->merge_parent = (int*)calloc(m, sizeof(int));
    s->topo_parent = (int*)calloc(m, sizeof(int));
    s->rate = rate;
    for (int k = 0; k < n; ++k) {
        for (int a = 0; a < 3; ++a) s->cen[3 * k + a] = centre[3 * k + a];
        if (s->L.d == 2) s->cen[3 * k + 2] = 0.0;
        s->rad[k] = radius[k];
        s->rem[k] = budget[k];
        s->nuc_node[k] = nearest_node(s, &s->cen[3 * k]);
        s->merge_parent[k] = k;
        s->topo_parent[k] = k;
    }

    /* Gas where the minimal-image distance to some centre is <= its radius. */
    const double zero[3] = {0.0, 0.0, 0.0};
    int64_t N = s->N;
    int q = s->L.q;
#pragma omp parallel for schedule(static)
    for (int64_t x = 0; x < N; ++x) {
        int c[3];
        node_coords(s, x, c);
        int gas = 0;
        for (int k = 0; k < n && !gas; ++k) {
            double dx = min_image((double)c[0] - s->cen[3 * k + 0], s->nx);
            double dy = min_image((double)c[1] - s->cen[3 * k + 1], s->ny);
            double dz = (s->L.d == 3) ? min_image((double)c[2] - s->cen[3 * k + 2], s->nz) : 0.0;
            if (s->rad[k] >= 0.0 && dx * dx + dy * dy + dz * dz <= s->rad[k] * s->rad[k]) gas = 1;
        }
        if (gas) {
            double rho = s->rho_g + s->amp * (2.0 * orc_uniform(s->seed, (uint64_t)x) - 1.0);
            for (int i = 0; i < q; ++i) s->f[(int64_t)i * N + x] = feq_one(&s->L, i, rho, zero);
            if (s->ncomp == 2)  /* the bubble is filled with the gas component */
                for (int i = 0; i < q; ++i)
                    s->fv[(int64_t)i * N + x] = feq_one(&s->L, i, s->rho_vap, zero);
        }
    }
    /* the buoyancy reference follows the seeded box when it is the mean density */
    if (s->rho0_auto) s->rho0 = mean_density(s);
    /* The pass run by seeding labels the painted bubbles but does not evaluate the criterion:
     * a painted step profile has no film yet, and p(rho_g) ~ p(rho_l) there. */
    return test_pass(s, 0);
}

/* ------------------------------------------------------------------------------------------ */
/* One time step: moments, pseudopotential, force, forced BGK collision, streaming.            */
/* ------------------------------------------------------------------------------------------ */
/* Cross interaction of the two-component mixture (Shan & Doolen): the force on component a at x
 * is -Gx rho_a(x) sum_{i != 0} w_i rho_b(x + e_i) e_i, b the other component (psi = rho). */
static void cross_force(const orc_sim* s, const double* rho_a, const double* rho_b, int64_t x,
                        double F[3])
{
    double acc[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < s->L.q; ++i) {
        if (s->L.e[i][0] == 0 && s->L.e[i][1] == 0 && s->L.e[i][2] == 0) continue;
        double rn = rho_b[neighbour(s, x, i)];
        for (int a = 0; a < 3; ++a) acc[a] += s->L.w[i] * rn * s->L.e[i][a];
    }
    for (int a = 0; a < 3; ++a) F[a] = -s->Gx * rho_a[x] * acc[a];
}

/* Two-component step: common velocity u' = sum_a (j_a / tau_a) / sum_a (rho_a / tau_a); each
 * component relaxes to its equilibrium at u' + tau_a F_a / rho_a with its own tau, then streams. */
static void collide_stream_2c(orc_sim* s)
{
    int64_t N = s->N;
    int q = s->L.q;
    double* rl = (double*)malloc(sizeof(double) * (size_t)N);
    double* rv = (double*)malloc(sizeof(double) * (size_t)N);
    for (int64_t x = 0; x < N; ++x) {
        rl[x] = node_density(s, s->f, x);
        rv[x] = node_density(s, s->fv, x);
    }
#pragma omp parallel for schedule(static)
    for (int64_t x = 0; x < N; ++x) {
        double jl[3], jv[3], Fl[3], Fv[3], up[3], ul[3], uv[3];
        node_momentum(s, s->f, x, jl);
        node_momentum(s, s->fv, x, jv);
        cross_force(s, rl, rv, x, Fl);
        cross_force(s, rv, rl, x, Fv);
        double den = rl[x] / s->tau + rv[x] / s->tau_v;
        for (int a = 0; a < 3; ++a) {
            up[a] = (jl[a] / s->tau + jv[a] / s->tau_v) / den;
            ul[a] = up[a] + s->tau * Fl[a] / rl[x];
            uv[a] = up[a] + s->tau_v * Fv[a] / rv[x];
        }
        for (int i = 0; i < q; ++i) {
            double fl = s->f[(int64_t)i * N + x], fv = s->fv[(int64_t)i * N + x];
            int64_t y = neighbour(s, x, i);
            s->fn[(int64_t)i * N + y] = fl - (fl - feq_one(&s->L, i, rl[x], ul)) / s->tau;
            s->fvn[(int64_t)i * N + y] = fv - (fv - feq_one(&s->L, i, rv[x], uv)) / s->tau_v;
        }
    }
    double* tmp = s->f; s->f = s->fn; s->fn = tmp;
    tmp = s->fv; s->fv = s->fvn; s->fvn = tmp;
    free(rl);
    free(rv);
}

static void collide_stream(orc_sim* s)
{
    if (s->ncomp == 2) {
        collide_stream_2c(s);
        return;
    }
    int64_t N = s->N;
    int q = s->L.q;
    double* psi = (double*)malloc(sizeof(double) * (size_t)N);

    /* psi(x) from rho(x) = sum_i f_i(x). */
    psi_field(s, psi);

#pragma omp parallel for schedule(static)
    for (int64_t x = 0; x < N; ++x) {
        double rho = node_density(s, s->f, x);
        double j[3], F[3], u[3], ueq[3];
        node_momentum(s, s->f, x, j);
        sc_force(s, psi, x, F);
        /* gravity: buoyancy body force relative to rho0 */
        for (int a = 0; a < 3; ++a) F[a] += (rho - s->rho0) * s->g[a];
        /* Original Shan-Chen forcing: the equilibrium velocity is shifted by tau F / rho. */
        for (int a = 0; a < 3; ++a) {
            u[a] = j[a] / rho;
            ueq[a] = u[a] + s->tau * F[a] / rho;
        }
        for (int i = 0; i < q; ++i) {
            double fi = s->f[(int64_t)i * N + x];
            double fstar = fi - (fi - feq_one(&s->L, i, rho, ueq)) / s->tau;
            /* streaming: the post-collision value moves to x + e_i */
            s->fn[(int64_t)i * N + neighbour(s, x, i)] = fstar;
        }
    }
    double* tmp = s->f; s->f = s->fn; s->fn = tmp;
    free(psi);
}

/* Virtual blowing agent (Sec. 3): after streaming, each bubble b receives
 * dm_b = sum_{k in S_b} min(rate, rem_k), spread as w_i dm_b / n_b over its gas nodes
 * (zero momentum); each contributing budget decreases by what it gave. */
static void growth_source(orc_sim* s)
{
    if (s->rate <= 0.0 || s->nb == 0) return;
    int64_t N = s->N;
    int q = s->L.q;
    double* add = (double*)calloc((size_t)s->nb, sizeof(double));
    for (int b = 0; b < s->nb; ++b) {
        double dm = 0.0;
        for (int k = 0; k < s->n_nuc; ++k) {
            if (s->comp[k] != s->bub[b].label) continue;
            double d = s->rem[k] < s->rate ? s->rem[k] : s->rate;
            dm += d;
            s->rem[k] -= d;
        }
        add[b] = dm / (double)s->bub[b].n;
    }
#pragma omp parallel for schedule(static)
    for (int64_t x = 0; x < N; ++x) {
        uint32_t lab = s->labels[x];
        if (lab == 0) continue;
        int b = s->bub_of_label[lab];
        if (b < 0 || add[b] == 0.0) continue;
        /* the agent's gas goes to the gas component when there is one */
        double* target = s->ncomp == 2 ? s->fv : s->f;
        for (int i = 0; i < q; ++i) target[(int64_t)i * N + x] += s->L.w[i] * add[b];
    }
    free(add);
}

/* EOS of the two-component mixture: p = (rho_l + rho_v)/3 + (Gx/3) rho_l rho_v (the bulk
 * pressure of the cross interaction with psi = rho and cs^2 = 1/3). */
static double pressure_2c(double rl, double rv, double Gx)
{
    return (rl + rv) / 3.0 + (Gx / 3.0) * rl * rv;
}

/* EOS pressure of node x: one- or two-component. */
static double node_pressure(const orc_sim* s, int64_t x)
{
    if (s->ncomp == 2)
        return pressure_2c(node_density(s, s->f, x), node_density(s, s->fv, x), s->Gx);
    return pressure_of(node_density(s, s->f, x), s->G);
}

int orc_set_two_component(orc_sim* s, double Gx, double tau_v, double rho_vapour,
                          double rho_dissolved)
{
    if (!isfinite(Gx) || !(tau_v > 0.5) || !(rho_vapour > 0.0) || !(rho_dissolved > 0.0))
        return -1;
    int64_t N = s->N;
    int q = s->L.q;
    s->fv = (double*)malloc(sizeof(double) * (size_t)q * (size_t)N);
    s->fvn = (double*)malloc(sizeof(double) * (size_t)q * (size_t)N);
    if (!s->fv || !s->fvn) return -2;
    s->ncomp = 2;
    s->Gx = Gx;
    s->tau_v = tau_v;
    s->rho_vap = rho_vapour;
    s->rho_dis = rho_dissolved;
    const double zero[3] = {0.0, 0.0, 0.0};
    /* the liquid holds rho_dissolved of the gas component everywhere until nuclei are painted */
    for (int64_t x = 0; x < N; ++x)
        for (int i = 0; i < q; ++i) s->fv[(int64_t)i * N + x] = feq_one(&s->L, i, rho_dissolved, zero);
    return 0;
}

int orc_set_gas_equilibrium(orc_sim* s, const double* rho_v)
{
    if (s->ncomp != 2) return -1;
    const double zero[3] = {0.0, 0.0, 0.0};
    for (int64_t x = 0; x < s->N; ++x)
        for (int i = 0; i < s->L.q; ++i)
            s->fv[(int64_t)i * s->N + x] = feq_one(&s->L, i, rho_v[x], zero);
    return 0;
}

void orc_gas_density(const orc_sim* s, double* rho_v)
{
    for (int64_t x = 0; x < s->N; ++x) rho_v[x] = s->ncomp == 2 ? node_density(s, s->fv, x) : 0.0;
}

/* ------------------------------------------------------------------------------------------ */
/* Gas-phase labelling: textbook breadth-first flood fill, seeds taken in increasing index so  */
/* the first node reached of each component is its smallest index.                            */
/* ------------------------------------------------------------------------------------------ */
static int64_t label_components(const lattice* L, int nx, int ny, int nz, const uint8_t* mask,
                                uint32_t* labels)
{
    orc_sim g;
    memset(&g, 0, sizeof(g));
    g.L = *L; g.nx = nx; g.ny = ny; g.nz = nz; g.N = (int64_t)nx * ny * nz;
    int64_t N = g.N, ncomp = 0;
    int64_t* queue = (int64_t*)malloc(sizeof(int64_t) * (size_t)(N > 0 ? N : 1));
    for (int64_t x = 0; x < N; ++x) labels[x] = 0;
    for (int64_t seed = 0; seed < N; ++seed) {
        if (!mask[seed] || labels[seed]) continue;
        uint32_t lab = (uint32_t)(seed + 1);
        int64_t head = 0, tail = 0;
        queue[tail++] = seed;
        labels[seed] = lab;
        while (head < tail) {
            int64_t x = queue[head++];
            for (int i = 0; i < L->q; ++i) {
                if (L->e[i][0] == 0 && L->e[i][1] == 0 && L->e[i][2] == 0) continue;
                int64_t y = neighbour(&g, x, i);
                if (mask[y] && !labels[y]) {
                    labels[y] = lab;
                    queue[tail++] = y;
                }
            }
        }
        ++ncomp;
    }
    free(queue);
    return ncomp;
}

int64_t orc_label_mask(int q, int nx, int ny, int nz, const uint8_t* mask, uint32_t* labels)
{
    lattice L;
    if (lattice_make(&L, q) != 0) return -1;
    return label_components(&L, nx, ny, nz, mask, labels);
}

static int uf_find(int* parent, int k)
{
    while (parent[k] != k) k = parent[k];
    return k;
}

static void push_event(orc_sim* s, const orc_event* e)
{
    if (s->nev == s->cap_ev) {
        s->cap_ev = s->cap_ev ? 2 * s->cap_ev : 16;
        s->ev = (orc_event*)realloc(s->ev, sizeof(orc_event) * (size_t)s->cap_ev);
    }
    s->ev[s->nev++] = *e;
}

static void push_topo(orc_sim* s, const orc_topo_event* e)
{
    if (s->ntev == s->cap_tev) {
        s->cap_tev = s->cap_tev ? 2 * s->cap_tev : 16;
        s->tev = (orc_topo_event*)realloc(s->tev, sizeof(orc_topo_event) * (size_t)s->cap_tev);
    }
    s->tev[s->ntev++] = *e;
}

static int cmp_u32(const void* a, const void* b)
{
    uint32_t x = *(const uint32_t*)a, y = *(const uint32_t*)b;
    return (x > y) - (x < y);
}

/* ------------------------------------------------------------------------------------------ */
/* Owner field of the barrier.  The paper keeps each bubble on its own lattice (Fig. 1 steps   */
/* 3-5); on one lattice this becomes an owner id per node.  A bubble owns its gas nodes and a  */
/* corona of `corona` liquid layers, grown one lattice-neighbour layer at a time: a node that  */
/* nobody owns takes the smallest id among its owned neighbours of the previous layer.  The id  */
/* of a bubble is 1 + the smallest nucleus index of the criterion-merged groups (eta_m = 0) its */
/* nuclei belong to, so merged bubbles share one lattice again.                                 */
/* ------------------------------------------------------------------------------------------ */
static void build_owner(orc_sim* s)
{
    int64_t N = s->N;
    int* id = (int*)malloc(sizeof(int) * (size_t)(s->nb > 0 ? s->nb : 1));
    for (int b = 0; b < s->nb; ++b) {
        int m = -1;
        for (int k = 0; k < s->n_nuc; ++k) {
            if (s->comp[k] != s->bub[b].label) continue;
            int g = uf_find(s->merge_parent, k);
            if (m < 0 || g < m) m = g;
        }
        id[b] = 1 + m;
    }
    for (int64_t x = 0; x < N; ++x) {
        uint32_t lab = s->labels[x];
        int b = lab ? s->bub_of_label[lab] : -1;
        s->owner[x] = b >= 0 ? id[b] : 0;
    }
    int32_t* next = (int32_t*)malloc(sizeof(int32_t) * (size_t)N);
    for (int r = 0; r < s->corona; ++r) {
        for (int64_t x = 0; x < N; ++x) {
            next[x] = s->owner[x];
            if (s->owner[x] != 0) continue;
            int32_t m = 0;
            for (int i = 0; i < s->L.q; ++i) {
                if (s->L.e[i][0] == 0 && s->L.e[i][1] == 0 && s->L.e[i][2] == 0) continue;
                int32_t o = s->owner[neighbour(s, x, i)];
                if (o != 0 && (m == 0 || o < m)) m = o;
            }
            next[x] = m;
        }
        memcpy(s->owner, next, sizeof(int32_t) * (size_t)N);
    }
    free(next);
    free(id);
}

int orc_set_barrier(orc_sim* s, int on, int corona)
{
    if (corona < 0) return -1;
    s->barrier = on ? 1 : 0;
    s->corona = corona;
    if (s->barrier) build_owner(s);
    else memset(s->owner, 0, sizeof(int32_t) * (size_t)s->N);
    return 0;
}

int orc_owner(const orc_sim* s, int32_t* owner)
{
    memcpy(owner, s->owner, sizeof(int32_t) * (size_t)s->N);
    return 0;
}

/* ------------------------------------------------------------------------------------------ */
/* Test pass (Fig. 1 step 7 and the eta_m switch of Sec. 3.1).                                  */
/* ------------------------------------------------------------------------------------------ */
static int test_pass(orc_sim* s, int with_criterion)
{
    int64_t N = s->N;
    int d = s->L.d;
    double* rho = (double*)malloc(sizeof(double) * (size_t)N);
    uint8_t* mask = (uint8_t*)malloc((size_t)N);

    /* 1-2. density and gas mask rho < theta */
    for (int64_t x = 0; x < N; ++x) {
        rho[x] = node_density(s, s->f, x);
        mask[x] = rho[x] < s->theta ? 1 : 0;
    }

    /* 6 (done early). FP64 totals; a non-finite total latches the numeric error. */
    {
        double M = 0.0, J[3] = {0.0, 0.0, 0.0};
        for (int64_t x = 0; x < N; ++x) {
            double j[3];
            node_momentum(s, s->f, x, j);
            M += rho[x];
            for (int a = 0; a < 3; ++a) J[a] += j[a];
            if (s->ncomp == 2) {
                node_momentum(s, s->fv, x, j);
                M += node_density(s, s->fv, x);
                for (int a = 0; a < 3; ++a) J[a] += j[a];
            }
        }
        if (!isfinite(M) || !isfinite(J[0]) || !isfinite(J[1]) || !isfinite(J[2]))
            s->numeric_error = 1;
    }

    /* 3. canonical labels */
    label_components(&s->L, s->nx, s->ny, s->nz, mask, s->labels);

    /* 4. nucleus map and bubbles (distinct nonzero labels held by nuclei, ascending) */
    for (int b = 0; b < s->nb; ++b) s->bub_of_label[s->bub[b].label] = -1;
    free(s->bub);
    s->bub = NULL;
    s->nb = 0;
    uint32_t* distinct = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)(s->n_nuc > 0 ? s->n_nuc : 1));
    int nd = 0;
    for (int k = 0; k < s->n_nuc; ++k) {
        s->comp[k] = s->labels[s->nuc_node[k]];
        if (s->comp[k] != 0) distinct[nd++] = s->comp[k];
    }
    qsort(distinct, (size_t)nd, sizeof(uint32_t), cmp_u32);
    s->bub = (orc_bubble*)calloc((size_t)(nd > 0 ? nd : 1), sizeof(orc_bubble));
    for (int i = 0; i < nd; ++i) {
        if (i > 0 && distinct[i] == distinct[i - 1]) continue;
        orc_bubble* B = &s->bub[s->nb];
        B->label = distinct[i];
        B->nucleus = -1;
        for (int k = 0; k < s->n_nuc; ++k) {
            if (s->comp[k] != B->label) continue;
            if (B->nucleus < 0) B->nucleus = k;
            B->n_nuclei++;
        }
        s->bub_of_label[B->label] = s->nb;
        s->nb++;
    }
    free(distinct);

    /* 5. statistics: n_b, centroid = anchor + mean integer minimal-image offset, radius */
    {
        int64_t* sum = (int64_t*)calloc((size_t)(3 * (s->nb > 0 ? s->nb : 1)), sizeof(int64_t));
        for (int64_t x = 0; x < N; ++x) {
            if (!s->labels[x]) continue;
            int b = s->bub_of_label[s->labels[x]];
            if (b < 0) continue;
            int c[3], a0[3];
            node_coords(s, x, c);
            node_coords(s, s->nuc_node[s->bub[b].nucleus], a0);
            s->bub[b].n++;
            sum[3 * b + 0] += min_image_int((int64_t)c[0] - a0[0], s->nx);
            sum[3 * b + 1] += min_image_int((int64_t)c[1] - a0[1], s->ny);
            sum[3 * b + 2] += min_image_int((int64_t)c[2] - a0[2], s->nz);
        }
        for (int b = 0; b < s->nb; ++b) {
            int a0[3];
            node_coords(s, s->nuc_node[s->bub[b].nucleus], a0);
            for (int a = 0; a < 3; ++a)
                s->bub[b].centroid[a] = (double)a0[a] + (double)sum[3 * b + a] / (double)s->bub[b].n;
            if (d == 2) {
                s->bub[b].centroid[2] = 0.0;
                s->bub[b].radius = sqrt((double)s->bub[b].n / M_PI);
            } else {
                s->bub[b].radius = cbrt(3.0 * (double)s->bub[b].n / (4.0 * M_PI));
            }
        }
        free(sum);
    }

    /* Topological merges: nuclei of one component join one group (smallest index leads). */
    for (int b = 0; b < s->nb; ++b) {
        int k0 = s->bub[b].nucleus;
        for (int k = k0 + 1; k < s->n_nuc; ++k) {
            if (s->comp[k] != s->bub[b].label) continue;
            int ra = uf_find(s->topo_parent, k0), rb = uf_find(s->topo_parent, k);
            if (ra == rb) continue;
            orc_topo_event te;
            te.step = s->t;
            te.nucleus_a = ra < rb ? ra : rb;
            te.nucleus_b = ra < rb ? rb : ra;
            push_topo(s, &te);
            s->topo_parent[te.nucleus_b] = te.nucleus_a;
        }
    }

    /* 7. merge criterion for each candidate pair (Sec. 3.1 eta_m; Sec. 4, Fig. 2) */
    if (with_criterion) {
        int nfire = 0;
        int* fire_a = (int*)malloc(sizeof(int) * (size_t)(s->nb * s->nb + 1));
        int* fire_b = (int*)malloc(sizeof(int) * (size_t)(s->nb * s->nb + 1));
        int64_t* walk = NULL;
        int walk_cap = 0;
        for (int a = 0; a < s->nb; ++a) {
            for (int b = a + 1; b < s->nb; ++b) {
                const orc_bubble* A = &s->bub[a];
                const orc_bubble* B = &s->bub[b];
                /* pairs already merged by the criterion are not tested again */
                if (uf_find(s->merge_parent, A->nucleus) == uf_find(s->merge_parent, B->nucleus))
                    continue;
                double dv[3];
                dv[0] = min_image(B->centroid[0] - A->centroid[0], s->nx);
                dv[1] = min_image(B->centroid[1] - A->centroid[1], s->ny);
                dv[2] = (d == 3) ? min_image(B->centroid[2] - A->centroid[2], s->nz) : 0.0;
                double dist = sqrt(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
                if (dist > A->radius + B->radius + (double)s->film_max) continue;
                int T = (int)ceil(dist);
                if (T <= 0) continue;
                /* walk of the centroid segment, rounded to nodes, consecutive repeats dropped */
                if (walk_cap < T + 1) {
                    walk_cap = T + 1;
                    walk = (int64_t*)realloc(walk, sizeof(int64_t) * (size_t)walk_cap);
                }
                int nw = 0;
                for (int k = 0; k <= T; ++k) {
                    double pt[3];
                    for (int ax = 0; ax < 3; ++ax)
                        pt[ax] = A->centroid[ax] + dv[ax] * (double)k / (double)T;
                    int64_t node = nearest_node(s, pt);
                    if (nw == 0 || walk[nw - 1] != node) walk[nw++] = node;
                }
                /* film run: strictly between the last a node and the first b node after it */
                int sa = -1, sb = -1;
                for (int k = 0; k < nw; ++k)
                    if (s->labels[walk[k]] == A->label) sa = k;
                if (sa < 0) continue;
                for (int k = sa + 1; k < nw; ++k)
                    if (s->labels[walk[k]] == B->label) { sb = k; break; }
                if (sb < 0) continue;
                int len = sb - sa - 1;
                if (len <= 0 || len > s->film_max) continue;
                int other = 0;
                for (int k = sa + 1; k < sb; ++k)
                    if (s->labels[walk[k]] != 0) other = 1;
                if (other) continue;
                /* film centre: densest run node, first on ties */
                int64_t cstar = walk[sa + 1];
                for (int k = sa + 2; k < sb; ++k)
                    if (rho[walk[k]] > rho[cstar]) cstar = walk[k];
                /* lattice Laplacian of the EOS pressure at c* */
                double pc = node_pressure(s, cstar), lap = 0.0;
                for (int i = 0; i < s->L.q; ++i) {
                    if (s->L.e[i][0] == 0 && s->L.e[i][1] == 0 && s->L.e[i][2] == 0) continue;
                    lap += s->L.w[i] * (node_pressure(s, neighbour(s, cstar, i)) - pc);
                }
                lap *= 6.0;
                if (lap >= 0.0) {
                    orc_event e;
                    memset(&e, 0, sizeof(e));
                    e.step = s->t;
                    e.nucleus_a = A->nucleus;
                    e.nucleus_b = B->nucleus;
                    e.label_a = A->label;
                    e.label_b = B->label;
                    e.film_node = cstar;
                    e.film_len = len;
                    e.lap_p = lap;
                    e.rho_film = rho[cstar];
                    push_event(s, &e);
                    fire_a[nfire] = A->nucleus;
                    fire_b[nfire] = B->nucleus;
                    ++nfire;
                }
            }
        }
        /* eta_m: 1 -> 0 for every fired pair, applied after all pairs were tested */
        for (int k = 0; k < nfire; ++k) {
            int ra = uf_find(s->merge_parent, fire_a[k]), rb = uf_find(s->merge_parent, fire_b[k]);
            if (ra == rb) continue;
            if (ra < rb) s->merge_parent[rb] = ra; else s->merge_parent[ra] = rb;
        }
        free(walk);
        free(fire_a);
        free(fire_b);
    }

    /* the lattices of the bubbles as they stand after this pass's merges */
    if (s->barrier) build_owner(s);

    free(rho);
    free(mask);
    return s->numeric_error ? -5 : 0;
}

int orc_test_pass(orc_sim* s) { return test_pass(s, 1); }

/* ------------------------------------------------------------------------------------------ */
/* Film geometry of a bubble pair (Sec. 3: the film is a disc of radius R_d and thickness h   */
/* between two interfaces; Sec. 4, Fig. 3: h_c against R_d, R_d against R_b at rupture).       */
/* ------------------------------------------------------------------------------------------ */
/* One line parallel to the centroid segment, shifted by off: walk the T+1 samples rounded to
 * nodes (consecutive repeats dropped), find the last node of A and the first node of B after it.
 * Returns the film length (liquid nodes strictly between), or 0 if the line does not cross a
 * film of 1..film_max liquid nodes free of other labels.  Walk nodes and their unwrapped
 * positions go to nodes/pos (capacity T+1) when given; *sa_out, *sb_out get the run ends. */
static int film_line(const orc_sim* s, const double cen[3], const double off[3],
                     const double dv[3], int T, uint32_t la, uint32_t lb, int64_t* nodes,
                     double (*pos)[3], int* sa_out, int* sb_out)
{
    int64_t prev = -1;
    int nw = 0, sa = -1, sb = -1;
    int64_t* wn = (int64_t*)malloc(sizeof(int64_t) * (size_t)(T + 1));
    double(*wp)[3] = (double(*)[3])malloc(sizeof(double) * 3 * (size_t)(T + 1));
    for (int k = 0; k <= T; ++k) {
        double q[3], r[3];
        for (int a = 0; a < 3; ++a) {
            q[a] = cen[a] + off[a] + dv[a] * (double)k / (double)T;
            r[a] = floor(q[a] + 0.5);
        }
        if (s->L.d == 2) r[2] = 0.0;
        int64_t node = node_index(s, wrap((int)r[0], s->nx), wrap((int)r[1], s->ny),
                                  s->L.d == 3 ? wrap((int)r[2], s->nz) : 0);
        if (node == prev) continue;
        prev = node;
        wn[nw] = node;
        for (int a = 0; a < 3; ++a) wp[nw][a] = r[a];
        ++nw;
    }
    for (int k = 0; k < nw; ++k)
        if (s->labels[wn[k]] == la) sa = k;
    if (sa >= 0)
        for (int k = sa + 1; k < nw; ++k)
            if (s->labels[wn[k]] == lb) { sb = k; break; }
    int len = (sa >= 0 && sb >= 0) ? sb - sa - 1 : 0;
    for (int k = sa + 1; len > 0 && k < sb; ++k)
        if (s->labels[wn[k]] != 0) len = 0;
    if (len > s->film_max) len = 0;
    if (nodes) for (int k = 0; k < nw; ++k) { nodes[k] = wn[k]; for (int a = 0; a < 3; ++a) pos[k][a] = wp[k][a]; }
    if (sa_out) *sa_out = sa;
    if (sb_out) *sb_out = sb;
    free(wn);
    free(wp);
    return len;
}

int orc_film_geometry(const orc_sim* s, int nucleus_a, int nucleus_b, double* h, double* r_disc,
                      int* n_lines)
{
    if (nucleus_a < 0 || nucleus_b < 0 || nucleus_a >= s->n_nuc || nucleus_b >= s->n_nuc)
        return -1;
    uint32_t la = s->comp[nucleus_a], lb = s->comp[nucleus_b];
    if (la == 0 || lb == 0 || la == lb) return -4;
    int ba = s->bub_of_label[la], bb = s->bub_of_label[lb];
    const orc_bubble* A = &s->bub[ba];
    const orc_bubble* B = &s->bub[bb];
    int d = s->L.d;
    double dv[3];
    dv[0] = min_image(B->centroid[0] - A->centroid[0], s->nx);
    dv[1] = min_image(B->centroid[1] - A->centroid[1], s->ny);
    dv[2] = (d == 3) ? min_image(B->centroid[2] - A->centroid[2], s->nz) : 0.0;
    double dist = sqrt(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
    int T = (int)ceil(dist);
    if (T <= 0) return -4;
    /* unit axis and an orthonormal basis of the perpendicular plane (2D: one vector) */
    double u[3] = {dv[0] / dist, dv[1] / dist, dv[2] / dist}, n1[3], n2[3] = {0.0, 0.0, 0.0};
    if (d == 2) {
        n1[0] = -u[1]; n1[1] = u[0]; n1[2] = 0.0;
    } else {
        /* n1 = u x z if that is not too short, else u x x */
        double c[3] = {u[1], -u[0], 0.0};
        if (c[0] * c[0] + c[1] * c[1] < 0.25) { c[0] = 0.0; c[1] = u[2]; c[2] = -u[1]; }
        double cl = sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
        for (int a = 0; a < 3; ++a) n1[a] = c[a] / cl;
        n2[0] = u[1] * n1[2] - u[2] * n1[1];
        n2[1] = u[2] * n1[0] - u[0] * n1[2];
        n2[2] = u[0] * n1[1] - u[1] * n1[0];
    }
    int K = (int)floor(A->radius < B->radius ? A->radius : B->radius);
    int count = 0;
    for (int i = -K; i <= K; ++i) {
        for (int j = (d == 3 ? -K : 0); j <= (d == 3 ? K : 0); ++j) {
            if (i * i + j * j > K * K) continue;
            double off[3];
            for (int a = 0; a < 3; ++a) off[a] = (double)i * n1[a] + (double)j * n2[a];
            if (film_line(s, A->centroid, off, dv, T, la, lb, NULL, NULL, NULL, NULL) > 0) ++count;
        }
    }
    *n_lines = count;
    *r_disc = (d == 2) ? 0.5 * (double)count : sqrt((double)count / M_PI);
    /* thickness on the centre line: distance between the rho = theta crossings, linear in the
     * walk's arc length between the node centres on either side of each interface */
    *h = -1.0;
    int64_t* nodes = (int64_t*)malloc(sizeof(int64_t) * (size_t)(T + 1));
    double(*pos)[3] = (double(*)[3])malloc(sizeof(double) * 3 * (size_t)(T + 1));
    double zero[3] = {0.0, 0.0, 0.0};
    int sa, sb;
    if (film_line(s, A->centroid, zero, dv, T, la, lb, nodes, pos, &sa, &sb) > 0) {
        double arc = 0.0, sA = 0.0, sB = 0.0;
        for (int k = 1; k <= sb; ++k) {
            double dx = pos[k][0] - pos[k - 1][0], dy = pos[k][1] - pos[k - 1][1],
                   dz = pos[k][2] - pos[k - 1][2];
            double seg = sqrt(dx * dx + dy * dy + dz * dz);
            double r0 = node_density(s, s->f, nodes[k - 1]), r1 = node_density(s, s->f, nodes[k]);
            if (k == sa + 1) sA = arc + seg * (s->theta - r0) / (r1 - r0);
            if (k == sb) sB = arc + seg * (r0 - s->theta) / (r0 - r1);
            arc += seg;
        }
        *h = sB - sA;
    }
    free(nodes);
    free(pos);
    return 0;
}

int orc_step(orc_sim* s, int nsteps)
{
    for (int n = 0; n < nsteps; ++n) {
        if (s->numeric_error) return -5;
        collide_stream(s);
        growth_source(s);
        s->t += 1;
        if (s->K > 0 && s->t % s->K == 0) {
            if (test_pass(s, 1) != 0) return -5;
        }
    }
    return s->numeric_error ? -5 : 0;
}

/* ------------------------------------------------------------------------------------------ */
/* Output fields                                                                               */
/* ------------------------------------------------------------------------------------------ */
static void fields_2c(const orc_sim* s, double* rho, double* u)
{
    int64_t N = s->N;
    int d = s->L.d;
    double* rl = (double*)malloc(sizeof(double) * (size_t)N);
    double* rv = (double*)malloc(sizeof(double) * (size_t)N);
    for (int64_t x = 0; x < N; ++x) {
        rl[x] = node_density(s, s->f, x);
        rv[x] = node_density(s, s->fv, x);
    }
    for (int64_t x = 0; x < N; ++x) {
        if (rho) rho[x] = rl[x];
        if (!u) continue;
        /* barycentric velocity of the mixture: (j_l + j_v + (F_l + F_v)/2) / (rho_l + rho_v) */
        double jl[3], jv[3], Fl[3], Fv[3];
        node_momentum(s, s->f, x, jl);
        node_momentum(s, s->fv, x, jv);
        cross_force(s, rl, rv, x, Fl);
        cross_force(s, rv, rl, x, Fv);
        for (int a = 0; a < d; ++a)
            u[(int64_t)a * N + x] = (jl[a] + jv[a] + 0.5 * (Fl[a] + Fv[a])) / (rl[x] + rv[x]);
    }
    free(rl);
    free(rv);
}

void orc_fields(const orc_sim* s, double* rho, double* u, double* totals)
{
    int64_t N = s->N;
    int d = s->L.d;
    double* psi = (double*)malloc(sizeof(double) * (size_t)N);
    psi_field(s, psi);
    if ((rho || u) && s->ncomp == 2) {
        fields_2c(s, rho, u);
    } else if (rho || u) {
#pragma omp parallel for schedule(static)
        for (int64_t x = 0; x < N; ++x) {
            double r = node_density(s, s->f, x);
            if (rho) rho[x] = r;
            if (u) {
                double j[3], F[3];
                node_momentum(s, s->f, x, j);
                sc_force(s, psi, x, F);
                for (int a = 0; a < 3; ++a) F[a] += (r - s->rho0) * s->g[a];
                /* reported velocity: (j + F/2) / rho, F with the body force */
                for (int a = 0; a < d; ++a) u[(int64_t)a * N + x] = (j[a] + 0.5 * F[a]) / r;
            }
        }
    }
    if (totals) {
        double M = 0.0, J[3] = {0.0, 0.0, 0.0};
        for (int64_t x = 0; x < N; ++x) {
            double j[3];
            node_momentum(s, s->f, x, j);
            M += node_density(s, s->f, x);
            for (int a = 0; a < 3; ++a) J[a] += j[a];
            if (s->ncomp == 2) {  /* totals of the mixture */
                node_momentum(s, s->fv, x, j);
                M += node_density(s, s->fv, x);
                for (int a = 0; a < 3; ++a) J[a] += j[a];
            }
        }
        totals[0] = M; totals[1] = J[0]; totals[2] = J[1]; totals[3] = J[2];
    }
    free(psi);
}

void orc_force(const orc_sim* s, double* F)
{
    int64_t N = s->N;
    int d = s->L.d;
    if (s->ncomp == 2) {  /* the mixture's total interaction force F_l + F_v */
        double* rl = (double*)malloc(sizeof(double) * (size_t)N);
        double* rv = (double*)malloc(sizeof(double) * (size_t)N);
        for (int64_t x = 0; x < N; ++x) {
            rl[x] = node_density(s, s->f, x);
            rv[x] = node_density(s, s->fv, x);
        }
        for (int64_t x = 0; x < N; ++x) {
            double Fl[3], Fv[3];
            cross_force(s, rl, rv, x, Fl);
            cross_force(s, rv, rl, x, Fv);
            for (int a = 0; a < d; ++a) F[(int64_t)a * N + x] = Fl[a] + Fv[a];
        }
        free(rl);
        free(rv);
        return;
    }
    double* psi = (double*)malloc(sizeof(double) * (size_t)N);
    psi_field(s, psi);
#pragma omp parallel for schedule(static)
    for (int64_t x = 0; x < N; ++x) {
        double Fx[3];
        sc_force(s, psi, x, Fx);
        for (int a = 0; a < d; ++a) F[(int64_t)a * N + x] = Fx[a];
    }
    free(psi);
}

void orc_laplacian_p(const orc_sim* s, double* p, double* lap)
{
    int64_t N = s->N;
    double* pp = (double*)malloc(sizeof(double) * (size_t)N);
#pragma omp parallel for schedule(static)
    for (int64_t x = 0; x < N; ++x) pp[x] = node_pressure(s, x);
    if (p) memcpy(p, pp, sizeof(double) * (size_t)N);
    if (lap) {
#pragma omp parallel for schedule(static)
        for (int64_t x = 0; x < N; ++x) {
            double acc = 0.0;
            for (int i = 0; i < s->L.q; ++i) {
                if (s->L.e[i][0] == 0 && s->L.e[i][1] == 0 && s->L.e[i][2] == 0) continue;
                acc += s->L.w[i] * (pp[neighbour(s, x, i)] - pp[x]);
            }
            /* 1/cs^2 = 3 and the factor 2 of the second-order expansion give 6 */
            lap[x] = 6.0 * acc;
        }
    }
    free(pp);
}

/* ------------------------------------------------------------------------------------------ */
/* State access                                                                                */
/* ------------------------------------------------------------------------------------------ */
void orc_get_f(const orc_sim* s, double* f)
{
    memcpy(f, s->f, sizeof(double) * (size_t)s->L.q * (size_t)s->N);
}

void orc_set_f(orc_sim* s, const double* f)
{
    memcpy(s->f, f, sizeof(double) * (size_t)s->L.q * (size_t)s->N);
}

void orc_set_equilibrium(orc_sim* s, const double* rho, const double* u)
{
    int64_t N = s->N;
    int d = s->L.d;
#pragma omp parallel for schedule(static)
    for (int64_t x = 0; x < N; ++x) {
        double v[3] = {0.0, 0.0, 0.0};
        if (u)
            for (int a = 0; a < d; ++a) v[a] = u[(int64_t)a * N + x];
        for (int i = 0; i < s->L.q; ++i) s->f[(int64_t)i * N + x] = feq_one(&s->L, i, rho[x], v);
    }
}

int64_t orc_time(const orc_sim* s) { return s->t; }
double orc_rho0(const orc_sim* s) { return s->rho0; }
int64_t orc_num_nodes(const orc_sim* s) { return s->N; }

int orc_labels(const orc_sim* s, uint32_t* labels)
{
    memcpy(labels, s->labels, sizeof(uint32_t) * (size_t)s->N);
    return 0;
}

int orc_bubbles(const orc_sim* s, orc_bubble* out, int cap)
{
    for (int b = 0; b < s->nb && b < cap; ++b) out[b] = s->bub[b];
    return s->nb;
}

int orc_events(const orc_sim* s, orc_event* out, int cap)
{
    for (int k = 0; k < s->nev && k < cap; ++k) out[k] = s->ev[k];
    return s->nev;
}

int orc_topo_events(const orc_sim* s, orc_topo_event* out, int cap)
{
    for (int k = 0; k < s->ntev && k < cap; ++k) out[k] = s->tev[k];
    return s->ntev;
}

int orc_nuclei(const orc_sim* s, uint32_t* comp, double* rem)
{
    for (int k = 0; k < s->n_nuc; ++k) {
        if (comp) comp[k] = s->comp[k];
        if (rem) rem[k] = s->rem[k];
    }
    return s->n_nuc;
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
