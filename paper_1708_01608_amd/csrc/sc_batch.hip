// sc_batch.hip -- many independent two-bubble D2Q9 boxes in one persistent kernel (gfx950).
//
// Each workgroup (256 threads) takes the next box from an atomic work queue and runs it to the
// end: fill and paint (Sec. 3.1), time steps (Fig. 1 step 6), and every K steps a test pass
// (gas labelling, two-bubble statistics, the film walk and the FP64 pressure-Laplacian criterion
// of Sec. 3.1 / Sec. 4).  A box stops at the first criterion firing, at the first test pass where
// both nuclei sit in one gas component, or after max_steps.  The workgroup barrier is the box's
// step barrier, so boxes of different sizes and run lengths never wait for one another; the
// queue hands out boxes largest first.  Every workgroup leaves the loop once the queue is empty.
//
// A box is at most 256 nodes wide: one thread per column, marching over the rows with the psi
// of four rows in LDS (the full row is in the block, so the x neighbours wrap inside LDS).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "sc_device.hpp"
#include "sc_internal.hpp"
#include "sc_stepcore.hpp"

namespace sc {

constexpr int kBatchThreads = 256;
constexpr uint32_t kNone = 0xffffffffu;

struct BatchInst {
    int32_t nx, ny;
    int64_t off;   // first float of the box's two population buffers [2][9][N]
    int64_t loff;  // first label of the box
    double tau, G, rho_l, rho_g, amp, theta;
    uint64_t seed;
    double cx[2], cy[2], R[2];
};

struct BatchOut {
    int64_t merge_step, topo_step, steps_run, film_node;
    int32_t film_len, status;
    double lap_p, rho_film;
    double totals[3];
};

struct BatchArgs {
    const BatchInst* inst;
    BatchOut* out;
    const int32_t* order;
    int n;
    float* pool;
    uint32_t* lab;
    unsigned int* counter;
    int K, film_max, max_steps;
};

__device__ __forceinline__ int wrapi(int a, int n)
{
    int r = a % n;
    return r < 0 ? r + n : r;
}

// ---- workgroup reductions (fixed order: deterministic) ----------------------------------------
// A butterfly within each wave (the value of lane 0, whose association order is fixed), then the
// waves in order.  All values of a test pass are reduced together behind one barrier.
template <typename T>
__device__ __forceinline__ T wave_sum(T v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

constexpr int kWaves = kBatchThreads / 64;

// ---- fill and paint (every node liquid plus noise, two balls of gas) -------------------------
__device__ void batch_init(float* f, const BatchInst& in)
{
#pragma clang fp contract(off)
    using L = lat<9>;
    const int nx = in.nx, ny = in.ny, N = nx * ny;
    for (int n = threadIdx.x; n < N; n += kBatchThreads) {
        const int x = n % nx, y = n / nx;
        bool gas = false;
        for (int b = 0; b < 2; ++b) {
            double dx = (double)x - in.cx[b], dy = (double)y - in.cy[b];
            dx = dx - nx * floor(dx / nx + 0.5);
            dy = dy - ny * floor(dy / ny + 0.5);
            if (in.R[b] >= 0.0 && dx * dx + dy * dy <= in.R[b] * in.R[b]) gas = true;
        }
        const double rho = (gas ? in.rho_g : in.rho_l) + in.amp * (2.0 * unit_noise(in.seed, n) - 1.0);
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            const int sx = wrap_once(x - L::ex[i], nx), sy = wrap_once(y - L::ey[i], ny);
            f[(int64_t)i * N + sx + nx * sy] = (float)(L::wd[i] * rho);
        }
    }
}

// ---- one time step of a whole box ------------------------------------------------------------
// The nodes of a box are walked in blocks of rb = max(1, 256 RB / nx) rows: a block has
// rb * nx <= 256 RB node slots j = t + 256 r (r < RB), slot j holding column j % nx of the
// block's row j / nx, so narrow boxes keep every lane busy.  Blocks are numbered virtually:
// block b holds rows w = (b - 1) rb + j / nx (row w mod ny of the box), so block 0 is the
// prologue (the rb rows before row 0) and blocks past the end wrap to the first rows.  psi of
// block b lives in LDS ring slot b mod 4.  Iteration b (1 <= b <= nblk) loads block b + 1 and
// collides block b; its one barrier separates the writes of slot (b+1) mod 4 from the reads of
// block b - 3, done in iteration b - 2.
template <typename A, int RB>
__device__ void batch_step(const float* __restrict__ src, float* __restrict__ dst, int nx, int ny,
                           const Coef<A>& c, A* __restrict__ ps)
{
    using L = lat<9>;
    constexpr int W = kBatchThreads * RB;  // node slots per block (and LDS entries per ring slot)
    const int N = nx * ny;
    const int rb = max(1, W / nx);
    const int nblk = (ny + rb - 1) / rb;
    const int t = threadIdx.x;
    int col[RB], row[RB], xm[RB], xp[RB];
    bool act[RB];
#pragma unroll
    for (int r = 0; r < RB; ++r) {
        const int j = t + kBatchThreads * r;
        row[r] = j / nx;
        col[r] = j - row[r] * nx;
        act[r] = row[r] < rb;
        xm[r] = wrap_once(col[r] - 1, nx);
        xp[r] = wrap_once(col[r] + 1, nx);
    }
    float cur[RB][9], nxt[RB][9];
    A dcur[RB], dnxt[RB];
    // populations (kept) and psi (into LDS) of block b's slot r
    auto load = [&](int blk, int r, float* g) -> A {
        int y = ((blk - 1) * rb + row[r]) % ny;
        if (y < 0) y += ny;
        pull_node<9>(src, N, nx, ny, col[r], xm[r], xp[r], y, wrap_once(y - 1, ny),
                        wrap_once(y + 1, ny), 0, 0, 0, g);
        const A d = sum_dev<9, A>(g);
        ps[(blk & 3) * W + t + kBatchThreads * r] = psi_f(c.rho_ref + d);
        return d;
    };
#pragma unroll
    for (int r = 0; r < RB; ++r) {
        if (act[r]) {
            float g[9];
            (void)load(0, r, g);
            dcur[r] = load(1, r, cur[r]);
        }
    }
    for (int blk = 1; blk <= nblk; ++blk) {
#pragma unroll
        for (int r = 0; r < RB; ++r)
            if (act[r]) dnxt[r] = load(blk + 1, r, nxt[r]);
        __syncthreads();
        const int sb = (blk & 3) * W, sn = ((blk + 1) & 3) * W, sp = ((blk + 3) & 3) * W;
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            const int y = (blk - 1) * rb + row[r];
            if (act[r] && y < ny) {
                // row starts of rows y - 1, y, y + 1 in the ring
                const int j0 = t + kBatchThreads * r - col[r];
                const int rc = sb + j0;
                const int ru = row[r] + 1 < rb ? rc + nx : sn;
                const int rd = row[r] > 0 ? rc - nx : sp + (rb - 1) * nx;
                const A pc = ps[rc + col[r]];
                A fx, fy, fz;  // the single-box kernel's grouped sum
                interaction_sum<9, A>(
                    [&](int i) {
                        const int rw = L::ey[i] > 0 ? ru : (L::ey[i] < 0 ? rd : rc);
                        const int xx = L::ex[i] > 0 ? xp[r] : (L::ex[i] < 0 ? xm[r] : col[r]);
                        return ps[rw + xx];
                    },
                    fx, fy, fz);
                const A gp = -c.G * pc;
                collide_store<9, A, float>(dst, N, (uint32_t)(col[r] + nx * y), cur[r], dcur[r],
                                           gp * fx, gp * fy, (A)0, c);
            }
        }
#pragma unroll
        for (int r = 0; r < RB; ++r) {
#pragma unroll
            for (int i = 0; i < 9; ++i) cur[r][i] = nxt[r][i];
            dcur[r] = dnxt[r];
        }
    }
    __syncthreads();  // this step's stores are the next step's loads
}

// ---- test pass of one box --------------------------------------------------------------------
__device__ __forceinline__ uint32_t ld_par(const uint32_t* p, int i)
{
    return __hip_atomic_load(p + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Root of x with path halving: each visited node is relinked to its grandparent.  Links only
// ever point to smaller indices and a relinked node keeps an ancestor, so concurrent unions
// (atomicMin on roots) and finds stay correct; chains get short after a few finds.
__device__ uint32_t batch_find(uint32_t* par, uint32_t x)
{
    while (true) {
        const uint32_t p = ld_par(par, x);
        if (p == x) return x;
        const uint32_t gp = ld_par(par, p);
        if (gp == p) return p;
        __hip_atomic_store(par + x, gp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        x = gp;
    }
}

// Label of node n once the unions are done: its root, or kNone for a liquid node.
__device__ __forceinline__ uint32_t batch_root(uint32_t* par, uint32_t n)
{
    return par[n] == kNone ? kNone : batch_find(par, n);
}

__device__ void batch_unite(uint32_t* par, uint32_t a, uint32_t b)
{
    while (true) {
        a = batch_find(par, a);
        b = batch_find(par, b);
        if (a == b) return;
        if (a > b) { const uint32_t t = a; a = b; b = t; }
        const uint32_t old = atomicMin(par + b, a);
        if (old == b) return;
        b = old;
    }
}

__device__ __forceinline__ double rho64(const float* f, int N, int nx, int ny, int x, int y)
{
    using L = lat<9>;
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < 9; ++i)
        s += (double)f[(int64_t)i * N + wrap_once(x - L::ex[i], nx) + nx * wrap_once(y - L::ey[i], ny)];
    return s;
}

// minimal-image offset of d in (-n, n) on a ring of n nodes (boxes are small: 32-bit is exact)
__device__ __forceinline__ int min_img_i(int d, int n)
{
    const int h = n / 2;
    int r = (d + h) % n;
    if (r < 0) r += n;
    return r - h;
}

struct Scratch {
    long long i[kWaves][6];  // per wave: count, x and y offset sums of both bubbles
    double d[kWaves][3];     // per wave: M, Jx, Jy
    int flag;
};

// Labels the gas (rho < theta, FP64), gathers the two bubbles and, if asked, applies the film
// criterion.  Returns (uniformly) whether the box stops.  Thread 0 updates `o`.
__device__ bool batch_test(const float* f, uint32_t* par, const BatchInst& in, int K, int film_max,
                           int64_t step, bool criterion, BatchOut& o, Scratch& sh)
{
#pragma clang fp contract(off)
    using L = lat<9>;
    const int nx = in.nx, ny = in.ny, N = nx * ny;
    const int t = threadIdx.x;
    // One sweep over the populations: the FP64 density of each node (in the oracle's order) for
    // the mask, and the box totals from the same pulled values (on a periodic box the pulled
    // populations of all nodes are all the populations).  The sweeps take U nodes per thread and
    // iteration, loads first: a workgroup carries one box, so without that each iteration would
    // wait out a full memory latency.
    double M = 0.0, Jx = 0.0, Jy = 0.0;
    constexpr int U1 = 2;
    for (int n0 = t; n0 < N; n0 += U1 * kBatchThreads) {
        float g[U1][9];
#pragma unroll
        for (int u = 0; u < U1; ++u) {
            const int n = n0 + u * kBatchThreads;
            if (n < N) {
                const int x = n % nx, y = n / nx;
#pragma unroll
                for (int i = 0; i < 9; ++i)
                    g[u][i] = f[(int64_t)i * N + wrap_once(x - L::ex[i], nx) +
                                nx * wrap_once(y - L::ey[i], ny)];
            }
        }
#pragma unroll
        for (int u = 0; u < U1; ++u) {
            const int n = n0 + u * kBatchThreads;
            if (n < N) {
                double r = 0.0, jx = 0.0, jy = 0.0;
#pragma unroll
                for (int i = 0; i < 9; ++i) {
                    const double v = (double)g[u][i];
                    r += v;
                    if (L::ex[i] > 0) jx += v; else if (L::ex[i] < 0) jx -= v;
                    if (L::ey[i] > 0) jy += v; else if (L::ey[i] < 0) jy -= v;
                }
                par[n] = r < in.theta ? (uint32_t)n : kNone;
                M += r;
                Jx += jx;
                Jy += jy;
            }
        }
    }
    __syncthreads();
    // runs along x: a wave holds 64 consecutive nodes, so one ballot of the gas mask (and one of
    // the row starts) gives every gas node the first node of its run within the wave's segment,
    // which becomes its parent; a run that began before the segment (the node before it gas, in
    // the same row: the carry into lane 0) continues from that node.  x-links then need no union,
    // except the periodic one from x = nx - 1 to 0.
    for (int n0 = t; n0 < ((N + 63) & ~63); n0 += kBatchThreads) {
        const int lane = n0 & 63;
        const int seg = n0 - lane;
        const bool gas = n0 < N && ld_par(par, n0) != kNone;
        const unsigned long long mask = __ballot(gas);
        const unsigned long long rows = __ballot(n0 < N && n0 % nx == 0);
        // gas stays gas while the wave before rewrites its parents, so this read is stable
        const unsigned long long cin =
            (seg > 0 && seg < N && seg % nx != 0 && ld_par(par, seg - 1) != kNone) ? 1ull : 0ull;
        const unsigned long long starts = mask & ~(((mask << 1) | cin) & ~rows);
        const unsigned long long upto = starts & (~0ull >> (63 - lane));
        if (gas) par[n0] = upto ? (uint32_t)(seg + 63 - __clzll(upto)) : (uint32_t)(seg - 1);
    }
    __syncthreads();
    // links to other rows: two adjacent runs always share a link at which one end starts its run
    // (x = 0 counts as a start, so every link across the periodic boundary qualifies): only those
    // are united, about one union per run instead of one per link
    constexpr int U2 = 8;
    for (int n0 = t; n0 < N; n0 += U2 * kBatchThreads) {
        // gas or liquid never changes in this pass: one mask bit per gas node of the group
        unsigned gas = 0;
#pragma unroll
        for (int u = 0; u < U2; ++u) {
            const int n = n0 + u * kBatchThreads;
            if (n < N && ld_par(par, n) != kNone) gas |= 1u << u;
        }
        while (gas) {
            const int u = __builtin_ctz(gas);
            gas &= gas - 1;
            const int n = n0 + u * kBatchThreads;
            const int x = n % nx, y = n / nx;
            const bool s0 = x == 0 || ld_par(par, n - 1) == kNone;
#pragma unroll
            for (int h = 0; h < L::nhalf; ++h) {
                const int i = L::half[h];
                if (L::ey[i] == 0 && x != nx - 1) continue;  // inside the row: the run
                const int mx = wrap_once(x + L::ex[i], nx);
                const int m = mx + nx * wrap_once(y + L::ey[i], ny);
                if (ld_par(par, m) == kNone) continue;
                if (L::ey[i] != 0 && !s0 && mx != 0 && ld_par(par, m - 1) != kNone) continue;
                batch_unite(par, (uint32_t)n, (uint32_t)m);
            }
        }
    }
    __syncthreads();
    // the trees are left unflattened (par is read-only from here on): a gas node's label is the
    // root its find returns

    // nucleus nodes and their components (root index, kNone if liquid)
    int nd[2];
    uint32_t comp[2];
    for (int b = 0; b < 2; ++b) {
        const int x = wrapi((int)floor(in.cx[b] + 0.5), nx);
        const int y = wrapi((int)floor(in.cy[b] + 0.5), ny);
        nd[b] = x + nx * y;
        comp[b] = batch_root(par, (uint32_t)nd[b]);
    }
    // statistics: counts and integer minimal-image offset sums from each bubble's anchor node
    // (the bubble of nucleus 1 is anchored at nucleus 0 when both share it)
    int ax[2], ay[2];
    for (int b = 0; b < 2; ++b) {
        const int a = (b == 1 && comp[1] == comp[0]) ? nd[0] : nd[b];
        ax[b] = a % nx;
        ay[b] = a / nx;
    }
    long long cnt[2] = {0, 0}, sx[2] = {0, 0}, sy[2] = {0, 0};
    constexpr int U3 = 8;
    for (int n0 = t; n0 < N; n0 += U3 * kBatchThreads) {
        unsigned gas = 0;
#pragma unroll
        for (int u = 0; u < U3; ++u) {
            const int n = n0 + u * kBatchThreads;
            if (n < N && par[n] != kNone) gas |= 1u << u;
        }
        while (gas) {
            const int u = __builtin_ctz(gas);
            gas &= gas - 1;
            const int n = n0 + u * kBatchThreads;
            const uint32_t p = batch_find(par, (uint32_t)n);
            const int y = n / nx, x = n - y * nx;
            for (int b = 0; b < 2; ++b) {
                if (p != comp[b]) continue;
                cnt[b] += 1;
                sx[b] += min_img_i(x - ax[b], nx);
                sy[b] += min_img_i(y - ay[b], ny);
            }
        }
    }
    {
        const long long vi[6] = {cnt[0], sx[0], sy[0], cnt[1], sx[1], sy[1]};
        const double vd[3] = {M, Jx, Jy};
        long long ri[6];
        double rd[3];
#pragma unroll
        for (int k = 0; k < 6; ++k) ri[k] = wave_sum(vi[k]);
#pragma unroll
        for (int k = 0; k < 3; ++k) rd[k] = wave_sum(vd[k]);
        if ((t & 63) == 0) {
            const int w = t >> 6;
#pragma unroll
            for (int k = 0; k < 6; ++k) sh.i[w][k] = ri[k];
#pragma unroll
            for (int k = 0; k < 3; ++k) sh.d[w][k] = rd[k];
        }
    }
    __syncthreads();
    // (sh is next written in the following test pass, behind further barriers)
    long long tot_i[6];
    double tot_d[3];
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        tot_i[k] = sh.i[0][k];
        for (int w = 1; w < kWaves; ++w) tot_i[k] += sh.i[w][k];
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        tot_d[k] = sh.d[0][k];
        for (int w = 1; w < kWaves; ++w) tot_d[k] += sh.d[w][k];
    }
    const double tM = tot_d[0], tJx = tot_d[1], tJy = tot_d[2];

    if (t == 0) {
        bool stop = false;
        o.totals[0] = tM; o.totals[1] = tJx; o.totals[2] = tJy;
        if (!(isfinite(tM) && isfinite(tJx) && isfinite(tJy))) {
            o.status = SC_E_NUMERIC;
            stop = true;
        }
        if (comp[0] != kNone && comp[0] == comp[1]) {
            if (o.topo_step < 0) o.topo_step = step;
            stop = true;
        } else if (criterion && comp[0] != kNone && comp[1] != kNone && !stop) {
            // bubbles in label order (smaller root first)
            const int A = comp[0] < comp[1] ? 0 : 1, B = 1 - A;
            double cen[2][2], rad[2];
            for (int b = 0; b < 2; ++b) {
                const long long n_b = tot_i[3 * b];
                cen[b][0] = (double)(nd[b] % nx) + (double)tot_i[3 * b + 1] / (double)n_b;
                cen[b][1] = (double)(nd[b] / nx) + (double)tot_i[3 * b + 2] / (double)n_b;
                rad[b] = __dsqrt_rn((double)n_b / M_PI);
            }
            double dv[2];
            dv[0] = cen[B][0] - cen[A][0];
            dv[0] = dv[0] - nx * floor(dv[0] / nx + 0.5);
            dv[1] = cen[B][1] - cen[A][1];
            dv[1] = dv[1] - ny * floor(dv[1] / ny + 0.5);
            const double dist = __dsqrt_rn(dv[0] * dv[0] + dv[1] * dv[1] + 0.0 * 0.0);
            const int T = (int)ceil(dist);
            if (dist <= rad[A] + rad[B] + (double)film_max && T > 0) {
                // walk the centroid segment (consecutive repeats dropped)
                int sa = -1, sb = -1, pos = -1, prev = -1;
                for (int pass = 0; pass < 2; ++pass) {
                    pos = -1;
                    prev = -1;
                    for (int k = 0; k <= T; ++k) {
                        const double px = cen[A][0] + dv[0] * (double)k / (double)T;
                        const double py = cen[A][1] + dv[1] * (double)k / (double)T;
                        const int node = wrapi((int)floor(px + 0.5), nx) +
                                         nx * wrapi((int)floor(py + 0.5), ny);
                        if (node == prev) continue;
                        prev = node;
                        ++pos;
                        if (pass == 0 && batch_root(par, (uint32_t)node) == comp[A]) sa = pos;
                        if (pass == 1 && pos > sa && sb < 0 && batch_root(par, (uint32_t)node) == comp[B]) sb = pos;
                    }
                    if (sa < 0) break;
                }
                const int len = sb - sa - 1;
                if (sa >= 0 && sb >= 0 && len >= 1 && len <= film_max) {
                    bool clean = true;
                    int cstar = -1;
                    double best = 0.0;
                    pos = -1;
                    prev = -1;
                    for (int k = 0; k <= T; ++k) {
                        const double px = cen[A][0] + dv[0] * (double)k / (double)T;
                        const double py = cen[A][1] + dv[1] * (double)k / (double)T;
                        const int node = wrapi((int)floor(px + 0.5), nx) +
                                         nx * wrapi((int)floor(py + 0.5), ny);
                        if (node == prev) continue;
                        prev = node;
                        ++pos;
                        if (pos <= sa || pos >= sb) continue;
                        if (par[node] != kNone) clean = false;
                        const double r = rho64(f, N, nx, ny, node % nx, node / nx);
                        if (cstar < 0 || r > best) { cstar = node; best = r; }
                    }
                    if (clean) {
                        const int x = cstar % nx, y = cstar / nx;
                        const double pc = pressure_d(best, in.G);
                        double acc = 0.0;
                        for (int i = 1; i < 9; ++i) {
                            const double r = rho64(f, N, nx, ny, wrap_once(x + L::ex[i], nx),
                                                   wrap_once(y + L::ey[i], ny));
                            acc += L::wd[i] * (pressure_d(r, in.G) - pc);
                        }
                        const double lap = 6.0 * acc;
                        if (lap >= 0.0) {
                            o.merge_step = step;
                            o.film_node = cstar;
                            o.film_len = len;
                            o.lap_p = lap;
                            o.rho_film = best;
                            stop = true;
                        }
                    }
                }
            }
        }
        sh.flag = stop ? 1 : 0;
    }
    __syncthreads();
    const bool stop = sh.flag != 0;
    __syncthreads();
    return stop;
}

// Waves per SIMD the compiler must fit (the second launch bound): one box per workgroup leaves
// latency to hide, so with one node slot per lane the registers are capped for three waves (a
// few spills, measured 16% faster than two); more slots need two.
template <typename A, int RB>
__global__ void __launch_bounds__(kBatchThreads, RB == 1 ? 3 : 2) k_batch(BatchArgs b)
{
    __shared__ A ps[4 * RB * kBatchThreads];
    __shared__ Scratch sh;
    __shared__ BatchOut s_out;
    __shared__ int s_idx;
    for (;;) {
        if (threadIdx.x == 0) s_idx = (int)atomicAdd(b.counter, 1u);
        __syncthreads();
        // the queue index is uniform over the workgroup: keep it (and the box record loaded
        // through it) in scalar registers
        const int q = __builtin_amdgcn_readfirstlane(s_idx);
        __syncthreads();
        if (q >= b.n) return;
        const int k = __builtin_amdgcn_readfirstlane(b.order[q]);
        const BatchInst in = b.inst[k];
        const int N = in.nx * in.ny;
        float* f0 = b.pool + in.off;
        float* f1 = f0 + (int64_t)9 * N;
        uint32_t* par = b.lab + in.loff;
        const Coef<A> c{(A)in.tau, (A)(1.0 / in.tau), (A)in.G, (A)0, (A)0};
        // the box's record is written by thread 0 only: keep it in LDS, not in every lane
        BatchOut& o = s_out;
        if (threadIdx.x == 0) {
            o.merge_step = -1; o.topo_step = -1; o.steps_run = 0; o.film_node = -1;
            o.film_len = 0; o.status = 0; o.lap_p = 0.0; o.rho_film = 0.0;
            o.totals[0] = o.totals[1] = o.totals[2] = 0.0;
        }

        batch_init(f0, in);
        __syncthreads();
        bool stop = batch_test(f0, par, in, b.K, b.film_max, 0, false, o, sh);
        int cur = 0;
        int64_t step = 0;
        while (!stop && step < b.max_steps) {
            batch_step<A, RB>(cur ? f1 : f0, cur ? f0 : f1, in.nx, in.ny, c, ps);
            cur ^= 1;
            ++step;
            if (b.K > 0 && step % b.K == 0)
                stop = batch_test(cur ? f1 : f0, par, in, b.K, b.film_max, step, true, o, sh);
        }
        if (threadIdx.x == 0) {
            o.steps_run = step;
            b.out[k] = o;
        }
        __syncthreads();
    }
}

__global__ void k_batch_reset(unsigned int* counter) { *counter = 0u; }

// Density of one box after a run (FP64 sum, FP32 out).
__global__ void k_batch_rho(const float* f, int nx, int ny, float* rho)
{
    const int N = nx * ny;
    for (int n = blockIdx.x * blockDim.x + threadIdx.x; n < N; n += gridDim.x * blockDim.x)
        rho[n] = (float)rho64(f, N, nx, ny, n % nx, n / nx);
}

}  // namespace sc

// ==============================================================================================
// C ABI of the batch
// ==============================================================================================
using namespace sc;

struct sc_batch {
    int n = 0;
    int K = 10, film_max = 8, max_steps = 5000, compute = SC_COMPUTE_F64;
    int rb = 2;  // rows per thread per iteration of the box step
    hipStream_t stream = nullptr;
    bool own_stream = false;
    sc_allocator alloc{};
    bool has_alloc = false;
    std::vector<BatchInst> inst;
    std::vector<int32_t> order;
    void *d_inst = nullptr, *d_out = nullptr, *d_order = nullptr, *d_pool = nullptr,
         *d_lab = nullptr, *d_counter = nullptr, *d_rho = nullptr;
    size_t pool_floats = 0, lab_count = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    std::vector<BatchOut> last;
    bool ran = false;
};

namespace {

void* balloc(sc_batch* b, size_t bytes)
{
    if (bytes == 0) bytes = 256;
    if (b->has_alloc) return b->alloc.alloc(bytes, b->alloc.user);
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return p;
}

void bfree(sc_batch* b, void* p)
{
    if (!p) return;
    if (b->has_alloc) b->alloc.free(p, b->alloc.user);
    else (void)hipFree(p);
}

void brelease(sc_batch* b)
{
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->ev0) (void)hipEventDestroy(b->ev0);
    if (b->ev1) (void)hipEventDestroy(b->ev1);
    for (void* p : {b->d_inst, b->d_out, b->d_order, b->d_pool, b->d_lab, b->d_counter, b->d_rho})
        bfree(b, p);
    if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
}

}  // namespace

namespace {

hipError_t batch_occupancy(int compute, int rb, int* per_cu)
{
#define SC_OCC(A, RB) return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k_batch<A, RB>, kBatchThreads, 0)
    if (compute == SC_COMPUTE_F32) {
        if (rb == 1) SC_OCC(float, 1);
        if (rb == 2) SC_OCC(float, 2);
        SC_OCC(float, 4);
    }
    if (rb == 1) SC_OCC(double, 1);
    if (rb == 2) SC_OCC(double, 2);
    SC_OCC(double, 4);
#undef SC_OCC
}

void batch_launch(int compute, int rb, int grid, hipStream_t st, const BatchArgs& a)
{
#define SC_LB(A, RB) hipLaunchKernelGGL((k_batch<A, RB>), dim3(grid), dim3(kBatchThreads), 0, st, a)
    if (compute == SC_COMPUTE_F32) {
        if (rb == 1) SC_LB(float, 1); else if (rb == 2) SC_LB(float, 2); else SC_LB(float, 4);
    } else {
        if (rb == 1) SC_LB(double, 1); else if (rb == 2) SC_LB(double, 2); else SC_LB(double, 4);
    }
#undef SC_LB
}

}  // namespace

#define BHIP(call)                                                                               \
    do {                                                                                         \
        hipError_t e_ = (call);                                                                  \
        if (e_ != hipSuccess) return set_error(SC_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

extern "C" {

int sc_batch_create(int32_t n, const sc_batch_instance* inst, int32_t test_every,
                    int32_t film_max, int32_t max_steps, int32_t compute, void* stream,
                    const sc_allocator* allocator, sc_batch** out)
{
    if (!out) return set_error(SC_E_INVAL, "NULL output handle");
    if (n < 1 || !inst) return set_error(SC_E_INVAL, "need n >= 1 instances");
    if (test_every < 1 || film_max < 1 || max_steps < 0)
        return set_error(SC_E_INVAL, "test_every >= 1, film_max >= 1, max_steps >= 0");
    if (compute != SC_COMPUTE_AUTO && compute != SC_COMPUTE_F32 && compute != SC_COMPUTE_F64)
        return set_error(SC_E_INVAL, "unknown compute type");
    if (allocator && (!allocator->alloc || !allocator->free))
        return set_error(SC_E_INVAL, "allocator needs alloc and free");
    for (int k = 0; k < n; ++k) {
        const sc_batch_instance& I = inst[k];
        if (I.nx < 4 || I.ny < 4 || I.nx > kBatchThreads)
            return set_error(SC_E_INVAL, "instance " + std::to_string(k) + ": need 4 <= nx <= 256, ny >= 4");
        if ((double)I.nx * I.ny > 2.0e9) return set_error(SC_E_INVAL, "instance too large");
        if (!(I.tau > 0.5) || !std::isfinite(I.G) || !(I.rho_liquid > 0) || !(I.rho_gas > 0) ||
            !(I.noise_amp >= 0) || !std::isfinite(I.gas_threshold))
            return set_error(SC_E_INVAL, "instance " + std::to_string(k) + ": bad physical parameters");
        for (int b = 0; b < 2; ++b)
            if (!std::isfinite(I.centre[b][0]) || !std::isfinite(I.centre[b][1]) ||
                !std::isfinite(I.radius[b]))
                return set_error(SC_E_INVAL, "instance " + std::to_string(k) + ": bad nucleus");
    }
    sc_batch* b = new sc_batch();
    b->n = n;
    b->K = test_every;
    b->film_max = film_max;
    b->max_steps = max_steps;
    b->compute = compute == SC_COMPUTE_F32 ? SC_COMPUTE_F32 : SC_COMPUTE_F64;
    if (allocator) {
        b->alloc = *allocator;
        b->has_alloc = true;
    }
    b->inst.resize(n);
    size_t off = 0, loff = 0;
    for (int k = 0; k < n; ++k) {
        const sc_batch_instance& I = inst[k];
        BatchInst& d = b->inst[k];
        d.nx = I.nx;
        d.ny = I.ny;
        d.off = (int64_t)off;
        d.loff = (int64_t)loff;
        d.tau = I.tau; d.G = I.G; d.rho_l = I.rho_liquid; d.rho_g = I.rho_gas; d.amp = I.noise_amp;
        d.theta = I.gas_threshold > 0.0 ? I.gas_threshold : 0.5 * (I.rho_liquid + I.rho_gas);
        d.seed = I.noise_seed;
        for (int q = 0; q < 2; ++q) {
            d.cx[q] = I.centre[q][0];
            d.cy[q] = I.centre[q][1];
            d.R[q] = I.radius[q];
        }
        const size_t N = (size_t)I.nx * I.ny;
        off += 2 * 9 * N;
        off = (off + 63) & ~size_t(63);  // 256-byte aligned buffers
        loff += (N + 63) & ~size_t(63);
    }
    b->pool_floats = off;
    b->lab_count = loff;
    // largest boxes first: the queue order of a longest-first schedule
    b->order.resize(n);
    std::iota(b->order.begin(), b->order.end(), 0);
    std::stable_sort(b->order.begin(), b->order.end(), [&](int a, int c) {
        return (int64_t)b->inst[a].nx * b->inst[a].ny > (int64_t)b->inst[c].nx * b->inst[c].ny;
    });
    auto cleanup = [&](int code, const std::string& m) {
        brelease(b);
        delete b;
        return set_error(code, m);
    };
    if (stream) {
        b->stream = (hipStream_t)stream;
    } else {
        if (hipStreamCreate(&b->stream) != hipSuccess) return cleanup(SC_E_DEVICE, "hipStreamCreate failed");
        b->own_stream = true;
    }
    b->d_inst = balloc(b, sizeof(BatchInst) * n);
    b->d_out = balloc(b, sizeof(BatchOut) * n);
    b->d_order = balloc(b, sizeof(int32_t) * n);
    b->d_pool = balloc(b, sizeof(float) * b->pool_floats);
    b->d_lab = balloc(b, sizeof(uint32_t) * b->lab_count);
    b->d_counter = balloc(b, 256);
    if (!b->d_inst || !b->d_out || !b->d_order || !b->d_pool || !b->d_lab || !b->d_counter)
        return cleanup(SC_E_NOMEM, "batch buffers");
    hipError_t e = hipMemcpyAsync(b->d_inst, b->inst.data(), sizeof(BatchInst) * n,
                                  hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->d_order, b->order.data(), sizeof(int32_t) * n,
                           hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e == hipSuccess) e = hipEventCreate(&b->ev0);
    if (e == hipSuccess) e = hipEventCreate(&b->ev1);
    if (e != hipSuccess) return cleanup(SC_E_DEVICE, std::string("batch setup: ") + hipGetErrorString(e));
    *out = b;
    return SC_OK;
}

int sc_batch_destroy(sc_batch* b)
{
    if (!b) return set_error(SC_E_INVAL, "NULL batch handle");
    brelease(b);
    delete b;
    return SC_OK;
}

int sc_batch_run(sc_batch* b, sc_batch_result* results, double* kernel_ms)
{
    if (!b) return set_error(SC_E_INVAL, "NULL batch handle");
    if (!b->exec) {
        // capture once: queue reset (a kernel, not a memset node) + the persistent kernel
        int dev = 0, cus = 0, per_cu = 0;
        BHIP(hipGetDevice(&dev));
        BHIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        BatchArgs a;
        a.inst = (const BatchInst*)b->d_inst;
        a.out = (BatchOut*)b->d_out;
        a.order = (const int32_t*)b->d_order;
        a.n = b->n;
        a.pool = (float*)b->d_pool;
        a.lab = (uint32_t*)b->d_lab;
        a.counter = (unsigned int*)b->d_counter;
        a.K = b->K;
        a.film_max = b->film_max;
        a.max_steps = b->max_steps;
        BHIP(batch_occupancy(b->compute, b->rb, &per_cu));
        const int grid = std::max(1, std::min(b->n, std::max(1, per_cu) * std::max(1, cus)));
        BHIP(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
        hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(1), 0, b->stream, (unsigned int*)b->d_counter);
        batch_launch(b->compute, b->rb, grid, b->stream, a);
        hipError_t le = hipGetLastError();
        hipError_t ce = hipStreamEndCapture(b->stream, &b->graph);
        if (le != hipSuccess) return set_error(SC_E_DEVICE, std::string("batch launch: ") + hipGetErrorString(le));
        if (ce != hipSuccess) return set_error(SC_E_DEVICE, std::string("capture: ") + hipGetErrorString(ce));
        BHIP(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    }
    BHIP(hipEventRecord(b->ev0, b->stream));
    BHIP(hipGraphLaunch(b->exec, b->stream));
    BHIP(hipEventRecord(b->ev1, b->stream));
    b->last.resize(b->n);
    BHIP(hipMemcpyAsync(b->last.data(), b->d_out, sizeof(BatchOut) * b->n, hipMemcpyDeviceToHost,
                        b->stream));
    BHIP(hipStreamSynchronize(b->stream));
    b->ran = true;
    if (kernel_ms) {
        float ms = 0.0f;
        BHIP(hipEventElapsedTime(&ms, b->ev0, b->ev1));
        *kernel_ms = ms;
    }
    if (results) {
        for (int k = 0; k < b->n; ++k) {
            const BatchOut& o = b->last[k];
            sc_batch_result& r = results[k];
            r.merge_step = o.merge_step;
            r.topo_step = o.topo_step;
            r.steps_run = o.steps_run;
            r.film_node = o.film_node;
            r.film_len = o.film_len;
            r.status = o.status;
            r.lap_p = o.lap_p;
            r.rho_film = o.rho_film;
            for (int c = 0; c < 3; ++c) r.totals[c] = o.totals[c];
        }
    }
    return SC_OK;
}

int sc_batch_tune(sc_batch* b, int32_t trial_steps, int32_t* rows_per_thread, double* ms_out)
{
    if (!b) return set_error(SC_E_INVAL, "NULL batch handle");
    if (trial_steps < 1) return set_error(SC_E_INVAL, "trial_steps >= 1");
    const int keep_steps = b->max_steps;
    const int keep_rb = b->rb;
    double best = 1e300;
    int best_rb = keep_rb;
    int rc = SC_OK;
    b->max_steps = trial_steps;
    for (int rb : {1, 2, 4}) {
        b->rb = rb;
        if (b->exec) { (void)hipGraphExecDestroy(b->exec); b->exec = nullptr; }
        if (b->graph) { (void)hipGraphDestroy(b->graph); b->graph = nullptr; }
        double ms = 0.0;
        rc = sc_batch_run(b, nullptr, &ms);
        if (rc != SC_OK) break;
        if (ms_out) ms_out[rb == 1 ? 0 : rb == 2 ? 1 : 2] = ms;
        if (ms < best) { best = ms; best_rb = rb; }
    }
    b->max_steps = keep_steps;
    b->rb = rc == SC_OK ? best_rb : keep_rb;
    if (b->exec) { (void)hipGraphExecDestroy(b->exec); b->exec = nullptr; }
    if (b->graph) { (void)hipGraphDestroy(b->graph); b->graph = nullptr; }
    b->ran = false;
    if (rows_per_thread) *rows_per_thread = b->rb;
    return rc;
}

int sc_batch_fields(sc_batch* b, int32_t k, float* rho)
{
    if (!b || !rho) return set_error(SC_E_INVAL, "NULL argument");
    if (k < 0 || k >= b->n) return set_error(SC_E_INVAL, "instance index out of range");
    if (!b->ran) return set_error(SC_E_STATE, "sc_batch_run has not run");
    const BatchInst& in = b->inst[k];
    const int N = in.nx * in.ny;
    const float* f = (const float*)b->d_pool + in.off + (b->last[k].steps_run % 2 ? (int64_t)9 * N : 0);
    if (!b->d_rho) {
        b->d_rho = balloc(b, sizeof(float) * (size_t)kBatchThreads * 65536);
        if (!b->d_rho) return set_error(SC_E_NOMEM, "density buffer");
    }
    if ((size_t)N > (size_t)kBatchThreads * 65536) return set_error(SC_E_INVAL, "instance too large");
    hipLaunchKernelGGL(k_batch_rho, dim3((N + 255) / 256), dim3(256), 0, b->stream, f, in.nx,
                       in.ny, (float*)b->d_rho);
    BHIP(hipGetLastError());
    BHIP(hipMemcpyAsync(rho, b->d_rho, sizeof(float) * N, hipMemcpyDeviceToHost, b->stream));
    BHIP(hipStreamSynchronize(b->stream));
    return SC_OK;
}

}  // extern "C"
