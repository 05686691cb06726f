// sc_test.hip -- output fields, FP64 EOS / Laplacian / totals, gas labelling, bubble statistics,
// merge criterion and blowing-agent source of libsc (gfx950).
//
// Every kernel reads the pull-layout populations: f_i(x, t) = stored_i(x - e_i) + w_i rho_ref.
#include <algorithm>

#include "sc_device.hpp"
#include "sc_internal.hpp"

namespace sc {

static dim3 grid_for(int64_t n)
{
    int64_t b = (n + 255) / 256;
    if (b > 65536) b = 65536;
    if (b < 1) b = 1;
    return dim3((unsigned)b);
}

// Coordinates of node n.  n < N <= 2^31 (sc_create bounds a population array to 2^32 bytes), so
// 32-bit unsigned division is exact, at a fraction of the cost of 64-bit division.
__device__ __forceinline__ void coords3(int64_t n, int nx, int ny, int& x, int& y, int& z)
{
    const uint32_t m = (uint32_t)n;
    const uint32_t r = m / (uint32_t)nx;
    x = (int)(m - r * (uint32_t)nx);
    y = (int)(r % (uint32_t)ny);
    z = (int)(r / (uint32_t)ny);
}

__device__ __forceinline__ int64_t idx3(int x, int y, int z, int nx, int ny)
{
    return (int64_t)x + (int64_t)nx * ((int64_t)y + (int64_t)ny * z);
}

// Node x + s * e_i (s = +1 downstream, -1 upstream), periodic.
template <int Q>
__device__ __forceinline__ int64_t shifted(int x, int y, int z, int i, int s, const FieldArgs& a)
{
    using L = lat<Q>;
    return idx3(wrap_once(x + s * L::ex[i], a.nx), wrap_once(y + s * L::ey[i], a.ny),
                wrap_once(z + s * L::ez[i], a.nz), a.nx, a.ny);
}

// FP32 deviation sum of node n (the same order as the step kernel).
template <int Q, typename S>
__device__ __forceinline__ float dev_sum_f(const S* f, int64_t n, const FieldArgs& a, float* g)
{
    int x, y, z;
    coords3(n, a.nx, a.ny, x, y, z);
    float s = 0.0f;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        g[i] = load_f(f[(int64_t)i * a.N + shifted<Q>(x, y, z, i, -1, a)]);
        s += g[i];
    }
    return s;
}

// Sum of the stored deviations of node n, in double.
template <int Q, typename S>
__device__ __forceinline__ double dev_d(const S* f, int64_t n, const FieldArgs& a)
{
    int x, y, z;
    coords3(n, a.nx, a.ny, x, y, z);
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < Q; ++i)
        s += (double)load_f(f[(int64_t)i * a.N + shifted<Q>(x, y, z, i, -1, a)]);
    return s;
}

// FP64 density of node n: rho_ref + sum of the stored deviations.
template <int Q, typename S>
__device__ __forceinline__ double rho_d(const S* f, int64_t n, const FieldArgs& a)
{
    return a.rho_ref_d + dev_d<Q, S>(f, n, a);
}

// EOS pressure at node n: one component, p = rho/3 + (G/6) psi^2; two components (the gas
// component in a.f2, same storage, shifted by a.rho_ref2), p = (rho_l + rho_v)/3 + (Gx/3) rho_l rho_v.
template <int Q, typename S>
__device__ __forceinline__ double pressure_at(const S* f, int64_t n, const FieldArgs& a)
{
    const double r = rho_d<Q, S>(f, n, a);
    if (a.f2) {
        const double rv = a.rho_ref2 + dev_d<Q, S>((const S*)a.f2, n, a);
        return (r + rv) / 3.0 + (a.Gx / 3.0) * r * rv;
    }
    return pressure_d(r, a.Gd);
}

// ---- psi and the reported fields (FP64 arithmetic, FP32 output) -------------------------------
template <int Q, typename S>
__global__ void k_psi(const S* f, double* psi, FieldArgs a)
{
    for (int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; n < a.N;
         n += (int64_t)gridDim.x * blockDim.x)
        psi[n] = psi_f(rho_d<Q, S>(f, n, a));
}

// rho and u = (j + F/2)/rho with the Shan-Chen force of the current state.
template <int Q, typename S>
__global__ void k_fields(const S* f, const double* psi, float* rho_out, float* u_out, FieldArgs a)
{
    using L = lat<Q>;
    for (int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; n < a.N;
         n += (int64_t)gridDim.x * blockDim.x) {
        int x, y, z;
        coords3(n, a.nx, a.ny, x, y, z);
        double g[Q];
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            g[i] = (double)load_f(f[(int64_t)i * a.N + shifted<Q>(x, y, z, i, -1, a)]);
            s += g[i];
        }
        const double rho = a.rho_ref_d + s;
        if (rho_out) rho_out[n] = (float)rho;
        if (!u_out) continue;
        double j[3] = {0.0, 0.0, 0.0}, F[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            j[0] += g[i] * L::ex[i];
            j[1] += g[i] * L::ey[i];
            j[2] += g[i] * L::ez[i];
        }
        const uint16_t oc = a.owner ? a.owner[n] : (uint16_t)0;
#pragma unroll
        for (int i = 1; i < Q; ++i) {
            const int64_t m = shifted<Q>(x, y, z, i, +1, a);
            double pn = psi[m];
            // barrier: a neighbour of another, un-merged bubble is seen as bulk liquid
            if (oc != 0) {
                const uint16_t on = a.owner[m];
                if (on != 0 && on != oc) pn = a.psi_ld;
            }
            F[0] += L::wd[i] * pn * L::ex[i];
            F[1] += L::wd[i] * pn * L::ey[i];
            F[2] += L::wd[i] * pn * L::ez[i];
        }
        const double pc = psi[n];
        for (int c = 0; c < L::d; ++c) {
            double Fc = -a.Gd * pc * F[c];
            if (a.grav) Fc += (rho - a.rho0d) * a.gd[c];  // gravity body force
            u_out[(int64_t)c * a.N + n] = (float)((j[c] + 0.5 * Fc) / rho);
        }
    }
}

// ---- FP64 EOS and its lattice Laplacian (Sec. 3.1, the criterion's operator) ----------------
template <int Q, typename S>
__global__ void k_pressure(const S* f, double* p, FieldArgs a)
{
    for (int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; n < a.N;
         n += (int64_t)gridDim.x * blockDim.x)
        p[n] = pressure_at<Q, S>(f, n, a);
}

template <int Q>
__global__ void k_laplacian(const double* p, double* lap, FieldArgs a)
{
    using L = lat<Q>;
    for (int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; n < a.N;
         n += (int64_t)gridDim.x * blockDim.x) {
        int x, y, z;
        coords3(n, a.nx, a.ny, x, y, z);
        const double pc = p[n];
        double acc = 0.0;
#pragma unroll
        for (int i = 1; i < Q; ++i) acc += L::wd[i] * (p[shifted<Q>(x, y, z, i, +1, a)] - pc);
        lap[n] = 6.0 * acc;
    }
}

// ---- wave-level aggregation of per-node atomics ------------------------------------------------
// Per-node contributions to per-bubble counters arrive from many nodes of the same bubble at
// once; one atomic per node onto a few hundred addresses serialises.  The lanes of a wave that
// carry the same key (a bubble slot, >= 0) sum their values with a butterfly and one lane adds the
// sum: one atomic per distinct key per wave.  Integer sums, so the result does not depend on the
// grouping.  Every lane of the wave must call these (the loops below are wave-uniform).
__device__ __forceinline__ long long wave_sum_i64(long long v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

template <int M, typename Flush>
__device__ __forceinline__ void wave_add_by_key(int key, const long long (&v)[M], Flush flush)
{
    const int lane = (int)(threadIdx.x & 63);
    unsigned long long pending = __ballot(key >= 0);
    while (pending) {
        const int leader = __ffsll(pending) - 1;
        const int k = __shfl(key, leader, 64);
        const bool mine = key == k;
        const unsigned long long grp = __ballot(mine);
        long long sum[M];
#pragma unroll
        for (int j = 0; j < M; ++j) sum[j] = wave_sum_i64(mine ? v[j] : 0ll);
        if (lane == leader) flush(k, sum);
        pending &= ~grp;
    }
}

// ---- FP64 totals: wave64 shuffles -> LDS -> one partial per block -> fixed-order final sum ---
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

constexpr int kTotBlocks = 1024;

int totals_blocks(int64_t N)
{
    int64_t b = (N + 255) / 256;
    return (int)(b < kTotBlocks ? (b < 1 ? 1 : b) : kTotBlocks);
}

// Sums the stored values directly (a permutation of the pulled ones): M = N rho_ref + sum g,
// J = sum_i e_i sum_y g_i(y).
template <int Q, typename S>
__global__ void __launch_bounds__(256) k_totals(const S* f, double* partials, FieldArgs a)
{
    using L = lat<Q>;
    double m = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
    for (int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; n < a.N;
         n += (int64_t)gridDim.x * blockDim.x) {
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const double g = (double)load_f(f[(int64_t)i * a.N + n]);
            m += g;
            jx += g * L::ex[i];
            jy += g * L::ey[i];
            jz += g * L::ez[i];
        }
    }
    __shared__ double red[4][4];
    m = wave_sum(m); jx = wave_sum(jx); jy = wave_sum(jy); jz = wave_sum(jz);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) { red[w][0] = m; red[w][1] = jx; red[w][2] = jy; red[w][3] = jz; }
    __syncthreads();
    if (threadIdx.x < 4) {
        double s = 0.0;
        for (int k = 0; k < 4; ++k) s += red[k][threadIdx.x];
        partials[(int64_t)blockIdx.x * 4 + threadIdx.x] = s;
    }
}

__global__ void k_totals_final(const double* partials, int nb, double* out, double base_mass)
{
    // one thread per component, blocks summed in index order; the loads of 16 partials are
    // issued together before their ordered adds, so the sum waits out one latency per 16
    const int c = threadIdx.x;
    if (c >= 4) return;
    double s = 0.0;
    int b = 0;
    for (; b + 16 <= nb; b += 16) {
        double v[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) v[k] = partials[(int64_t)(b + k) * 4 + c];
#pragma unroll
        for (int k = 0; k < 16; ++k) s += v[k];
    }
    for (; b < nb; ++b) s += partials[(int64_t)b * 4 + c];
    out[c] = (c == 0) ? base_mass + s : s;
}

// ---- gas labelling: lock-free union-find, roots linked towards the smaller index ------------
constexpr uint32_t kLiquid = 0xffffffffu;

template <int Q, typename S>
__global__ void k_mask_rho(const S* f, uint32_t* parent, FieldArgs a)
{
    for (int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; n < a.N;
         n += (int64_t)gridDim.x * blockDim.x)
        parent[n] = (rho_d<Q, S>(f, n, a) < a.theta) ? (uint32_t)n : kLiquid;
}

// The test pass's mask and FP64 totals from one sweep of pulled populations: parent[n] exactly as
// k_mask_rho (same density, same order of the sum), and per block the partial sums of the pulled
// values and their momenta, as k_totals forms them from the stored values (the pulled values are a
// permutation of the stored ones, so the totals are the same sums in another order).
template <int Q, typename S>
__global__ void __launch_bounds__(256) k_mask_totals(const S* f, uint32_t* parent,
                                                     double* partials, FieldArgs a)
{
    using L = lat<Q>;
    double m = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
    // two nodes per pass, loads of both first (one block carries many nodes, so each pass would
    // otherwise wait out a full memory latency); the sums keep the node order
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t n0 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; n0 < a.N; n0 += 2 * stride) {
        float g[2][Q];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int64_t n = n0 + u * stride;
            if (n < a.N) {
                int x, y, z;
                coords3(n, a.nx, a.ny, x, y, z);
#pragma unroll
                for (int i = 0; i < Q; ++i)
                    g[u][i] = load_f(f[(int64_t)i * a.N + shifted<Q>(x, y, z, i, -1, a)]);
            }
        }
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int64_t n = n0 + u * stride;
            if (n >= a.N) continue;
            double s = 0.0, sx = 0.0, sy = 0.0, sz = 0.0;
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                const double v = (double)g[u][i];
                s += v;
                sx += v * L::ex[i];
                sy += v * L::ey[i];
                sz += v * L::ez[i];
            }
            parent[n] = (a.rho_ref_d + s < a.theta) ? (uint32_t)n : kLiquid;
            m += s;
            jx += sx;
            jy += sy;
            jz += sz;
        }
    }
    __shared__ double red[4][4];
    m = wave_sum(m); jx = wave_sum(jx); jy = wave_sum(jy); jz = wave_sum(jz);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) { red[w][0] = m; red[w][1] = jx; red[w][2] = jy; red[w][3] = jz; }
    __syncthreads();
    if (threadIdx.x < 4) {
        double t = 0.0;
        for (int k = 0; k < 4; ++k) t += red[k][threadIdx.x];
        partials[(int64_t)blockIdx.x * 4 + threadIdx.x] = t;
    }
}

__global__ void k_mask_bytes(const uint8_t* mask, uint32_t* parent, int64_t N)
{
    for (int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; n < N;
         n += (int64_t)gridDim.x * blockDim.x)
        parent[n] = mask[n] ? (uint32_t)n : kLiquid;
}

__device__ __forceinline__ uint32_t load_parent(const uint32_t* parent, uint32_t x)
{
    return __hip_atomic_load(parent + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint32_t find_root(const uint32_t* parent, uint32_t x)
{
    uint32_t p = load_parent(parent, x);
    while (p != x) {
        x = p;
        p = load_parent(parent, x);
    }
    return x;
}

// parent values only decrease and always point inside the same set, so a stale read is still an
// ancestor; atomicMin links root b under a and reports a concurrent re-link through its result.
__device__ void unite(uint32_t* parent, uint32_t a, uint32_t b)
{
    while (true) {
        a = find_root(parent, a);
        b = find_root(parent, b);
        if (a == b) return;
        if (a > b) { const uint32_t t = a; a = b; b = t; }
        const uint32_t old = atomicMin(parent + b, a);
        if (old == b) return;
        b = old;
    }
}

__global__ void k_flatten(const uint32_t* parent, uint32_t* labels, uint32_t* ncomp, int64_t N)
{
    for (int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; n < N;
         n += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t p = parent[n];
        if (p == kLiquid) {
            labels[n] = 0;
            continue;
        }
        uint32_t r = (uint32_t)n, q = p;
        while (q != r) {
            r = q;
            q = parent[r];
        }
        labels[n] = r + 1;
        if (r == (uint32_t)n) atomicAdd(ncomp, 1u);
    }
}

// Tiled labelling.  A plain union over every lattice link sends all of them through global
// atomics and pointer chases; on a gas-rich box that is most of the test pass.  Instead each block
// first unites the links inside its tile in LDS (local indices follow the global index order
// within a tile, so a local root is the smallest global index of its local set) and writes the
// local roots to parent; a second kernel unites only the links that leave a tile (or wrap around
// the box) through the global structure.  Roots still link to smaller indices, so the labels
// stay the canonical 1 + smallest index of each component.
template <int Q>
struct UnionTile;
template <>
struct UnionTile<9> {
    static constexpr int TX = 32, TY = 32, TZ = 1, THREADS = 1024;  // one node per thread
};
template <>
struct UnionTile<19> {
    static constexpr int TX = 16, TY = 16, TZ = 16, THREADS = 256;  // sixteen nodes per thread
};

__device__ __forceinline__ uint32_t lds_load(const uint32_t* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ uint32_t lds_root(const uint32_t* lp, uint32_t x)
{
    uint32_t p = lds_load(lp + x);
    while (p != x) {
        x = p;
        p = lds_load(lp + x);
    }
    return x;
}

__device__ void lds_unite(uint32_t* lp, uint32_t a, uint32_t b)
{
    while (true) {
        a = lds_root(lp, a);
        b = lds_root(lp, b);
        if (a == b) return;
        if (a > b) { const uint32_t t = a; a = b; b = t; }
        const uint32_t old = atomicMin(lp + b, a);
        if (old == b) return;
        b = old;
    }
}

// Neighbour (x + e_i) of a tile node stays inside the tile and the box: a local link.
template <int Q>
__device__ __forceinline__ bool local_link(int lx, int ly, int lz, int x, int y, int z, int i,
                                           const FieldArgs& a)
{
    using L = lat<Q>;
    using T = UnionTile<Q>;
    const int mx = lx + L::ex[i], my = ly + L::ey[i], mz = lz + L::ez[i];
    return mx >= 0 && mx < T::TX && my >= 0 && my < T::TY && mz >= 0 && mz < T::TZ &&
           x + L::ex[i] >= 0 && x + L::ex[i] < a.nx && y + L::ey[i] >= 0 &&
           y + L::ey[i] < a.ny && z + L::ez[i] >= 0 && z + L::ez[i] < a.nz;
}

template <int Q>
__global__ void __launch_bounds__(UnionTile<Q>::THREADS) k_union_local(uint32_t* parent,
                                                                       uint32_t* zero_counter,
                                                                       FieldArgs a)
{
    // the component counter of the flatten that follows starts at zero
    if (zero_counter && blockIdx.x == 0 && threadIdx.x == 0) *zero_counter = 0u;
    using L = lat<Q>;
    using T = UnionTile<Q>;
    constexpr int NT = T::TX * T::TY * T::TZ;
    __shared__ uint32_t lp[NT];
    const int gx = (a.nx + T::TX - 1) / T::TX, gy = (a.ny + T::TY - 1) / T::TY;
    const int b = blockIdx.x;
    const int x0 = (b % gx) * T::TX, y0 = ((b / gx) % gy) * T::TY, z0 = (b / (gx * gy)) * T::TZ;
    auto node = [&](int li, int& lx, int& ly, int& lz, int& x, int& y, int& z) {
        lx = li % T::TX;
        ly = (li / T::TX) % T::TY;
        lz = li / (T::TX * T::TY);
        x = x0 + lx; y = y0 + ly; z = z0 + lz;
        return x < a.nx && y < a.ny && z < a.nz;
    };
    static_assert(64 % T::TX == 0, "a wave holds whole tile rows");
    // runs along x: a wave holds 64 consecutive tile nodes, whole rows, so one ballot of the gas
    // mask gives every gas node the first node of its run, which becomes its parent (x-links
    // need no union at all)
    constexpr uint64_t kRowStarts = T::TX == 32 ? 0x0000000100000001ull
                                                : 0x0001000100010001ull;  // lanes with lx == 0
    static_assert(T::TX == 32 || T::TX == 16, "row-start mask for 16- or 32-node rows");
    for (int li = threadIdx.x; li < NT; li += blockDim.x) {
        int lx, ly, lz, x, y, z;
        const bool in = node(li, lx, ly, lz, x, y, z);
        const bool gas = in && parent[idx3(x, y, z, a.nx, a.ny)] != kLiquid;
        const uint64_t mask = __ballot(gas);
        const uint64_t starts = mask & ~((mask << 1) & ~kRowStarts);
        const int lane = li & 63;
        const uint64_t upto = ~0ull >> (63 - lane);
        lp[li] = gas ? (uint32_t)((li & ~63) + 63 - __clzll(starts & upto)) : kLiquid;
    }
    __syncthreads();
    // links to other rows: two adjacent runs always have a link at which one end starts its run
    // (the later-starting run's first node lies within the other's neighbourhood window, or the
    // other's first node touches it), so only such links are united -- per run, not per node
    auto starts_run = [&](int li, int lx) {
        return lx == 0 || lds_load(lp + li - 1) == kLiquid;
    };
    for (int li = threadIdx.x; li < NT; li += blockDim.x) {
        if (lds_load(lp + li) == kLiquid) continue;
        int lx, ly, lz, x, y, z;
        node(li, lx, ly, lz, x, y, z);
        const bool s0 = starts_run(li, lx);
#pragma unroll
        for (int h = 0; h < L::nhalf; ++h) {
            const int i = L::half[h];
            if (L::ey[i] == 0 && L::ez[i] == 0) continue;  // along the row: the run
            if (!local_link<Q>(lx, ly, lz, x, y, z, i, a)) continue;
            const int lj = li + L::ex[i] + T::TX * (L::ey[i] + T::TY * L::ez[i]);
            if (lds_load(lp + lj) == kLiquid) continue;
            if (!s0 && !starts_run(lj, lx + L::ex[i])) continue;
            lds_unite(lp, (uint32_t)li, (uint32_t)lj);
        }
    }
    __syncthreads();
    for (int li = threadIdx.x; li < NT; li += blockDim.x) {
        if (lp[li] == kLiquid) continue;
        int lx, ly, lz, x, y, z;
        node(li, lx, ly, lz, x, y, z);
        const uint32_t r = lds_root(lp, (uint32_t)li);
        const int rx = x0 + (int)(r % T::TX), ry = y0 + (int)((r / T::TX) % T::TY);
        const int rz = z0 + (int)(r / (T::TX * T::TY));
        parent[idx3(x, y, z, a.nx, a.ny)] = (uint32_t)idx3(rx, ry, rz, a.nx, a.ny);
    }
}

// The links the tiles could not see: those that leave a tile or wrap around the box.  As inside
// the tiles, only links at which one end starts its run along x (the first gas node of a tile
// row, or one whose left neighbour is liquid) are united: an x-link across a tile face always
// ends at such a node, and two adjacent runs of different rows always share such a link.
template <int Q>
__global__ void k_union_cross(uint32_t* parent, FieldArgs a)
{
    using L = lat<Q>;
    using T = UnionTile<Q>;
    for (int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; n < a.N;
         n += (int64_t)gridDim.x * blockDim.x) {
        if (load_parent(parent, (uint32_t)n) == kLiquid) continue;
        int x, y, z;
        coords3(n, a.nx, a.ny, x, y, z);
        const int lx = x % T::TX, ly = y % T::TY, lz = z % T::TZ;
        const bool s0 = lx == 0 || load_parent(parent, (uint32_t)(n - 1)) == kLiquid;
#pragma unroll
        for (int h = 0; h < L::nhalf; ++h) {
            const int i = L::half[h];
            if (local_link<Q>(lx, ly, lz, x, y, z, i, a)) continue;
            const int64_t m = shifted<Q>(x, y, z, i, +1, a);
            if (m == n) continue;
            if (load_parent(parent, (uint32_t)m) == kLiquid) continue;
            if (!s0) {
                const int mx = wrap_once(x + L::ex[i], a.nx);
                if (mx % T::TX != 0 && load_parent(parent, (uint32_t)(m - 1)) != kLiquid) continue;
            }
            unite(parent, (uint32_t)n, (uint32_t)m);
        }
    }
}

// ---- bubble statistics ------------------------------------------------------------------------
__global__ void k_gather(const uint32_t* labels, const int64_t* nodes, uint32_t* out, int n,
                         int64_t N)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int64_t nd = nodes[k];
    out[k] = (nd >= 0 && nd < N) ? labels[nd] : 0u;
}

__global__ void k_set_slots(int32_t* slot_of_root, const uint32_t* labs, int nb, int clear)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < nb) slot_of_root[labs[b] - 1] = clear ? -1 : b;
}

__device__ __forceinline__ int64_t min_image_i(int64_t d, int n)
{
    const int64_t h = n / 2;
    int64_t r = (d + h) % n;
    if (r < 0) r += n;
    return r - h;
}

__global__ void k_stats(const uint32_t* labels, const int32_t* slot_of_root, const int32_t* anchors,
                        unsigned long long* count, unsigned long long* sums, FieldArgs a)
{
    // block-uniform trip count, so every lane of a wave reaches the aggregation
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t n0 = blockIdx.x * (int64_t)blockDim.x; n0 < a.N; n0 += stride) {
        const int64_t n = n0 + threadIdx.x;
        int b = -1;
        long long v[4] = {0, 0, 0, 0};
        if (n < a.N) {
            const uint32_t L = labels[n];
            if (L) b = slot_of_root[L - 1];
            if (b >= 0) {
                int x, y, z;
                coords3(n, a.nx, a.ny, x, y, z);
                v[0] = 1;
                v[1] = min_image_i((int64_t)x - anchors[3 * b + 0], a.nx);
                v[2] = min_image_i((int64_t)y - anchors[3 * b + 1], a.ny);
                v[3] = min_image_i((int64_t)z - anchors[3 * b + 2], a.nz);
            }
        }
        // two's-complement wrap-around makes unsigned adds exact signed sums
        wave_add_by_key<4>(b, v, [&](int k, const long long* s) {
            const size_t o = (size_t)k * kStatStride;
            atomicAdd(count + o, (unsigned long long)s[0]);
            atomicAdd(sums + o + 0, (unsigned long long)s[1]);
            atomicAdd(sums + o + 1, (unsigned long long)s[2]);
            atomicAdd(sums + o + 2, (unsigned long long)s[3]);
        });
    }
}

// Gas-node list of the fed bubbles, in node order, without a global atomic per node or per wave:
// every block owns a contiguous chunk of nodes; the blocks count their fed gas nodes, one wave
// turns the counts into offsets, and each block writes its nodes from its offset on.
constexpr int kListBlocks = 1024;

static int64_t list_chunk(int64_t N)
{
    return ((N + (int64_t)kListBlocks * 256 - 1) / ((int64_t)kListBlocks * 256)) * 256;
}

__device__ __forceinline__ bool fed_gas(const uint32_t* labels, const int32_t* slot_of_root,
                                        const int32_t* feed, int64_t n, int64_t N, int& b)
{
    b = -1;
    if (n >= N) return false;
    const uint32_t L = labels[n];
    if (!L) return false;
    const int s = slot_of_root[L - 1];
    if (s < 0 || !feed[s]) return false;
    b = s;
    return true;
}

__global__ void __launch_bounds__(256) k_gas_count(const uint32_t* labels,
                                                   const int32_t* slot_of_root,
                                                   const int32_t* feed, unsigned int* counts,
                                                   int64_t N, int64_t chunk)
{
    const int64_t begin = blockIdx.x * chunk;
    unsigned int c = 0;
    for (int64_t n0 = begin; n0 < begin + chunk && n0 < N; n0 += 256) {
        int b;
        c += (unsigned int)__syncthreads_count(
            fed_gas(labels, slot_of_root, feed, n0 + threadIdx.x, N, b));
    }
    if (threadIdx.x == 0) counts[blockIdx.x] = c;
}

// One wave: exclusive prefix sums of the block counts in place, and their total.
__global__ void __launch_bounds__(64) k_gas_scan(unsigned int* counts, int n, unsigned int* total)
{
    const int lane = (int)threadIdx.x;
    unsigned int carry = 0;
    for (int c0 = 0; c0 < n; c0 += 64) {
        const int i = c0 + lane;
        const unsigned int v = i < n ? counts[i] : 0u;
        unsigned int x = v;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const unsigned int y = __shfl_up(x, off, 64);
            if (lane >= off) x += y;
        }
        if (i < n) counts[i] = carry + x - v;
        carry += __shfl(x, 63, 64);
    }
    if (lane == 0) *total = carry;
}

__global__ void __launch_bounds__(256) k_gas_write(const uint32_t* labels,
                                                   const int32_t* slot_of_root,
                                                   const int32_t* feed,
                                                   const unsigned int* offsets,
                                                   uint32_t* list_node, int32_t* list_slot,
                                                   int64_t N, int64_t chunk)
{
    __shared__ unsigned int wcnt[4];
    const int lane = (int)(threadIdx.x & 63), w = (int)(threadIdx.x >> 6);
    const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    unsigned int base = offsets[blockIdx.x];
    const int64_t begin = blockIdx.x * chunk;
    for (int64_t n0 = begin; n0 < begin + chunk && n0 < N; n0 += 256) {
        const int64_t n = n0 + threadIdx.x;
        int b;
        const bool g = fed_gas(labels, slot_of_root, feed, n, N, b);
        const unsigned long long m = __ballot(g);
        if (lane == 0) wcnt[w] = (unsigned int)__popcll(m);
        __syncthreads();
        unsigned int off = base;
        for (int k = 0; k < w; ++k) off += wcnt[k];
        const unsigned int tot = wcnt[0] + wcnt[1] + wcnt[2] + wcnt[3];
        if (g) {
            const unsigned int k = off + (unsigned int)__popcll(m & below);
            list_node[k] = (uint32_t)n;
            list_slot[k] = b;
        }
        base += tot;
        __syncthreads();  // wcnt is rewritten by the next pass
    }
}

// ---- merge criterion (Sec. 3.1 eta_m, Sec. 4): one thread per candidate pair -----------------
template <int Q>
__device__ __forceinline__ int64_t walk_node(const MergePair& pr, int k, const FieldArgs& a)
{
#pragma clang fp contract(off)
    double pt[3];
    for (int c = 0; c < 3; ++c) pt[c] = pr.cen_a[c] + pr.dv[c] * (double)k / (double)pr.T;
    int x = (int)floor(pt[0] + 0.5) % a.nx; if (x < 0) x += a.nx;
    int y = (int)floor(pt[1] + 0.5) % a.ny; if (y < 0) y += a.ny;
    int z = 0;
    if (lat<Q>::d == 3) { z = (int)floor(pt[2] + 0.5) % a.nz; if (z < 0) z += a.nz; }
    return idx3(x, y, z, a.nx, a.ny);
}

// One wave tests one pair: the lanes take consecutive samples of the walk, so the walk's node
// arithmetic and label loads run side by side instead of one after another.  Repeats of the
// previous sample's node are dropped and positions counted over the kept samples, exactly as a
// sequential walk would; the densest film node is the first of the maxima in walk order, and the
// Laplacian's terms are summed by lane 0 in direction order.  Every lane of the wave must call
// this; all of them return the same result.
__device__ __forceinline__ int wave_max_i(int v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = max(v, __shfl_xor(v, off, 64));
    return v;
}
__device__ __forceinline__ int wave_min_i(int v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = min(v, __shfl_xor(v, off, 64));
    return v;
}
__device__ __forceinline__ double wave_max_d(double v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

template <int Q, typename S>
__device__ MergeResult merge_pair_wave(const MergePair& pr, const uint32_t* labels, const S* f,
                                       int film_max, const FieldArgs& a)
{
    using L = lat<Q>;
    const int lane = (int)(threadIdx.x & 63);
    const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const int nk = pr.T + 1;
    MergeResult r;
    r.fired = 0; r.film_len = -1; r.film_node = -1; r.lap_p = 0.0; r.rho_film = 0.0;
    // Visits the kept samples chunk by chunk: fn(kept, pos, node) per lane, with the chunk's
    // lanes in walk order; fn returns false (wave-uniformly) to stop.
    auto walk = [&](auto fn) {
        int64_t carry_node = -1;
        int carry_pos = -1;
        for (int k0 = 0; k0 < nk; k0 += 64) {
            const int k = k0 + lane;
            const bool in = k < nk;
            const int64_t nd = in ? walk_node<Q>(pr, k, a) : (int64_t)-2;
            int64_t prev = __shfl_up(nd, 1, 64);
            if (lane == 0) prev = carry_node;
            const bool keep = in && nd != prev;
            const unsigned long long km = __ballot(keep);
            const int pos = carry_pos + __popcll(km & below) + 1;
            if (!fn(keep, pos, nd)) return;
            carry_pos += __popcll(km);
            const int last = min(63, nk - 1 - k0);
            carry_node = __shfl(nd, last, 64);
        }
    };
    // last node of a; then the first node of b after it
    int sa = -1;
    walk([&](bool keep, int pos, int64_t nd) {
        const int c = (keep && labels[nd] == pr.label_a) ? pos : -1;
        sa = max(sa, wave_max_i(c));
        return true;
    });
    if (sa < 0) return r;
    int sb = -1;
    walk([&](bool keep, int pos, int64_t nd) {
        const int c = (keep && pos > sa && labels[nd] == pr.label_b) ? pos : 0x7fffffff;
        const int m = wave_min_i(c);
        if (m != 0x7fffffff) sb = m;
        return sb < 0;
    });
    const int len = sb - sa - 1;
    if (sb < 0 || len < 1 || len > film_max) return r;
    // film run: positions sa+1 .. sb-1; liquid only; densest node first on ties
    bool clean = true;
    int64_t cstar = -1;
    double best = 0.0;
    walk([&](bool keep, int pos, int64_t nd) {
        const bool film = keep && pos > sa && pos < sb;
        if (__ballot(film && labels[nd] != 0)) clean = false;
        const double rho = film ? rho_d<Q, S>(f, nd, a) : -INFINITY;
        const double m = wave_max_d(rho);
        const unsigned long long at = __ballot(film && rho == m);
        if (at) {
            const int l0 = __ffsll(at) - 1;
            const int64_t node = __shfl(nd, l0, 64);
            if (cstar < 0 || m > best) {
                cstar = node;
                best = m;
            }
        }
        return true;
    });
    if (!clean) return r;
    int x, y, z;
    coords3(cstar, a.nx, a.ny, x, y, z);
    const double pc = pressure_at<Q, S>(f, cstar, a);
    double term = 0.0;
    if (lane >= 1 && lane < Q) {
        const int64_t m = shifted<Q>(x, y, z, lane, +1, a);
        term = L::wd[lane] * (pressure_at<Q, S>(f, m, a) - pc);
    }
    double acc = 0.0;
    for (int i = 1; i < Q; ++i) acc += __shfl(term, i, 64);
    const double lap = 6.0 * acc;
    r.film_len = len;
    r.film_node = cstar;
    r.lap_p = lap;
    r.rho_film = best;
    r.fired = lap >= 0.0 ? 1 : 0;
    return r;
}

// One wave (one block of 64) per candidate pair, over the first min(*count_d, npairs) pairs.
template <int Q, typename S>
__global__ void __launch_bounds__(64) k_merge(const S* f, const uint32_t* labels,
                                              const MergePair* pairs, MergeResult* res,
                                              int npairs, const int32_t* count_d, int film_max,
                                              FieldArgs a)
{
    const int p = blockIdx.x;
    if (count_d && *count_d < npairs) npairs = *count_d;
    if (p >= npairs) return;
    const MergeResult r = merge_pair_wave<Q, S>(pairs[p], labels, f, film_max, a);
    if (threadIdx.x == 0) res[p] = r;
}

// ---- blowing-agent source (Sec. 3): f_i(x) += w_i dm_b / n_b on the gas nodes of bubble b ----
// Each step bubble b is owed T_b = owed_b + dm_b: what earlier steps could not place plus this
// step's release.  Every listed node adds w_i T_b / n_b to its populations and rounds the sum
// into the storage type: to nearest for FP32, stochastically for FP16/BF16, whose spacing at a
// gas node (~5e-4 at -0.59 in FP16) exceeds the per-step increment (~1e-7) by orders of
// magnitude, so rounding to nearest would drop every increment.  The exact gain of the stored
// values (FP64 differences) is summed per bubble in fixed point (2^-40 units, integer atomics,
// so the sum does not depend on the order of the nodes), and k_source_close then sets
// owed_b = T_b - gain_b: the ledger carries what the storage could not take into the next step.

// The storage value next to the 16-bit pattern b toward +inf (up) or -inf: sign-magnitude
// layout, so moving away from zero adds one to the magnitude; +-0 steps to +-the smallest
// subnormal.
__device__ __forceinline__ uint16_t next_bits16(uint16_t b, bool up)
{
    const bool neg = (b & 0x8000u) != 0;
    if ((b & 0x7fffu) == 0) return up ? 0x0001u : 0x8001u;
    return (up != neg) ? (uint16_t)(b + 1u) : (uint16_t)(b - 1u);
}

// v rounded into the storage type.  FP32: to nearest.  FP16 / BF16: stochastically, to one of
// the two storage values lo <= v <= hi, hi with probability (v - lo) / (hi - lo), u in [0, 1),
// so the expected stored value is v.  (S)(float)v is one of lo, hi even where rounding twice
// picks the farther one; which of them it is follows from comparing it with v.
template <typename S>
__device__ __forceinline__ S round_into(double v, double u)
{
    const S h = static_cast<S>(static_cast<float>(v));
    const double hd = (double)static_cast<float>(h);
    if (hd == v) return h;
    const bool below = hd < v;
    const S o = __builtin_bit_cast(S, next_bits16(__builtin_bit_cast(uint16_t, h), below));
    const double od = (double)static_cast<float>(o);
    const double lo = below ? hd : od, hi = below ? od : hd;
    const bool take_hi = u < (v - lo) / (hi - lo);
    return take_hi ? (below ? o : h) : (below ? h : o);
}
template <>
__device__ __forceinline__ float round_into<float>(double v, double) { return (float)v; }

constexpr double kGainUnit = 1.0 / 1099511627776.0;  // 2^-40
constexpr double kGainScale = 1099511627776.0;

template <int Q, typename S>
__global__ void k_source(S* f, const uint32_t* list_node, const int32_t* list_slot, int64_t count,
                         SourceLedger led, int64_t t, FieldArgs a)
{
    using L = lat<Q>;
    // block-uniform trip count, so every lane of a wave reaches the aggregation of the gains
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k0 = blockIdx.x * (int64_t)blockDim.x; k0 < count; k0 += stride) {
        const int64_t k = k0 + threadIdx.x;
        int b = -1;
        long long gfx[1] = {0};
        if (k < count) {
            b = list_slot[k];
            const double T = led.owed[b] + led.dm[b];
            if (T == 0.0) {
                b = -1;
            } else {
                const double ab = T / led.nodes[b];
                const int64_t n = list_node[k];
                int x, y, z;
                coords3(n, a.nx, a.ny, x, y, z);
                // population i streams into n from n - e_i: 32-bit offsets per axis (indexed by
                // e + 1), as in the step kernel
                const uint32_t nx = a.nx, plane = (uint32_t)a.nx * (uint32_t)a.ny;
                const uint32_t xo[3] = {(uint32_t)wrap_once(x + 1, a.nx), (uint32_t)x,
                                        (uint32_t)wrap_once(x - 1, a.nx)};
                const uint32_t yo[3] = {(uint32_t)wrap_once(y + 1, a.ny) * nx, (uint32_t)y * nx,
                                        (uint32_t)wrap_once(y - 1, a.ny) * nx};
                const uint32_t zo[3] = {(uint32_t)wrap_once(z + 1, a.nz) * plane,
                                        (uint32_t)z * plane,
                                        (uint32_t)wrap_once(z - 1, a.nz) * plane};
                // every population of the node is loaded before any is stored (the stores
                // would otherwise order each load behind the previous direction's store)
                S* slot[Q];
                S old[Q];
#pragma unroll
                for (int i = 0; i < Q; ++i) {
                    slot[i] = f + (int64_t)i * a.N +
                              (xo[L::ex[i] + 1] + yo[L::ey[i] + 1] + zo[L::ez[i] + 1]);
                    old[i] = *slot[i];
                }
                double gain = 0.0;
#pragma unroll
                for (int i = 0; i < Q; ++i) {
                    const double oldd = (double)load_f(old[i]);
                    const double u = unit_noise(
                        led.key, ((uint64_t)t * (uint64_t)a.N + (uint64_t)n) * (uint64_t)Q +
                                     (uint64_t)i);
                    const S nw = round_into<S>(oldd + L::wd[i] * ab, u);
                    *slot[i] = nw;
                    gain += (double)load_f(nw) - oldd;
                }
                gfx[0] = (long long)rint(gain * kGainScale);
            }
        }
        wave_add_by_key<1>(b, gfx, [&](int kb, const long long* s) {
            atomicAdd(&led.gain[(size_t)kb * kLedgerGainStride], (unsigned long long)s[0]);
        });
    }
}

// Closes the step's ledger once every node has added: owed_b = T_b - gain_b, gains back to zero.
__global__ void __launch_bounds__(256) k_source_close(SourceLedger led)
{
    for (int b = threadIdx.x; b < led.nb; b += blockDim.x) {
        const long long g = (long long)led.gain[(size_t)b * kLedgerGainStride];
        const double T = led.owed[b] + led.dm[b];
        led.owed[b] = T - (double)g * kGainUnit;
        led.gain[(size_t)b * kLedgerGainStride] = 0ull;
    }
}

// ---- film geometry of a bubble pair (Sec. 3 film disc; Fig. 3) --------------------------------
// Node of sample k on the line shifted by off, and its rounded (unwrapped) position r.
template <int Q>
__device__ __forceinline__ int64_t film_node(const FilmArgs& g, const double off[3], int k,
                                             const FieldArgs& a, double r[3])
{
#pragma clang fp contract(off)
    for (int c = 0; c < 3; ++c) {
        const double q = g.cen[c] + off[c] + g.dv[c] * (double)k / (double)g.T;
        r[c] = floor(q + 0.5);
    }
    if (lat<Q>::d == 2) r[2] = 0.0;
    int x = (int)r[0] % a.nx; if (x < 0) x += a.nx;
    int y = (int)r[1] % a.ny; if (y < 0) y += a.ny;
    int z = 0;
    if (lat<Q>::d == 3) { z = (int)r[2] % a.nz; if (z < 0) z += a.nz; }
    return idx3(x, y, z, a.nx, a.ny);
}

// One thread per line (offset (i, j)); the centre line also measures h.  Three walks per line,
// consecutive repeats dropped: the last node of bubble a, the first node of b after it, then the
// run between (liquid only) and, on the centre line, the arc positions of the two crossings.
template <int Q, typename S>
__global__ void k_film(const S* f, const uint32_t* labels, FilmArgs g, FilmOut* out,
                       FieldArgs a)
{
#pragma clang fp contract(off)
    const int side = 2 * g.K + 1;
    const int nlines = g.dim == 3 ? side * side : side;
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < nlines;
         t += gridDim.x * blockDim.x) {
        const int i = t % side - g.K;
        const int j = g.dim == 3 ? t / side - g.K : 0;
        if (i * i + j * j > g.K * g.K) continue;
        double off[3], r[3];
        for (int c = 0; c < 3; ++c) off[c] = (double)i * g.n1[c] + (double)j * g.n2[c];
        int sa = -1, sb = -1, pos = -1;
        int64_t prev = -1;
        for (int k = 0; k <= g.T; ++k) {
            const int64_t nd = film_node<Q>(g, off, k, a, r);
            if (nd == prev) continue;
            prev = nd;
            ++pos;
            if (labels[nd] == g.label_a) sa = pos;
        }
        if (sa < 0) continue;
        prev = -1; pos = -1;
        for (int k = 0; k <= g.T && sb < 0; ++k) {
            const int64_t nd = film_node<Q>(g, off, k, a, r);
            if (nd == prev) continue;
            prev = nd;
            ++pos;
            if (pos > sa && labels[nd] == g.label_b) sb = pos;
        }
        const int len = sb >= 0 ? sb - sa - 1 : 0;
        if (len < 1 || len > g.film_max) continue;
        const bool centre = i == 0 && j == 0;
        bool clean = true;
        double arc = 0.0, sA = 0.0, sB = 0.0, rp[3] = {0.0, 0.0, 0.0}, rho_p = 0.0;
        prev = -1; pos = -1;
        for (int k = 0; k <= g.T && pos < sb; ++k) {
            const int64_t nd = film_node<Q>(g, off, k, a, r);
            if (nd == prev) continue;
            prev = nd;
            ++pos;
            if (pos > sa && pos < sb && labels[nd] != 0) clean = false;
            if (centre) {
                const double rho = rho_d<Q, S>(f, nd, a);
                if (pos >= 1) {
                    const double dx = r[0] - rp[0], dy = r[1] - rp[1], dz = r[2] - rp[2];
                    const double seg = sqrt(dx * dx + dy * dy + dz * dz);
                    if (pos == sa + 1) sA = arc + seg * (a.theta - rho_p) / (rho - rho_p);
                    if (pos == sb) sB = arc + seg * (rho_p - a.theta) / (rho_p - rho);
                    arc += seg;
                }
                rho_p = rho;
                for (int c = 0; c < 3; ++c) rp[c] = r[c];
            }
        }
        if (!clean) continue;
        atomicAdd(&out->count, 1u);
        if (centre) out->h = sB - sA;
    }
}

// ---- barrier owner field ---------------------------------------------------------------------
// Seed: a gas node of a bubble (a component holding nuclei) gets that bubble's owner id.
__global__ void k_owner_seed(const uint32_t* labels, const int32_t* slot_of_root,
                             const uint16_t* ids, int nb, uint16_t* owner, int64_t N)
{
    for (int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; n < N;
         n += (int64_t)gridDim.x * blockDim.x) {
        uint16_t o = 0;
        if (nb > 0) {
            const uint32_t l = labels[n];
            if (l != 0) {
                const int32_t b = slot_of_root[l - 1];
                if (b >= 0) o = ids[b];
            }
        }
        owner[n] = o;
    }
}

// One corona layer: a node nobody owns takes the smallest owner id among its lattice
// neighbours (the velocity set is symmetric, so x + e_i covers the same nodes as x - e_i).
template <int Q>
__global__ void k_owner_grow(const uint16_t* in, uint16_t* out, FieldArgs a)
{
    for (int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; n < a.N;
         n += (int64_t)gridDim.x * blockDim.x) {
        uint16_t o = in[n];
        if (o == 0) {
            int x, y, z;
            coords3(n, a.nx, a.ny, x, y, z);
#pragma unroll
            for (int i = 1; i < Q; ++i) {
                const uint16_t v = in[shifted<Q>(x, y, z, i, +1, a)];
                if (v != 0 && (o == 0 || v < o)) o = v;
            }
        }
        out[n] = o;
    }
}

// Frontier nodes: owned nodes with a lattice neighbour owned by a different bubble (the only
// nodes whose force the barrier changes), appended in any order.
template <int Q>
__global__ void k_frontier_list(const uint16_t* owner, uint32_t* list, unsigned int* count,
                                FieldArgs a)
{
    for (int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; n < a.N;
         n += (int64_t)gridDim.x * blockDim.x) {
        const uint16_t o = owner[n];
        if (o == 0) continue;
        int x, y, z;
        coords3(n, a.nx, a.ny, x, y, z);
        bool frontier = false;
#pragma unroll
        for (int i = 1; i < Q; ++i) {
            const uint16_t v = owner[shifted<Q>(x, y, z, i, +1, a)];
            if (v != 0 && v != o) frontier = true;
        }
        if (frontier) list[atomicAdd(count, 1u)] = (uint32_t)n;
    }
}

__global__ void k_fill_i32(int32_t* p, int32_t v, int64_t n)
{
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n;
         k += (int64_t)gridDim.x * blockDim.x)
        p[k] = v;
}

__global__ void k_fill_u64(unsigned long long* p, unsigned long long v, int64_t n)
{
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n;
         k += (int64_t)gridDim.x * blockDim.x)
        p[k] = v;
}

// ---- launchers ------------------------------------------------------------------------------
#define SC_DISPATCH(q, storage, CALL)                                                             \
    do {                                                                                          \
        if (q == 9 && storage == SC_STORE_F32) { constexpr int QQ = 9; using SS = float; CALL; }  \
        else if (q == 9 && storage == SC_STORE_F16) { constexpr int QQ = 9; using SS = _Float16; CALL; } \
        else if (q == 9 && storage == SC_STORE_BF16) { constexpr int QQ = 9; using SS = __bf16; CALL; } \
        else if (q == 19 && storage == SC_STORE_F32) { constexpr int QQ = 19; using SS = float; CALL; } \
        else if (q == 19 && storage == SC_STORE_F16) { constexpr int QQ = 19; using SS = _Float16; CALL; } \
        else if (q == 19 && storage == SC_STORE_BF16) { constexpr int QQ = 19; using SS = __bf16; CALL; } \
        else return hipErrorInvalidValue;                                                         \
    } while (0)

hipError_t launch_psi(int q, int storage, const void* f, double* psi, const FieldArgs& a,
                      hipStream_t st)
{
    SC_DISPATCH(q, storage,
                hipLaunchKernelGGL((k_psi<QQ, SS>), grid_for(a.N), dim3(256), 0, st,
                                   (const SS*)f, psi, a));
    return hipGetLastError();
}

hipError_t launch_fields(int q, int storage, const void* f, const double* psi, float* rho,
                         float* u, const FieldArgs& a, hipStream_t st)
{
    SC_DISPATCH(q, storage,
                hipLaunchKernelGGL((k_fields<QQ, SS>), grid_for(a.N), dim3(256), 0, st,
                                   (const SS*)f, psi, rho, u, a));
    return hipGetLastError();
}

hipError_t launch_pressure(int q, int storage, const void* f, double* p, const FieldArgs& a,
                           hipStream_t st)
{
    SC_DISPATCH(q, storage,
                hipLaunchKernelGGL((k_pressure<QQ, SS>), grid_for(a.N), dim3(256), 0, st,
                                   (const SS*)f, p, a));
    return hipGetLastError();
}

hipError_t launch_laplacian(int q, const double* p, double* lap, const FieldArgs& a,
                            hipStream_t st)
{
    if (q == 9)
        hipLaunchKernelGGL((k_laplacian<9>), grid_for(a.N), dim3(256), 0, st, p, lap, a);
    else if (q == 19)
        hipLaunchKernelGGL((k_laplacian<19>), grid_for(a.N), dim3(256), 0, st, p, lap, a);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_totals(int q, int storage, const void* f, double* partials, double* out_d,
                         const FieldArgs& a, hipStream_t st)
{
    const int nb = totals_blocks(a.N);
    SC_DISPATCH(q, storage,
                hipLaunchKernelGGL((k_totals<QQ, SS>), dim3(nb), dim3(256), 0, st, (const SS*)f,
                                   partials, a));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_totals_final, dim3(1), dim3(64), 0, st, partials, nb, out_d,
                       (double)a.N * a.rho_ref_d);
    return hipGetLastError();
}

hipError_t launch_mask_from_rho(int q, int storage, const void* f, uint32_t* parent,
                                const FieldArgs& a, hipStream_t st)
{
    SC_DISPATCH(q, storage,
                hipLaunchKernelGGL((k_mask_rho<QQ, SS>), grid_for(a.N), dim3(256), 0, st,
                                   (const SS*)f, parent, a));
    return hipGetLastError();
}

hipError_t launch_mask_totals(int q, int storage, const void* f, uint32_t* parent,
                              double* partials, double* out_d, const FieldArgs& a, hipStream_t st)
{
    const int nb = totals_blocks(a.N);
    SC_DISPATCH(q, storage,
                hipLaunchKernelGGL((k_mask_totals<QQ, SS>), dim3(nb), dim3(256), 0, st,
                                   (const SS*)f, parent, partials, a));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_totals_final, dim3(1), dim3(64), 0, st, partials, nb, out_d,
                       (double)a.N * a.rho_ref_d);
    return hipGetLastError();
}

hipError_t launch_mask_from_bytes(const uint8_t* mask_d, uint32_t* parent, int64_t N,
                                  hipStream_t st)
{
    hipLaunchKernelGGL(k_mask_bytes, grid_for(N), dim3(256), 0, st, mask_d, parent, N);
    return hipGetLastError();
}

template <int Q>
static hipError_t launch_union_tiled(uint32_t* parent, uint32_t* zero_counter, const FieldArgs& a,
                                     hipStream_t st)
{
    using T = UnionTile<Q>;
    const int64_t tiles = (int64_t)((a.nx + T::TX - 1) / T::TX) * ((a.ny + T::TY - 1) / T::TY) *
                          ((a.nz + T::TZ - 1) / T::TZ);
    if (tiles > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_union_local<Q>), dim3((unsigned)tiles), dim3(T::THREADS), 0, st,
                       parent, zero_counter, a);
    hipLaunchKernelGGL((k_union_cross<Q>), grid_for(a.N), dim3(256), 0, st, parent, a);
    return hipGetLastError();
}

hipError_t launch_union(int q, uint32_t* parent, uint32_t* zero_counter, const FieldArgs& a,
                        hipStream_t st)
{
    if (q == 9) return launch_union_tiled<9>(parent, zero_counter, a, st);
    if (q == 19) return launch_union_tiled<19>(parent, zero_counter, a, st);
    return hipErrorInvalidValue;
}

hipError_t launch_flatten(uint32_t* parent, uint32_t* labels, uint32_t* ncomp_d, int64_t N,
                          hipStream_t st)
{
    hipLaunchKernelGGL(k_flatten, grid_for(N), dim3(256), 0, st, parent, labels, ncomp_d, N);
    return hipGetLastError();
}

hipError_t launch_gather_labels(const uint32_t* labels, const int64_t* nodes_d, uint32_t* out_d,
                                int n, int64_t N, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather, dim3((n + 255) / 256), dim3(256), 0, st, labels, nodes_d, out_d,
                       n, N);
    return hipGetLastError();
}

hipError_t launch_set_slots(int32_t* slot_of_root, const uint32_t* labs_d, int nb, int clear,
                            hipStream_t st)
{
    if (nb <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_set_slots, dim3((nb + 255) / 256), dim3(256), 0, st, slot_of_root,
                       labs_d, nb, clear);
    return hipGetLastError();
}

hipError_t launch_stats(const uint32_t* labels, const int32_t* slot_of_root,
                        const int32_t* anchors_d, unsigned long long* count_d,
                        unsigned long long* sums_d, const FieldArgs& a, hipStream_t st)
{
    hipLaunchKernelGGL(k_stats, grid_for(a.N), dim3(256), 0, st, labels, slot_of_root, anchors_d,
                       count_d, sums_d, a);
    return hipGetLastError();
}

int gas_list_scratch_words() { return kListBlocks; }

hipError_t launch_gas_list(const uint32_t* labels, const int32_t* slot_of_root,
                           const int32_t* feed_d, uint32_t* list_node, int32_t* list_slot,
                           unsigned int* count_d, unsigned int* block_counts, int64_t N,
                           hipStream_t st)
{
    const int64_t chunk = list_chunk(N);
    hipLaunchKernelGGL(k_gas_count, dim3(kListBlocks), dim3(256), 0, st, labels, slot_of_root,
                       feed_d, block_counts, N, chunk);
    hipLaunchKernelGGL(k_gas_scan, dim3(1), dim3(64), 0, st, block_counts, kListBlocks, count_d);
    hipLaunchKernelGGL(k_gas_write, dim3(kListBlocks), dim3(256), 0, st, labels, slot_of_root,
                       feed_d, block_counts, list_node, list_slot, N, chunk);
    return hipGetLastError();
}

hipError_t launch_merge_counted(int q, int storage, const void* f, const uint32_t* labels,
                                const MergePair* pairs_d, MergeResult* res_d, int cap,
                                const int32_t* count_d, int film_max, const FieldArgs& a,
                                hipStream_t st)
{
    if (cap <= 0) return hipSuccess;
    const dim3 g((unsigned)cap);
    SC_DISPATCH(q, storage,
                hipLaunchKernelGGL((k_merge<QQ, SS>), g, dim3(64), 0, st, (const SS*)f, labels,
                                   pairs_d, res_d, cap, count_d, film_max, a));
    return hipGetLastError();
}

// ---- read-back of a test pass ----------------------------------------------------------------
__device__ void stage_out_body(const StageOut& o)
{
    const int t = threadIdx.x;
    if (t < 4) o.dst_tot[t] = o.tot[t];
    if (t >= 4 && t < 8 && o.tot2) o.dst_tot[t] = o.tot2[t - 4];
    if (o.head && t < 16) o.dst_head[t] = o.head[t];
    for (int k = t; k < o.n; k += blockDim.x) {
        o.dst_comp[k] = o.comp[k];
        o.dst_count[k] = o.count[(size_t)k * kStatStride];
        o.dst_sums[3 * k + 0] = o.sums[(size_t)k * kStatStride + 0];
        o.dst_sums[3 * k + 1] = o.sums[(size_t)k * kStatStride + 1];
        o.dst_sums[3 * k + 2] = o.sums[(size_t)k * kStatStride + 2];
    }
    for (int k = t; k < o.ledger_nb; k += blockDim.x) o.dst_owed[k] = o.owed[k];
    for (int k = t; k < o.npairs; k += blockDim.x) {
        o.dst_pairs[k] = o.pairs[k];
        o.dst_ab[2 * k] = o.ab[2 * k];
        o.dst_ab[2 * k + 1] = o.ab[2 * k + 1];
        o.dst_res[k] = o.res[k];
    }
}

__global__ void __launch_bounds__(256) k_stage_out(StageOut o) { stage_out_body(o); }

hipError_t launch_stage_out(const StageOut& o, hipStream_t st)
{
    hipLaunchKernelGGL(k_stage_out, dim3(1), dim3(256), 0, st, o);
    return hipGetLastError();
}

// ---- device bubble table and candidate pairs --------------------------------------------------
static size_t tab_align(size_t b) { return (b + 255) & ~size_t(255); }

size_t bubble_tab_bytes(int n)
{
    const size_t m = (size_t)(n > 0 ? n : 1);
    return tab_align(64) + tab_align(4 * m) * 4 + tab_align(12 * m) +
           tab_align(8 * kStatStride * m) + tab_align(24 * m) + tab_align(8 * m);
}

BubbleTab bubble_tab_view(void* base, int n)
{
    const size_t m = (size_t)(n > 0 ? n : 1);
    char* p = (char*)base;
    BubbleTab t;
    t.head = (int32_t*)p; p += tab_align(64);
    t.comp = (uint32_t*)p; p += tab_align(4 * m);
    t.distinct = (uint32_t*)p; p += tab_align(4 * m);
    t.lead = (int32_t*)p; p += tab_align(4 * m);
    t.first = (int32_t*)p; p += tab_align(4 * m);
    t.anchors = (int32_t*)p; p += tab_align(12 * m);
    t.count = (unsigned long long*)p; p += tab_align(8 * kStatStride * m);
    t.sums = t.count + 1;
    t.cen = (double*)p; p += tab_align(24 * m);
    t.rad = (double*)p;
    return t;
}

// One block.  A bubble is a distinct nonzero label held by a nucleus node; its slot is the rank
// of its label among them and its lead nucleus the smallest index holding it (both O(n^2 / 1024)
// comparisons, a few microseconds for hundreds of nuclei).
__global__ void __launch_bounds__(1024) k_bubble_table(const uint32_t* labels,
                                                       const int64_t* nuc_node, int n, int64_t N,
                                                       BubbleTab prev, BubbleTab t,
                                                       int32_t* slot_of_root, int nx, int ny)
{
    __shared__ int nb;
    // the previous pass's bubbles leave the slot map first (prev: the same buffer laid out for
    // the nucleus count of that pass; its head is zero before the first pass)
    const int nb_prev = prev.head[0];
    for (int b = threadIdx.x; b < nb_prev; b += blockDim.x)
        slot_of_root[prev.distinct[b] - 1] = -1;
    __syncthreads();
    if (threadIdx.x == 0) nb = 0;
    for (int k = threadIdx.x; k < n; k += blockDim.x) {
        const int64_t nd = nuc_node[k];
        t.comp[k] = (nd >= 0 && nd < N) ? labels[nd] : 0u;
    }
    __syncthreads();
    for (int k = threadIdx.x; k < n; k += blockDim.x) {
        const uint32_t c = t.comp[k];
        int first = c != 0u;
        for (int j = 0; j < k && first; ++j)
            if (t.comp[j] == c) first = 0;
        t.first[k] = first;
        if (first) atomicAdd(&nb, 1);
    }
    __syncthreads();
    for (int k = threadIdx.x; k < n; k += blockDim.x) {
        if (!t.first[k]) continue;
        const uint32_t c = t.comp[k];
        int b = 0;
        for (int j = 0; j < n; ++j)
            if (t.first[j] && t.comp[j] < c) ++b;
        t.distinct[b] = c;
        t.lead[b] = k;
        const int64_t a0 = nuc_node[k];
        t.anchors[3 * b + 0] = (int32_t)(a0 % nx);
        t.anchors[3 * b + 1] = (int32_t)((a0 / nx) % ny);
        t.anchors[3 * b + 2] = (int32_t)(a0 / ((int64_t)nx * ny));
        t.count[(size_t)b * kStatStride] = 0ull;
        t.sums[(size_t)b * kStatStride + 0] = 0ull;
        t.sums[(size_t)b * kStatStride + 1] = 0ull;
        t.sums[(size_t)b * kStatStride + 2] = 0ull;
        slot_of_root[c - 1] = b;
    }
    if (threadIdx.x == 0) {
        t.head[0] = nb;
        t.head[1] = 0;
    }
}

hipError_t launch_bubble_table(const uint32_t* labels, const int64_t* nuc_node, int n,
                               const BubbleTab& prev, const BubbleTab& t, int32_t* slot_of_root,
                               const FieldArgs& a, hipStream_t st)
{
    hipLaunchKernelGGL(k_bubble_table, dim3(1), dim3(1024), 0, st, labels, nuc_node, n, a.N,
                       prev, t, slot_of_root, a.nx, a.ny);
    return hipGetLastError();
}

__device__ __forceinline__ double min_image_d(double d, int n)
{
#pragma clang fp contract(off)
    return d - n * floor(d / n + 0.5);
}

// One block: centroid = anchor + (sum of integer offsets) / n and the equal-area (2D) or
// equal-volume (3D) radius, in the host's operation order; then the candidate pairs.
__device__ void find_pairs(const BubbleTab& t, const int32_t* group, int dim, int film_max,
                           MergePair* pairs, int32_t* ab, int cap, int nx, int ny, int nz)
{
#pragma clang fp contract(off)
    const int nb = t.head[0];
    for (int b = threadIdx.x; b < nb; b += blockDim.x) {
        const double n = (double)t.count[(size_t)b * kStatStride];
        for (int c = 0; c < 3; ++c)
            t.cen[3 * b + c] = (double)t.anchors[3 * b + c] +
                               (double)(long long)t.sums[(size_t)b * kStatStride + c] / n;
        if (dim == 2) {
            t.cen[3 * b + 2] = 0.0;
            t.rad[b] = sqrt(n / M_PI);
        } else {
            t.rad[b] = cbrt(3.0 * n / (4.0 * M_PI));
        }
    }
    __syncthreads();
    const int64_t total = (int64_t)nb * nb;
    for (int64_t p = threadIdx.x; p < total; p += blockDim.x) {
        const int a = (int)(p / nb), b = (int)(p % nb);
        if (b <= a) continue;
        if (group[t.lead[a]] == group[t.lead[b]]) continue;
        double dv[3];
        dv[0] = min_image_d(t.cen[3 * b + 0] - t.cen[3 * a + 0], nx);
        dv[1] = min_image_d(t.cen[3 * b + 1] - t.cen[3 * a + 1], ny);
        dv[2] = (dim == 3) ? min_image_d(t.cen[3 * b + 2] - t.cen[3 * a + 2], nz) : 0.0;
        const double dist = sqrt(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
        if (dist > t.rad[a] + t.rad[b] + (double)film_max + 1e-6) continue;
        const int T = (int)ceil(dist);
        if (T <= 0) continue;
        const int k = atomicAdd(&t.head[1], 1);
        if (k >= cap) continue;
        MergePair mp;
        for (int c = 0; c < 3; ++c) {
            mp.cen_a[c] = t.cen[3 * a + c];
            mp.dv[c] = dv[c];
        }
        mp.label_a = t.distinct[a];
        mp.label_b = t.distinct[b];
        mp.T = T;
        mp.pad = 0;
        pairs[k] = mp;
        ab[2 * k] = a;
        ab[2 * k + 1] = b;
    }
}

__global__ void __launch_bounds__(1024) k_pairs(BubbleTab t, const int32_t* group, int dim,
                                                int film_max, MergePair* pairs, int32_t* ab,
                                                int cap, int nx, int ny, int nz)
{
    find_pairs(t, group, dim, film_max, pairs, ab, cap, nx, ny, nz);
}

hipError_t launch_pairs(const BubbleTab& t, const int32_t* group, int dim, int film_max,
                        MergePair* pairs, int32_t* ab, int cap, const FieldArgs& a,
                        hipStream_t st)
{
    hipLaunchKernelGGL(k_pairs, dim3(1), dim3(1024), 0, st, t, group, dim, film_max, pairs, ab,
                       cap, a.nx, a.ny, a.nz);
    return hipGetLastError();
}

// The tail of a test pass in one block: candidate pairs, their merge test (one wave per pair,
// sixteen at a time) and the read-back into pinned host memory.
template <int Q, typename S>
__global__ void __launch_bounds__(1024) k_pass_tail(BubbleTab t, const int32_t* group, int dim,
                                                    int film_max, MergePair* pairs, int32_t* ab,
                                                    MergeResult* res, int cap, int do_pairs,
                                                    StageOut o, const S* f,
                                                    const uint32_t* labels, FieldArgs a)
{
    if (do_pairs) {
        find_pairs(t, group, dim, film_max, pairs, ab, cap, a.nx, a.ny, a.nz);
        __syncthreads();
        const int found = min(t.head[1], cap);
        const int w = (int)(threadIdx.x >> 6), nw = (int)(blockDim.x >> 6);
        for (int p = w; p < found; p += nw) {
            const MergeResult r = merge_pair_wave<Q, S>(pairs[p], labels, f, film_max, a);
            if ((threadIdx.x & 63) == 0) res[p] = r;
        }
        __syncthreads();
    }
    stage_out_body(o);
}

hipError_t launch_pass_tail(int q, int storage, const BubbleTab& t, const int32_t* group,
                            int film_max, MergePair* pairs, int32_t* ab, MergeResult* res,
                            int cap, int do_pairs, const StageOut& o, const void* f,
                            const uint32_t* labels, const FieldArgs& a, hipStream_t st)
{
    const int dim = q == 9 ? 2 : 3;
    SC_DISPATCH(q, storage,
                hipLaunchKernelGGL((k_pass_tail<QQ, SS>), dim3(1), dim3(1024), 0, st, t, group,
                                   dim, film_max, pairs, ab, res, cap, do_pairs, o,
                                   (const SS*)f, labels, a));
    return hipGetLastError();
}

hipError_t launch_source(int q, int storage, void* f, const uint32_t* list_node,
                         const int32_t* list_slot, int64_t count, const SourceLedger& led,
                         int64_t t, const FieldArgs& a, hipStream_t st)
{
    if (count <= 0) return hipSuccess;
    SC_DISPATCH(q, storage,
                hipLaunchKernelGGL((k_source<QQ, SS>), grid_for(count), dim3(256), 0, st, (SS*)f,
                                   list_node, list_slot, count, led, t, a));
    hipLaunchKernelGGL(k_source_close, dim3(1), dim3(256), 0, st, led);
    return hipGetLastError();
}

hipError_t launch_owner_seed(const uint32_t* labels, const int32_t* slot_of_root,
                             const uint16_t* ids_d, int nb, uint16_t* owner, int64_t N,
                             hipStream_t st)
{
    hipLaunchKernelGGL(k_owner_seed, grid_for(N), dim3(256), 0, st, labels, slot_of_root, ids_d,
                       nb, owner, N);
    return hipGetLastError();
}

hipError_t launch_film(int q, int storage, const void* f, const uint32_t* labels,
                       const FilmArgs& g, FilmOut* out_d, const FieldArgs& a, hipStream_t st)
{
    const int side = 2 * g.K + 1;
    const int nlines = g.dim == 3 ? side * side : side;
    const dim3 grid((unsigned)std::max(1, std::min(1024, (nlines + 255) / 256)));
    SC_DISPATCH(q, storage,
                hipLaunchKernelGGL((k_film<QQ, SS>), grid, dim3(256), 0, st, (const SS*)f,
                                   labels, g, out_d, a));
    return hipGetLastError();
}

hipError_t launch_frontier_list(int q, const uint16_t* owner, uint32_t* list,
                                unsigned int* count_d, const FieldArgs& a, hipStream_t st)
{
    if (q == 9)
        hipLaunchKernelGGL((k_frontier_list<9>), grid_for(a.N), dim3(256), 0, st, owner, list,
                           count_d, a);
    else if (q == 19)
        hipLaunchKernelGGL((k_frontier_list<19>), grid_for(a.N), dim3(256), 0, st, owner, list,
                           count_d, a);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_owner_grow(int q, const uint16_t* in, uint16_t* out, const FieldArgs& a,
                             hipStream_t st)
{
    if (q == 9)
        hipLaunchKernelGGL((k_owner_grow<9>), grid_for(a.N), dim3(256), 0, st, in, out, a);
    else if (q == 19)
        hipLaunchKernelGGL((k_owner_grow<19>), grid_for(a.N), dim3(256), 0, st, in, out, a);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_i32, grid_for(n), dim3(256), 0, st, p, v, n);
    return hipGetLastError();
}

hipError_t launch_fill_u64(unsigned long long* p, unsigned long long v, int64_t n,
                           hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u64, grid_for(n), dim3(256), 0, st, p, v, n);
    return hipGetLastError();
}

}  // namespace sc
