// sc_stepcore.hpp -- pieces of the Shan-Chen step shared by the step kernels (one and two
// components) and the batched kernel: the XCD-aware tile order, pulled loads, deviation sums,
// the grouped interaction sum and the forced BGK collision.
#pragma once

#include <type_traits>

#include "sc_device.hpp"
#include "sc_internal.hpp"

namespace sc {

// The value itself, opaque to the optimizer: what is derived from it is computed where it is used
// instead of being hoisted out of a loop, or shared with an earlier use, and kept live (with 128
// VGPRs, spilled) across the collision.
__device__ __forceinline__ int opaque(int v)
{
    asm volatile("" : "+v"(v));
    return v;
}
__device__ __forceinline__ float opaque(float v)
{
    asm volatile("" : "+v"(v));
    return v;
}

struct StepGrid {
    int gx, gy, gz;  // tiles along x, y and plane chunks
    int remap;       // 1: contiguous tile ranges per XCD (8 XCDs, round-robin dispatch)
};

// Logical tile of this block.  Blocks are dispatched round-robin over the 8 XCDs, so block b
// runs on XCD b % 8; with remap, XCD k processes the contiguous logical range
// [k * n/8, (k+1) * n/8) and neighbouring tiles share that XCD's L2.
__device__ __forceinline__ int logical_block(const StepGrid& g)
{
    const int b = blockIdx.x;
    const int n = g.gx * g.gy * g.gz;
    if (!g.remap) return b;
    return (b & 7) * (n >> 3) + (b >> 3);
}

// Pulled populations g_i = stored_i(x - e_i) of one node: unsigned 32-bit byte offsets from a
// per-direction base, so one vector add per load and the 64-bit bases stay in scalar registers.
// The byte offset of any node is below N sizeof(S) <= 2^32 (the library rejects larger boxes).
template <int Q, typename S>
__device__ __forceinline__ void pull_node(const S* __restrict__ src, int64_t N, int nx, int ny,
                                          int x, int xm, int xp, int y, int ym, int yp, int z,
                                          int zm, int zp, float* g)
{
    using L = lat<Q>;
    const uint32_t plane = (uint32_t)nx * (uint32_t)ny;
    const uint32_t xo[3] = {(uint32_t)xp, (uint32_t)x, (uint32_t)xm};   // by -e_x: +1 -> xm
    const uint32_t yo[3] = {(uint32_t)yp * nx, (uint32_t)y * nx, (uint32_t)ym * nx};
    const uint32_t zo[3] = {(uint32_t)zp * plane, (uint32_t)z * plane, (uint32_t)zm * plane};
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const uint32_t off = (xo[L::ex[i] + 1] + yo[L::ey[i] + 1] + zo[L::ez[i] + 1]) *
                             (uint32_t)sizeof(S);
        const char* base = reinterpret_cast<const char*>(src + (int64_t)i * N);
        g[i] = load_f(*reinterpret_cast<const S*>(base + off));
    }
}

// Index of the lattice velocity (dx, dy, dz) in lat<Q> (compile time).
template <int Q>
__device__ __host__ constexpr int dir_of(int dx, int dy, int dz)
{
    for (int i = 0; i < Q; ++i)
        if (lat<Q>::ex[i] == dx && lat<Q>::ey[i] == dy && lat<Q>::ez[i] == dz) return i;
    return -1;
}

// Interaction sum S = sum_{i != 0} w_i psi(x + e_i) e_i (the Shan-Chen force is -G psi(x) S),
// grouped by the lattice's symmetry: opposite axis neighbours enter as one difference, and the
// four diagonals of each coordinate plane as two differences that the plane's two components
// share (a1 = psi(+x+y) - psi(-x-y) counts for +x and +y, a2 = psi(+x-y) - psi(-x+y) for +x and
// -y).  24 operations in D3Q19 and 10 in D2Q9, against 48 and 20 for the plain sum.  psi(i)
// returns the pseudopotential seen at neighbour i; every direction is asked once.
template <int Q, typename A, typename P>
__device__ __forceinline__ void interaction_sum(P psi, A& sx, A& sy, A& sz)
{
    constexpr int E = dir_of<Q>(1, 0, 0), W = dir_of<Q>(-1, 0, 0);
    constexpr int N = dir_of<Q>(0, 1, 0), S = dir_of<Q>(0, -1, 0);
    const A w1 = weight<Q, A>(E), w2 = weight<Q, A>(dir_of<Q>(1, 1, 0));
    const A a1 = psi(dir_of<Q>(1, 1, 0)) - psi(dir_of<Q>(-1, -1, 0));
    const A a2 = psi(dir_of<Q>(1, -1, 0)) - psi(dir_of<Q>(-1, 1, 0));
    if constexpr (Q == 9) {
        sx = fmad(w1, psi(E) - psi(W), w2 * (a1 + a2));
        sy = fmad(w1, psi(N) - psi(S), w2 * (a1 - a2));
        sz = (A)0;
    } else {
        constexpr int T = dir_of<Q>(0, 0, 1), B = dir_of<Q>(0, 0, -1);
        const A b1 = psi(dir_of<Q>(1, 0, 1)) - psi(dir_of<Q>(-1, 0, -1));
        const A b2 = psi(dir_of<Q>(1, 0, -1)) - psi(dir_of<Q>(-1, 0, 1));
        const A c1 = psi(dir_of<Q>(0, 1, 1)) - psi(dir_of<Q>(0, -1, -1));
        const A c2 = psi(dir_of<Q>(0, 1, -1)) - psi(dir_of<Q>(0, -1, 1));
        sx = fmad(w1, psi(E) - psi(W), w2 * ((a1 + a2) + (b1 + b2)));
        sy = fmad(w1, psi(N) - psi(S), w2 * ((a1 - a2) + (c1 + c2)));
        sz = fmad(w1, psi(T) - psi(B), w2 * ((b1 - b2) + (c1 - c2)));
    }
}

// 1/rho through the hardware reciprocal and Newton steps (each doubles the correct bits): two
// in FP64, a faithful result for the densities here at half the cost of IEEE division; one in
// FP32 (3 instructions instead of the 10 of IEEE division, within an ulp).
__device__ __forceinline__ double recip(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}
__device__ __forceinline__ float recip(float x)
{
    const float r = __builtin_amdgcn_rcpf(x);
    return fmaf(r, fmaf(-x, r, 1.0f), r);
}

// Deviation sum sum_i g_i in the arithmetic type A (fixed order: the ring and the owner of a
// node obtain the same value).
template <int Q, typename A>
__device__ __forceinline__ A sum_dev(const float* g)
{
    A s = (A)0;
#pragma unroll
    for (int i = 0; i < Q; ++i) s += (A)g[i];
    return s;
}

// Scalar coefficients in the arithmetic type.
template <typename A>
struct Coef {
    A tau, omega, G, rho_ref, psi_l;
    A gx, gy, gz, rho0;  // gravity (used by the extended kernels when grav != 0)
    int grav;
};
__device__ __forceinline__ Coef<float> coef_of(const StepArgs& a, float)
{
    return Coef<float>{a.tau, a.omega, a.G, a.rho_ref, a.psi_l,
                       a.g[0], a.g[1], a.g[2], a.rho0, a.grav};
}
__device__ __forceinline__ Coef<double> coef_of(const StepArgs& a, double)
{
    return Coef<double>{a.taud, a.omegad, a.Gd, a.rho_refd, a.psi_ld,
                        a.gd[0], a.gd[1], a.gd[2], a.rho0d, a.grav};
}


// Forced BGK collision on deviations g_i = f_i - w_i rho_ref; writes f_i* - w_i rho_ref.
// With h_i = g_i - w_i drho (one fused rounding), the relaxation
//   f_i* = f_i - (f_i - f_i^eq)/tau,  f_i^eq - w_i rho_ref = w_i drho + w_i rho P_i,
//   P_i = 3 e.u + 4.5 (e.u)^2 - 1.5 u^2,
// becomes g_i* = g_i + omega (w_i rho P_i - h_i): every intermediate is small, so rounding
// happens at the scale of the non-equilibrium part instead of w_i rho.
// Store of one post-collision population; NT = non-temporal (streaming) store of FP32 values,
// which are not read again before the next step, so they need not displace loads from L2.
template <bool NT, typename S>
__device__ __forceinline__ void put(S* p, S v)
{
    *p = v;
}
template <>
__device__ __forceinline__ void put<true, float>(float* p, float v)
{
    __builtin_nontemporal_store(v, p);
}
template <>
__device__ __forceinline__ void put<true, _Float16>(_Float16* p, _Float16 v)
{
    __builtin_nontemporal_store(__builtin_bit_cast(uint16_t, v), reinterpret_cast<uint16_t*>(p));
}
template <>
__device__ __forceinline__ void put<true, __bf16>(__bf16* p, __bf16 v)
{
    __builtin_nontemporal_store(__builtin_bit_cast(uint16_t, v), reinterpret_cast<uint16_t*>(p));
}

// e_i . u with the exactly-zero components left out (a product with 0 would have to be kept
// under IEEE rules; dropping it changes no value).
template <int Q, typename A>
__device__ __forceinline__ A e_dot(int i, A ux, A uy, A uz)
{
    using L = lat<Q>;
    const bool hx = L::ex[i] != 0, hy = L::ey[i] != 0, hz = L::ez[i] != 0;
    A s = (A)0;
    if (hx) s = L::ex[i] > 0 ? ux : -ux;
    if (hy) s = hx ? (L::ey[i] > 0 ? s + uy : s - uy) : (L::ey[i] > 0 ? uy : -uy);
    if (hz) s = (hx || hy) ? (L::ez[i] > 0 ? s + uz : s - uz) : (L::ez[i] > 0 ? uz : -uz);
    return s;
}

// BGK relaxation towards f^eq(rho, u_eq) and the store of node `lane`:
// g_i* = g_i + omega (f_i^eq - f_i), written as deviations (the stored shift cancels in the
// difference: f_i - f_i^eq = g_i - (w_i drho + w_i rho P_i)).  In FP32 the w_i drho term takes
// the weight as a pair of floats.  Population i goes to byte offset
// lane sizeof(S) from the direction's base dst + i N (below 2^32, as for the loads).
//
// With 16-bit storage the stored value's rounding (2^-11 or 2^-8 relative) dwarfs the FP32
// arithmetic's, so the collision there takes the short form
//   g_i* = g_i + omega (w_i (drho + rho P_i) - g_i)
// with P of an opposite pair sharing its even part (P_i = S + 3 e.u, P_ibar = S - 3 e.u,
// S = 4.5 (e.u)^2 - 1.5 u^2): three FMAs a direction instead of five.
template <int Q, typename A, typename S, bool NT = false, bool RECVT = false>
__device__ __forceinline__ void relax_store(S* __restrict__ dst, int64_t N, uint32_t lane,
                                            const float* g, A drho, A rho, A ux, A uy, A uz,
                                            A omega)
{
    constexpr bool three = Q == 19;
    const A usq15 = (A)1.5 * (three ? ux * ux + uy * uy + uz * uz : ux * ux + uy * uy);
    const uint32_t boff = lane * (uint32_t)sizeof(S);
    if constexpr (sizeof(S) == 2) {
        // rest population, then the opposite pairs (i odd, i + 1 its reverse)
        auto put_one = [&](int i, A P) {
            const A gi = (A)g[i];
            const A feq = weight<Q, A>(i) * fmad(rho, P, drho);
            const A gs = fmad(omega, feq - gi, gi);
            char* base = reinterpret_cast<char*>(dst + (int64_t)i * N);
            put<NT, S>(reinterpret_cast<S*>(base + boff), store_f<S>((float)gs));
        };
        put_one(0, -usq15);
#pragma unroll
        for (int i = 1; i < Q; i += 2) {
            const A eu = e_dot<Q, A>(i, ux, uy, uz);
            const A even = fmad((A)4.5 * eu, eu, -usq15);
            put_one(i, fmad((A)3, eu, even));
            put_one(i + 1, fmad((A)-3, eu, even));
        }
        return;
    }
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const A eu = e_dot<Q, A>(i, ux, uy, uz);
        const A P = fmad(eu, fmad((A)4.5, eu, (A)3), -usq15);
        const A w = weight<Q, A>(i);
        // RECVT: converted again here rather than kept from the momentum sums (with FP64, 19
        // doubles live through the velocity spill in a 1024-thread block)
        const A gi = RECVT ? (A)opaque(g[i]) : (A)g[i];
        A h = fmad(-w, drho, gi);
        if constexpr (std::is_same<A, float>::value) h = fmad(-weight_lo<Q>(i), drho, h);
        const A d = fmad(w * rho, P, -h);
        const A gs = fmad(omega, d, gi);
        char* base = reinterpret_cast<char*>(dst + (int64_t)i * N);
        put<NT, S>(reinterpret_cast<S*>(base + boff), store_f<S>((float)gs));
    }
}

// Forced collision of one component: velocity-shift forcing u_eq = (j + tau F) / rho, then the
// BGK relaxation and the store.
template <int Q, typename A, typename S, bool NT = false, bool EXT = false, bool RECVT = false>
__device__ __forceinline__ void collide_store(S* __restrict__ dst, int64_t N, uint32_t lane,
                                              const float* g, A drho, A Fx, A Fy, A Fz,
                                              const Coef<A>& c)
{
    using L = lat<Q>;
    constexpr bool three = Q == 19;
    const A rho = c.rho_ref + drho;
    if constexpr (EXT) {
        if (c.grav) {  // gravity: buoyancy body force relative to rho0
            const A dr = (c.rho_ref - c.rho0) + drho;
            Fx = fmad(dr, c.gx, Fx);
            Fy = fmad(dr, c.gy, Fy);
            if (three) Fz = fmad(dr, c.gz, Fz);
        }
    }
    A jx = (A)0, jy = (A)0, jz = (A)0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        if (L::ex[i] > 0) jx += (A)g[i]; else if (L::ex[i] < 0) jx -= (A)g[i];
        if (L::ey[i] > 0) jy += (A)g[i]; else if (L::ey[i] < 0) jy -= (A)g[i];
        if (L::ez[i] > 0) jz += (A)g[i]; else if (L::ez[i] < 0) jz -= (A)g[i];
    }
    const A inv = recip(rho);
    // velocity-shift forcing: u_eq = (j + tau F) / rho
    const A ux = fmad(c.tau, Fx, jx) * inv;
    const A uy = fmad(c.tau, Fy, jy) * inv;
    const A uz = three ? fmad(c.tau, Fz, jz) * inv : (A)0;
    relax_store<Q, A, S, NT, RECVT>(dst, N, lane, g, drho, rho, ux, uy, uz, c.omega);
}

}  // namespace sc
