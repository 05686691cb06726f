// sc_device.hpp -- lattice tables and device helpers shared by the HIP kernels of libsc.
//
// Velocity sets (D2Q9, D3Q19) in this library's order: rest first, then opposite pairs next to
// each other (i odd, i+1 is its reverse).  Weights: D2Q9 4/9, 1/9, 1/36; D3Q19 1/3, 1/18, 1/36.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sc {

template <int Q>
struct lat;

template <>
struct lat<9> {
    static constexpr int d = 2;
    static constexpr int ex[9] = {0, 1, -1, 0, 0, 1, -1, 1, -1};
    static constexpr int ey[9] = {0, 0, 0, 1, -1, 1, -1, -1, 1};
    static constexpr int ez[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    static constexpr float wf[9] = {4.f / 9.f, 1.f / 9.f, 1.f / 9.f, 1.f / 9.f, 1.f / 9.f,
                                    1.f / 36.f, 1.f / 36.f, 1.f / 36.f, 1.f / 36.f};
    static constexpr double wd[9] = {4.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0,
                                     1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
    // Half of the neighbour directions (one of each opposite pair), for union-find.
    static constexpr int nhalf = 4;
    static constexpr int half[4] = {1, 3, 5, 7};
};

template <>
struct lat<19> {
    static constexpr int d = 3;
    static constexpr int ex[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
    static constexpr int ey[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
    static constexpr int ez[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
    static constexpr float wf[19] = {1.f / 3.f,  1.f / 18.f, 1.f / 18.f, 1.f / 18.f, 1.f / 18.f,
                                     1.f / 18.f, 1.f / 18.f, 1.f / 36.f, 1.f / 36.f, 1.f / 36.f,
                                     1.f / 36.f, 1.f / 36.f, 1.f / 36.f, 1.f / 36.f, 1.f / 36.f,
                                     1.f / 36.f, 1.f / 36.f, 1.f / 36.f, 1.f / 36.f};
    static constexpr double wd[19] = {1.0 / 3.0,  1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0,
                                      1.0 / 18.0, 1.0 / 18.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0,
                                      1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0,
                                      1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
    static constexpr int nhalf = 9;
    static constexpr int half[9] = {1, 3, 5, 7, 9, 11, 13, 15, 17};
};

// ---- storage conversion (FP32 arithmetic, FP32 / FP16 / BF16 storage) ----------------------
template <typename S>
__device__ __forceinline__ float load_f(S v) { return static_cast<float>(v); }
template <typename S>
__device__ __forceinline__ S store_f(float v) { return static_cast<S>(v); }

// ---- periodic coordinates ------------------------------------------------------------------
__device__ __forceinline__ int wrap_once(int a, int n)
{
    // a in [-n, 2n): one conditional correction
    return a < 0 ? a + n : (a >= n ? a - n : a);
}

struct Box {
    int nx, ny, nz;
    int64_t N;
};

__device__ __forceinline__ int64_t node_of(const Box& b, int x, int y, int z)
{
    return (int64_t)x + (int64_t)b.nx * ((int64_t)y + (int64_t)b.ny * z);
}

// psi(rho) = 1 - exp(-rho) (Sec. 3.1), in the arithmetic type of the kernel.
__device__ __forceinline__ float psi_f(float rho) { return 1.0f - expf(-rho); }
__device__ __forceinline__ double psi_f(double rho) { return 1.0 - exp(-rho); }

// Fused multiply-add in the arithmetic type (one rounding).
__device__ __forceinline__ float fmad(float a, float b, float c) { return fmaf(a, b, c); }
__device__ __forceinline__ double fmad(double a, double b, double c) { return fma(a, b, c); }

// Lattice weight in the arithmetic type.
template <int Q, typename A>
__device__ __forceinline__ A weight(int i);
template <>
__device__ __forceinline__ float weight<9, float>(int i) { return lat<9>::wf[i]; }
template <>
__device__ __forceinline__ double weight<9, double>(int i) { return lat<9>::wd[i]; }
template <>
__device__ __forceinline__ float weight<19, float>(int i) { return lat<19>::wf[i]; }
template <>
__device__ __forceinline__ double weight<19, double>(int i) { return lat<19>::wd[i]; }

// The FP32 weight's rounding error w - (float)w: with it, w x takes two FMAs to the accuracy of
// an FP64 weight.  1/9, 1/18 and 1/36 are not binary fractions; their FP32 rounding (relative
// ~3e-8) would otherwise bias every node's equilibrium by the same amount at every step.
template <int Q>
__device__ __forceinline__ float weight_lo(int i)
{
    return (float)(lat<Q>::wd[i] - (double)lat<Q>::wf[i]);
}

// p(rho) = rho/3 + (G/6) psi^2 in FP64 (Sec. 3.1 EOS; 0.166 read as G cs^2 / 2).
__device__ __forceinline__ double pressure_d(double rho, double G)
{
    double ps = 1.0 - exp(-rho);
    return rho / 3.0 + (G / 6.0) * ps * ps;
}

// SplitMix64: k-th output of the stream seeded with s (state s + k * golden gamma, then the
// 64-bit finaliser), and U in [0,1) from its top 53 bits.
__device__ __forceinline__ uint64_t splitmix64_at(uint64_t s, uint64_t k)
{
    uint64_t z = s + k * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ double unit_noise(uint64_t seed, int64_t idx)
{
    return (double)(splitmix64_at(seed, (uint64_t)idx + 1ull) >> 11) * (1.0 / 9007199254740992.0);
}

}  // namespace sc
