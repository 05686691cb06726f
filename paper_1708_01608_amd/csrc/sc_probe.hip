// sc_probe.hip -- HBM bandwidth probes: the achievable ceilings the step kernel is judged
// against.  A float4 grid-stride copy (read + write) and a float4 read-only pass over a device
// buffer; and the D3Q19 step's own memory pattern without its arithmetic: every population of
// every node pulled from its upstream neighbour and stored, once flat (one node per thread) and
// once marching the step kernel's tiles through the planes.
#include <hip/hip_runtime.h>

#include <string>

#include "sc_device.hpp"
#include "sc_internal.hpp"

namespace sc {

__global__ void k_probe_copy(const float4* __restrict__ a, float4* __restrict__ b, size_t n)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        b[i] = a[i];
}

__global__ void k_probe_read(const float4* __restrict__ a, float* __restrict__ sink, size_t n)
{
    float s = 0.0f;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        const float4 v = a[i];
        s += v.x + v.y + v.z + v.w;
    }
    if (s == -1.0f) sink[0] = s;  // keeps the loads; the buffers hold zeros
}

__global__ void k_probe_fill(float4* a, size_t n)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        a[i] = make_float4(0.f, 0.f, 0.f, 0.f);
}

// The step's data movement without its arithmetic: population i of node (x, y, z) becomes the
// stored population i of its upstream neighbour (periodic), written with non-temporal stores
// like the step's.  Addressing as in the step kernel: 32-bit byte offsets from per-direction
// bases (the box holds at most 2^32 bytes per direction), the plane offsets uniform.
template <typename T>
__device__ __forceinline__ void pattern_node(const T* __restrict__ s, T* __restrict__ d,
                                             int64_t N, uint32_t nx, uint32_t plane, uint32_t x,
                                             uint32_t xm, uint32_t xp, uint32_t y, uint32_t ym,
                                             uint32_t yp, uint32_t z, uint32_t zm, uint32_t zp)
{
    using L = lat<19>;
    const uint32_t xo[3] = {xp, x, xm};  // indexed by e_x + 1: the node pulls from x - e_x
    const uint32_t yo[3] = {yp * nx, y * nx, ym * nx};
    const uint32_t zo[3] = {zp * plane, z * plane, zm * plane};
    T v[19];
#pragma unroll
    for (int i = 0; i < 19; ++i) {
        const uint32_t off = (xo[L::ex[i] + 1] + yo[L::ey[i] + 1] + zo[L::ez[i] + 1]) *
                             (uint32_t)sizeof(T);
        v[i] = *reinterpret_cast<const T*>(reinterpret_cast<const char*>(s + (int64_t)i * N) +
                                           off);
    }
    const uint32_t off = (x + y * nx + z * plane) * (uint32_t)sizeof(T);
#pragma unroll
    for (int i = 0; i < 19; ++i)
        __builtin_nontemporal_store(
            v[i], reinterpret_cast<T*>(reinterpret_cast<char*>(d + (int64_t)i * N) + off));
}

// one node per thread: blocks of 256 along x, the grid's y and z the box's rows and planes
template <typename T>
__global__ void __launch_bounds__(256) k_pattern_flat(const T* __restrict__ s, T* __restrict__ d,
                                                      int nx, int ny, int nz)
{
    const int x = blockIdx.x * 256 + threadIdx.x;
    if (x >= nx) return;
    const int y = blockIdx.y, z = blockIdx.z;
    pattern_node(s, d, (int64_t)nx * ny * nz, nx, (uint32_t)nx * ny, x, wrap_once(x - 1, nx),
                 wrap_once(x + 1, nx), y, wrap_once(y - 1, ny), wrap_once(y + 1, ny), z,
                 wrap_once(z - 1, nz), wrap_once(z + 1, nz));
}

// tiles of tx x ty nodes marching tz planes, in the step kernel's block order (contiguous tile
// ranges per XCD when the tile count divides by 8)
template <typename T>
__global__ void __launch_bounds__(1024) k_pattern_march(const T* __restrict__ s,
                                                        T* __restrict__ d, int nx, int ny, int nz,
                                                        int tx, int ty, int tz)
{
    const int gx = (int)(((int64_t)nx + tx - 1) / tx), gy = (int)(((int64_t)ny + ty - 1) / ty),
              gz = (int)(((int64_t)nz + tz - 1) / tz);
    const int nb = gx * gy * gz;
    const int b = (nb % 8 == 0) ? (int)(blockIdx.x & 7) * (nb >> 3) + (int)(blockIdx.x >> 3)
                                : (int)blockIdx.x;
    const int bx = b % gx, by = (b / gx) % gy, bz = b / (gx * gy);
    const int x = bx * tx + (int)threadIdx.x % tx, y = by * ty + (int)threadIdx.x / tx;
    if (x >= nx || y >= ny) return;
    const int64_t N = (int64_t)nx * ny * nz;
    const uint32_t plane = (uint32_t)nx * ny;
    const int xm = wrap_once(x - 1, nx), xp = wrap_once(x + 1, nx);
    const int ym = wrap_once(y - 1, ny), yp = wrap_once(y + 1, ny);
    const int ze = min(bz * tz + tz, nz);
    for (int z = bz * tz; z < ze; ++z)
        pattern_node(s, d, N, nx, plane, x, xm, xp, y, ym, yp, z, wrap_once(z - 1, nz),
                     wrap_once(z + 1, nz));
}

}  // namespace sc

using namespace sc;

extern "C" int sc_hbm_probe(size_t bytes, int32_t reps, double* copy_GBps, double* read_GBps)
{
    if (bytes < 1024 * 1024 || reps < 1) return set_error(SC_E_INVAL, "bytes >= 1 MiB, reps >= 1");
    const size_t n = bytes / 16;
    float4 *a = nullptr, *b = nullptr;
    float* sink = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = SC_OK;
    auto ck = [&](hipError_t e, const char* what) {
        if (e != hipSuccess && rc == SC_OK) rc = set_error(SC_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
        return e == hipSuccess;
    };
    if (ck(hipMalloc(&a, n * 16), "hipMalloc") && ck(hipMalloc(&b, n * 16), "hipMalloc") &&
        ck(hipMalloc(&sink, 64), "hipMalloc") && ck(hipEventCreate(&e0), "event") &&
        ck(hipEventCreate(&e1), "event")) {
        const dim3 grid(1024), block(256);
        hipLaunchKernelGGL(k_probe_fill, grid, block, 0, 0, a, n);
        hipLaunchKernelGGL(k_probe_fill, grid, block, 0, 0, b, n);
        ck(hipGetLastError(), "fill");
        for (int which = 0; which < 2 && rc == SC_OK; ++which) {
            float best = 1e30f;
            for (int r = 0; r <= reps && rc == SC_OK; ++r) {
                ck(hipEventRecord(e0, 0), "record");
                if (which == 0)
                    hipLaunchKernelGGL(k_probe_copy, grid, block, 0, 0, a, b, n);
                else
                    hipLaunchKernelGGL(k_probe_read, grid, block, 0, 0, a, sink, n);
                ck(hipGetLastError(), "probe launch");
                ck(hipEventRecord(e1, 0), "record");
                ck(hipEventSynchronize(e1), "sync");
                float ms = 0.f;
                ck(hipEventElapsedTime(&ms, e0, e1), "elapsed");
                if (r > 0 && ms < best) best = ms;  // the first pass warms up
            }
            const double moved = (which == 0 ? 2.0 : 1.0) * (double)(n * 16);
            double* out = which == 0 ? copy_GBps : read_GBps;
            if (out && rc == SC_OK) *out = moved / (best * 1e-3) / 1e9;
        }
    }
    if (a) (void)hipFree(a);
    if (b) (void)hipFree(b);
    if (sink) (void)hipFree(sink);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    return rc;
}

extern "C" int sc_pattern_probe(int32_t nx, int32_t ny, int32_t nz, int32_t storage,
                                int32_t tile_x, int32_t tile_y, int32_t tile_z, int32_t reps,
                                double* flat_GBps, double* march_GBps)
{
    if (nx < 1 || ny < 1 || nz < 1 || reps < 1 || tile_x < 1 || tile_y < 1 || tile_z < 1 ||
        (int64_t)tile_x * tile_y > 1024 || storage < SC_STORE_F32 || storage > SC_STORE_BF16)
        return set_error(SC_E_INVAL, "pattern probe: bad box, tile, storage or reps");
    const int64_t N = (int64_t)nx * ny * nz;
    const size_t es = storage == SC_STORE_F32 ? 4 : 2;
    if ((size_t)N * es > ((size_t)1 << 32) || nx > (1 << 30) || ny > 65535 || nz > 65535)
        return set_error(SC_E_INVAL, "pattern probe: box too large");
    const size_t bytes = 19 * (size_t)N * es;
    void *a = nullptr, *b = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = SC_OK;
    auto ck = [&](hipError_t e, const char* what) {
        if (e != hipSuccess && rc == SC_OK)
            rc = set_error(SC_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
        return e == hipSuccess;
    };
    const int64_t tiles = (((int64_t)nx + tile_x - 1) / tile_x) *
                          (((int64_t)ny + tile_y - 1) / tile_y) *
                          (((int64_t)nz + tile_z - 1) / tile_z);
    if (tiles > 0x7fffffff) return set_error(SC_E_INVAL, "pattern probe: too many tiles");
    if (ck(hipMalloc(&a, bytes), "hipMalloc") && ck(hipMalloc(&b, bytes), "hipMalloc") &&
        ck(hipMemset(a, 0, bytes), "memset") && ck(hipEventCreate(&e0), "event") &&
        ck(hipEventCreate(&e1), "event")) {
        for (int which = 0; which < 2 && rc == SC_OK; ++which) {
            float best = 1e30f;
            for (int r = 0; r <= reps && rc == SC_OK; ++r) {
                ck(hipEventRecord(e0, 0), "record");
                if (which == 0) {
                    const dim3 grid((unsigned)(((int64_t)nx + 255) / 256), (unsigned)ny,
                                    (unsigned)nz);
                    if (es == 4)
                        hipLaunchKernelGGL(k_pattern_flat<uint32_t>, grid, dim3(256), 0, 0,
                                           (const uint32_t*)a, (uint32_t*)b, nx, ny, nz);
                    else
                        hipLaunchKernelGGL(k_pattern_flat<uint16_t>, grid, dim3(256), 0, 0,
                                           (const uint16_t*)a, (uint16_t*)b, nx, ny, nz);
                } else {
                    const dim3 grid((unsigned)tiles), block((unsigned)(tile_x * tile_y));
                    if (es == 4)
                        hipLaunchKernelGGL(k_pattern_march<uint32_t>, grid, block, 0, 0,
                                           (const uint32_t*)a, (uint32_t*)b, nx, ny, nz, tile_x,
                                           tile_y, tile_z);
                    else
                        hipLaunchKernelGGL(k_pattern_march<uint16_t>, grid, block, 0, 0,
                                           (const uint16_t*)a, (uint16_t*)b, nx, ny, nz, tile_x,
                                           tile_y, tile_z);
                }
                ck(hipGetLastError(), "pattern probe launch");
                ck(hipEventRecord(e1, 0), "record");
                ck(hipEventSynchronize(e1), "sync");
                float ms = 0.f;
                ck(hipEventElapsedTime(&ms, e0, e1), "elapsed");
                if (r > 0 && ms < best) best = ms;  // the first pass warms up
            }
            double* out = which == 0 ? flat_GBps : march_GBps;
            if (out && rc == SC_OK) *out = 2.0 * (double)bytes / (best * 1e-3) / 1e9;
        }
    }
    if (a) (void)hipFree(a);
    if (b) (void)hipFree(b);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    return rc;
}
