// sc_probe.hip -- HBM bandwidth probe: the achievable ceiling the step kernel is judged against.
// A float4 grid-stride copy (read + write) and a float4 read-only pass over a device buffer.
#include <hip/hip_runtime.h>

#include <string>

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
