// lds_peak.hip -- measured LDS bandwidth of the part, the denominator of the
// attempt kernel's LDS roofline.  Not part of the REWL method: the benchmark
// loads this library on its own.
//
// Every workgroup (8 wavefronts) owns 64 KiB of LDS and streams through it:
// mode 0 reads 16 bytes per lane per instruction (ds_read_b128), mode 1
// writes 8 bytes per lane (ds_write_b64), 16 independent accesses per thread
// and pass.  Consecutive lanes touch consecutive 16 (8) byte words, so a
// wavefront instruction covers 1 KiB (512 B) without bank conflicts.  Two
// workgroups per CU (128 KiB of the 160 KiB, 16 wavefronts), a grid of two
// workgroups per compute unit; each thread folds what it read into one word
// that it stores, and the address of every access is opaque to the compiler,
// so no access is dropped or merged with another.
//
//   int lds_peak(int mode, int iters, double *bytes_per_s, double *ms)
//
// runs one warm-up and one timed launch on the null stream (iters passes of
// 16 accesses per thread) and returns the LDS bytes moved per second
// of the timed launch; 0 on success, -1 on a HIP error or invalid argument.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

constexpr int kThreads = 512;
constexpr int kBytes = 64 * 1024;
constexpr int kUnroll = 16;

__global__ __launch_bounds__(kThreads) void k_lds_stream(int mode, int iters, uint32_t *out) {
    extern __shared__ __align__(16) unsigned char lds[];
    const int t = threadIdx.x;
    uint4 *v16 = (uint4 *)lds;
    uint2 *v8 = (uint2 *)lds;
    for (int i = t; i < kBytes / 16; i += kThreads) v16[i] = make_uint4(i, i ^ 1, i ^ 2, i ^ 3);
    __syncthreads();
    uint32_t acc = 0;
    if (mode == 0) {
        for (int it = 0; it < iters; ++it) {
            // kUnroll independent reads in flight per thread; each address is
            // opaque to the compiler (every pass reads words it read before,
            // which it would otherwise load once and reuse)
            uint4 x[kUnroll];
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                int j = (t + u * kThreads + it * 64) & (kBytes / 16 - 1);
                asm volatile("" : "+v"(j));
                x[u] = v16[j];
            }
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) acc ^= x[u].x ^ x[u].y ^ x[u].z ^ x[u].w;
        }
    } else {
        uint2 x = make_uint2(t, ~t);
        for (int it = 0; it < iters; ++it) {
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                int j = (t + u * kThreads + it * 64) & (kBytes / 8 - 1);
                asm volatile("" : "+v"(j));
                v8[j] = x;
                x.x += 1u;
            }
        }
        __syncthreads();
        acc = v8[t].x;
    }
    out[blockIdx.x * kThreads + t] = acc;
}

}  // namespace

extern "C" int lds_peak(int mode, int iters, double *bytes_per_s, double *ms) {
    if ((mode != 0 && mode != 1) || iters < 1 || !bytes_per_s || !ms) return -1;
    int dev = 0, ncu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return -1;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return -1;
    if (hipFuncSetAttribute((const void *)k_lds_stream, hipFuncAttributeMaxDynamicSharedMemorySize, kBytes) !=
        hipSuccess)
        return -1;
    const int grid = 2 * ncu;
    uint32_t *out = nullptr;
    if (hipMalloc((void **)&out, sizeof(uint32_t) * (size_t)grid * kThreads) != hipSuccess) return -1;
    hipEvent_t a = nullptr, b = nullptr;
    int rc = -1;
    if (hipEventCreate(&a) == hipSuccess && hipEventCreate(&b) == hipSuccess) {
        hipLaunchKernelGGL(k_lds_stream, dim3(grid), dim3(kThreads), kBytes, 0, mode, iters, out);
        hipEventRecord(a, 0);
        hipLaunchKernelGGL(k_lds_stream, dim3(grid), dim3(kThreads), kBytes, 0, mode, iters, out);
        hipEventRecord(b, 0);
        float t = 0.0f;
        if (hipGetLastError() == hipSuccess && hipEventSynchronize(b) == hipSuccess &&
            hipEventElapsedTime(&t, a, b) == hipSuccess && t > 0.0f) {
            const double per_access = mode == 0 ? 16.0 : 8.0;
            const double bytes = (double)grid * kThreads * kUnroll * iters * per_access;
            *ms = t;
            *bytes_per_s = bytes / (t * 1e-3);
            rc = 0;
        }
    }
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    (void)hipFree(out);
    return rc;
}
