// misc_kernels.hip — small fill / conversion kernels used around the sweep.
#include "internal.h"

namespace pbit {

namespace {

__global__ void k_fill_i32(int32_t *__restrict__ p, int64_t n, int32_t v)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_widen(const int32_t *__restrict__ s, int64_t *__restrict__ d, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) d[i] = s[i];
}

// hit = sweep if min_r E[r] <= target and no earlier sweep has hit (one workgroup).
__global__ __launch_bounds__(256) void k_check_target(const int32_t *__restrict__ E, int R, int64_t target,
                                                      int32_t sweep, int32_t *__restrict__ hit)
{
    __shared__ int32_t wmin[4];
    int32_t m = INT32_MAX;
    for (int r = threadIdx.x; r < R; r += 256) m = min(m, E[r]);
    for (int off = 32; off > 0; off >>= 1) m = min(m, __shfl_xor(m, off, 64));
    if ((threadIdx.x & 63) == 0) wmin[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        m = min(min(wmin[0], wmin[1]), min(wmin[2], wmin[3]));
        if ((int64_t)m <= target && *hit == INT32_MAX) *hit = sweep;
    }
}

}  // namespace

hipError_t check_target(const int32_t *E, int R, int64_t target, int32_t sweep, int32_t *hit, hipStream_t st)
{
    hipLaunchKernelGGL(k_check_target, dim3(1), dim3(256), 0, st, E, R, target, sweep, hit);
    return hipGetLastError();
}

hipError_t fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}

hipError_t widen_i32_i64(const int32_t *src, int64_t *dst, int64_t n, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_widen, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, src, dst, n);
    return hipGetLastError();
}

}  // namespace pbit
