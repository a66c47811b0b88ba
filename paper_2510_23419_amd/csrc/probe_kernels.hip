// probe_kernels.hip — the ceilings the sweep kernels are measured against, as
// kernels of their own: Philox4x32-10 alone (the random words every update
// needs), a plain device copy (the memory roof the stencil's bytes move at),
// and a loop of int8 MFMAs (the matrix-core roof of the biclique fields).
// pbit_probe times them with HIP events on the context's stream.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "../../include/pbit.h"
#include "device.h"
#include "runtime_internal.h"

using namespace pbit;

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

constexpr int kProbeThreads = 256;

// Each thread draws `blocks` Philox blocks with the counter layout of the
// sweep (site, sweep, replica group, domain 0) and folds the words into one
// output word, so that no draw can be dropped.
__global__ __launch_bounds__(kProbeThreads) void k_probe_philox(uint32_t *__restrict__ out, int blocks, uint32_t k0,
                                                                 uint32_t k1)
{
    const uint32_t gid = blockIdx.x * kProbeThreads + threadIdx.x;
    uint32_t acc = 0u;
    for (int b = 0; b < blocks; ++b) {
        const Block4 x = philox(gid, (uint32_t)b, gid >> 6, kDomainSweep, k0, k1);
        acc ^= __builtin_amdgcn_bitop3_b32(x.w[0], x.w[1], x.w[2], 0x96) ^ x.w[3];
    }
    out[gid] = acc;
}

// One 16-byte element per thread, one thread per element (faster than a grid-stride
// loop over a fixed grid: 6.2 against 4.6 TB/s at 1 GiB).
__global__ __launch_bounds__(kProbeThreads) void k_probe_copy(const uint4 *__restrict__ src, uint4 *__restrict__ dst,
                                                               int64_t n16)
{
    const int64_t i = (int64_t)blockIdx.x * kProbeThreads + threadIdx.x;
    if (i < n16) dst[i] = src[i];
}

// Four independent accumulator chains of v_mfma_i32_32x32x32_i8 per wave,
// `iters` steps each; the operands stay in registers.
__global__ __launch_bounds__(kProbeThreads) void k_probe_mfma(int32_t *__restrict__ out, int iters, int seed)
{
    const int lane = threadIdx.x & 63;
    const v4i a = {lane + seed, lane ^ seed, lane * 3, seed};
    const v4i b = {seed, lane + 1, lane ^ 5, lane * seed};
    v16i c0 = {0}, c1 = {0}, c2 = {0}, c3 = {0};
    for (int k = 0; k < iters; ++k) {
        c0 = __builtin_amdgcn_mfma_i32_32x32x32_i8(a, b, c0, 0, 0, 0);
        c1 = __builtin_amdgcn_mfma_i32_32x32x32_i8(b, a, c1, 0, 0, 0);
        c2 = __builtin_amdgcn_mfma_i32_32x32x32_i8(a, a, c2, 0, 0, 0);
        c3 = __builtin_amdgcn_mfma_i32_32x32x32_i8(b, b, c3, 0, 0, 0);
    }
    int s = 0;
#pragma unroll
    for (int j = 0; j < 16; ++j) s += c0[j] ^ c1[j] ^ c2[j] ^ c3[j];
    out[blockIdx.x * kProbeThreads + threadIdx.x] = s;
}

}  // namespace

extern "C" int pbit_probe(pbit_ctx *ctx, int32_t probe, int64_t size, int32_t reps, double *ms_per_launch,
                          double *work_per_launch)
{
    try {
        PBIT_ENTER(ctx);
        if (!ms_per_launch || !work_per_launch || reps < 1 || size < 1)
            return fail(PBIT_E_ARG, "pbit_probe: bad arguments");
        hipDeviceProp_t prop;
        hipError_t e = hipGetDeviceProperties(&prop, ctx->device);
        if (e != hipSuccess) return device_fail(ctx, e, "hipGetDeviceProperties");
        const int cus = prop.multiProcessorCount;
        const hipStream_t st = ctx->stream;
        void *buf = nullptr;
        int rc;
        double work = 0.0;
        unsigned grid = 0;
        int64_t n16 = 0;
        int blocks = 0, iters = 0;
        if (probe == PBIT_PROBE_PHILOX) {
            // size: Philox blocks per thread; 8 workgroups of 256 threads per CU
            if (size > (1 << 24)) return fail(PBIT_E_ARG, "pbit_probe: at most 2^24 blocks per thread");
            blocks = (int)size;
            grid = (unsigned)(8 * cus);
            rc = scratch(ctx, Slot::Aux, sizeof(uint32_t) * grid * kProbeThreads, &buf);
            work = 4.0 * blocks * grid * kProbeThreads;  // words
        } else if (probe == PBIT_PROBE_COPY) {
            // size: bytes copied (two buffers of `size` bytes, rounded to 16); launches
            // alternate direction, so that each reads what the one before wrote, as the
            // half-sweeps of a sweep do
            if (size > ((int64_t)1 << 36)) return fail(PBIT_E_ARG, "pbit_probe: at most 64 GiB");
            n16 = (size + 15) / 16;
            grid = (unsigned)((n16 + kProbeThreads - 1) / kProbeThreads);
            rc = scratch(ctx, Slot::Aux, (size_t)(32 * n16), &buf);
            work = 32.0 * (double)n16;  // bytes read plus bytes written
        } else if (probe == PBIT_PROBE_MFMA) {
            // size: MFMA steps per chain; one workgroup of four waves per SIMD quad, two per CU
            if (size > (1 << 24)) return fail(PBIT_E_ARG, "pbit_probe: at most 2^24 steps");
            iters = (int)size;
            grid = (unsigned)(2 * cus);
            rc = scratch(ctx, Slot::Aux, sizeof(int32_t) * grid * kProbeThreads, &buf);
            work = 4.0 * 65536.0 * (double)iters * grid * (kProbeThreads / 64);  // int8 ops (2 per multiply-add)
        } else {
            return fail(PBIT_E_ARG, "pbit_probe: unknown probe %d", probe);
        }
        if (rc) return rc;
        int parity = 0;
        auto launch = [&]() {
            if (probe == PBIT_PROBE_PHILOX)
                hipLaunchKernelGGL(k_probe_philox, dim3(grid), dim3(kProbeThreads), 0, st, (uint32_t *)buf, blocks,
                                   0x12345678u, 0x9abcdef0u);
            else if (probe == PBIT_PROBE_COPY) {
                const uint4 *a = (const uint4 *)buf + (parity ? n16 : 0);
                uint4 *b = (uint4 *)buf + (parity ? 0 : n16);
                parity ^= 1;
                hipLaunchKernelGGL(k_probe_copy, dim3(grid), dim3(kProbeThreads), 0, st, a, b, n16);
            }
            else
                hipLaunchKernelGGL(k_probe_mfma, dim3(grid), dim3(kProbeThreads), 0, st, (int32_t *)buf, iters, 7);
            return hipGetLastError();
        };
        hipEvent_t e0, e1;
        e = hipEventCreate(&e0);
        if (e != hipSuccess) return device_fail(ctx, e, "hipEventCreate");
        e = hipEventCreate(&e1);
        if (e != hipSuccess) {
            (void)hipEventDestroy(e0);
            return device_fail(ctx, e, "hipEventCreate");
        }
        e = launch();  // warm-up
        if (e == hipSuccess) e = hipEventRecord(e0, st);
        for (int k = 0; k < reps && e == hipSuccess; ++k) e = launch();
        if (e == hipSuccess) e = hipEventRecord(e1, st);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        if (e != hipSuccess) return device_fail(ctx, e, "probe");
        *ms_per_launch = (double)ms / reps;
        *work_per_launch = work;
        return PBIT_OK;
    } catch (...) {
        return fail(PBIT_E_ARG, "pbit_probe: internal error");
    }
}
