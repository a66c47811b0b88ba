// noalloc.cpp — the anneal entry point that allocates no device memory.
//
// pbit_anneal_dev needs device buffers beyond the caller's spins and energies:
// the kernels' own spin layout, a bit copy of biclique spins, per-replica
// energy accumulators and the threshold table.  It takes them from the
// context's scratch slots, which grow with hipMalloc.  Callers that cannot
// allocate get the same anneal with those buffers carved from one fixed array
// in device memory, `scratch`, of PBIT_NOALLOC_SCRATCH_BYTES.  Each GPU the library
// runs on holds its own copy of the array (at its own address) until the
// process ends.
#include <hip/hip_runtime.h>

#include <mutex>
#include <new>

#include "../../include/pbit.h"
#include "runtime_internal.h"

using namespace pbit;

// The array.  Host code names it only to look up its device address (as
// ::scratch: inside namespace pbit the name would find the scratch-slot function).
static __device__ __align__(256) uint8_t scratch[PBIT_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;

// Device address of `scratch` on each device (null until looked up), and a lock
// per device: calls on one device share its array, so they run one at a time.
std::mutex g_lookup_mu;
void *g_scratch_ptr[kMaxDevices] = {};
std::mutex g_device_mu[kMaxDevices];

}  // namespace

namespace pbit {

// Look up the device address of `scratch` on `device`, which must be current.
// The name of the array is only a host-side handle; kernels and copies get
// this address.
int noalloc_setup(int device)
{
    if (device < 0 || device >= kMaxDevices) return fail(PBIT_E_ARG, "device %d beyond %d", device, kMaxDevices);
    std::lock_guard<std::mutex> lk(g_lookup_mu);
    if (g_scratch_ptr[device]) return PBIT_OK;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(::scratch));
    if (e != hipSuccess || !p)
        return fail(PBIT_E_DEVICE, "hipGetSymbolAddress of the static scratch on device %d failed (%s)", device,
                    hipGetErrorString(e));
    g_scratch_ptr[device] = p;
    return PBIT_OK;
}

}  // namespace pbit

extern "C" int pbit_anneal_dev_noalloc(pbit_ctx *ctx, uint64_t problem, const pbit_anneal_desc *desc, void *d_spins,
                                       int32_t spins_in, void *d_energies, void *hip_stream)
{
    try {
        PBIT_ENTER(ctx);
        int rc = check_desc(desc, "pbit_anneal_dev_noalloc");
        if (rc) return rc;
        if (!d_spins) return fail(PBIT_E_ARG, "pbit_anneal_dev_noalloc: d_spins is NULL");
        if (desc->init_spins)
            return fail(PBIT_E_ARG, "pbit_anneal_dev_noalloc: pass initial spins in d_spins (spins_in)");
        if (desc->trace_every || desc->has_target)
            return fail(PBIT_E_ARG, "pbit_anneal_dev_noalloc: traces and targets need pbit_anneal");
        Problem *P = find_problem(ctx, problem);
        if (!P) return fail(PBIT_E_HANDLE, "pbit_anneal_dev_noalloc: unknown problem handle");
        const size_t need = anneal_dev_bytes(ctx, *P, desc);
        if (need > (size_t)PBIT_NOALLOC_SCRATCH_BYTES)
            return fail(PBIT_E_UNSUPPORTED,
                        "pbit_anneal_dev_noalloc: %lld spins x %d replicas over %d sweeps need %llu bytes of scratch, "
                        "more than the %llu of the static array (use pbit_anneal_dev)",
                        (long long)P->N, desc->n_replicas, desc->n_sweeps, (unsigned long long)need,
                        (unsigned long long)PBIT_NOALLOC_SCRATCH_BYTES);
        rc = noalloc_setup(ctx->device);  // normally done by pbit_create already
        if (rc) return rc;
        std::lock_guard<std::mutex> dev_lock(g_device_mu[ctx->device]);
        Arena arena;
        arena.base = g_scratch_ptr[ctx->device];
        arena.bytes = (size_t)PBIT_NOALLOC_SCRATCH_BYTES;
        // no timing windows (their events would be created here)
        const int prof = ctx->prof_every;
        ctx->prof_every = 0;
        hipStream_t st = hip_stream ? (hipStream_t)hip_stream : ctx->stream;
        rc = run_device(ctx, *P, desc, (int8_t *)d_spins, spins_in != 0, (int64_t *)d_energies, st, &arena);
        ctx->prof_every = prof;
        return rc;
    } catch (const std::bad_alloc &) {
        return fail(PBIT_E_NOMEM, "pbit_anneal_dev_noalloc: host allocation failed");
    } catch (...) {
        return fail(PBIT_E_ARG, "pbit_anneal_dev_noalloc: internal error");
    }
}
