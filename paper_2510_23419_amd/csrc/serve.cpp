// serve.cpp — job submission and polling (continuous batching of anneal jobs).
#include "runtime_internal.h"

using namespace pbit;

namespace pbit {
void serve_shutdown(pbit_ctx *) {}
}  // namespace pbit

extern "C" int pbit_submit(pbit_ctx *ctx, uint64_t, const pbit_anneal_desc *, uint64_t *)
{
    if (!ctx) return fail(PBIT_E_ARG, "pbit_submit: context is NULL");
    return fail(PBIT_E_UNSUPPORTED, "pbit_submit: serving is not built yet");
}

extern "C" int pbit_poll(pbit_ctx *ctx, uint64_t, pbit_result *)
{
    if (!ctx) return fail(PBIT_E_ARG, "pbit_poll: context is NULL");
    return fail(PBIT_E_HANDLE, "pbit_poll: unknown job");
}

extern "C" int pbit_progress(pbit_ctx *ctx)
{
    if (!ctx) return fail(PBIT_E_ARG, "pbit_progress: context is NULL");
    return PBIT_OK;
}
