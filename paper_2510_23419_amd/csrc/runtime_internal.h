// runtime_internal.h — host-side state of a libpbit context.
#pragma once

#include <hip/hip_runtime.h>

#include <array>
#include <map>
#include <mutex>
#include <vector>

#include "../../include/pbit.h"
#include "bq.h"
#include "host.h"

namespace pbit {

struct Problem {
    int kind = 0;
    int64_t N = 0;
    int amax = 0;  // largest possible |I|
    EaView ea{};
    BqView bq{};
    GraphView graph{};
    const uint32_t *tile_sites = nullptr;  // cube site list for the batched tiles (N < 65536), else null
    std::vector<int32_t> class_start;  // host copy behind graph.class_start
    std::vector<uint8_t> colour;       // colouring used (graph problems)
    std::vector<void *> allocs;
    int jobs = 0;  // serving jobs that still reference the problem
};

enum class Slot : int { Spins = 0, Table, E32, Stage, Aux, Snap, Hit, Count };

struct Scratch {
    void *ptr = nullptr;
    size_t bytes = 0;
};

struct ServeState;

// A fixed device region that an anneal carves its buffers from instead of
// allocating them (the no-allocation entry point).
struct Arena {
    void *base = nullptr;
    size_t bytes = 0;
    size_t used = 0;
};

}  // namespace pbit

struct pbit_ctx {
    std::mutex mu;
    int device = 0;
    uint32_t serial = 0;
    uint64_t budget = 0;
    uint64_t in_use = 0;
    bool poisoned = false;
    hipStream_t stream = nullptr;
    uint64_t next_handle = 0;
    std::map<uint64_t, pbit::Problem> problems;
    std::map<void *, size_t> sizes;
    std::array<pbit::Scratch, (int)pbit::Slot::Count> scratch{};
    std::vector<uint32_t> host_table;
    pbit::ServeState *serve = nullptr;
    // profiling: event pairs around sampled half-sweep launches
    int prof_every = 0;
    std::vector<hipEvent_t> prof_pool;
    size_t prof_used = 0;
    std::vector<int> prof_kind;      // kind of each pending pair
    std::vector<int> prof_launches;  // launches inside each pending pair
    int prof_open = -1;              // pool index of the pair whose end is not recorded yet
    double prof_ms[4] = {0, 0, 0, 0};       // by problem kind (PBIT_EA3D, PBIT_BICLIQUE, PBIT_GRAPH)
    int64_t prof_count[4] = {0, 0, 0, 0};
    // biclique kernel variant: forced (PBIT_BQ_VARIANT) or autotuned per shape
    pbit::BqVariant bq_forced = pbit::BqVariant::Auto;
    int bq_last_variant = 0;  // biclique half-sweep variant of the latest biclique anneal (0: none yet)
    int bq_bits_rt = 0;       // replicas per tile of the bit kernel (PBIT_BQ_BITS_RT: 64, 128, 256; 0 = by size)
    int bq_slab_rs = 0;       // replicas per slice of the LDS-resident kernel (PBIT_BQ_SLAB_RS: 16, 8; 0 = timed)
    bool ea_stream_forced = false;  // cubes always take the streaming stencil (PBIT_EA_STREAM=1)
    int ea_rows = 0;                // lattice rows per workgroup of the streaming stencil (PBIT_EA_ROWS; 0 = default)
    int ea_mfma = -1;  // matrix-core cube half-sweep: -1 timed against the stencil, 1 every cube, 0 none (PBIT_EA_MFMA)
    std::map<std::array<int, 4>, bool> ea_tuned;  // (Lx, Ly, Lz, replicas padded to 128) -> matrix cores faster
    // pbit_anneal_dev's sweep launches as one HIP graph (PBIT_GRAPH=1), kept for replay
    bool use_graph = false;
    bool tile_tune = true;  // batched tile sizes timed per shape (PBIT_TILE_TUNE=0: the fixed rule)
    void *graph_exec = nullptr;  // hipGraphExec_t
    uint64_t graph_key = 0;
    int64_t graph_captures = 0, graph_launches = 0;
    int ea_last_path = 0;           // cube path of the latest cube anneal: 1 stream, 2 LDS-resident (0: none)
    int graph_last_path = 0;        // graph path of the latest graph anneal: 1 per class, 2 LDS-resident (0: none)
    bool graph_slab = true;         // graphs that fit LDS run there (PBIT_GRAPH_SLAB=0: one launch per class)
    int graph_slab_rs = 0;          // its tile width when forced (PBIT_GRAPH_SLAB=4, 8 or 16; 0: by the rule)
    // (na_p, nb_p, Rp, LDS form possible) -> fastest kernel and its replica tile (bit kernel) or
    // slice (LDS-resident kernel)
    std::map<std::array<int, 4>, std::pair<pbit::BqVariant, int>> bq_tuned;
};

namespace pbit {

int device_fail(pbit_ctx *ctx, hipError_t e, const char *where);
int dev_alloc(pbit_ctx *ctx, size_t bytes, void **out);
void dev_free(pbit_ctx *ctx, void *p);
int scratch(pbit_ctx *ctx, Slot slot, size_t bytes, void **out);
Problem *find_problem(pbit_ctx *ctx, uint64_t handle);
int check_desc(const pbit_anneal_desc *d, const char *who);
void serve_shutdown(pbit_ctx *ctx);
int spins_in_range(const int8_t *s, size_t n);
hipError_t prof_begin(pbit_ctx *ctx, int kind, hipStream_t st);
hipError_t prof_count_launch(pbit_ctx *ctx, hipStream_t st);
hipError_t prof_close(pbit_ctx *ctx, hipStream_t st);
hipError_t prof_harvest(pbit_ctx *ctx);
void prof_release(pbit_ctx *ctx);
int run_device(pbit_ctx *ctx, const Problem &P, const pbit_anneal_desc *d, int8_t *d_spins, bool spins_in,
               int64_t *d_energies, hipStream_t st, Arena *arena);
size_t anneal_dev_bytes(const pbit_ctx *ctx, const Problem &P, const pbit_anneal_desc *d);
int noalloc_setup(int device);

}  // namespace pbit

// Entry of every context call: a context, its lock, not poisoned, its device current.
#define PBIT_ENTER(ctx)                                                                     \
    if (!(ctx)) return pbit::fail(PBIT_E_ARG, "%s: context is NULL", __func__);             \
    std::lock_guard<std::mutex> lock_((ctx)->mu);                                           \
    if ((ctx)->poisoned) return pbit::fail(PBIT_E_DEVICE, "%s: context is poisoned", __func__); \
    {                                                                                       \
        hipError_t se_ = hipSetDevice((ctx)->device);                                       \
        if (se_ != hipSuccess) return pbit::device_fail((ctx), se_, "hipSetDevice");        \
    }
