// serve.cpp — batched anneals and the serving scheduler (continuous batching).
//
// Jobs are cut into replica tiles; a round advances every running job by one
// chunk of sweeps with one persistent kernel per tile kind (cube tiles, and
// biclique tiles of 64 or 32 replicas), each on its own stream so the kinds
// overlap on the device.  Between rounds the scheduler harvests energies
// (traces, targets), retires finished jobs, and admits queued ones when their
// device memory fits the context's budget.  A job's arithmetic and random
// counters do not depend on the round it runs in, so results are the same
// alone and in any mix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <atomic>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <new>
#include <thread>
#include <vector>

#include "batch.h"
#include "runtime_internal.h"
#include "serve_sched.h"

using namespace pbit;

namespace pbit {

int spins_in_range(const int8_t *s, size_t n);  // runtime.cpp

namespace {

constexpr int kMaxLdsTile = 160 * 1024 - 4096;
// tile kinds, one persistent launch and one stream each: cube tiles (4, 8 or 16
// replicas, one launch); 128-, 64- and 32-replica biclique tiles; general-graph
// tiles (4, 8 or 16 replicas, one launch); cube tiles whose rows need more than
// kEaLargeTileLds of LDS (one workgroup per CU, launched with more threads; apart
// from the small ones, whose launch then keeps several workgroups per CU)
constexpr int kKinds = 6;
constexpr int kGraphKind = 4;
constexpr int kCubeLargeKind = 5;
inline int kind_of_rs(int rs) { return rs == 128 ? 1 : (rs == 64 ? 2 : 3); }
constexpr double kItemOps = 1.5e11;  // multiply-adds of one biclique tile over its anneal
inline int rs_of_kind(int k) { return k == 1 ? 128 : (k == 2 ? 64 : 32); }

struct BJob : SchedJob {
    uint64_t id = 0;
    uint64_t problem = 0;
    Problem *P = nullptr;
    pbit_anneal_desc d{};
    std::vector<double> beta;
    std::vector<int8_t> init;
    std::vector<uint32_t> table;  // threshold rows built ahead of admission (batch calls), else empty
    int kind = 0, N = 0, R = 0, S = 0;
    int rs = 4, tiles = 0, width = 1, chunk = 1;
    int mode = kTileInt8;  // biclique tile operands: int8 rows (default) or spin bits
    // device memory (released when the job finishes)
    void *d_table = nullptr, *d_state = nullptr, *d_energy = nullptr;
    size_t bytes = 0;
    bool admitted = false, started = false;
    bool filled = false;  // batch API: result copied out and device memory released
    int s_done = 0, sweeps_done = 0;
    std::vector<int32_t> energy;  // latest per-replica energies
    std::vector<int64_t> etrace;  // [trace_len][R]
    int trace_len = 0, trace_cap = 0;
    pbit_result *user = nullptr;  // batch API: result filled at completion
};

}  // namespace

struct ServeState {
    SchedQueues<BJob> q;  // queue, running jobs, round in flight
    std::map<uint64_t, std::unique_ptr<BJob>> jobs;
    uint64_t next_id = 1;
    int max_queue = 4096, round_sweeps = 500;
    // one stream per tile kind
    hipStream_t st[kKinds] = {};
    hipEvent_t fork = nullptr, join[kKinds] = {};
    std::vector<BJob *> round_jobs;
    std::vector<int> round_end;
    // device work lists (grown on demand)
    void *d_ea_jobs = nullptr, *d_bq_jobs[3] = {}, *d_graph_jobs = nullptr;  // per tile kind
    void *d_items[kKinds] = {};
    size_t cap_ea_jobs = 0, cap_bq_jobs[3] = {}, cap_graph_jobs = 0, cap_items[kKinds] = {};
    int32_t *d_meta = nullptr;  // counters[kKinds], n_items[kKinds]
    bool lds_ready = false;
    // tile autotuner: (kind, shape, threshold width, replicas rounded to a power of two,
    // operand mode) -> replicas per tile; the rule picks when PBIT_TILE_TUNE=0 or a round
    // is in flight (the timing would share the device)
    std::map<std::array<int, 6>, int> tile_tuned;
    bool tune = true;
    int64_t tunings = 0;
};

static int grow(pbit_ctx *ctx, void **p, size_t *cap, size_t need)
{
    if (*cap >= need && *p) return PBIT_OK;
    if (*p) {
        hipError_t e = hipDeviceSynchronize();
        if (e != hipSuccess) return device_fail(ctx, e, "hipDeviceSynchronize");
        dev_free(ctx, *p);
        *p = nullptr;
        *cap = 0;
    }
    size_t want = std::max(need, (size_t)4096);
    int rc = dev_alloc(ctx, want, p);
    if (rc) return rc;
    *cap = want;
    return PBIT_OK;
}

static int serve_init(pbit_ctx *ctx)
{
    if (ctx->serve) return PBIT_OK;
    std::unique_ptr<ServeState> s(new (std::nothrow) ServeState());
    if (!s) return fail(PBIT_E_NOMEM, "serving state: host allocation failed");
    hipError_t e = hipSuccess;
    for (int k = 0; k < kKinds && e == hipSuccess; ++k) e = hipStreamCreateWithFlags(&s->st[k], hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&s->fork, hipEventDisableTiming);
    for (int k = 0; k < kKinds && e == hipSuccess; ++k) e = hipEventCreateWithFlags(&s->join[k], hipEventDisableTiming);
    if (e != hipSuccess) return device_fail(ctx, e, "serving streams");
    s->tune = ctx->tile_tune;
    void *meta = nullptr;
    int rc = dev_alloc(ctx, 64, &meta);
    if (rc) return rc;
    s->d_meta = (int32_t *)meta;
    ctx->serve = s.release();
    return PBIT_OK;
}

void serve_shutdown(pbit_ctx *ctx)
{
    ServeState *s = ctx->serve;
    if (!s) return;
    (void)hipDeviceSynchronize();
    for (auto &kv : s->jobs) {
        BJob *j = kv.second.get();
        dev_free(ctx, j->d_table);
        dev_free(ctx, j->d_state);
        dev_free(ctx, j->d_energy);
        if (j->P) j->P->jobs--;
    }
    dev_free(ctx, s->d_ea_jobs);
    dev_free(ctx, s->d_graph_jobs);
    for (int k = 0; k < 3; ++k) dev_free(ctx, s->d_bq_jobs[k]);
    for (int k = 0; k < kKinds; ++k) dev_free(ctx, s->d_items[k]);
    dev_free(ctx, s->d_meta);
    for (int k = 0; k < kKinds; ++k) {
        if (s->st[k]) (void)hipStreamDestroy(s->st[k]);
        if (s->join[k]) (void)hipEventDestroy(s->join[k]);
    }
    if (s->fork) (void)hipEventDestroy(s->fork);
    delete s;
    ctx->serve = nullptr;
}

// ---------------------------------------------------------------- job set-up

// Bytes of one biclique replica row in a tile: one byte per site, or one bit.
static int bq_row_bytes(const BJob &j)
{
    const int n = j.P->bq.na_p + j.P->bq.nb_p;
    return j.mode == kTileBits ? n / 8 : n;
}

// Operand mode of a context's biclique tiles: int8 rows unless the bit variant is
// forced.  Bit rows let 128 replicas share each coupling fragment at any
// side length, but on the bag's sides (n <= 1024) a tile's Philox draws and
// decisions cost about as much as its MFMAs, and the int8 rows' smaller tiles
// spread a job over more CUs: measured, int8 rows are the faster default there.
static int tile_mode(const pbit_ctx *ctx)
{
    if (ctx->bq_forced == BqVariant::Bits) return kTileBits;
    return kTileInt8;
}

static size_t tile_bytes(const BJob &j)
{
    return j.kind != PBIT_BICLIQUE ? (size_t)j.rs * j.N : (size_t)j.rs * bq_row_bytes(j);
}

static int tune_tile(pbit_ctx *ctx, ServeState &s, BJob &j, const std::vector<int> &cands, int *pick);

static int plan_job(pbit_ctx *ctx, ServeState &s, BJob &j)
{
    const Problem &P = *j.P;
    j.kind = P.kind;
    j.N = (int)P.N;
    j.R = j.d.n_replicas;
    j.S = j.d.n_sweeps;
    j.width = j.S > 0 ? table_width(j.beta.data(), j.S, P.amax) : 1;
    j.mode = tile_mode(ctx);
    std::vector<int> cands;  // tile sizes the job can take (the autotuner times them)
    if (j.width > kMaxTableWidth) return fail(PBIT_E_UNSUPPORTED, "threshold rows of %d entries are too wide", j.width);
    if (P.kind == PBIT_GRAPH) {
        // the widest tile (16, 8 or 4 replicas of every site) that the job fills and the LDS holds
        if (graph_tile_lds(P.N, 4) > (size_t)kMaxLdsTile)
            return fail(PBIT_E_UNSUPPORTED, "graph of %lld spins is too large for a batched tile", (long long)P.N);
        if (j.width > kGraphMaxDegree + 2)
            return fail(PBIT_E_UNSUPPORTED, "threshold rows of %d entries are too wide", j.width);
        j.rs = 4;
        for (int rs : {16, 8})
            if (j.R >= rs && graph_tile_lds(P.N, rs) <= (size_t)kMaxLdsTile) {
                j.rs = rs;
                break;
            }
        for (int rs : {16, 8, 4})
            if (rs <= std::max(j.R, 4) && graph_tile_lds(P.N, rs) <= (size_t)kMaxLdsTile) cands.push_back(rs);
    } else if (P.kind == PBIT_EA3D) {
        if (ea_tile_lds(P.N, 4) > (size_t)kMaxLdsTile || P.ea.Lx > 1024 || P.ea.Ly > 1024)
            return fail(PBIT_E_UNSUPPORTED, "cube of %lld sites is too large for a batched tile", (long long)P.N);
        // the widest tile (16, 8 or 4 replicas: a 16-, 8- or 4-byte row per site) that the
        // job fills and the LDS holds
        if (!P.tile_sites)
            return fail(PBIT_E_UNSUPPORTED, "cube of %lld sites has no site list", (long long)P.N);
        j.rs = 4;
        for (int rs : {16, 8})
            if (j.R >= rs && ea_tile_lds(P.N, rs) <= (size_t)kMaxLdsTile) {
                j.rs = rs;
                break;
            }
        for (int rs : {16, 8, 4})
            if (rs <= std::max(j.R, 4) && ea_tile_lds(P.N, rs) <= (size_t)kMaxLdsTile) cands.push_back(rs);
    } else {
        // the largest tile that the replicas fill, the LDS holds and whose whole anneal
        // stays below kItemOps multiply-adds: larger tiles stream fewer coupling bytes
        // per replica, but a tile is one workgroup for all of its sweeps, so a big job
        // is cut into more, smaller tiles that run side by side
        const int na_p = P.bq.na_p, nb_p = P.bq.nb_p;
        j.rs = 0;
        for (int rs : {128, 64, 32}) {
            if (rs == 128 && j.mode != kTileBits) continue;  // int8 rows: 64 and 32 replicas
            if (bq_tile_lds(rs, na_p, nb_p, j.width, j.mode) > (size_t)kMaxLdsTile) continue;
            j.rs = rs;  // the smallest that fits, if none passes the tests below
            const double item = 2.0 * na_p * nb_p * rs * std::max(j.S, 1);
            if ((j.R >= rs || rs == 32) && item <= kItemOps) break;
        }
        if (j.rs == 0)
            return fail(PBIT_E_UNSUPPORTED, "biclique %d x %d is too large for a batched tile", P.bq.na, P.bq.nb);
        for (int rs : {128, 64, 32})
            if ((rs != 128 || j.mode == kTileBits) && (rs == 32 || rs <= j.R) &&
                bq_tile_lds(rs, na_p, nb_p, j.width, j.mode) <= (size_t)kMaxLdsTile)
                cands.push_back(rs);
    }
    if (cands.size() > 1 && s.tune && j.S > 0) {
        int R2 = 1;
        while (R2 < j.R) R2 *= 2;
        const std::array<int, 6> key{P.kind, P.kind == PBIT_BICLIQUE ? P.bq.na_p : (int)P.N,
                                     P.kind == PBIT_BICLIQUE ? P.bq.nb_p : 0, j.width, R2, j.mode};
        auto it = s.tile_tuned.find(key);
        if (it != s.tile_tuned.end()) {
            j.rs = it->second;
        } else if (!s.q.in_flight) {
            int pick = j.rs;
            int rc = tune_tile(ctx, s, j, cands, &pick);
            if (rc) return rc;
            j.rs = pick;
            s.tile_tuned[key] = pick;
        }
    }
    j.tiles = (j.R + j.rs - 1) / j.rs;
    j.bytes = sizeof(uint32_t) * (size_t)std::max(j.S, 1) * j.width + (size_t)j.tiles * tile_bytes(j) +
              sizeof(int32_t) * (size_t)j.tiles * j.rs;
    const bool check = j.d.has_target || j.d.trace_every > 0;
    j.chunk = check ? (j.d.trace_every > 0 ? j.d.trace_every : PBIT_CHECK_SWEEPS) : std::max(j.S, 1);
    j.trace_cap = j.d.trace_every > 0 ? j.S / j.d.trace_every : 0;
    (void)ctx;
    return PBIT_OK;
}

// [R][N] host rows <-> tile layout
static void rows_to_tiles(const BJob &j, const int8_t *rows, std::vector<int8_t> &tiles_out)
{
    const Problem &P = *j.P;
    if (P.kind != PBIT_BICLIQUE) {  // cubes and graphs: [tile][site][replica in tile]
        tiles_out.assign((size_t)j.tiles * j.rs * j.N, 1);
        for (int r = 0; r < j.R; ++r)
            for (int i = 0; i < j.N; ++i)
                tiles_out[((size_t)(r / j.rs) * j.N + i) * j.rs + (r % j.rs)] = rows[(size_t)r * j.N + i];
    } else {
        // spin bits (set = -1, bit col % 8 of byte col / 8: the little-endian words the
        // kernel reads) or int8 spins
        const int Pw = bq_row_bytes(j);
        tiles_out.assign((size_t)j.tiles * j.rs * Pw, 0);
        for (int r = 0; r < j.R; ++r)
            for (int i = 0; i < j.N; ++i) {
                const int col = i < P.bq.na ? i : P.bq.na_p + (i - P.bq.na);
                const int8_t m = rows[(size_t)r * j.N + i] > 0 ? 1 : -1;
                const size_t row = (size_t)(r / j.rs) * j.rs + (r % j.rs);
                if (j.mode == kTileBits)
                    tiles_out[row * Pw + col / 8] |= (uint8_t)((m < 0 ? 1 : 0) << (col % 8));
                else
                    tiles_out[row * Pw + col] = m;
            }
    }
}

static void tiles_to_rows(const BJob &j, const int8_t *tl, int8_t *rows)
{
    const Problem &P = *j.P;
    if (P.kind != PBIT_BICLIQUE) {
        for (int r = 0; r < j.R; ++r)
            for (int i = 0; i < j.N; ++i)
                rows[(size_t)r * j.N + i] = tl[((size_t)(r / j.rs) * j.N + i) * j.rs + (r % j.rs)];
    } else {
        const int Pw = bq_row_bytes(j);
        for (int r = 0; r < j.R; ++r)
            for (int i = 0; i < j.N; ++i) {
                const int col = i < P.bq.na ? i : P.bq.na_p + (i - P.bq.na);
                const size_t row = (size_t)(r / j.rs) * j.rs + (r % j.rs);
                if (j.mode == kTileBits) {
                    rows[(size_t)r * j.N + i] = ((uint8_t)tl[row * Pw + col / 8] >> (col % 8)) & 1 ? -1 : 1;
                } else {
                    rows[(size_t)r * j.N + i] = tl[row * Pw + col];
                }
            }
    }
}

static int admit(pbit_ctx *ctx, BJob &j)
{
    int rc = dev_alloc(ctx, sizeof(uint32_t) * (size_t)std::max(j.S, 1) * j.width, &j.d_table);
    if (rc == PBIT_OK) rc = dev_alloc(ctx, (size_t)j.tiles * tile_bytes(j), &j.d_state);
    if (rc == PBIT_OK) rc = dev_alloc(ctx, sizeof(int32_t) * (size_t)j.tiles * j.rs, &j.d_energy);
    if (rc != PBIT_OK) {
        dev_free(ctx, j.d_table);
        dev_free(ctx, j.d_state);
        dev_free(ctx, j.d_energy);
        j.d_table = j.d_state = j.d_energy = nullptr;
        return rc;
    }
    std::vector<uint32_t> tab;
    if (j.table.size() == (size_t)std::max(j.S, 1) * j.width) {
        tab.swap(j.table);
    } else {
        tab.assign((size_t)std::max(j.S, 1) * j.width, 0u);
        if (j.S > 0) build_table(j.beta.data(), j.S, j.width, tab.data());
    }
    hipError_t e = hipMemcpy(j.d_table, tab.data(), sizeof(uint32_t) * tab.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess && !j.init.empty()) {
        std::vector<int8_t> tl;
        rows_to_tiles(j, j.init.data(), tl);
        e = hipMemcpy(j.d_state, tl.data(), tl.size(), hipMemcpyHostToDevice);
        j.started = true;
    }
    if (e != hipSuccess) return device_fail(ctx, e, "job upload");
    j.admitted = true;
    j.energy.assign(j.R, 0);
    return PBIT_OK;
}

// Threshold tables of a batch's jobs, built side by side on up to 16 host threads (one
// job per thread at a time) before admission, up to 1 GiB of them; admission builds the
// rest (and any a thread could not allocate).
static void prebuild_tables(const std::vector<BJob *> &js)
{
    std::vector<BJob *> todo;
    size_t bytes = 0;
    for (BJob *j : js) {
        const size_t b = sizeof(uint32_t) * (size_t)std::max(j->S, 1) * j->width;
        if (j->S <= 0 || bytes + b > ((size_t)1 << 30)) continue;
        bytes += b;
        todo.push_back(j);
    }
    std::atomic<size_t> next{0};
    auto work = [&]() {
        for (size_t q; (q = next++) < todo.size();) {
            BJob &j = *todo[q];
            try {
                j.table.assign((size_t)j.S * j.width, 0u);
                build_table(j.beta.data(), j.S, j.width, j.table.data(), 1);
            } catch (...) {
                std::vector<uint32_t>().swap(j.table);
            }
        }
    };
    const int nt = (int)std::min<size_t>({(size_t)16, (size_t)std::max(1u, std::thread::hardware_concurrency()),
                                          todo.size()});
    std::vector<std::thread> pool;
    for (int t = 1; t < nt; ++t) {
        try {
            pool.emplace_back(work);
        } catch (...) {
            break;
        }
    }
    work();
    for (std::thread &th : pool) th.join();
}

static void release(pbit_ctx *ctx, BJob &j)
{
    dev_free(ctx, j.d_table);
    dev_free(ctx, j.d_state);
    dev_free(ctx, j.d_energy);
    j.d_table = j.d_state = j.d_energy = nullptr;
    if (j.P) {
        j.P->jobs--;
        j.P = nullptr;
    }
}

// ---------------------------------------------------------------- rounds

static int launch_round(pbit_ctx *ctx, ServeState &s, const std::vector<BJob *> &running, bool &launched)
{
    launched = false;
    s.round_jobs.clear();
    s.round_end.clear();
    std::vector<EaJobDev> ea;
    std::vector<GraphJobDev> gr;
    std::vector<BqJobDev> bq[3];
    std::vector<WorkItem> items[kKinds];
    std::vector<double> cost[kKinds];
    size_t lds[kKinds] = {};
    for (BJob *j : running) {
        if (j->finished) continue;
        const int s0 = j->s_done;
        const int s1 = std::min(j->S, s0 + j->chunk);
        if (s1 <= s0) continue;
        s.round_jobs.push_back(j);
        s.round_end.push_back(s1);
        const Key key{(uint32_t)j->d.seed, (uint32_t)(j->d.seed >> 32)};
        if (j->kind == PBIT_EA3D) {
            const EaView &v = j->P->ea;
            EaJobDev jd{reinterpret_cast<const uint2 *>(j->P->tile_sites),
                        (const uint32_t *)j->d_table,
                        (int8_t *)j->d_state,
                        (int32_t *)j->d_energy,
                        v.Lx, v.Ly, v.Lz, j->width, j->rs, v.dense ? 1 : 0,
                        (uint32_t)j->d.sweep_offset, (uint32_t)j->d.replica_offset >> 2, key.k0, key.k1};
            const int idx = (int)ea.size();
            ea.push_back(jd);
            const int k = ea_tile_lds(j->N, j->rs) > kEaLargeTileLds ? kCubeLargeKind : 0;
            for (int t = 0; t < j->tiles; ++t) {
                items[k].push_back(WorkItem{idx, t, s0, s1, j->started ? 0 : 1, {0, 0, 0}});
                cost[k].push_back((double)(s1 - s0) * j->N * j->rs);
            }
            lds[k] = std::max(lds[k], ea_tile_lds(j->N, j->rs));
        } else if (j->kind == PBIT_GRAPH) {
            const GraphView &v = j->P->graph;
            GraphJobDev jd{reinterpret_cast<const int4 *>(v.site_meta), v.adj, v.class_start_dev, v.bi, v.bj, v.bJ,
                           v.h, (const uint32_t *)j->d_table, (int8_t *)j->d_state, (int32_t *)j->d_energy,
                           v.n, v.n_bonds, v.n_colours, j->width, j->rs,
                           (uint32_t)j->d.sweep_offset, (uint32_t)j->d.replica_offset >> 2, key.k0, key.k1};
            const int idx = (int)gr.size();
            gr.push_back(jd);
            const int k = kGraphKind;
            for (int t = 0; t < j->tiles; ++t) {
                items[k].push_back(WorkItem{idx, t, s0, s1, j->started ? 0 : 1, {0, 0, 0}});
                cost[k].push_back((double)(s1 - s0) * ((double)j->N + 2.0 * v.n_bonds) * j->rs);
            }
            lds[k] = std::max(lds[k], graph_tile_lds(j->N, j->rs));
        } else {
            const BqView &v = j->P->bq;
            const int k = kind_of_rs(j->rs);
            BqJobDev jd{v.J, v.JT, v.Jb, v.JTb, v.hA2, v.hB2, v.J2, v.JT2, v.hA, v.hB,
                        (const uint32_t *)j->d_table, (uint8_t *)j->d_state,
                        (int32_t *)j->d_energy, v.na, v.nb, v.na_p, v.nb_p, j->width,
                        (uint32_t)j->d.sweep_offset, (uint32_t)j->d.replica_offset >> 2, key.k0, key.k1};
            const int idx = (int)bq[k - 1].size();
            bq[k - 1].push_back(jd);
            for (int t = 0; t < j->tiles; ++t) {
                items[k].push_back(WorkItem{idx, t, s0, s1, j->started ? 0 : 1, {0, 0, 0}});
                cost[k].push_back((double)(s1 - s0) * (double)v.na_p * v.nb_p * j->rs);
            }
            lds[k] = std::max(lds[k], bq_tile_lds(j->rs, v.na_p, v.nb_p, j->width, j->mode));
        }
    }
    if (s.round_jobs.empty()) return PBIT_OK;

    // longest items first, so that the persistent workgroups finish together
    for (int k = 0; k < kKinds; ++k) {
        std::vector<size_t> ord(items[k].size());
        for (size_t q = 0; q < ord.size(); ++q) ord[q] = q;
        std::stable_sort(ord.begin(), ord.end(), [&](size_t a, size_t b) { return cost[k][a] > cost[k][b]; });
        std::vector<WorkItem> sorted(items[k].size());
        for (size_t q = 0; q < ord.size(); ++q) sorted[q] = items[k][ord[q]];
        items[k].swap(sorted);
    }
    int rc = grow(ctx, &s.d_ea_jobs, &s.cap_ea_jobs, sizeof(EaJobDev) * std::max<size_t>(ea.size(), 1));
    if (rc == PBIT_OK)
        rc = grow(ctx, &s.d_graph_jobs, &s.cap_graph_jobs, sizeof(GraphJobDev) * std::max<size_t>(gr.size(), 1));
    for (int k = 0; k < 3 && rc == PBIT_OK; ++k)
        rc = grow(ctx, &s.d_bq_jobs[k], &s.cap_bq_jobs[k], sizeof(BqJobDev) * std::max<size_t>(bq[k].size(), 1));
    for (int k = 0; k < kKinds && rc == PBIT_OK; ++k)
        rc = grow(ctx, &s.d_items[k], &s.cap_items[k], sizeof(WorkItem) * std::max<size_t>(items[k].size(), 1));
    if (rc) return rc;
    if (!s.lds_ready) {
        hipError_t e = tiles_set_lds_limit();
        if (e != hipSuccess) return device_fail(ctx, e, "tile LDS limit");
        s.lds_ready = true;
    }
    int32_t meta[2 * kKinds] = {0};
    for (int k = 0; k < kKinds; ++k) meta[kKinds + k] = (int32_t)items[k].size();
    hipError_t e = hipMemcpy(s.d_meta, meta, sizeof meta, hipMemcpyHostToDevice);
    if (e == hipSuccess && !ea.empty())
        e = hipMemcpy(s.d_ea_jobs, ea.data(), sizeof(EaJobDev) * ea.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess && !gr.empty())
        e = hipMemcpy(s.d_graph_jobs, gr.data(), sizeof(GraphJobDev) * gr.size(), hipMemcpyHostToDevice);
    for (int k = 0; k < 3 && e == hipSuccess; ++k)
        if (!bq[k].empty()) e = hipMemcpy(s.d_bq_jobs[k], bq[k].data(), sizeof(BqJobDev) * bq[k].size(), hipMemcpyHostToDevice);
    for (int k = 0; k < kKinds && e == hipSuccess; ++k)
        if (!items[k].empty()) e = hipMemcpy(s.d_items[k], items[k].data(), sizeof(WorkItem) * items[k].size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) return device_fail(ctx, e, "round upload");

    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, ctx->device);
    if (e != hipSuccess) return device_fail(ctx, e, "hipGetDeviceProperties");
    const int cus = prop.multiProcessorCount;
    for (int k = 0; k < kKinds; ++k) {
        if (items[k].empty()) continue;
        const size_t per_cu_lds = std::max<size_t>(lds[k] + 2048, 1);
        const int per_cu = std::max(1, std::min(4, (int)((160 * 1024) / per_cu_lds)));
        const int grid = std::max(1, std::min((int)items[k].size(), cus * per_cu));
        if (k == 0 || k == kCubeLargeKind)
            e = ea_tiles((const EaJobDev *)s.d_ea_jobs, (const WorkItem *)s.d_items[k], s.d_meta + kKinds + k,
                         s.d_meta + k, grid, lds[k], s.st[k]);
        else if (k == kGraphKind)
            e = graph_tiles((const GraphJobDev *)s.d_graph_jobs, (const WorkItem *)s.d_items[k], s.d_meta + kKinds + k,
                            s.d_meta + k, grid, lds[k], s.st[k]);
        else
            e = bq_tiles((const BqJobDev *)s.d_bq_jobs[k - 1], (const WorkItem *)s.d_items[k], s.d_meta + kKinds + k,
                         s.d_meta + k, rs_of_kind(k), tile_mode(ctx), grid, lds[k], s.st[k]);
        if (e == hipSuccess) e = hipEventRecord(s.join[k], s.st[k]);
        if (e != hipSuccess) return device_fail(ctx, e, "tile kernel launch");
    }
    launched = true;
    return PBIT_OK;
}

// The tile autotuner: one tile of each candidate size runs a couple of the job's
// sweeps alone on the device (from a random start, on scratch memory), timed with
// HIP events.  The job's cost with that size is its number of tiles times the tile
// time over the number of tiles the device holds at once (the device time the job
// takes from a full batch), and the cheapest size is kept; a smaller size must be
// at least 2 % cheaper, as larger tiles stream fewer bytes per replica.
static int tune_tile(pbit_ctx *ctx, ServeState &s, BJob &j, const std::vector<int> &cands, int *pick)
{
    const Problem &P = *j.P;
    constexpr int kSweeps = 2;
    if (!s.lds_ready) {
        hipError_t e = tiles_set_lds_limit();
        if (e != hipSuccess) return device_fail(ctx, e, "tile LDS limit");
        s.lds_ready = true;
    }
    std::vector<uint32_t> tab((size_t)kSweeps * j.width);
    std::vector<double> beta(kSweeps, j.beta[0]);
    for (int k = 1; k < kSweeps && k < j.S; ++k) beta[k] = j.beta[k];
    build_table(beta.data(), kSweeps, j.width, tab.data(), 1);
    hipDeviceProp_t prop;
    hipError_t e = hipGetDeviceProperties(&prop, ctx->device);
    if (e != hipSuccess) return device_fail(ctx, e, "hipGetDeviceProperties");
    const int cus = prop.multiProcessorCount;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e != hipSuccess) return device_fail(ctx, e, "hipEventCreate (tile tuning)");
    const hipStream_t st = ctx->stream;
    double best_t = 0.0;
    int rc = PBIT_OK;
    for (int rs : cands) {
        BJob t = j;  // the job's shape with this tile size
        t.rs = rs;
        const size_t state = tile_bytes(t);
        const size_t lds = P.kind == PBIT_EA3D ? ea_tile_lds(P.N, rs)
                           : P.kind == PBIT_GRAPH ? graph_tile_lds(P.N, rs)
                                                  : bq_tile_lds(rs, P.bq.na_p, P.bq.nb_p, j.width, j.mode);
        // scratch: job descriptor, item, counter and item count, energies, table, state
        const size_t off_item = 512, off_meta = off_item + 64, off_en = off_meta + 64,
                     off_tab = off_en + ((sizeof(int32_t) * rs + 255) & ~(size_t)255),
                     off_state = off_tab + ((sizeof(uint32_t) * tab.size() + 255) & ~(size_t)255);
        void *buf = nullptr;
        rc = scratch(ctx, Slot::Stage, off_state + state, &buf);
        if (rc) break;
        uint8_t *b = (uint8_t *)buf;
        const WorkItem item{0, 0, 0, kSweeps, 1, {0, 0, 0}};
        const int32_t meta[2] = {0, 1};
        e = hipMemcpy(b + off_tab, tab.data(), sizeof(uint32_t) * tab.size(), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(b + off_item, &item, sizeof item, hipMemcpyHostToDevice);
        if (e == hipSuccess) {
            if (P.kind == PBIT_EA3D) {
                const EaView &v = P.ea;
                const EaJobDev jd{reinterpret_cast<const uint2 *>(P.tile_sites), (const uint32_t *)(b + off_tab),
                                  (int8_t *)(b + off_state), (int32_t *)(b + off_en), v.Lx, v.Ly, v.Lz, j.width, rs,
                                  v.dense ? 1 : 0, 0u, 0u, 0u, 0u};
                e = hipMemcpy(b, &jd, sizeof jd, hipMemcpyHostToDevice);
            } else if (P.kind == PBIT_GRAPH) {
                const GraphView &v = P.graph;
                const GraphJobDev jd{reinterpret_cast<const int4 *>(v.site_meta), v.adj, v.class_start_dev, v.bi,
                                     v.bj, v.bJ, v.h, (const uint32_t *)(b + off_tab), (int8_t *)(b + off_state),
                                     (int32_t *)(b + off_en), v.n, v.n_bonds, v.n_colours, j.width, rs,
                                     0u, 0u, 0u, 0u};
                e = hipMemcpy(b, &jd, sizeof jd, hipMemcpyHostToDevice);
            } else {
                const BqView &v = P.bq;
                const BqJobDev jd{v.J, v.JT, v.Jb, v.JTb, v.hA2, v.hB2, v.J2, v.JT2, v.hA, v.hB,
                                  (const uint32_t *)(b + off_tab), (uint8_t *)(b + off_state),
                                  (int32_t *)(b + off_en), v.na, v.nb, v.na_p, v.nb_p, j.width, 0u, 0u, 0u, 0u};
                e = hipMemcpy(b, &jd, sizeof jd, hipMemcpyHostToDevice);
            }
        }
        float ms = 0.f;
        for (int rep = 0; rep < 2 && e == hipSuccess; ++rep) {  // the first run warms up
            e = hipMemcpyAsync(b + off_meta, meta, sizeof meta, hipMemcpyHostToDevice, st);
            if (e == hipSuccess) e = hipEventRecord(e0, st);
            if (e == hipSuccess) {
                const WorkItem *it = (const WorkItem *)(b + off_item);
                int32_t *ctr = (int32_t *)(b + off_meta);
                if (P.kind == PBIT_EA3D)
                    e = ea_tiles((const EaJobDev *)b, it, ctr + 1, ctr, 1, lds, st);
                else if (P.kind == PBIT_GRAPH)
                    e = graph_tiles((const GraphJobDev *)b, it, ctr + 1, ctr, 1, lds, st);
                else
                    e = bq_tiles((const BqJobDev *)b, it, ctr + 1, ctr, rs, j.mode, 1, lds, st);
            }
            if (e == hipSuccess) e = hipEventRecord(e1, st);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        }
        if (e != hipSuccess) {
            rc = device_fail(ctx, e, "tile tuning");
            break;
        }
        // device time the job's tiles take: tiles x tile time over the tiles the device holds at once
        const int per_cu = std::max(1, std::min(4, (int)((160 * 1024) / (lds + 2048))));
        const int slots = cus * per_cu, tiles = (j.R + rs - 1) / rs;
        const double est = (double)tiles * ms / slots;
        if (rs == cands[0] || est < best_t * 0.98) {
            best_t = est;
            *pick = rs;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc == PBIT_OK) ++s.tunings;
    return rc;
}

static bool round_done(ServeState &s)
{
    for (int k = 0; k < kKinds; ++k)
        if (hipEventQuery(s.join[k]) == hipErrorNotReady) return false;
    return true;
}

static int harvest(pbit_ctx *ctx, ServeState &s)
{
    hipError_t e = hipSuccess;
    for (int k = 0; k < kKinds && e == hipSuccess; ++k) e = hipStreamSynchronize(s.st[k]);
    if (e != hipSuccess) return device_fail(ctx, e, "round");
    std::vector<int32_t> tile_e;
    for (size_t q = 0; q < s.round_jobs.size(); ++q) {
        BJob &j = *s.round_jobs[q];
        j.s_done = s.round_end[q];
        j.started = true;
        tile_e.resize((size_t)j.tiles * j.rs);
        e = hipMemcpy(tile_e.data(), j.d_energy, sizeof(int32_t) * tile_e.size(), hipMemcpyDeviceToHost);
        if (e != hipSuccess) return device_fail(ctx, e, "energy readback");
        for (int r = 0; r < j.R; ++r) j.energy[r] = tile_e[r];
        if (j.d.trace_every > 0 && j.s_done % j.d.trace_every == 0 && j.trace_len < j.trace_cap) {
            for (int r = 0; r < j.R; ++r) j.etrace.push_back(j.energy[r]);
            ++j.trace_len;
        }
        const bool hit = j.d.has_target && *std::min_element(j.energy.begin(), j.energy.end()) <= j.d.target_energy;
        if (hit || j.s_done >= j.S) {
            // the job's device state stays until it is polled (spins are read back only if asked for)
            j.finished = true;
            j.sweeps_done = j.s_done;
        }
    }
    return PBIT_OK;
}

// The device side of a scheduling step (see serve_sched.h).
struct ServeDevice {
    pbit_ctx *ctx;
    ServeState &s;
    bool round_done() { return pbit::round_done(s); }
    int harvest() { return pbit::harvest(ctx, s); }
    int admit(BJob *j)
    {
        if (ctx->budget && ctx->in_use + j->bytes > ctx->budget)
            return fail(PBIT_E_NOMEM, "job %llu needs %llu bytes; %llu of the %llu-byte budget are in use",
                        (unsigned long long)j->id, (unsigned long long)j->bytes, (unsigned long long)ctx->in_use,
                        (unsigned long long)ctx->budget);
        return pbit::admit(ctx, *j);
    }
    void drop(BJob *j) { release(ctx, *j); }
    int launch_round(const std::vector<BJob *> &running, bool &launched)
    {
        return pbit::launch_round(ctx, s, running, launched);
    }
};

// One scheduling step.  With wait = true it blocks until the round it launched
// (or the one in flight) has been harvested.
static int step(pbit_ctx *ctx, ServeState &s, bool wait)
{
    ServeDevice dev{ctx, s};
    return sched_step(s.q, dev, wait);
}

static int new_job(pbit_ctx *ctx, ServeState &s, uint64_t problem, const pbit_anneal_desc *desc, BJob **out)
{
    int rc = check_desc(desc, "pbit_submit");
    if (rc) return rc;
    Problem *P = find_problem(ctx, problem);
    if (!P) return fail(PBIT_E_HANDLE, "pbit_submit: unknown problem handle");
    if (desc->init_spins && !spins_in_range(desc->init_spins, (size_t)desc->n_replicas * P->N))
        return fail(PBIT_E_RANGE, "pbit_submit: init_spins must be +-1");
    if (desc->n_sweeps < 1) return fail(PBIT_E_ARG, "pbit_submit: a job needs at least one sweep");
    std::unique_ptr<BJob> j(new (std::nothrow) BJob());
    if (!j) return fail(PBIT_E_NOMEM, "pbit_submit: host allocation failed");
    j->d = *desc;
    j->beta.assign(desc->beta, desc->beta + desc->n_sweeps);
    j->d.beta = j->beta.data();
    if (desc->init_spins) j->init.assign(desc->init_spins, desc->init_spins + (size_t)desc->n_replicas * P->N);
    j->d.init_spins = nullptr;
    j->P = P;
    j->problem = problem;
    rc = plan_job(ctx, s, *j);
    if (rc) return rc;
    if (ctx->budget && j->bytes + 65536 > ctx->budget)
        return fail(PBIT_E_NOMEM, "job needs %llu bytes of device memory, more than the budget",
                    (unsigned long long)j->bytes);
    j->id = ((uint64_t)ctx->serial << 40) | (s.next_id++);
    P->jobs++;
    s.q.queue.push_back(j.get());
    *out = j.get();
    s.jobs[j->id] = std::move(j);
    return PBIT_OK;
}

// Copy a finished job's results out and release its device memory.
static int fill_result(pbit_ctx *ctx, BJob &j, pbit_result *res)
{
    if (res && res->spins && j.d_state) {
        std::vector<int8_t> tl((size_t)j.tiles * tile_bytes(j));
        hipError_t e = hipMemcpy(tl.data(), j.d_state, tl.size(), hipMemcpyDeviceToHost);
        if (e != hipSuccess) return device_fail(ctx, e, "spin readback");
        tiles_to_rows(j, tl.data(), res->spins);
    }
    release(ctx, j);
    if (!res) return PBIT_OK;
    int best = 0;
    for (int r = 0; r < j.R; ++r) {
        if (res->energies) res->energies[r] = j.energy[r];
        if (j.energy[r] < j.energy[best]) best = r;
    }
    res->best_energy = j.energy[best];
    res->best_replica = best;
    res->sweeps_done = j.sweeps_done;
    const int n = std::min(j.trace_len, std::max(res->trace_cap, 0));
    if (res->energy_trace)
        for (int k = 0; k < n; ++k)
            for (int r = 0; r < j.R; ++r) res->energy_trace[(size_t)k * j.R + r] = j.etrace[(size_t)k * j.R + r];
    res->trace_len = res->energy_trace ? n : 0;
    return PBIT_OK;
}

// Take a failing batch call's jobs out of the scheduler: finish the round in
// flight (it may use their memory), then drop them from the queue and the running
// list and release their device memory and problem references.  Their result
// structs are not touched.
static void withdraw(pbit_ctx *ctx, ServeState &s, const std::vector<BJob *> &mine)
{
    if (s.q.in_flight) {
        if (harvest(ctx, s) != PBIT_OK)
            for (int k = 0; k < kKinds; ++k) (void)hipStreamSynchronize(s.st[k]);
        s.q.in_flight = false;
        s.q.running.erase(std::remove_if(s.q.running.begin(), s.q.running.end(), [](BJob *j) { return j->finished; }),
                          s.q.running.end());
    }
    for (BJob *m : mine) {
        s.q.queue.erase(std::remove(s.q.queue.begin(), s.q.queue.end(), m), s.q.queue.end());
        s.q.running.erase(std::remove(s.q.running.begin(), s.q.running.end(), m), s.q.running.end());
        release(ctx, *m);
    }
}

}  // namespace pbit

#define PBIT_SERVE_ENTER(ctx)                                                                \
    if (!(ctx)) return fail(PBIT_E_ARG, "%s: context is NULL", __func__);                    \
    std::lock_guard<std::mutex> lock_((ctx)->mu);                                            \
    if ((ctx)->poisoned) return fail(PBIT_E_DEVICE, "%s: context is poisoned", __func__);    \
    {                                                                                        \
        hipError_t se_ = hipSetDevice((ctx)->device);                                        \
        if (se_ != hipSuccess) return device_fail((ctx), se_, "hipSetDevice");               \
    }                                                                                        \
    {                                                                                        \
        int ir_ = serve_init(ctx);                                                           \
        if (ir_) return ir_;                                                                 \
    }

extern "C" int pbit_submit(pbit_ctx *ctx, uint64_t problem, const pbit_anneal_desc *desc, uint64_t *job_out)
{
    try {
        PBIT_SERVE_ENTER(ctx);
        if (!job_out) return fail(PBIT_E_ARG, "pbit_submit: job_out is NULL");
        ServeState &s = *ctx->serve;
        if ((int)s.q.queue.size() >= s.max_queue)
            return fail(PBIT_E_BUSY, "pbit_submit: queue full (%d jobs)", s.max_queue);
        BJob *j = nullptr;
        int rc = new_job(ctx, s, problem, desc, &j);
        if (rc) return rc;
        // jobs without checks advance round_sweeps at a time, so that jobs arriving
        // later join the running ones at the next round
        if (!j->d.has_target && j->d.trace_every == 0) j->chunk = std::min(j->chunk, s.round_sweeps);
        *job_out = j->id;
        return step(ctx, s, false);
    } catch (const std::bad_alloc &) {
        return fail(PBIT_E_NOMEM, "pbit_submit: host allocation failed");
    } catch (...) {
        return fail(PBIT_E_ARG, "pbit_submit: internal error");
    }
}

extern "C" int pbit_poll(pbit_ctx *ctx, uint64_t job, pbit_result *result)
{
    try {
        PBIT_SERVE_ENTER(ctx);
        ServeState &s = *ctx->serve;
        auto it = s.jobs.find(job);
        if (it == s.jobs.end()) return fail(PBIT_E_HANDLE, "pbit_poll: unknown job");
        int rc = step(ctx, s, false);
        if (rc) return rc;
        BJob &j = *it->second;
        if (!j.finished) return PBIT_PENDING;
        if (j.status != PBIT_OK) {
            const int st = j.status;
            const unsigned long long bytes = (unsigned long long)j.bytes;
            s.jobs.erase(it);
            return fail(st, "pbit_poll: the job (%llu bytes of device memory) could not be admitted while no "
                        "other job ran", bytes);
        }
        rc = fill_result(ctx, j, result);
        s.jobs.erase(it);
        return rc;
    } catch (...) {
        return fail(PBIT_E_ARG, "pbit_poll: internal error");
    }
}

extern "C" int pbit_progress(pbit_ctx *ctx)
{
    try {
        PBIT_SERVE_ENTER(ctx);
        return step(ctx, *ctx->serve, false);
    } catch (...) {
        return fail(PBIT_E_ARG, "pbit_progress: internal error");
    }
}

extern "C" int pbit_serve_config(pbit_ctx *ctx, int32_t max_queue, int32_t max_running, int32_t round_sweeps)
{
    PBIT_SERVE_ENTER(ctx);
    if (max_queue < 0 || max_running < 0 || round_sweeps < 0) return fail(PBIT_E_ARG, "pbit_serve_config: negative limit");
    ServeState &s = *ctx->serve;
    if (max_queue) s.max_queue = max_queue;
    if (max_running) s.q.max_running = max_running;
    if (round_sweeps) s.round_sweeps = round_sweeps;
    return PBIT_OK;
}

extern "C" int pbit_profile_tiles(pbit_ctx *ctx, int64_t *tunings, int32_t *shapes)
{
    PBIT_SERVE_ENTER(ctx);
    if (tunings) *tunings = ctx->serve->tunings;
    if (shapes) *shapes = (int32_t)ctx->serve->tile_tuned.size();
    return PBIT_OK;
}

extern "C" int pbit_anneal_batch(pbit_ctx *ctx, const pbit_batch_job *jobs, int32_t n_jobs)
{
    try {
        PBIT_SERVE_ENTER(ctx);
        if (n_jobs < 0 || (n_jobs > 0 && !jobs)) return fail(PBIT_E_ARG, "pbit_anneal_batch: bad job list");
        ServeState &s = *ctx->serve;
        std::vector<BJob *> mine;
        for (int k = 0; k < n_jobs; ++k) {
            if (!jobs[k].result) return fail(PBIT_E_ARG, "pbit_anneal_batch: job %d has no result", k);
            if (jobs[k].result->spin_trace) return fail(PBIT_E_ARG, "pbit_anneal_batch: spin traces are not supported");
        }
        for (int k = 0; k < n_jobs; ++k) {
            BJob *j = nullptr;
            int rc = new_job(ctx, s, jobs[k].problem, jobs[k].desc, &j);
            if (rc) {
                // withdraw the jobs queued by this call
                for (BJob *m : mine) {
                    s.q.queue.erase(std::remove(s.q.queue.begin(), s.q.queue.end(), m), s.q.queue.end());
                    if (m->P) m->P->jobs--;
                    s.jobs.erase(m->id);
                }
                return rc;
            }
            j->user = jobs[k].result;
            mine.push_back(j);
        }
        prebuild_tables(mine);
        int frc = PBIT_OK;
        for (;;) {
            // copy finished jobs out at once: their device memory then serves the jobs
            // still queued
            bool all = true;
            for (BJob *m : mine) {
                if (m->finished && !m->filled) {
                    m->filled = true;
                    const int rc = m->status != PBIT_OK ? m->status : fill_result(ctx, *m, m->user);
                    if (rc && frc == PBIT_OK) {
                        frc = rc;
                        if (m->status != PBIT_OK)
                            fail(rc, "pbit_anneal_batch: job %d needs %llu bytes of device memory and could not "
                                 "be admitted while no other job ran", (int)(std::find(mine.begin(), mine.end(), m) -
                                                                             mine.begin()),
                                 (unsigned long long)m->bytes);
                    }
                }
                all = all && m->finished;
            }
            if (all || frc != PBIT_OK) break;
            frc = step(ctx, s, true);
        }
        if (frc != PBIT_OK) withdraw(ctx, s, mine);
        for (BJob *m : mine) s.jobs.erase(m->id);
        return frc;
    } catch (const std::bad_alloc &) {
        return fail(PBIT_E_NOMEM, "pbit_anneal_batch: host allocation failed");
    } catch (...) {
        return fail(PBIT_E_ARG, "pbit_anneal_batch: internal error");
    }
}
