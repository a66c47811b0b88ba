// runtime.cpp — host side of libpbit: contexts, problem upload and validation,
// the FP64 threshold table, device-memory budget, and the anneal driver that
// enqueues the HIP kernels.  Every entry point is extern "C", returns a status
// code and never lets an exception cross the boundary.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "../../include/pbit.h"
#include "batch.h"
#include "internal.h"
#include "runtime_internal.h"

using namespace pbit;

// ---------------------------------------------------------------- errors

namespace pbit {

int device_fail(pbit_ctx *ctx, hipError_t e, const char *where)
{
    ctx->poisoned = true;
    return fail(PBIT_E_DEVICE, "%s: HIP error %d (%s); context poisoned", where, (int)e, hipGetErrorString(e));
}

}  // namespace pbit

// ---------------------------------------------------------------- device memory

namespace pbit {

static std::atomic<uint32_t> g_ctx_serial{1};

int dev_alloc(pbit_ctx *ctx, size_t bytes, void **out)
{
    *out = nullptr;
    if (bytes == 0) return PBIT_OK;
    if (ctx->budget && ctx->in_use + bytes > ctx->budget)
        return fail(PBIT_E_NOMEM, "device budget exhausted: %llu in use + %llu requested > %llu",
                    (unsigned long long)ctx->in_use, (unsigned long long)bytes, (unsigned long long)ctx->budget);
    hipError_t e = hipMalloc(out, bytes);
    if (e == hipErrorOutOfMemory) {
        (void)hipGetLastError();
        *out = nullptr;
        return fail(PBIT_E_NOMEM, "hipMalloc of %llu bytes failed: out of device memory", (unsigned long long)bytes);
    }
    if (e != hipSuccess) return device_fail(ctx, e, "hipMalloc");
    ctx->in_use += bytes;
    ctx->sizes[*out] = bytes;
    return PBIT_OK;
}

void dev_free(pbit_ctx *ctx, void *p)
{
    if (!p) return;
    auto it = ctx->sizes.find(p);
    if (it != ctx->sizes.end()) {
        ctx->in_use -= it->second;
        ctx->sizes.erase(it);
    }
    (void)hipFree(p);
}

int scratch(pbit_ctx *ctx, Slot slot, size_t bytes, void **out)
{
    Scratch &s = ctx->scratch[(int)slot];
    if (s.bytes >= bytes && s.ptr) {
        *out = s.ptr;
        return PBIT_OK;
    }
    if (s.ptr) {
        hipError_t e = hipStreamSynchronize(ctx->stream);
        if (e != hipSuccess) return device_fail(ctx, e, "hipStreamSynchronize");
        dev_free(ctx, s.ptr);
        s.ptr = nullptr;
        s.bytes = 0;
    }
    size_t want = std::max(bytes, (size_t)256);
    int rc = dev_alloc(ctx, want, &s.ptr);
    if (rc != PBIT_OK) return rc;
    s.bytes = want;
    *out = s.ptr;
    return PBIT_OK;
}

void release_scratch(pbit_ctx *ctx)
{
    for (auto &s : ctx->scratch) {
        dev_free(ctx, s.ptr);
        s.ptr = nullptr;
        s.bytes = 0;
    }
}

}  // namespace pbit

// ---------------------------------------------------------------- context

extern "C" int pbit_create(pbit_ctx **out, int device, uint64_t hbm_budget_bytes)
{
    if (!out) return fail(PBIT_E_ARG, "pbit_create: out is NULL");
    *out = nullptr;
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess || count <= 0) {
        (void)hipGetLastError();
        return fail(PBIT_E_DEVICE, "pbit_create: no HIP device available (%s)", hipGetErrorString(e));
    }
    if (device < 0 || device >= count) return fail(PBIT_E_ARG, "pbit_create: device %d out of range [0, %d)", device, count);
    e = hipSetDevice(device);
    if (e != hipSuccess) return fail(PBIT_E_DEVICE, "pbit_create: hipSetDevice failed (%s)", hipGetErrorString(e));
    pbit_ctx *ctx = new (std::nothrow) pbit_ctx();
    if (!ctx) return fail(PBIT_E_NOMEM, "pbit_create: host allocation failed");
    ctx->device = device;
    ctx->budget = hbm_budget_bytes;
    if (const char *v = std::getenv("PBIT_BQ_VARIANT")) {  // tuning override: 1..4 (see BqVariant)
        const int k = std::atoi(v);
        if (k >= 1 && k <= 4) ctx->bq_forced = (BqVariant)k;
    }
    if (const char *v = std::getenv("PBIT_BQ_BITS_RT")) ctx->bq_bits_rt = std::atoi(v);  // tuning override
    if (const char *v = std::getenv("PBIT_GRAPH_SLAB")) {  // tuning override: 0 off, 4 / 8 / 16 a tile width
        const int k = std::atoi(v);
        ctx->graph_slab = k != 0;
        ctx->graph_slab_rs = k == 4 || k == 8 || k == 16 ? k : 0;
    }
    if (const char *v = std::getenv("PBIT_BQ_SLAB_RS")) {  // tuning override: 16 or 8
        const int k = std::atoi(v);
        ctx->bq_slab_rs = k == 16 || k == 8 ? k : 0;
    }
    if (const char *v = std::getenv("PBIT_EA_STREAM")) ctx->ea_stream_forced = std::atoi(v) != 0;
    if (const char *v = std::getenv("PBIT_EA_ROWS")) ctx->ea_rows = std::max(0, std::atoi(v));  // tuning override
    if (const char *v = std::getenv("PBIT_GRAPH")) ctx->use_graph = std::atoi(v) != 0;
    if (const char *v = std::getenv("PBIT_TILE_TUNE")) ctx->tile_tune = std::atoi(v) != 0;
    if (const char *v = std::getenv("PBIT_EA_MFMA")) ctx->ea_mfma = std::atoi(v) < 0 ? -1 : (std::atoi(v) ? 1 : 0);
    ctx->serial = g_ctx_serial.fetch_add(1);
    int rc = noalloc_setup(device);  // device address of the static scratch of pbit_anneal_dev_noalloc
    if (rc) {
        delete ctx;
        return rc;
    }
    e = hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
        delete ctx;
        return fail(PBIT_E_DEVICE, "pbit_create: hipStreamCreate failed (%s)", hipGetErrorString(e));
    }
    *out = ctx;
    return PBIT_OK;
}

namespace pbit {
void free_problem(pbit_ctx *ctx, Problem &p)
{
    for (void *q : p.allocs) dev_free(ctx, q);
    p.allocs.clear();
}
}  // namespace pbit

extern "C" void pbit_destroy(pbit_ctx *ctx)
{
    if (!ctx) return;
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        (void)hipSetDevice(ctx->device);
        (void)hipStreamSynchronize(ctx->stream);
        serve_shutdown(ctx);
        for (auto &kv : ctx->problems) free_problem(ctx, kv.second);
        ctx->problems.clear();
        release_scratch(ctx);
        prof_release(ctx);
        if (ctx->graph_exec) (void)hipGraphExecDestroy((hipGraphExec_t)ctx->graph_exec);
        (void)hipStreamDestroy(ctx->stream);
    }
    delete ctx;
}

extern "C" uint64_t pbit_bytes_in_use(const pbit_ctx *ctx) { return ctx ? ctx->in_use : 0; }

// ---------------------------------------------------------------- problems

namespace pbit {

static bool in_unit_range(const int8_t *v, size_t n)
{
    for (size_t k = 0; k < n; ++k)
        if (v[k] < -1 || v[k] > 1) return false;
    return true;
}

static int upload(pbit_ctx *ctx, Problem &p, const void *host, size_t bytes, void **dev)
{
    int rc = dev_alloc(ctx, bytes, dev);
    if (rc != PBIT_OK) return rc;
    p.allocs.push_back(*dev);
    hipError_t e = hipMemcpy(*dev, host, bytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) return device_fail(ctx, e, "hipMemcpy (problem upload)");
    return PBIT_OK;
}

static int load_ea(pbit_ctx *ctx, const pbit_problem_desc *d, Problem &p)
{
    const int Lx = d->dims[0], Ly = d->dims[1], Lz = d->dims[2];
    if (Lx < 1 || Ly < 1 || Lz < 1) return fail(PBIT_E_ARG, "EA dims must be positive (got %d %d %d)", Lx, Ly, Lz);
    if ((Lx | Ly | Lz) & 1)
        return fail(PBIT_E_COLOURING, "EA sides must be even for a two-colour checkerboard (got %d %d %d)", Lx, Ly, Lz);
    const int64_t N = (int64_t)Lx * Ly * Lz;
    if (N > (int64_t)1 << 28) return fail(PBIT_E_UNSUPPORTED, "EA lattice of %lld sites is too large", (long long)N);
    if (!d->J) return fail(PBIT_E_ARG, "EA couplings are NULL");
    if (!in_unit_range(d->J, (size_t)(3 * N))) return fail(PBIT_E_RANGE, "EA couplings must be in {-1, 0, +1}");
    if (d->h && !in_unit_range(d->h, (size_t)N)) return fail(PBIT_E_RANGE, "fields must be in {-1, 0, +1}");

    std::vector<uint32_t> code((size_t)N);
    int amax = 0;
    bool dense = true;
    const int64_t plane = (int64_t)Lx * Ly;
    for (int z = 0; z < Lz; ++z)
        for (int y = 0; y < Ly; ++y)
            for (int x = 0; x < Lx; ++x) {
                const int64_t i = x + (int64_t)Lx * y + plane * z;
                const int64_t xm = (x == 0 ? Lx - 1 : x - 1) + (int64_t)Lx * y + plane * z;
                const int64_t ym = x + (int64_t)Lx * (y == 0 ? Ly - 1 : y - 1) + plane * z;
                const int64_t zm = x + (int64_t)Lx * y + plane * (z == 0 ? Lz - 1 : z - 1);
                const int8_t Jd[6] = {d->J[i], d->J[xm], d->J[N + i], d->J[N + ym], d->J[2 * N + i], d->J[2 * N + zm]};
                uint32_t c = 0;
                int nnz = 0;
                for (int k = 0; k < 6; ++k) {
                    if (Jd[k] != 0) {
                        c |= 1u << k;
                        ++nnz;
                    }
                    if (Jd[k] < 0) c |= 1u << (kCodeFlipShift + k);
                }
                const int hv = d->h ? d->h[i] : 0;
                c |= (uint32_t)(uint8_t)(int8_t)(nnz + hv) << kCodeBaseShift;
                c |= (uint32_t)(8 * (7 - nnz + hv)) << kCodePosShift;  // in [0, 64]
                dense = dense && nnz == 6;
                code[(size_t)i] = c;
                amax = std::max(amax, nnz + std::abs(hv));
            }
    void *dc = nullptr, *dJ = nullptr, *dh = nullptr, *ds = nullptr;
    int rc = upload(ctx, p, code.data(), sizeof(uint32_t) * (size_t)N, &dc);
    if (rc == PBIT_OK) rc = upload(ctx, p, d->J, (size_t)(3 * N), &dJ);
    if (rc == PBIT_OK && d->h) rc = upload(ctx, p, d->h, (size_t)N, &dh);
    EaView v{Lx, Ly, Lz, N, (const uint32_t *)dc, (const int8_t *)dJ, (const int8_t *)dh, dense, nullptr,
             nullptr, nullptr, nullptr, 0, 0};
    if (rc == PBIT_OK && N < 65536) {
        // the LDS-resident kernels' site list: class position -> site, wrap flags, code
        const int64_t half = N / 2, hx = Lx / 2;
        std::vector<uint32_t> sites((size_t)4 * half);
        for (int c = 0; c < 2; ++c)
            for (int64_t j = 0; j < half; ++j) {
                const int kx = (int)(j % hx), row = (int)(j / hx);
                const int y = row % Ly, z = row / Ly;
                const int x = 2 * kx + ((c + y + z) & 1);
                const int64_t i = x + (int64_t)Lx * y + plane * z;
                const uint32_t wrap = (x + 1 == Lx ? 1u : 0u) | (x == 0 ? 2u : 0u) | (y + 1 == Ly ? 4u : 0u) |
                                      (y == 0 ? 8u : 0u) | (z + 1 == Lz ? 16u : 0u) | (z == 0 ? 32u : 0u);
                sites[(size_t)2 * (c * half + j)] = (uint32_t)i | wrap << 16;
                sites[(size_t)2 * (c * half + j) + 1] = code[(size_t)i];
            }
        rc = upload(ctx, p, sites.data(), sizeof(uint32_t) * sites.size(), &ds);
        p.tile_sites = (const uint32_t *)ds;
        if (ea_slab_fits(v)) v.slab_sites = (const uint32_t *)ds;
    }
    // the matrix-core half-sweep's tiles (about 24 bytes per site), where the shape
    // allows them and the path may run: every cube with PBIT_EA_MFMA=1; by default the
    // cubes too large for the LDS-resident path, up to 2^21 sites
    const bool mfma_wanted = !ctx->ea_stream_forced && (ctx->ea_mfma == 1 ||
                             (ctx->ea_mfma != 0 && N > kEaSlabMaxSites && N <= ((int64_t)1 << 21)));
    if (rc == PBIT_OK && mfma_wanted) {
        EaMfmaHost mh;
        if (ea_mfma_build(Lx, Ly, Lz, d->J, d->h, mh)) {
            void *dt = nullptr, *dp = nullptr, *df = nullptr;
            rc = upload(ctx, p, mh.tiles.data(), sizeof(int32_t) * mh.tiles.size(), &dt);
            if (rc == PBIT_OK) rc = upload(ctx, p, mh.pos.data(), sizeof(int32_t) * mh.pos.size(), &dp);
            if (rc == PBIT_OK) rc = upload(ctx, p, mh.bonds.data(), sizeof(uint16_t) * mh.bonds.size(), &df);
            v.mfma_tiles = (const int32_t *)dt;
            v.mfma_pos = (const int2 *)dp;
            v.mfma_bonds = df;
            v.mfma_nb = mh.nb;
            v.mfma_n_tiles = mh.n_tiles;
        }
    }
    if (rc != PBIT_OK) return rc;
    p.kind = PBIT_EA3D;
    p.N = N;
    p.amax = amax;
    p.ea = v;
    return PBIT_OK;
}

static int round_up(int v, int m) { return (v + m - 1) / m * m; }

static int load_biclique(pbit_ctx *ctx, const pbit_problem_desc *d, Problem &p)
{
    const int na = d->dims[0], nb = d->dims[1];
    if (na < 1 || nb < 1) return fail(PBIT_E_ARG, "biclique sides must be >= 1 (got %d %d)", na, nb);
    if ((int64_t)na * nb > ((int64_t)1 << 30))
        return fail(PBIT_E_UNSUPPORTED, "biclique with %d x %d couplings is too large", na, nb);
    if (!d->J) return fail(PBIT_E_ARG, "biclique couplings are NULL");
    if (!in_unit_range(d->J, (size_t)na * nb)) return fail(PBIT_E_RANGE, "biclique couplings must be in {-1, 0, +1}");
    if (d->h && !in_unit_range(d->h, (size_t)na + nb)) return fail(PBIT_E_RANGE, "fields must be in {-1, 0, +1}");
    const int pad = std::min(na, nb) >= kBqLargeSide ? kBqPadLarge : kBqPad;
    const int na_p = round_up(na, pad), nb_p = round_up(nb, pad);
    std::vector<int8_t> J((size_t)na_p * nb_p, 0), JT((size_t)nb_p * na_p, 0), hA(na_p, 0), hB(nb_p, 0);
    std::vector<int> rowsum(na, 0), colsum(nb, 0);
    for (int a = 0; a < na; ++a)
        for (int b = 0; b < nb; ++b) {
            const int8_t v = d->J[(size_t)a * nb + b];
            J[(size_t)a * nb_p + b] = v;
            JT[(size_t)b * na_p + a] = v;
            rowsum[a] += std::abs(v);
            colsum[b] += std::abs(v);
        }
    int amax = 0;
    for (int a = 0; a < na; ++a) {
        hA[a] = d->h ? d->h[a] : 0;
        amax = std::max(amax, rowsum[a] + std::abs(hA[a]));
    }
    for (int b = 0; b < nb; ++b) {
        hB[b] = d->h ? d->h[na + b] : 0;
        amax = std::max(amax, colsum[b] + std::abs(hB[b]));
    }
    void *dJ = nullptr, *dJT = nullptr, *dhA = nullptr, *dhB = nullptr;
    int rc = upload(ctx, p, J.data(), J.size(), &dJ);
    if (rc == PBIT_OK) rc = upload(ctx, p, JT.data(), JT.size(), &dJT);
    if (rc == PBIT_OK) rc = upload(ctx, p, hA.data(), hA.size(), &dhA);
    if (rc == PBIT_OK) rc = upload(ctx, p, hB.data(), hB.size(), &dhB);
    void *dJb = nullptr, *dJTb = nullptr, *dhA2 = nullptr, *dhB2 = nullptr;
    if (rc == PBIT_OK) {
        // the kernels on spin bits (per-instance half-sweep and batched tiles): K byte p = 16 g + 4 j + i of every group of 32
        // columns holds column 8 i + 4 g + j of the group times 2^(3 - j) (the spin
        // byte it meets holds the bit times 2^j), and each field carries the coupling
        // sum of its site
        auto permute = [](const std::vector<int8_t> &M, int rows, int cols, std::vector<int8_t> &out) {
            out.assign(M.size(), 0);
            for (int r = 0; r < rows; ++r)
                for (int c0 = 0; c0 < cols; c0 += 32)
                    for (int q = 0; q < 32; ++q) {
                        const int g = q >> 4, j = (q >> 2) & 3, i = q & 3;
                        out[(size_t)r * cols + c0 + q] =
                            (int8_t)(M[(size_t)r * cols + c0 + 8 * i + 4 * g + j] * (1 << (3 - j)));
                    }
        };
        std::vector<int8_t> Jb, JTb;
        permute(J, na_p, nb_p, Jb);
        permute(JT, nb_p, na_p, JTb);
        std::vector<int32_t> hA2(na_p, 0), hB2(nb_p, 0);
        for (int a = 0; a < na; ++a) {
            hA2[a] = hA[a];
            for (int b = 0; b < nb; ++b) hA2[a] += J[(size_t)a * nb_p + b];
        }
        for (int b = 0; b < nb; ++b) {
            hB2[b] = hB[b];
            for (int a = 0; a < na; ++a) hB2[b] += JT[(size_t)b * na_p + a];
        }
        rc = upload(ctx, p, Jb.data(), Jb.size(), &dJb);
        if (rc == PBIT_OK) rc = upload(ctx, p, JTb.data(), JTb.size(), &dJTb);
        if (rc == PBIT_OK) rc = upload(ctx, p, hA2.data(), sizeof(int32_t) * hA2.size(), &dhA2);
        if (rc == PBIT_OK) rc = upload(ctx, p, hB2.data(), sizeof(int32_t) * hB2.size(), &dhB2);
    }
    void *dJ2 = nullptr, *dJT2 = nullptr;
    if (rc == PBIT_OK) {
        // two-bit couplings for the batched int8 tiles: J + 1 in {0, 1, 2}, padding included
        // (J = 0 there, so the code is 1: the tiles subtract every spin of the other side,
        // and padding spins take arbitrary values after the first update), 16 per word in
        // fragment order: word ((blk nku + u) 2 + g) 32 + l holds row 32 blk + l, columns
        // 32 u + 16 g + 4 j + i, as bits 2 j (low) and 2 j + 1 (high) of byte i
        auto pack2 = [](const std::vector<int8_t> &M, int rows, int cols, std::vector<uint32_t> &out) {
            const int nku = cols / 32;
            out.assign((size_t)rows * cols / 16, 0u);
            for (int r = 0; r < rows; ++r)
                for (int c = 0; c < cols; ++c) {
                    const uint32_t v = (uint32_t)(M[(size_t)r * cols + c] + 1);
                    const int blk = r / 32, l = r % 32, u = c / 32, g = (c / 16) % 2, j = (c / 4) % 4, i = c % 4;
                    out[(((size_t)blk * nku + u) * 2 + g) * 32 + l] |= v << (8 * i + 2 * j);
                }
        };
        std::vector<uint32_t> J2, JT2;
        pack2(J, na_p, nb_p, J2);
        pack2(JT, nb_p, na_p, JT2);
        rc = upload(ctx, p, J2.data(), sizeof(uint32_t) * J2.size(), &dJ2);
        if (rc == PBIT_OK) rc = upload(ctx, p, JT2.data(), sizeof(uint32_t) * JT2.size(), &dJT2);
    }
    if (rc != PBIT_OK) return rc;
    p.kind = PBIT_BICLIQUE;
    p.N = (int64_t)na + nb;
    p.amax = amax;
    p.bq = BqView{na, nb, na_p, nb_p, (const int8_t *)dJ, (const int8_t *)dJT, (const int8_t *)dhA,
                  (const int8_t *)dhB, (const int8_t *)dJb, (const int8_t *)dJTb, (const int32_t *)dhA2, (const int32_t *)dhB2,
                  (const uint32_t *)dJ2, (const uint32_t *)dJT2};
    return PBIT_OK;
}

static int load_graph(pbit_ctx *ctx, const pbit_graph_desc *d, Problem &p)
{
    const int n = d->n_spins, nb = d->n_bonds;
    if (n < 1 || nb < 0 || (nb > 0 && (!d->bond_i || !d->bond_j || !d->bond_J)))
        return fail(PBIT_E_ARG, "graph: need n_spins >= 1 and bond arrays");
    if ((int64_t)n * 16 > ((int64_t)1 << 31)) return fail(PBIT_E_UNSUPPORTED, "graph of %d spins is too large", n);
    for (int b = 0; b < nb; ++b) {
        if (d->bond_i[b] < 0 || d->bond_i[b] >= n || d->bond_j[b] < 0 || d->bond_j[b] >= n)
            return fail(PBIT_E_ARG, "graph: bond %d joins a vertex outside [0, %d)", b, n);
        if (d->bond_i[b] == d->bond_j[b]) return fail(PBIT_E_ARG, "graph: bond %d is a self-loop", b);
    }
    if (nb > 0 && !in_unit_range(d->bond_J, (size_t)nb)) return fail(PBIT_E_RANGE, "graph couplings must be in {-1, 0, +1}");
    if (d->h && !in_unit_range(d->h, (size_t)n)) return fail(PBIT_E_RANGE, "fields must be in {-1, 0, +1}");
    std::vector<int32_t> deg((size_t)n, 0);
    for (int b = 0; b < nb; ++b) {
        ++deg[d->bond_i[b]];
        ++deg[d->bond_j[b]];
    }
    const int maxdeg = n > 0 ? *std::max_element(deg.begin(), deg.end()) : 0;
    if (maxdeg > kGraphMaxDegree)
        return fail(PBIT_E_UNSUPPORTED, "graph: a vertex has %d bonds (at most %d)", maxdeg, kGraphMaxDegree);
    p.colour.assign((size_t)n, 0);
    int ncol = 0;
    if (d->colour) {
        if (d->n_colours < 1 || d->n_colours > 255) return fail(PBIT_E_ARG, "graph: n_colours must be 1..255");
        for (int i = 0; i < n; ++i)
            if (d->colour[i] >= d->n_colours) return fail(PBIT_E_COLOURING, "graph: colour of vertex %d out of range", i);
        for (int b = 0; b < nb; ++b)
            if (d->colour[d->bond_i[b]] == d->colour[d->bond_j[b]])
                return fail(PBIT_E_COLOURING, "graph: bond %d joins two vertices of colour %d", b, d->colour[d->bond_i[b]]);
        std::copy(d->colour, d->colour + n, p.colour.begin());
        ncol = d->n_colours;
    } else {
        int rc = greedy_colouring(n, nb, d->bond_i, d->bond_j, p.colour.data(), &ncol);
        if (rc) return rc;
    }
    // colour classes, then per position (class-major, ascending site inside a class) the
    // site's id, its adjacency range and base = nnz + h, and the adjacency in that order,
    // each entry one word: a kernel thread reaches its site's whole neighbourhood through
    // two dependent loads
    std::vector<int32_t> start((size_t)n + 1, 0);
    for (int i = 0; i < n; ++i) start[(size_t)i + 1] = start[i] + deg[i];
    std::vector<uint32_t> word((size_t)2 * nb);
    std::vector<int32_t> fill(start.begin(), start.end() - 1);
    std::vector<int32_t> base((size_t)n, 0);
    int amax = 0;
    for (int b = 0; b < nb; ++b) {
        const int8_t J = d->bond_J[b];
        const uint32_t c = (J != 0 ? 1u : 0u) | (J < 0 ? 2u : 0u);
        const int i = d->bond_i[b], j = d->bond_j[b];
        word[(size_t)fill[i]++] = (uint32_t)j << 2 | c;
        word[(size_t)fill[j]++] = (uint32_t)i << 2 | c;
        if (J != 0) {
            ++base[i];
            ++base[j];
        }
    }
    for (int i = 0; i < n; ++i) {
        const int hv = d->h ? d->h[i] : 0;
        amax = std::max(amax, base[i] + std::abs(hv));
        base[i] += hv;
    }
    p.class_start.assign((size_t)ncol + 1, 0);
    for (int i = 0; i < n; ++i) ++p.class_start[(size_t)p.colour[i] + 1];
    for (int c = 0; c < ncol; ++c) p.class_start[(size_t)c + 1] += p.class_start[c];
    std::vector<int32_t> cls((size_t)n), cfill(p.class_start.begin(), p.class_start.end() - 1);
    for (int i = 0; i < n; ++i) cls[(size_t)cfill[p.colour[i]]++] = i;
    std::vector<int32_t> meta((size_t)4 * n);
    std::vector<uint32_t> adj((size_t)2 * nb);
    size_t at = 0;
    for (int j = 0; j < n; ++j) {
        const int i = cls[(size_t)j];
        meta[(size_t)4 * j] = i;
        meta[(size_t)4 * j + 1] = (int32_t)at;
        for (int e = start[i]; e < start[(size_t)i + 1]; ++e) adj[at++] = word[(size_t)e];
        meta[(size_t)4 * j + 2] = (int32_t)at;
        meta[(size_t)4 * j + 3] = base[i];
    }

    void *dmeta = nullptr, *dadj = nullptr, *dbi = nullptr, *dbj = nullptr, *dbJ = nullptr, *dh = nullptr;
    int rc = upload(ctx, p, meta.data(), sizeof(int32_t) * meta.size(), &dmeta);
    if (rc == PBIT_OK && nb > 0) rc = upload(ctx, p, adj.data(), sizeof(uint32_t) * adj.size(), &dadj);
    if (rc == PBIT_OK && nb > 0) rc = upload(ctx, p, d->bond_i, sizeof(int32_t) * (size_t)nb, &dbi);
    if (rc == PBIT_OK && nb > 0) rc = upload(ctx, p, d->bond_j, sizeof(int32_t) * (size_t)nb, &dbj);
    if (rc == PBIT_OK && nb > 0) rc = upload(ctx, p, d->bond_J, (size_t)nb, &dbJ);
    if (rc == PBIT_OK && d->h) rc = upload(ctx, p, d->h, (size_t)n, &dh);
    void *dcs = nullptr;
    if (rc == PBIT_OK) rc = upload(ctx, p, p.class_start.data(), sizeof(int32_t) * p.class_start.size(), &dcs);
    if (rc != PBIT_OK) return rc;
    p.kind = PBIT_GRAPH;
    p.N = n;
    p.amax = amax;
    p.graph = GraphView{n, nb, ncol, maxdeg, p.class_start.data(), (const int32_t *)dmeta, (const uint32_t *)dadj,
                        (const int32_t *)dbi, (const int32_t *)dbj, (const int8_t *)dbJ, (const int8_t *)dh,
                        (const int32_t *)dcs};
    // the cube's layout kernels (init, transposes) are reused with N = n
    p.ea = EaView{0, 0, 0, (int64_t)n, nullptr, nullptr, nullptr, false, nullptr, nullptr, nullptr, nullptr, 0, 0};
    return PBIT_OK;
}

Problem *find_problem(pbit_ctx *ctx, uint64_t handle)
{
    auto it = ctx->problems.find(handle);
    return it == ctx->problems.end() ? nullptr : &it->second;
}

}  // namespace pbit


extern "C" int pbit_load_problem(pbit_ctx *ctx, const pbit_problem_desc *desc, uint64_t *problem_out)
{
    try {
        PBIT_ENTER(ctx);
        if (!desc || !problem_out) return fail(PBIT_E_ARG, "pbit_load_problem: NULL argument");
        Problem p;
        int rc;
        if (desc->kind == PBIT_EA3D)
            rc = load_ea(ctx, desc, p);
        else if (desc->kind == PBIT_BICLIQUE)
            rc = load_biclique(ctx, desc, p);
        else
            rc = fail(PBIT_E_ARG, "pbit_load_problem: unknown kind %d", desc->kind);
        if (rc != PBIT_OK) {
            free_problem(ctx, p);
            return rc;
        }
        const uint64_t h = ((uint64_t)ctx->serial << 40) | (++ctx->next_handle);
        ctx->problems.emplace(h, std::move(p));
        *problem_out = h;
        return PBIT_OK;
    } catch (const std::bad_alloc &) {
        return fail(PBIT_E_NOMEM, "pbit_load_problem: host allocation failed");
    } catch (...) {
        return fail(PBIT_E_ARG, "pbit_load_problem: internal error");
    }
}

extern "C" int pbit_load_graph(pbit_ctx *ctx, const pbit_graph_desc *desc, uint64_t *problem_out)
{
    try {
        PBIT_ENTER(ctx);
        if (!desc || !problem_out) return fail(PBIT_E_ARG, "pbit_load_graph: NULL argument");
        Problem p;
        int rc = load_graph(ctx, desc, p);
        if (rc != PBIT_OK) {
            free_problem(ctx, p);
            return rc;
        }
        const uint64_t h = ((uint64_t)ctx->serial << 40) | (++ctx->next_handle);
        auto it = ctx->problems.emplace(h, std::move(p)).first;
        it->second.graph.class_start = it->second.class_start.data();  // the vector moved
        *problem_out = h;
        return PBIT_OK;
    } catch (const std::bad_alloc &) {
        return fail(PBIT_E_NOMEM, "pbit_load_graph: host allocation failed");
    } catch (...) {
        return fail(PBIT_E_ARG, "pbit_load_graph: internal error");
    }
}

extern "C" int pbit_problem_colouring(pbit_ctx *ctx, uint64_t problem, uint8_t *colour_out, int32_t *n_colours_out)
{
    PBIT_ENTER(ctx);
    Problem *P = find_problem(ctx, problem);
    if (!P) return fail(PBIT_E_HANDLE, "pbit_problem_colouring: unknown problem handle");
    int ncol = 2;
    if (P->kind == PBIT_GRAPH) {
        ncol = P->graph.n_colours;
        if (colour_out) std::copy(P->colour.begin(), P->colour.end(), colour_out);
    } else if (colour_out) {
        if (P->kind == PBIT_EA3D) {
            const EaView &v = P->ea;
            for (int64_t i = 0; i < P->N; ++i) {
                const int64_t x = i % v.Lx, y = (i / v.Lx) % v.Ly, z = i / ((int64_t)v.Lx * v.Ly);
                colour_out[i] = (uint8_t)((x + y + z) & 1);
            }
        } else {
            for (int64_t i = 0; i < P->N; ++i) colour_out[i] = i < P->bq.na ? 0 : 1;
        }
    }
    if (n_colours_out) *n_colours_out = ncol;
    return PBIT_OK;
}

extern "C" int pbit_unload_problem(pbit_ctx *ctx, uint64_t problem)
{
    PBIT_ENTER(ctx);
    Problem *p = find_problem(ctx, problem);
    if (!p) return fail(PBIT_E_HANDLE, "pbit_unload_problem: unknown problem handle");
    if (p->jobs > 0) return fail(PBIT_E_BUSY, "pbit_unload_problem: %d job(s) still use the problem", p->jobs);
    hipError_t e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return device_fail(ctx, e, "hipStreamSynchronize");
    free_problem(ctx, *p);
    ctx->problems.erase(problem);
    return PBIT_OK;
}

extern "C" int64_t pbit_problem_spins(pbit_ctx *ctx, uint64_t problem)
{
    PBIT_ENTER(ctx);
    Problem *p = find_problem(ctx, problem);
    if (!p) return fail(PBIT_E_HANDLE, "pbit_problem_spins: unknown problem handle");
    return p->N;
}

// ---------------------------------------------------------------- anneal

namespace pbit {

int check_desc(const pbit_anneal_desc *d, const char *who)
{
    if (!d) return fail(PBIT_E_ARG, "%s: descriptor is NULL", who);
    if (d->n_sweeps < 0 || d->sweep_offset < 0) return fail(PBIT_E_ARG, "%s: sweep count and offset must be >= 0", who);
    if ((int64_t)d->sweep_offset + d->n_sweeps > (int64_t)UINT32_MAX)
        return fail(PBIT_E_ARG, "%s: sweep index exceeds 32 bits", who);
    if (d->n_replicas < 1 || d->n_replicas > (1 << 30))
        return fail(PBIT_E_ARG, "%s: n_replicas must be in [1, 2^30]", who);
    if (d->replica_offset < 0 || d->replica_offset % 4 != 0)
        return fail(PBIT_E_ARG, "%s: replica_offset must be a non-negative multiple of 4", who);
    if (d->n_sweeps > 0 && !d->beta) return fail(PBIT_E_ARG, "%s: beta is NULL", who);
    if (d->trace_every < 0) return fail(PBIT_E_ARG, "%s: trace_every must be >= 0", who);
    for (int s = 0; s < d->n_sweeps; ++s)
        if (!(d->beta[s] >= 0.0) || std::isinf(d->beta[s]))
            return fail(PBIT_E_RANGE, "%s: beta[%d] must be finite and >= 0", who, s);
    return PBIT_OK;
}

int spins_in_range(const int8_t *s, size_t n)
{
    for (size_t k = 0; k < n; ++k)
        if (s[k] != 1 && s[k] != -1) return 0;
    return 1;
}

// State of one anneal on the device, in the kernels' own layouts.
struct DevState {
    int R = 0, Rp = 0;
    int8_t *spins = nullptr;  // EA: [N][Rp]
    int8_t *MA = nullptr, *MB = nullptr;  // biclique int8 spins (staging when held as bits)
    bool bits = false;                    // biclique spins held as bits
    uint32_t *MAb = nullptr, *MBb = nullptr;
    uint32_t *table = nullptr;
    int width = 1;
    int32_t *E32 = nullptr;
    int8_t *stage = nullptr;  // [R][N] host-layout staging
    BqVariant variant = BqVariant::Auto;
    int bits_rt = 0;  // replicas per tile of the bit kernel (0: its launcher's rule)
    int slab_rs = 0;  // replicas per slice of the LDS-resident biclique kernel (0: its launcher's rule)
    bool slab = false;        // cube, graph or small biclique held in LDS for runs of sweeps
    int graph_rs = 0;         // replicas per workgroup of the LDS-resident graph sweep (graph_slab)
    int32_t *graph_energy = nullptr;  // its per-replica energies (not used by the runtime)
    bool mfma = false;        // cube fields on the matrix cores (ea_mfma.hip), spins [2][Rp][N / 2]
    Arena *arena = nullptr;   // set: buffers are carved from it (no allocation, no kernel timing)
};

// Device buffers of an anneal: carved from the arena when there is one, else the
// context's scratch slots (grown on demand).
static int take(pbit_ctx *ctx, DevState &ds, Slot slot, size_t bytes, void **out)
{
    if (!ds.arena) return scratch(ctx, slot, bytes, out);
    const size_t at = (ds.arena->used + 255) & ~(size_t)255;
    if (at + bytes > ds.arena->bytes)
        return fail(PBIT_E_UNSUPPORTED, "the anneal needs more than the %llu bytes of static scratch",
                    (unsigned long long)ds.arena->bytes);
    *out = static_cast<uint8_t *>(ds.arena->base) + at;
    ds.arena->used = at + bytes;
    return PBIT_OK;
}

constexpr int kSlabChunk = 1000;  // sweeps per launch of the LDS-resident cube, graph and biclique kernels
constexpr size_t kGraphSlabLds = 160 * 1024 - 4096;  // spin rows of a graph tile in LDS (beside its decision words)

// Pick the biclique kernel variant for this shape: the forced one, a cached
// choice, or the fastest of the candidates timed here on the (not yet
// initialised) spin buffers, whose contents do not affect the timing.
static int tune_biclique(pbit_ctx *ctx, const Problem &P, DevState &ds, hipStream_t st, int n_sweeps)
{
    // the DMA and bit tiles need sides padded to 128 (and the bit tiles a bit copy of
    // the spins, made where the replicas pad to 256); the LDS-resident form sides of
    // at most 512 and its decision words in LDS
    const bool large = P.bq.na_p % 128 == 0 && P.bq.nb_p % 128 == 0;
    const bool slab_ok = bq_slab_supported(P.bq, ds.Rp, ds.width, ctx->bq_slab_rs);
    const BqVariant f = ctx->bq_forced;
    ds.bits_rt = ctx->bq_bits_rt;
    ds.slab_rs = ctx->bq_slab_rs;
    if (f == BqVariant::Small || (f == BqVariant::Dma && large) || (f == BqVariant::Bits && ds.MAb) ||
        (f == BqVariant::Slab && slab_ok)) {
        ds.variant = f;  // a forced kernel the shape cannot take falls back to the tuned choice
        return PBIT_OK;
    }
    const std::array<int, 4> shape{P.bq.na_p, P.bq.nb_p, ds.Rp, slab_ok ? 1 : 0};
    auto it = ctx->bq_tuned.find(shape);
    if (it != ctx->bq_tuned.end()) {
        ds.variant = it->second.first;
        (ds.variant == BqVariant::Slab ? ds.slab_rs : ds.bits_rt) = it->second.second;
        return PBIT_OK;
    }
    if (!large && !slab_ok) {
        ds.variant = BqVariant::Small;
        ctx->bq_tuned[shape] = {ds.variant, 0};
        return PBIT_OK;
    }
    if (ds.arena) {
        // no timing here (it would create events and wait for the stream): the kernel
        // the tuner keeps at the benchmark's shapes (the LDS-resident form where it
        // runs, else the bit tile), else the DMA or 64 x 64 tile; not cached
        ds.variant = slab_ok ? BqVariant::Slab : ds.MAb ? BqVariant::Bits : large ? BqVariant::Dma : BqVariant::Small;
        return PBIT_OK;
    }
    const BqVariant cand[] = {BqVariant::Small, BqVariant::Dma, BqVariant::Bits, BqVariant::Slab};
    hipEvent_t e0, e1;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e != hipSuccess) return device_fail(ctx, e, "hipEventCreate (tuning)");
    const Key key{0u, 0u};
    // the LDS-resident form loads its couplings once per launch of up to kSlabChunk sweeps:
    // timed over 1 and 1 + m sweeps, and its cost for this call's sweeps set against the
    // others' per half-sweep (table rows up to n_sweeps are read)
    // (32 more sweeps: enough that a traced run's longer launches do not flip its slice choice)
    const int S = std::max(1, n_sweeps), m = std::min(32, S - 1);
    float best_ms = 0.f;
    BqVariant best = BqVariant::Small;
    int best_rt = 0;
    bool have = false;
    int rt = 0;  // the bit kernel's replica tile or the LDS-resident kernel's slice being timed
    // one warm-up pass, then the best of three (a profiler's tracing stretches single launches)
    auto time_it = [&](BqVariant v, int slab_sweeps, float *best_pass) {
        *best_pass = 0.f;
        for (int rep = 0; rep < 4 && e == hipSuccess; ++rep) {
            float one_pass = 0.f, *ms = &one_pass;
            e = hipEventRecord(e0, st);
            if (v == BqVariant::Slab) {
                if (e == hipSuccess)
                    e = bq_slab(P.bq, ds.MA, ds.MB, ds.Rp, ds.table, ds.width, 0, slab_sweeps, 0u, 0u, key, st,
                                rt);
            } else {
                for (int k = 0; k < 4 && e == hipSuccess; ++k)
                    e = v == BqVariant::Bits
                            ? bqb_halfsweep(P.bq, k & 1, ds.MAb, ds.MBb, ds.Rp, ds.table, ds.width, 0u, 0u, key, st,
                                            rt)
                            : bq_halfsweep(P.bq, k & 1, ds.MA, ds.MB, ds.R, ds.Rp, ds.table, ds.width, 0u, 0u, key,
                                           st, v);
            }
            if (e == hipSuccess) e = hipEventRecord(e1, st);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            if (e == hipSuccess) e = hipEventElapsedTime(ms, e0, e1);
            if (rep == 1 || (rep > 1 && one_pass < *best_pass)) *best_pass = one_pass;
        }
    };
    // the bit kernel in each replica tile that divides Rp, and the LDS-resident kernel in
    // slices of 16 and 8 replicas (unless forced): more tiles or slices fill more CUs,
    // larger ones read the couplings fewer times or use more of the MFMA's rows
    std::vector<std::pair<BqVariant, int>> runs;
    for (BqVariant v : cand) {
        if ((v == BqVariant::Dma && !large) || (v == BqVariant::Bits && !ds.MAb) || (v == BqVariant::Slab && !slab_ok))
            continue;  // the shape cannot take it
        if (v == BqVariant::Bits && ds.bits_rt == 0) {
            for (int w : {256, 128, 64})
                if (ds.Rp % w == 0) runs.push_back({v, w});
        } else if (v == BqVariant::Slab && ds.slab_rs == 0) {
            for (int w : {16, 8})
                if (bq_slab_supported(P.bq, ds.Rp, ds.width, w)) runs.push_back({v, w});
        } else {
            runs.push_back({v, v == BqVariant::Slab ? ds.slab_rs : ds.bits_rt});
        }
    }
    for (const auto &run : runs) {
        const BqVariant v = run.first;
        rt = run.second;
        float ms = 0.f;
        if (v == BqVariant::Slab) {
            float t1 = 0.f, t2 = 0.f;
            time_it(v, 1, &t1);
            if (m > 0) time_it(v, 1 + m, &t2);
            const double per_sweep = m > 0 ? std::max(0.0, (double)(t2 - t1) / m) : t1;
            const double load = m > 0 ? std::max(0.0, t1 - per_sweep) : 0.0;
            const double total = (double)((S + kSlabChunk - 1) / kSlabChunk) * load + S * per_sweep;
            ms = (float)(total * 2.0 / S);  // per four half-sweeps, as the others
        } else {
            time_it(v, 0, &ms);
        }
        if (e != hipSuccess) break;
        if (!have || ms < best_ms) {
            best_ms = ms;
            best = v;
            best_rt = rt;
            have = true;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess) return device_fail(ctx, e, "biclique kernel tuning");
    ds.variant = best;
    if (best == BqVariant::Bits) ds.bits_rt = best_rt;
    if (best == BqVariant::Slab) ds.slab_rs = best_rt;
    ctx->bq_tuned[shape] = {ds.variant, best == BqVariant::Slab ? ds.slab_rs : ds.bits_rt};
    return PBIT_OK;
}

// Cube path for a shape that both one-launch-per-half-sweep kernels can take: the
// streaming stencil or the matrix-core half-sweep, whichever ran faster when timed
// here (four half-sweeps each, after a warm-up pass) on `spins`, zeroed first (zero
// bytes are valid +1 spins for both kernels) and at least N x round_up(R, 128)
// bytes.  The choice is cached per shape and replica count.
static int tune_cube(pbit_ctx *ctx, const Problem &P, int R, int8_t *spins, hipStream_t st, bool *mfma)
{
    const int Rs = round_up(R, kEaRPad), Rm = round_up(R, kEaMfmaRPad);
    const std::array<int, 4> shape{P.ea.Lx, P.ea.Ly, P.ea.Lz, Rm};
    auto it = ctx->ea_tuned.find(shape);
    if (it != ctx->ea_tuned.end()) {
        *mfma = it->second;
        return PBIT_OK;
    }
    hipError_t e = fill_i32((int32_t *)spins, (int64_t)((size_t)P.N * Rm / 4), 0, st);
    if (e != hipSuccess) return device_fail(ctx, e, "spin buffer clear (tuning)");
    hipEvent_t e0, e1;
    e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e != hipSuccess) return device_fail(ctx, e, "hipEventCreate (tuning)");
    EaRow row;
    for (uint64_t &v : row.s) v = (uint64_t)1 << 31;
    const Key key{0u, 0u};
    float ms[2] = {0.f, 0.f};
    for (int m = 0; m < 2 && e == hipSuccess; ++m)
        for (int rep = 0; rep < 2 && e == hipSuccess; ++rep) {  // the first pass warms up
            e = hipEventRecord(e0, st);
            for (int k = 0; k < 4 && e == hipSuccess; ++k)
                e = m ? eam_halfsweep(P.ea, (uint8_t *)spins, Rm, k & 1, row, 0u, 0u, key, st)
                      : ea_halfsweep(P.ea, spins, Rs, k & 1, row, 0u, 0u, key, st, ctx->ea_rows);
            if (e == hipSuccess) e = hipEventRecord(e1, st);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            if (e == hipSuccess) e = hipEventElapsedTime(&ms[m], e0, e1);
        }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess) return device_fail(ctx, e, "cube kernel tuning");
    *mfma = ms[1] < ms[0];
    ctx->ea_tuned[shape] = *mfma;
    return PBIT_OK;
}

static int prepare(pbit_ctx *ctx, const Problem &P, const pbit_anneal_desc *d, hipStream_t st, DevState &ds,
                   const void *dev_init)
{
    const int R = d->n_replicas;
    ds.R = R;
    void *v = nullptr;
    int rc;
    if (P.kind == PBIT_EA3D || P.kind == PBIT_GRAPH) {
        // the stencil and the gather address the spin matrix with 32-bit byte offsets
        if ((uint64_t)P.N * (((uint64_t)R + kEaRPad - 1) / kEaRPad * kEaRPad) >= ((uint64_t)1 << 32))
            return fail(PBIT_E_UNSUPPORTED, "%lld spins x %d replicas exceed 4 GiB of int8 spins",
                        (long long)P.N, R);
        // cube paths: PBIT_EA_STREAM=1 takes the stencil; PBIT_EA_MFMA=1 the matrix cores
        // wherever built; by default cubes that fit LDS stay there, and for larger ones
        // the stencil and the matrix cores (where built) are timed against each other
        // (PBIT_EA_MFMA=0: the stencil)
        const bool cube = P.kind == PBIT_EA3D, tiles = cube && P.ea.mfma_tiles;
        bool tune = false;
        if (cube && !ctx->ea_stream_forced) {
            ds.mfma = tiles && ctx->ea_mfma == 1;
            ds.slab = !ds.mfma && P.ea.slab_sites;
            tune = !ds.mfma && !ds.slab && tiles && ctx->ea_mfma != 0 && d->n_sweeps > 0;
        }
        // the tuner times both layouts in one buffer: spins for replicas padded to 128
        ds.Rp = round_up(R, ds.mfma || tune ? kEaMfmaRPad : kEaRPad);
        rc = take(ctx, ds, Slot::Spins, (size_t)P.N * ds.Rp, &v);
        if (rc) return rc;
        ds.spins = (int8_t *)v;
        if (tune) {
            if (ds.arena)
                ds.mfma = R <= 1024;  // no timing without allocation: the measured default, not cached
            else if ((rc = tune_cube(ctx, P, R, ds.spins, st, &ds.mfma)))
                return rc;
            ds.Rp = round_up(R, ds.mfma ? kEaMfmaRPad : kEaRPad);
        }
    } else {
        // int8 spins, plus a bit copy where the sides are padded to 128 and the replicas to 256
        // (the tuner then times the bit kernel, whose tiles hold 256 replicas: a forced bit
        // kernel pads to that)
        const bool bits_forced = ctx->bq_forced == BqVariant::Bits && P.bq.Jb;
        ds.Rp = round_up(R, bits_forced ? 256 : kBqRPad);
        const size_t a = (size_t)ds.Rp * P.bq.na_p, b = (size_t)ds.Rp * P.bq.nb_p;
        rc = take(ctx, ds, Slot::Spins, a + b, &v);
        if (rc) return rc;
        ds.MA = (int8_t *)v;
        ds.MB = ds.MA + a;
        // padding sites must hold zero (a fill kernel: no memset node if a caller captures the stream)
        hipError_t e = fill_i32((int32_t *)ds.MA, (int64_t)((a + b) / 4), 0, st);
        if (e != hipSuccess) return device_fail(ctx, e, "spin buffer clear");
        if (bqb_supported(P.bq, ds.Rp) &&
                   (ctx->bq_forced == BqVariant::Auto || ctx->bq_forced == BqVariant::Bits)) {
            rc = take(ctx, ds, Slot::Aux, (a + b) / 8, &v);
            if (rc) return rc;
            ds.MAb = (uint32_t *)v;
            ds.MBb = ds.MAb + a / 32;
            e = fill_i32((int32_t *)ds.MAb, (int64_t)((a + b) / 32), 0, st);
            if (e != hipSuccess) return device_fail(ctx, e, "spin bit buffer clear");
        }
    }
    if (P.kind == PBIT_GRAPH && ctx->graph_slab) {
        // the whole graph for a tile of replicas in LDS, runs of sweeps per launch: the
        // narrowest tile (4, 8 or 16 replicas) that fits and leaves at most two workgroups
        // per compute unit, else the widest that fits.  Measured on the L = 14 dimerized
        // cube: a workgroup's sweep costs about the same at any tile width up to two per
        // CU, so narrow tiles spread small replica counts over more CUs, and past two per
        // CU the wider tile wins.
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device) != hipSuccess) cus = 256;
        for (int rs : {4, 8, 16}) {
            if (ds.Rp % rs != 0 || graph_tile_lds(P.N, rs) > kGraphSlabLds) continue;
            if (ctx->graph_slab_rs && rs != ctx->graph_slab_rs) continue;
            ds.graph_rs = rs;
            if (ds.Rp / rs <= 2 * cus) break;
        }
        if (ds.graph_rs) {
            rc = take(ctx, ds, Slot::Aux, sizeof(int32_t) * (size_t)ds.Rp, &v);
            if (rc) return rc;
            ds.graph_energy = (int32_t *)v;
            ds.slab = true;
        }
    }
    rc = take(ctx, ds, Slot::E32, sizeof(int32_t) * (size_t)ds.Rp, &v);
    if (rc) return rc;
    ds.E32 = (int32_t *)v;

    // threshold table for this call's sweeps (built on the host in FP64)
    const int S = d->n_sweeps;
    ds.width = S > 0 ? table_width(d->beta, S, P.amax) : 1;
    if (ds.width > kMaxTableWidth)
        return fail(PBIT_E_UNSUPPORTED, "threshold rows of %d entries exceed the %d the kernels stage in LDS "
                    "(raise the smallest beta)", ds.width, kMaxTableWidth);
    ctx->host_table.resize((size_t)std::max(S, 1) * ds.width);
    if (S > 0) build_table(d->beta, S, ds.width, ctx->host_table.data());
    rc = take(ctx, ds, Slot::Table, sizeof(uint32_t) * ctx->host_table.size(), &v);
    if (rc) return rc;
    ds.table = (uint32_t *)v;
    hipError_t e = hipMemcpyAsync(ds.table, ctx->host_table.data(), sizeof(uint32_t) * ctx->host_table.size(),
                                  hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return device_fail(ctx, e, "hipMemcpyAsync (table)");

    if (P.kind == PBIT_BICLIQUE && d->n_sweeps > 0) {
        rc = tune_biclique(ctx, P, ds, st, d->n_sweeps);
        if (rc) return rc;
    }
    ds.bits = P.kind == PBIT_BICLIQUE && ds.variant == BqVariant::Bits;
    if (P.kind == PBIT_BICLIQUE && ds.variant == BqVariant::Slab) ds.slab = true;  // runs of sweeps per launch
    if (P.kind == PBIT_EA3D && d->n_sweeps > 0) ctx->ea_last_path = ds.slab ? 2 : (ds.mfma ? 3 : 1);
    if (P.kind == PBIT_GRAPH && d->n_sweeps > 0) ctx->graph_last_path = ds.slab ? 2 : 1;
    if (P.kind == PBIT_BICLIQUE && d->n_sweeps > 0) ctx->bq_last_variant = (int)ds.variant;

    const Key key{(uint32_t)d->seed, (uint32_t)(d->seed >> 32)};
    const uint32_t rq0 = (uint32_t)d->replica_offset >> 2;
    const int8_t *init_rows = (const int8_t *)dev_init;
    if (d->init_spins) {
        rc = take(ctx, ds, Slot::Stage, (size_t)R * P.N, &v);
        if (rc) return rc;
        ds.stage = (int8_t *)v;
        e = hipMemcpyAsync(ds.stage, d->init_spins, (size_t)R * P.N, hipMemcpyHostToDevice, st);
        if (e != hipSuccess) return device_fail(ctx, e, "hipMemcpyAsync (init spins)");
        init_rows = ds.stage;
    }
    const bool rowlayout = P.kind != PBIT_BICLIQUE;  // cube and graph share the [N][Rp] layout
    if (ds.mfma)
        e = init_rows ? eam_from_rows(P.ea, init_rows, R, (uint8_t *)ds.spins, ds.Rp, st)
                      : eam_init(P.ea, (uint8_t *)ds.spins, ds.Rp, rq0, key, st);
    else if (rowlayout)
        e = init_rows ? ea_from_rows(P.ea, init_rows, R, ds.spins, ds.Rp, st)
                      : ea_init(P.ea, ds.spins, ds.Rp, rq0, key, st);
    else
        e = init_rows ? bq_from_rows(P.bq, init_rows, R, ds.MA, ds.MB, st) : bq_init(P.bq, ds.MA, ds.MB, R, rq0, key, st);
    if (e == hipSuccess && ds.bits) e = bqb_pack(P.bq, ds.MA, ds.MB, ds.MAb, ds.MBb, ds.Rp, st);
    if (e != hipSuccess) return device_fail(ctx, e, "spin initialisation launch");
    return PBIT_OK;
}

static hipError_t sweep(pbit_ctx *ctx, const Problem &P, DevState &ds, int s, uint32_t t, uint32_t rq0, Key key,
                        hipStream_t st)
{
    const uint32_t *row = ds.table + (size_t)s * ds.width;
    hipError_t e = hipSuccess;
    const int ncol = P.kind == PBIT_GRAPH ? P.graph.n_colours : 2;
    EaRow earow;
    if (P.kind == PBIT_EA3D) earow = ea_row(ctx->host_table.data() + (size_t)s * ds.width, ds.width);
    for (int c = 0; c < ncol && e == hipSuccess; ++c) {
        if (ctx->prof_every > 0 && ctx->prof_open < 0 && (ncol * s + c) % ctx->prof_every == 0) {
            e = prof_begin(ctx, P.kind, st);
            if (e != hipSuccess) return e;
        }
        if (ds.mfma)
            e = eam_halfsweep(P.ea, (uint8_t *)ds.spins, ds.Rp, c, earow, t, rq0, key, st);
        else if (P.kind == PBIT_EA3D)
            e = ea_halfsweep(P.ea, ds.spins, ds.Rp, c, earow, t, rq0, key, st, ctx->ea_rows);
        else if (P.kind == PBIT_GRAPH)
            e = graph_halfsweep(P.graph, c, ds.spins, ds.Rp, row, ds.width, t, rq0, key, st);
        else if (ds.bits)
            e = bqb_halfsweep(P.bq, c, ds.MAb, ds.MBb, ds.Rp, row, ds.width, t, rq0, key, st, ds.bits_rt);
        else
            e = bq_halfsweep(P.bq, c, ds.MA, ds.MB, ds.R, ds.Rp, row, ds.width, t, rq0, key, st, ds.variant);
        if (e == hipSuccess) e = prof_count_launch(ctx, st);
    }
    return e;
}

// Sweeps [s0, s1): one launch of the LDS-resident cube kernel, or a launch per
// half-sweep.  A timing window brackets the resident launch, counted as its half-sweeps.
static hipError_t sweeps(pbit_ctx *ctx, const Problem &P, DevState &ds, int s0, int s1, uint32_t sweep0,
                         uint32_t rq0, Key key, hipStream_t st)
{
    if (!ds.slab) {
        for (int s = s0; s < s1; ++s) {
            hipError_t e = sweep(ctx, P, ds, s, sweep0 + (uint32_t)s, rq0, key, st);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    }
    hipError_t e = hipSuccess;
    const bool timed = ctx->prof_every > 0 && ctx->prof_open < 0;
    if (timed) e = prof_begin(ctx, P.kind, st);
    if (e == hipSuccess) {
        if (P.kind == PBIT_BICLIQUE) {
            e = bq_slab(P.bq, ds.MA, ds.MB, ds.Rp, ds.table, ds.width, s0, s1, sweep0, rq0, key, st, ds.slab_rs);
        } else if (P.kind == PBIT_GRAPH) {
            const GraphView &g = P.graph;
            GraphJobDev jb{reinterpret_cast<const int4 *>(g.site_meta), g.adj, g.class_start_dev, g.bi, g.bj, g.bJ,
                           g.h, ds.table, ds.spins, ds.graph_energy, g.n, g.n_bonds, g.n_colours, ds.width,
                           ds.graph_rs, sweep0, rq0, key.k0, key.k1};
            jb.row_stride = ds.Rp;
            e = graph_slab(jb, ds.Rp / ds.graph_rs, s0, s1, st);
        } else {
            e = ea_slab(P.ea, ds.spins, ds.Rp, ds.table, ds.width, s0, s1, sweep0, rq0, key, st);
        }
    }
    if (e == hipSuccess && timed) {
        // counted as its class updates: two per sweep for a cube or biclique, one per colour class
        ctx->prof_launches.back() += (P.kind == PBIT_GRAPH ? P.graph.n_colours : 2) * (s1 - s0);
        e = prof_close(ctx, st);
    }
    return e;
}

static hipError_t energies(const Problem &P, DevState &ds, hipStream_t st)
{
    if (P.kind == PBIT_GRAPH) return graph_energy(P.graph, ds.spins, ds.Rp, ds.R, ds.E32, st);
    if (ds.mfma) return eam_energy(P.ea, (const uint8_t *)ds.spins, ds.Rp, ds.R, ds.E32, st);
    if (P.kind == PBIT_EA3D) return ea_energy(P.ea, ds.spins, ds.Rp, ds.R, ds.E32, st);
    if (ds.bits) {
        hipError_t e = bqb_unpack(P.bq, ds.MAb, ds.MBb, ds.MA, ds.MB, ds.Rp, st);
        if (e != hipSuccess) return e;
    }
    return bq_energy(P.bq, ds.MA, ds.MB, ds.R, ds.Rp, ds.E32, st);
}

static hipError_t to_rows(const Problem &P, DevState &ds, int8_t *dst, hipStream_t st)
{
    if (ds.mfma) return eam_to_rows(P.ea, (const uint8_t *)ds.spins, ds.Rp, dst, ds.R, st);
    if (P.kind != PBIT_BICLIQUE) return ea_to_rows(P.ea, ds.spins, ds.Rp, dst, ds.R, st);
    if (ds.bits) {
        hipError_t e = bqb_unpack(P.bq, ds.MAb, ds.MBb, ds.MA, ds.MB, ds.Rp, st);
        if (e != hipSuccess) return e;
    }
    return bq_to_rows(P.bq, ds.MA, ds.MB, dst, ds.R, st);
}

static int fetch_energies(pbit_ctx *ctx, const Problem &P, DevState &ds, hipStream_t st, std::vector<int32_t> &out)
{
    hipError_t e = prof_close(ctx, st);  // a timing window covers sweep launches only
    if (e == hipSuccess) e = energies(P, ds, st);
    if (e == hipSuccess) {
        out.resize(ds.R);
        e = hipMemcpyAsync(out.data(), ds.E32, sizeof(int32_t) * ds.R, hipMemcpyDeviceToHost, st);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e == hipSuccess) e = prof_harvest(ctx);
    if (e != hipSuccess) return device_fail(ctx, e, "energy evaluation");
    return PBIT_OK;
}

// The device state an anneal's next sweep depends on (the spin layout the sweep kernels read).
static void state_span(const Problem &P, const DevState &ds, void **ptr, size_t *bytes)
{
    if (P.kind != PBIT_BICLIQUE) {
        *ptr = ds.spins;
        *bytes = (size_t)P.N * ds.Rp;
    } else {
        const size_t ab = (size_t)ds.Rp * (P.bq.na_p + P.bq.nb_p);
        *ptr = ds.bits ? (void *)ds.MAb : (void *)ds.MA;
        *bytes = ds.bits ? ab / 8 : ab;
    }
}

// Sweeps with a target checked after every sweep, without a host round trip per
// sweep: chunks of sweeps are enqueued with a from-scratch energy pass and an
// on-device check after each sweep that records the first sweep meeting the
// target, and the host reads that once per chunk.  The state at the start of a
// chunk is kept; when a sweep inside the chunk met the target, the state is
// restored and the chunk re-run up to that sweep, which reproduces it exactly
// (the random words depend only on spin, sweep and replica).  Returns the
// sweeps done.
static int run_to_target(pbit_ctx *ctx, const Problem &P, const pbit_anneal_desc *d, DevState &ds, hipStream_t st,
                         Key key, uint32_t rq0, int *done_out)
{
    constexpr int kChunk = 32;
    void *state = nullptr, *snap = nullptr, *hitp = nullptr;
    size_t bytes = 0;
    state_span(P, ds, &state, &bytes);
    int rc = scratch(ctx, Slot::Snap, bytes, &snap);
    if (rc == PBIT_OK) rc = scratch(ctx, Slot::Hit, sizeof(int32_t), &hitp);
    if (rc) return rc;
    int32_t *hit_dev = (int32_t *)hitp;
    hipError_t e = fill_i32(hit_dev, 1, INT32_MAX, st);
    if (e != hipSuccess) return device_fail(ctx, e, "target flag");
    int done = 0;
    for (int s0 = 0; s0 < d->n_sweeps;) {
        const int s1 = std::min(d->n_sweeps, s0 + kChunk);
        e = hipMemcpyAsync(snap, state, bytes, hipMemcpyDeviceToDevice, st);
        for (int s = s0; s < s1 && e == hipSuccess; ++s) {
            e = sweeps(ctx, P, ds, s, s + 1, (uint32_t)d->sweep_offset, rq0, key, st);
            if (e == hipSuccess) e = prof_close(ctx, st);
            if (e == hipSuccess) e = energies(P, ds, st);
            if (e == hipSuccess) e = check_target(ds.E32, ds.R, d->target_energy, s + 1, hit_dev, st);
        }
        int32_t hit = INT32_MAX;
        if (e == hipSuccess) e = hipMemcpyAsync(&hit, hit_dev, sizeof hit, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e == hipSuccess) e = prof_harvest(ctx);
        if (e != hipSuccess) return device_fail(ctx, e, "sweeps with a target");
        if (hit != INT32_MAX) {
            // back to the chunk's start, then forward to the first sweep that met the target
            e = hipMemcpyAsync(state, snap, bytes, hipMemcpyDeviceToDevice, st);
            if (e == hipSuccess) e = sweeps(ctx, P, ds, s0, hit, (uint32_t)d->sweep_offset, rq0, key, st);
            if (e != hipSuccess) return device_fail(ctx, e, "target replay");
            done = hit;
            break;
        }
        done = s0 = s1;
    }
    *done_out = done;
    return PBIT_OK;
}

int run_blocking(pbit_ctx *ctx, const Problem &P, const pbit_anneal_desc *d, pbit_result *res)
{
    const hipStream_t st = ctx->stream;
    DevState ds;
    int rc = prepare(ctx, P, d, st, ds, nullptr);
    if (rc) return rc;
    const Key key{(uint32_t)d->seed, (uint32_t)(d->seed >> 32)};
    const uint32_t rq0 = (uint32_t)d->replica_offset >> 2;
    const int check = d->has_target ? (d->trace_every > 0 ? d->trace_every : 1) : d->trace_every;
    std::vector<int32_t> e32;
    int done = 0, trace_len = 0;
    bool hit = false;
    if (d->has_target && d->trace_every == 0) {
        rc = run_to_target(ctx, P, d, ds, st, key, rq0, &done);
        if (rc) return rc;
        hit = true;  // the loop below has nothing left to do
    }
    for (int s = 0; s < d->n_sweeps && !hit;) {
        // up to the next energy check (every sweep on the per-half-sweep path)
        int s1 = ds.slab ? std::min(d->n_sweeps, s + kSlabChunk) : s + 1;
        if (check > 0) s1 = std::min(s1, (s / check + 1) * check);
        hipError_t e = sweeps(ctx, P, ds, s, s1, (uint32_t)d->sweep_offset, rq0, key, st);
        if (e != hipSuccess) return device_fail(ctx, e, "sweep launch");
        s = s1;
        done = s;
        if (check > 0 && done % check == 0) {
            rc = fetch_energies(ctx, P, ds, st, e32);
            if (rc) return rc;
            if (d->trace_every > 0 && done % d->trace_every == 0 && trace_len < res->trace_cap) {
                if (res->energy_trace)
                    for (int r = 0; r < ds.R; ++r) res->energy_trace[(size_t)trace_len * ds.R + r] = e32[r];
                if (res->spin_trace) {
                    void *v = nullptr;
                    rc = scratch(ctx, Slot::Stage, (size_t)ds.R * P.N, &v);
                    if (rc) return rc;
                    e = to_rows(P, ds, (int8_t *)v, st);
                    if (e == hipSuccess)
                        e = hipMemcpyAsync(res->spin_trace + (size_t)trace_len * ds.R * P.N, v, (size_t)ds.R * P.N,
                                           hipMemcpyDeviceToHost, st);
                    if (e == hipSuccess) e = hipStreamSynchronize(st);
                    if (e != hipSuccess) return device_fail(ctx, e, "spin trace");
                }
                ++trace_len;
            }
            if (d->has_target && *std::min_element(e32.begin(), e32.end()) <= d->target_energy) hit = true;
        }
    }
    rc = fetch_energies(ctx, P, ds, st, e32);
    if (rc) return rc;
    if (res->spins) {
        void *v = nullptr;
        rc = scratch(ctx, Slot::Stage, (size_t)ds.R * P.N, &v);
        if (rc) return rc;
        hipError_t e = to_rows(P, ds, (int8_t *)v, st);
        if (e == hipSuccess) e = hipMemcpyAsync(res->spins, v, (size_t)ds.R * P.N, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return device_fail(ctx, e, "spin readback");
    }
    int best = 0;
    for (int r = 0; r < ds.R; ++r) {
        if (res->energies) res->energies[r] = e32[r];
        if (e32[r] < e32[best]) best = r;
    }
    res->best_energy = e32[best];
    res->best_replica = best;
    res->sweeps_done = done;
    res->trace_len = trace_len;
    return PBIT_OK;
}

// The sweep launches of pbit_anneal_dev as one HIP graph (PBIT_GRAPH=1 when the
// context is created): captured from the stream, instantiated and launched.  The
// executable graph is kept and replayed while the next call would capture the
// same launches: same problem, schedule, sweeps, replicas, seed, kernel path and
// device buffers (the sweep kernels take the decision words of the cube and the
// buffer addresses as launch arguments).
static uint64_t launch_key(const Problem &P, const pbit_anneal_desc *d, const DevState &ds, hipStream_t st)
{
    uint64_t h = 1469598103934665603ull;
    auto mix = [&h](const void *p, size_t n) {
        const unsigned char *b = (const unsigned char *)p;
        for (size_t k = 0; k < n; ++k) h = (h ^ b[k]) * 1099511628211ull;
    };
    const void *ptrs[] = {&P, ds.spins, ds.MA, ds.MAb, ds.table, ds.E32, (void *)st};
    mix(ptrs, sizeof ptrs);
    mix(d->beta, sizeof(double) * (size_t)d->n_sweeps);
    const int64_t f[] = {d->n_sweeps, d->sweep_offset, d->n_replicas, d->replica_offset, (int64_t)d->seed,
                         ds.Rp, ds.width, (int64_t)ds.variant, ds.slab, ds.bits, ds.mfma};
    mix(f, sizeof f);
    return h;
}

template <class Loop>
static int graph_sweeps(pbit_ctx *ctx, const Problem &P, const pbit_anneal_desc *d, DevState &ds, hipStream_t st,
                        Loop &loop)
{
    const uint64_t key = launch_key(P, d, ds, st);
    if (!ctx->graph_exec || ctx->graph_key != key) {
        if (ctx->graph_exec) (void)hipGraphExecDestroy((hipGraphExec_t)ctx->graph_exec);
        ctx->graph_exec = nullptr;
        const int prof = ctx->prof_every;
        ctx->prof_every = 0;  // no event records inside the graph
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
        hipError_t el = e == hipSuccess ? loop() : e;
        if (e == hipSuccess) e = hipStreamEndCapture(st, &g);
        ctx->prof_every = prof;
        if (e == hipSuccess) e = el;
        hipGraphExec_t x = nullptr;
        if (e == hipSuccess) e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
        if (g) (void)hipGraphDestroy(g);
        if (e != hipSuccess) return device_fail(ctx, e, "sweep graph capture");
        ctx->graph_exec = x;
        ctx->graph_key = key;
        ++ctx->graph_captures;
    }
    hipError_t e = hipGraphLaunch((hipGraphExec_t)ctx->graph_exec, st);
    if (e != hipSuccess) return device_fail(ctx, e, "sweep graph launch");
    ++ctx->graph_launches;
    return PBIT_OK;
}

int run_device(pbit_ctx *ctx, const Problem &P, const pbit_anneal_desc *d, int8_t *d_spins, bool spins_in,
               int64_t *d_energies, hipStream_t st, Arena *arena)
{
    DevState ds;
    ds.arena = arena;
    int rc = prepare(ctx, P, d, st, ds, spins_in ? d_spins : nullptr);
    if (rc) return rc;
    const Key key{(uint32_t)d->seed, (uint32_t)(d->seed >> 32)};
    const uint32_t rq0 = (uint32_t)d->replica_offset >> 2;
    auto loop = [&]() -> hipError_t {
        for (int s = 0; s < d->n_sweeps;) {
            const int s1 = ds.slab ? std::min(d->n_sweeps, s + kSlabChunk) : s + 1;
            hipError_t e = sweeps(ctx, P, ds, s, s1, (uint32_t)d->sweep_offset, rq0, key, st);
            if (e != hipSuccess) return e;
            s = s1;
        }
        return hipSuccess;
    };
    if (ctx->use_graph && !arena && d->n_sweeps > 0) {
        rc = graph_sweeps(ctx, P, d, ds, st, loop);
        if (rc) return rc;
    } else {
        hipError_t e = loop();
        if (e != hipSuccess) return device_fail(ctx, e, "sweep launch");
    }
    hipError_t e = prof_close(ctx, st);  // a timing window covers sweep launches only
    if (e == hipSuccess) e = to_rows(P, ds, d_spins, st);
    if (e == hipSuccess && d_energies) {
        e = energies(P, ds, st);
        if (e == hipSuccess) e = widen_i32_i64(ds.E32, d_energies, ds.R, st);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e == hipSuccess) e = prof_harvest(ctx);
    if (e != hipSuccess) return device_fail(ctx, e, "anneal (device buffers)");
    return PBIT_OK;
}

// Device bytes the buffers of pbit_anneal_dev take for this request (an upper
// bound: each buffer is counted with its 256-byte alignment).
size_t anneal_dev_bytes(const pbit_ctx *ctx, const Problem &P, const pbit_anneal_desc *d)
{
    const size_t R = (size_t)d->n_replicas;
    size_t spins, Rp;
    if (P.kind == PBIT_BICLIQUE) {
        const bool bits = ctx->bq_forced == BqVariant::Bits && P.bq.Jb;
        Rp = (R + (bits ? 255 : kBqRPad - 1)) / (bits ? 256 : kBqRPad) * (bits ? 256 : kBqRPad);
        const size_t ab = Rp * (size_t)(P.bq.na_p + P.bq.nb_p);
        spins = ab + (bqb_supported(P.bq, (int)Rp) ? ab / 8 + 256 : 0);
    } else {
        Rp = (R + kEaMfmaRPad - 1) / kEaMfmaRPad * kEaMfmaRPad;  // the larger of the cube paths' paddings
        spins = (size_t)P.N * Rp;
    }
    const int width = d->n_sweeps > 0 ? table_width(d->beta, d->n_sweeps, P.amax) : 1;
    const size_t table = sizeof(uint32_t) * (size_t)std::max(d->n_sweeps, 1) * (size_t)width;
    return spins + 256 + sizeof(int32_t) * Rp + 256 + table + 256;
}

}  // namespace pbit

extern "C" int pbit_anneal(pbit_ctx *ctx, uint64_t problem, const pbit_anneal_desc *desc, pbit_result *result)
{
    try {
        PBIT_ENTER(ctx);
        int rc = check_desc(desc, "pbit_anneal");
        if (rc) return rc;
        if (!result) return fail(PBIT_E_ARG, "pbit_anneal: result is NULL");
        Problem *P = find_problem(ctx, problem);
        if (!P) return fail(PBIT_E_HANDLE, "pbit_anneal: unknown problem handle");
        if (result->trace_cap < 0) return fail(PBIT_E_ARG, "pbit_anneal: trace_cap must be >= 0");
        if (desc->init_spins && !spins_in_range(desc->init_spins, (size_t)desc->n_replicas * P->N))
            return fail(PBIT_E_RANGE, "pbit_anneal: init_spins must be +-1");
        return run_blocking(ctx, *P, desc, result);
    } catch (const std::bad_alloc &) {
        return fail(PBIT_E_NOMEM, "pbit_anneal: host allocation failed");
    } catch (...) {
        return fail(PBIT_E_ARG, "pbit_anneal: internal error");
    }
}

extern "C" int pbit_anneal_dev(pbit_ctx *ctx, uint64_t problem, const pbit_anneal_desc *desc, void *d_spins,
                               int32_t spins_in, void *d_energies, void *hip_stream)
{
    try {
        PBIT_ENTER(ctx);
        int rc = check_desc(desc, "pbit_anneal_dev");
        if (rc) return rc;
        if (!d_spins) return fail(PBIT_E_ARG, "pbit_anneal_dev: d_spins is NULL");
        if (desc->init_spins) return fail(PBIT_E_ARG, "pbit_anneal_dev: pass initial spins in d_spins (spins_in)");
        if (desc->trace_every || desc->has_target)
            return fail(PBIT_E_ARG, "pbit_anneal_dev: traces and targets need pbit_anneal");
        Problem *P = find_problem(ctx, problem);
        if (!P) return fail(PBIT_E_HANDLE, "pbit_anneal_dev: unknown problem handle");
        hipStream_t st = hip_stream ? (hipStream_t)hip_stream : ctx->stream;
        return run_device(ctx, *P, desc, (int8_t *)d_spins, spins_in != 0, (int64_t *)d_energies, st, nullptr);
    } catch (const std::bad_alloc &) {
        return fail(PBIT_E_NOMEM, "pbit_anneal_dev: host allocation failed");
    } catch (...) {
        return fail(PBIT_E_ARG, "pbit_anneal_dev: internal error");
    }
}

extern "C" int pbit_energy(pbit_ctx *ctx, uint64_t problem, const int8_t *spins, int32_t R, int64_t *out)
{
    try {
        PBIT_ENTER(ctx);
        if (!spins || !out || R < 1) return fail(PBIT_E_ARG, "pbit_energy: bad arguments");
        Problem *P = find_problem(ctx, problem);
        if (!P) return fail(PBIT_E_HANDLE, "pbit_energy: unknown problem handle");
        if (!spins_in_range(spins, (size_t)R * P->N)) return fail(PBIT_E_RANGE, "pbit_energy: spins must be +-1");
        pbit_anneal_desc d{};
        d.n_replicas = R;
        d.init_spins = spins;
        DevState ds;
        int rc = prepare(ctx, *P, &d, ctx->stream, ds, nullptr);
        if (rc) return rc;
        std::vector<int32_t> e32;
        rc = fetch_energies(ctx, *P, ds, ctx->stream, e32);
        if (rc) return rc;
        for (int r = 0; r < R; ++r) out[r] = e32[r];
        return PBIT_OK;
    } catch (const std::bad_alloc &) {
        return fail(PBIT_E_NOMEM, "pbit_energy: host allocation failed");
    } catch (...) {
        return fail(PBIT_E_ARG, "pbit_energy: internal error");
    }
}

// ---------------------------------------------------------------- profiling

namespace pbit {

// A window of up to kProfWindow consecutive half-sweep launches is bracketed by
// one pair of events, so that the events' own cost is shared by the window.
constexpr int kProfWindow = 8;

hipError_t prof_begin(pbit_ctx *ctx, int kind, hipStream_t st)
{
    const size_t need = ctx->prof_used + 2;
    while (ctx->prof_pool.size() < need) {
        hipEvent_t ev;
        hipError_t e = hipEventCreate(&ev);
        if (e != hipSuccess) return e;
        ctx->prof_pool.push_back(ev);
    }
    const int k = (int)ctx->prof_used;
    ctx->prof_used += 2;
    ctx->prof_kind.push_back(kind);
    ctx->prof_launches.push_back(0);
    ctx->prof_open = k;
    return hipEventRecord(ctx->prof_pool[k], st);
}

hipError_t prof_count_launch(pbit_ctx *ctx, hipStream_t st)
{
    if (ctx->prof_open < 0) return hipSuccess;
    const int w = std::min(kProfWindow, ctx->prof_every);
    if (++ctx->prof_launches.back() < w) return hipSuccess;
    const int k = ctx->prof_open;
    ctx->prof_open = -1;
    return hipEventRecord(ctx->prof_pool[k + 1], st);
}

hipError_t prof_close(pbit_ctx *ctx, hipStream_t st)
{
    if (ctx->prof_open < 0) return hipSuccess;
    const int k = ctx->prof_open;
    ctx->prof_open = -1;
    return hipEventRecord(ctx->prof_pool[k + 1], st);
}

hipError_t prof_harvest(pbit_ctx *ctx)
{
    for (size_t k = 0; k < ctx->prof_kind.size(); ++k) {
        float ms = 0.f;
        hipError_t e = hipEventElapsedTime(&ms, ctx->prof_pool[2 * k], ctx->prof_pool[2 * k + 1]);
        if (e != hipSuccess) return e;
        const int kind = ctx->prof_kind[k];
        ctx->prof_ms[kind] += ms;
        ctx->prof_count[kind] += ctx->prof_launches[k];
    }
    ctx->prof_kind.clear();
    ctx->prof_launches.clear();
    ctx->prof_used = 0;
    return hipSuccess;
}

void prof_release(pbit_ctx *ctx)
{
    for (hipEvent_t ev : ctx->prof_pool) (void)hipEventDestroy(ev);
    ctx->prof_pool.clear();
    ctx->prof_kind.clear();
    ctx->prof_launches.clear();
    ctx->prof_used = 0;
    ctx->prof_open = -1;
}

}  // namespace pbit

extern "C" int pbit_profile_enable(pbit_ctx *ctx, int32_t every)
{
    PBIT_ENTER(ctx);
    if (every < 0) return fail(PBIT_E_ARG, "pbit_profile_enable: every must be >= 0");
    ctx->prof_every = every;
    return PBIT_OK;
}

extern "C" int pbit_profile_variant(pbit_ctx *ctx, int32_t *variant)
{
    PBIT_ENTER(ctx);
    if (!variant) return fail(PBIT_E_ARG, "pbit_profile_variant: variant is NULL");
    *variant = ctx->bq_last_variant;
    return PBIT_OK;
}

extern "C" int pbit_profile_graph(pbit_ctx *ctx, int64_t *captures, int64_t *launches)
{
    PBIT_ENTER(ctx);
    if (captures) *captures = ctx->graph_captures;
    if (launches) *launches = ctx->graph_launches;
    return PBIT_OK;
}

extern "C" int pbit_profile_ea_path(pbit_ctx *ctx, int32_t *path)
{
    PBIT_ENTER(ctx);
    if (!path) return fail(PBIT_E_ARG, "pbit_profile_ea_path: path is NULL");
    *path = ctx->ea_last_path;
    return PBIT_OK;
}

extern "C" int pbit_profile_graph_path(pbit_ctx *ctx, int32_t *path)
{
    PBIT_ENTER(ctx);
    if (!path) return fail(PBIT_E_ARG, "pbit_profile_graph_path: path is NULL");
    *path = ctx->graph_last_path;
    return PBIT_OK;
}

extern "C" int pbit_profile_read(pbit_ctx *ctx, int32_t kind, double *total_ms, int64_t *launches, int32_t reset)
{
    PBIT_ENTER(ctx);
    if (kind != PBIT_EA3D && kind != PBIT_BICLIQUE && kind != PBIT_GRAPH)
        return fail(PBIT_E_ARG, "pbit_profile_read: unknown kind %d", kind);
    const int k = kind;
    if (total_ms) *total_ms = ctx->prof_ms[k];
    if (launches) *launches = ctx->prof_count[k];
    if (reset) {
        ctx->prof_ms[k] = 0;
        ctx->prof_count[k] = 0;
    }
    return PBIT_OK;
}
