// graph_kernels.hip — general sparse graphs with k update groups (paper Sec. 1.2.2
// greedy colouring; Sec. 4.2 general QUBOs; odd cubes need more than two groups).
//
// Spins use the cube's layout, int8 [N][Rp] with replicas fastest, and one
// launch updates one colour class: a thread takes one site of the class and 16
// replicas, gathers its neighbours' 16-byte replica rows through the class-major
// adjacency, and counts negative products bytewise (degree <= 127 keeps the byte
// sums below 256).  Classes are visited in ascending colour order.
//
// The sweep of a sparse graph is bound by the latency of its gathers, so the
// adjacency is laid out for few dependent loads: the site's record (id,
// adjacency range, field base) is one 16-byte load, every adjacency entry one
// word (neighbour and coupling code), and the rows of four neighbours are in
// flight at once.  With at least 8 chunks of 16 replicas, blockIdx.x mod 8 (the
// XCD a workgroup is dispatched to) picks one replica slab, so that an XCD's L2
// holds its slab of every row and the neighbours a class shares are fetched
// there once.
#include "device.h"
#include "internal.h"

namespace pbit {

namespace {

constexpr int kThreads = 256;
constexpr int kMaxOff = kGraphMaxDegree + 1;          // |I| <= degree + |h|
constexpr int kSlots = 2 * kMaxOff + 1;

// Decision: the table holds, for every field value I, the 64-bit word S(I) = Tm
// for I >= 0 and 2^32 - Tm for I < 0; the new spin is -1 exactly when w + S(I)
// carries into bit 32 (the heat-bath rule with the uniform word w), one
// v_mad_u64_u32 per update (`one` is 1, passed in so that the multiply-add is
// kept as that instruction).
__global__ __launch_bounds__(kThreads) void k_graph_halfsweep(int8_t *__restrict__ spins,
                                                              const int4 *__restrict__ meta, uint32_t n_class,
                                                              const uint32_t *__restrict__ adj,
                                                              const uint32_t *__restrict__ trow, int width, int Rp,
                                                              int lg_nsl, uint32_t sweep, uint32_t rq0, uint32_t k0,
                                                              uint32_t k1, uint32_t one)
{
    const uint32_t cs = (uint32_t)(Rp / 16) >> lg_nsl;  // chunks of 16 replicas per slab
    const uint32_t slab = blockIdx.x & ((1u << lg_nsl) - 1u);
    const uint32_t gid = (blockIdx.x >> lg_nsl) * kThreads + threadIdx.x;  // (site, chunk) inside the slab
    const bool live = gid < n_class * cs;
    const uint32_t j = gid / cs;
    // the site record first, so that its latency overlaps the table build
    int4 m = make_int4(0, 0, 0, 0);  // site, first entry, end entry, base = nnz + h
    if (live) m = meta[j];
    // decision words by descending field value: entry k is S(I) for I = kMaxOff - k
    __shared__ uint64_t tab[kSlots];
    for (int k = threadIdx.x; k < kSlots; k += kThreads) {
        const int I = kMaxOff - k;
        const uint32_t T = trow[min(I >= 0 ? I : -I, width - 1)];
        tab[k] = I >= 0 ? (uint64_t)T : ((uint64_t)1 << 32) - T;
    }
    __syncthreads();
    if (!live) return;
    const uint32_t q = slab * cs + (gid - j * cs);
    const int i = m.x;
    const int last = m.z - 1;
    uint32_t cnt[4] = {0u, 0u, 0u, 0u};
    for (int e = m.y; e <= last; e += 4) {
        // four entries, then their four rows; an entry past the end repeats the last one
        // with its coupling code cleared, so it adds nothing and every load is in range
        uint32_t w[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const uint32_t x = adj[min(e + k, last)];
            w[k] = e + k <= last ? x : x & ~3u;
        }
        uint4 v[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) v[k] = *reinterpret_cast<const uint4 *>(spins + (size_t)(w[k] >> 2) * Rp + 16 * q);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            // 0x02 in every byte where J != 0 (keep) and where J = -1 (flip)
            const uint32_t keep = (uint32_t)((int32_t)(w[k] << 31) >> 31) & 0x02020202u;
            const uint32_t flip = (uint32_t)((int32_t)(w[k] << 30) >> 31) & 0x02020202u;
            cnt[0] += (v[k].x & keep) ^ flip;
            cnt[1] += (v[k].y & keep) ^ flip;
            cnt[2] += (v[k].z & keep) ^ flip;
            cnt[3] += (v[k].w & keep) ^ flip;
        }
    }
    // a byte c of cnt (two per negative product) gives I = base - c: table entry
    // kMaxOff - base + c
    const char *tb = reinterpret_cast<const char *>(tab) + 8 * (kMaxOff - m.w);
    uint32_t out[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const Block4 b = philox((uint32_t)i, sweep, rq0 + 4u * q + (uint32_t)k, kDomainSweep, k0, k1);
        uint32_t sgn[4];  // 1: the replica's new spin is -1
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            const uint32_t c = (cnt[k] >> (8 * p)) & 0xFFu;
            const uint64_t S = *static_cast<const uint64_t *>(__builtin_assume_aligned(tb + 8 * c, 8));
            sgn[p] = (uint32_t)(((uint64_t)b.w[p] * one + S) >> 32);
        }
        // gather the four low bytes, then map 0 -> 0x01 and 1 -> 0xFF
        const uint32_t lo = __builtin_amdgcn_perm(sgn[1], sgn[0], 0x0C0C0400u);
        const uint32_t hi = __builtin_amdgcn_perm(sgn[3], sgn[2], 0x0C0C0400u);
        out[k] = __builtin_amdgcn_perm(0u, 0xFF01u, __builtin_amdgcn_perm(hi, lo, 0x05040100u));
    }
    *reinterpret_cast<uint4 *>(spins + (size_t)i * Rp + 16 * q) = make_uint4(out[0], out[1], out[2], out[3]);
}

// E[r] += -sum over a chunk of bonds of J m_i m_j, plus -h_i m_i for a chunk of sites
__global__ __launch_bounds__(kThreads) void k_graph_energy(const int8_t *__restrict__ spins,
                                                           const int32_t *__restrict__ bi,
                                                           const int32_t *__restrict__ bj,
                                                           const int8_t *__restrict__ bJ, int n_bonds,
                                                           const int8_t *__restrict__ h, int n, int Rp, int R,
                                                           int chunk, int32_t *__restrict__ E)
{
    const int r = blockIdx.x * kThreads + threadIdx.x;
    if (r >= R) return;
    const int64_t b0 = (int64_t)blockIdx.y * chunk;
    int32_t e = 0;
    for (int64_t b = b0; b < b0 + chunk && b < n_bonds; ++b)
        e -= bJ[b] * spins[(size_t)bi[b] * Rp + r] * spins[(size_t)bj[b] * Rp + r];
    if (h)
        for (int64_t i = b0; i < b0 + chunk && i < n; ++i) e -= h[i] * spins[(size_t)i * Rp + r];
    atomicAdd(E + r, e);
}

}  // namespace

hipError_t graph_halfsweep(const GraphView &g, int colour, int8_t *spins, int Rp, const uint32_t *trow, int width,
                           uint32_t sweep, uint32_t rq0, Key key, hipStream_t st)
{
    if (width < 1 || width > kMaxOff + 1 || Rp % 16 != 0) return hipErrorInvalidValue;
    const int n_class = g.class_start[colour + 1] - g.class_start[colour];
    if (n_class == 0) return hipSuccess;
    const int chunks = Rp / 16;
    const int lg_nsl = chunks % 8 == 0 ? 3 : 0;  // 8 replica slabs, one per XCD
    const int64_t work = (int64_t)n_class * (chunks >> lg_nsl);
    if (work > 0xFFFFFF00LL) return hipErrorInvalidValue;  // 32-bit thread indices
    const int64_t blocks = ((work + kThreads - 1) / kThreads) << lg_nsl;
    hipLaunchKernelGGL(k_graph_halfsweep, dim3((unsigned)blocks), dim3(kThreads), 0, st, spins,
                       reinterpret_cast<const int4 *>(g.site_meta) + g.class_start[colour], (uint32_t)n_class, g.adj,
                       trow, width, Rp, lg_nsl, sweep, rq0, key.k0, key.k1, 1u);
    return hipGetLastError();
}

hipError_t graph_energy(const GraphView &g, const int8_t *spins, int Rp, int R, int32_t *E, hipStream_t st)
{
    hipError_t e = fill_i32(E, R, 0, st);
    if (e != hipSuccess) return e;
    const int64_t items = g.n_bonds > g.n ? g.n_bonds : g.n;
    const int chunk = (int)((items + 65534) / 65535 > 256 ? (items + 65534) / 65535 : 256);
    dim3 grid((unsigned)((R + kThreads - 1) / kThreads), (unsigned)((items + chunk - 1) / chunk));
    hipLaunchKernelGGL(k_graph_energy, grid, dim3(kThreads), 0, st, spins, g.bi, g.bj, g.bJ, g.n_bonds, g.h, g.n,
                       Rp, R, chunk, E);
    return hipGetLastError();
}

}  // namespace pbit
