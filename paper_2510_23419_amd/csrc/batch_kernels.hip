// batch_kernels.hip — persistent batched sweep for many independent jobs.
//
// Each workgroup repeatedly takes a work item (job, replica tile, sweep range)
// from a device queue and runs it with the tile's spins held in LDS, so the
// half-sweeps of a tile need only workgroup barriers, never a grid-wide one:
// replicas are independent runs (paper Sec. 1.3.3), and inside a tile the two
// update groups alternate (Sec. 1.2.2).  Jobs of uneven sizes therefore share
// one launch.  The arithmetic, the Philox counters and the decision rule are
// the same as in the per-instance kernels, so a job's result does not depend on
// which items it was batched with.
#include <type_traits>

#include "batch.h"
#include "device.h"
#include "bq.h"

namespace pbit {

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

typedef unsigned v2u __attribute__((ext_vector_type(2)));
typedef unsigned v4u __attribute__((ext_vector_type(4)));

// 8- and 16-byte global loads (vector types: uint2 and uint4 do not bind to an
// address-space-qualified reference)
__device__ __forceinline__ uint2 load_u2(const void *p)
{
    const v2u v = load_global<v2u>(p);
    return make_uint2(v.x, v.y);
}
__device__ __forceinline__ uint4 load_u4(const void *p)
{
    const v4u v = load_global<v4u>(p);
    return make_uint4(v.x, v.y, v.z, v.w);
}

__device__ __forceinline__ int take_item(int32_t *counter, int *slot)
{
    if (threadIdx.x == 0) *slot = atomicAdd(counter, 1);
    __syncthreads();
    const int it = __builtin_amdgcn_readfirstlane(*slot);
    __syncthreads();
    return it;
}

// ---------------------------------------------------------------- cube tiles

constexpr int kFieldOff = 7;
constexpr int kFieldSlots = 2 * kFieldOff + 1;

__device__ __forceinline__ uint32_t neg2(uint32_t m, uint32_t keep, uint32_t flip) { return (m & keep) ^ flip; }

// Sign mask of bit k of c: 0 or 0xFFFFFFFF.
__device__ __forceinline__ uint32_t bit_mask(uint32_t c, int k) { return (uint32_t)((int32_t)(c << (31 - k)) >> 31); }

// Cube tiles: the spins of 4W replicas (W = 1, 2 or 4) of the whole lattice live in
// LDS as W dwords per site (byte p of dword k = replica 4k + p, +1 = 0x01, -1 = 0xFF;
// for W = 4 the layout of the per-instance LDS-resident cube kernel), and the
// problem's site list gives each class position's site index, wrap flags and code,
// so that one site's addresses and code serve 4W updates.  The field and the
// decision use the cube stencil's arithmetic: bit 4 of a spin byte marks -1, one
// bitop3 per neighbour gives 0x10 per byte where J m = +1, and the sum with the
// site's base byte is 8 (I + 7), the LDS byte offset of the word S(I) (Tm for
// I >= 0, 2^32 - Tm for I < 0) whose sum with the random word carries into bit 32
// exactly when the new spin is -1.  `one` is 1 (passed in so that w * one + S is a
// single v_mad_u64_u32).
template <int W, int TPB>
__device__ __forceinline__ void ea_tile_item(const WorkItem &w, const EaJobDev &jb, uint4 *tile_rows,
                                             uint64_t *stab, int32_t *eacc, uint32_t one)
{
    typedef uint32_t V __attribute__((ext_vector_type(W)));
    constexpr int RS = 4 * W;  // replicas in the tile
    V *rows = reinterpret_cast<V *>(tile_rows);  // [N]: the tile's replicas of every site
    const int tid = threadIdx.x;
    const char *tb = reinterpret_cast<const char *>(stab);
    const int Lx = jb.Lx, Ly = jb.Ly, Lz = jb.Lz;
    const int plane = Lx * Ly, N = plane * Lz, half = N / 2;
    const uint32_t rgw = jb.rq0 + (uint32_t)W * (uint32_t)w.tile;  // Philox counter word 2 of the tile's first group
    V *gst = reinterpret_cast<V *>(jb.state) + (size_t)w.tile * N;
    // neighbour d of site i: i + step[d], or i + step[d] + fix[d] across the boundary
    const int step[6] = {1, -1, Lx, -Lx, plane, -plane};
    const int fix[6] = {-Lx, Lx, -plane, plane, -N, N};

    if (w.init) {
        for (int i = tid; i < N; i += TPB) {
            V d;
#pragma unroll
            for (int k = 0; k < W; ++k) {
                const Block4 b = philox((uint32_t)i, 0u, rgw + (uint32_t)k, kDomainInit, jb.k0, jb.k1);
                uint32_t packed = 0;
#pragma unroll
                for (int p = 0; p < 4; ++p) packed |= (uint32_t)(uint8_t)init_spin(b.w[p]) << (8 * p);
                d[k] = packed;
            }
            rows[i] = d;
        }
    } else {
        for (int i = tid; i < N; i += TPB) rows[i] = load_global<V>(gst + i);
    }

    for (int s = w.s_begin; s < w.s_end; ++s) {
        __syncthreads();
        if (tid < kFieldSlots) {
            const uint32_t *trow = jb.table + (size_t)s * jb.width;
            const int I = tid - kFieldOff;
            const uint32_t T = load_global<uint32_t>(trow + min(I >= 0 ? I : -I, jb.width - 1));
            stab[tid] = I >= 0 ? (uint64_t)T : ((uint64_t)1 << 32) - T;
        }
        __syncthreads();
        const uint32_t t = jb.sweep0 + (uint32_t)s;
        auto half_sweep = [&](int c, auto dense_tag) {
            constexpr bool DENSE = decltype(dense_tag)::value;
            for (int j = tid; j < half; j += TPB) {
                const uint2 e = load_u2(jb.sites + (size_t)c * half + j);
                const int i = (int)(e.x & 0xFFFFu);
                const uint32_t wrap = e.x >> 16, code = e.y;
                V v[6];
#pragma unroll
                for (int d = 0; d < 6; ++d) v[d] = rows[i + step[d] + (((wrap >> d) & 1u) ? fix[d] : 0)];
                Block4 b[W];
#pragma unroll
                for (int r = 0; r < W; ++r)
                    b[r] = philox((uint32_t)i, t, rgw + (uint32_t)r, kDomainSweep, jb.k0, jb.k1);
                uint32_t tt[6][W];
#pragma unroll
                for (int d = 0; d < 6; ++d) {
                    const uint32_t F = bit_mask(code, kCodeFlipShift + d);
                    const uint32_t K = DENSE ? 0x10101010u : (bit_mask(code, d) & 0x10101010u);
#pragma unroll
                    for (int r = 0; r < W; ++r) tt[d][r] = __builtin_amdgcn_bitop3_b32(v[d][r], F, K, 0x82);
                }
                const uint32_t pos8 = __builtin_amdgcn_perm(0u, code, 0x03030303u);  // base byte in every byte
                V out;
#pragma unroll
                for (int r = 0; r < W; ++r) {
                    const uint32_t idx =
                        (tt[0][r] + tt[1][r] + tt[2][r]) + (tt[3][r] + tt[4][r] + tt[5][r]) + pos8;
                    uint32_t sgn[4];  // 1: the replica's new spin is -1
#pragma unroll
                    for (int p = 0; p < 4; ++p) {
                        const uint64_t S = *static_cast<const uint64_t *>(
                            __builtin_assume_aligned(tb + ((idx >> (8 * p)) & 0xFFu), 8));
                        sgn[p] = (uint32_t)(((uint64_t)b[r].w[p] * one + S) >> 32);
                    }
                    const uint32_t lo = __builtin_amdgcn_perm(sgn[1], sgn[0], 0x0C0C0400u);
                    const uint32_t hi = __builtin_amdgcn_perm(sgn[3], sgn[2], 0x0C0C0400u);
                    out[r] = __builtin_amdgcn_perm(0u, 0xFF01u, __builtin_amdgcn_perm(hi, lo, 0x05040100u));
                }
                rows[i] = out;
            }
        };
        for (int c = 0; c < 2; ++c) {
            if (jb.dense)
                half_sweep(c, std::true_type{});
            else
                half_sweep(c, std::false_type{});
            __syncthreads();
        }
    }

    // energies of the tile's replicas: every bond has exactly one end of colour 1 (the
    // second half of the site list), so E = -sum_{i in colour 1} m_i sum_j J_ij m_j
    // - sum_i h_i m_i
    if (tid < RS) eacc[tid] = 0;
    __syncthreads();
    int32_t er[RS];
#pragma unroll
    for (int r = 0; r < RS; ++r) er[r] = 0;
    for (int j = tid; j < N; j += TPB) {
        const int c = j < half ? 0 : 1;
        const uint2 e = load_u2(jb.sites + j);  // colour 0 first, then colour 1
        const int i = (int)(e.x & 0xFFFFu);
        const uint32_t wrap = e.x >> 16, code = e.y;
        const int nnz = __builtin_popcount(code & 63u);
        const int hv = (int)(int8_t)(code >> kCodeBaseShift) - nnz;
        const V mi = rows[i];
        uint32_t cnt[W];
#pragma unroll
        for (int k = 0; k < W; ++k) cnt[k] = 0u;
        if (c == 1) {
#pragma unroll
            for (int d = 0; d < 6; ++d) {
                const V v = rows[i + step[d] + (((wrap >> d) & 1u) ? fix[d] : 0)];
                const uint32_t keep = ((code >> d) & 1u) * 0x02020202u;
                const uint32_t flip = ((code >> (kCodeFlipShift + d)) & 1u) * 0x02020202u;
#pragma unroll
                for (int k = 0; k < W; ++k) cnt[k] += neg2(v[k], keep, flip);
            }
        }
#pragma unroll
        for (int k = 0; k < W; ++k)
#pragma unroll
            for (int p = 0; p < 4; ++p) {
                const int m = (int)(int8_t)(mi[k] >> (8 * p));
                const int bonds = c == 1 ? nnz - (int)((cnt[k] >> (8 * p)) & 0xFFu) : 0;
                er[4 * k + p] -= m * (bonds + hv);
            }
    }
#pragma unroll
    for (int r = 0; r < RS; ++r) {
        int v = er[r];
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        if ((tid & 63) == 0) atomicAdd(&eacc[r], v);
    }
    __syncthreads();
    if (tid < RS) jb.energy[RS * w.tile + tid] = eacc[tid];
    for (int i = tid; i < N; i += TPB) gst[i] = rows[i];
}

// Persistent cube-tile kernel: items of any tile width share the launch.  TPB is
// 512, or 1024 for tiles whose LDS rows leave room for one workgroup per CU only
// (four waves per SIMD instead of two).
template <int TPB>
__global__ __launch_bounds__(TPB) void k_ea_tiles(const EaJobDev *__restrict__ jobs,
                                                  const WorkItem *__restrict__ items,
                                                  const int32_t *__restrict__ n_items_p,
                                                  int32_t *__restrict__ counter, uint32_t one)
{
    extern __shared__ uint4 tile_rows[];
    __shared__ uint64_t stab[kFieldSlots];
    __shared__ int32_t eacc[16];
    __shared__ int slot;
    const int n_items = *n_items_p;
    for (;;) {
        const int it = take_item(counter, &slot);
        if (it >= n_items) break;
        const WorkItem w = items[it];
        const EaJobDev jb = jobs[w.job];
        if (jb.rs == 16)
            ea_tile_item<4, TPB>(w, jb, tile_rows, stab, eacc, one);
        else if (jb.rs == 8)
            ea_tile_item<2, TPB>(w, jb, tile_rows, stab, eacc, one);
        else
            ea_tile_item<1, TPB>(w, jb, tile_rows, stab, eacc, one);
        __syncthreads();  // the next item's first LDS writes wait for this item's last reads
    }
}

// ---------------------------------------------------------------- graph tiles

// General graphs with k update groups (Sec. 1.2.2): the spins of 4W replicas of
// the whole graph live in LDS as W dwords per site, in the layout of the cube
// tiles (byte p of dword k = replica 4k + p, +1 = 0x01, -1 = 0xFF).  The classes
// are swept in ascending colour order with a workgroup barrier between them; a
// thread takes one site of the class at a time, reads its record and adjacency
// words from global memory (class-major, as for the per-instance sweep) and its
// neighbours' rows from LDS, and counts negative products bytewise exactly as
// the per-instance kernel does (0x02 per negative product, degree <= 127), so
// that the field, the Philox counters and the carry decision are the same.
constexpr int kGraphOff = kGraphMaxDegree + 1;  // |I| <= degree + |h|
constexpr int kGraphSlots = 2 * kGraphOff + 1;

template <int W>
__device__ __forceinline__ void graph_tile_item(const WorkItem &w, const GraphJobDev &jb, uint4 *tile_rows,
                                                uint64_t *gtab, int32_t *eacc, uint32_t one)
{
    typedef uint32_t V __attribute__((ext_vector_type(W)));
    constexpr int RS = 4 * W;
    V *rows = reinterpret_cast<V *>(tile_rows);  // [n]
    const int tid = threadIdx.x;
    const int n = jb.n;
    const uint32_t rgw = jb.rq0 + (uint32_t)W * (uint32_t)w.tile;  // Philox counter word 2 of the tile's first group
    // the tile's rows: contiguous (batch state) or strided columns of the per-instance spins
    const size_t rstride = jb.row_stride ? (size_t)jb.row_stride : (size_t)RS;
    int8_t *gst = jb.state + (size_t)w.tile * (jb.row_stride ? (size_t)RS : (size_t)n * RS);

    if (w.init) {
        for (int i = tid; i < n; i += kGraphTileThreads) {
            V d;
#pragma unroll
            for (int k = 0; k < W; ++k) {
                const Block4 b = philox((uint32_t)i, 0u, rgw + (uint32_t)k, kDomainInit, jb.k0, jb.k1);
                uint32_t packed = 0;
#pragma unroll
                for (int p = 0; p < 4; ++p) packed |= (uint32_t)(uint8_t)init_spin(b.w[p]) << (8 * p);
                d[k] = packed;
            }
            rows[i] = d;
        }
    } else {
        for (int i = tid; i < n; i += kGraphTileThreads) rows[i] = load_global<V>(gst + rstride * i);
    }

    for (int s = w.s_begin; s < w.s_end; ++s) {
        __syncthreads();
        // decision words by descending field value: entry k is S(I) for I = kGraphOff - k
        const uint32_t *trow = jb.table + (size_t)s * jb.width;
        for (int k = tid; k < kGraphSlots; k += kGraphTileThreads) {
            const int I = kGraphOff - k;
            const uint32_t T = load_global<uint32_t>(trow + min(I >= 0 ? I : -I, jb.width - 1));
            gtab[k] = I >= 0 ? (uint64_t)T : ((uint64_t)1 << 32) - T;
        }
        __syncthreads();
        const uint32_t t = jb.sweep0 + (uint32_t)s;
        for (int c = 0; c < jb.n_colours; ++c) {
            const int p0 = load_global<int32_t>(jb.class_start + c), p1 = load_global<int32_t>(jb.class_start + c + 1);
            for (int j = p0 + tid; j < p1; j += kGraphTileThreads) {
                const v4i mv = load_global<v4i>(jb.meta + j);  // site, first entry, end entry, nnz + h
                const int4 m = make_int4(mv[0], mv[1], mv[2], mv[3]);
                const int i = m.x;
                uint32_t cnt[W];
#pragma unroll
                for (int k = 0; k < W; ++k) cnt[k] = 0u;
                // four adjacency entries, then their four rows, in flight together; an entry
                // past the end reads as 0 (row 0, no coupling), so it adds nothing
                for (int e = m.y; e < m.z; e += 4) {
                    uint32_t a[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) a[u] = e + u < m.z ? load_global<uint32_t>(jb.adj + e + u) : 0u;
                    V v[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) v[u] = rows[a[u] >> 2];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        // 0x02 in every byte where J != 0 (keep) and where J = -1 (flip)
                        const uint32_t keep = (uint32_t)((int32_t)(a[u] << 31) >> 31) & 0x02020202u;
                        const uint32_t flip = (uint32_t)((int32_t)(a[u] << 30) >> 31) & 0x02020202u;
#pragma unroll
                        for (int k = 0; k < W; ++k) cnt[k] += neg2(v[u][k], keep, flip);
                    }
                }
                // a byte c of cnt (two per negative product) gives I = base - c: entry kGraphOff - base + c
                const char *tb = reinterpret_cast<const char *>(gtab) + 8 * (kGraphOff - m.w);
                V out;
#pragma unroll
                for (int k = 0; k < W; ++k) {
                    const Block4 b = philox((uint32_t)i, t, rgw + (uint32_t)k, kDomainSweep, jb.k0, jb.k1);
                    uint32_t sgn[4];  // 1: the replica's new spin is -1
#pragma unroll
                    for (int p = 0; p < 4; ++p) {
                        const uint32_t cb = (cnt[k] >> (8 * p)) & 0xFFu;
                        const uint64_t S = *static_cast<const uint64_t *>(__builtin_assume_aligned(tb + 8 * cb, 8));
                        sgn[p] = (uint32_t)(((uint64_t)b.w[p] * one + S) >> 32);
                    }
                    const uint32_t lo = __builtin_amdgcn_perm(sgn[1], sgn[0], 0x0C0C0400u);
                    const uint32_t hi = __builtin_amdgcn_perm(sgn[3], sgn[2], 0x0C0C0400u);
                    out[k] = __builtin_amdgcn_perm(0u, 0xFF01u, __builtin_amdgcn_perm(hi, lo, 0x05040100u));
                }
                rows[i] = out;
            }
            __syncthreads();
        }
    }

    // energies from scratch: E = -sum_bonds J m_i m_j - sum_i h_i m_i; a product is -1
    // where the two bytes differ (bit 1 of their xor)
    if (tid < RS) eacc[tid] = 0;
    __syncthreads();
    int32_t er[RS];
#pragma unroll
    for (int r = 0; r < RS; ++r) er[r] = 0;
    for (int b = tid; b < jb.n_bonds; b += kGraphTileThreads) {
        const int J = load_global<int8_t>(jb.bJ + b);
        if (J == 0) continue;
        const V mi = rows[load_global<int32_t>(jb.bi + b)], mj = rows[load_global<int32_t>(jb.bj + b)];
#pragma unroll
        for (int k = 0; k < W; ++k) {
            const uint32_t d = ((mi[k] ^ mj[k]) >> 1) & 0x01010101u;
#pragma unroll
            for (int p = 0; p < 4; ++p) er[4 * k + p] -= J * (1 - 2 * (int)((d >> (8 * p)) & 1u));
        }
    }
    if (jb.h)
        for (int i = tid; i < n; i += kGraphTileThreads) {
            const int hv = load_global<int8_t>(jb.h + i);
            if (hv == 0) continue;
            const V mi = rows[i];
#pragma unroll
            for (int k = 0; k < W; ++k)
#pragma unroll
                for (int p = 0; p < 4; ++p) er[4 * k + p] -= hv * (int)(int8_t)(mi[k] >> (8 * p));
        }
#pragma unroll
    for (int r = 0; r < RS; ++r) {
        int v = er[r];
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        if ((tid & 63) == 0) atomicAdd(&eacc[r], v);
    }
    __syncthreads();
    if (tid < RS) jb.energy[RS * w.tile + tid] = eacc[tid];
    for (int i = tid; i < n; i += kGraphTileThreads) *reinterpret_cast<V *>(gst + rstride * i) = rows[i];
}

// Persistent graph-tile kernel: items of any tile width share the launch.
__global__ __launch_bounds__(kGraphTileThreads) void k_graph_tiles(const GraphJobDev *__restrict__ jobs,
                                                                   const WorkItem *__restrict__ items,
                                                                   const int32_t *__restrict__ n_items_p,
                                                                   int32_t *__restrict__ counter, uint32_t one)
{
    extern __shared__ uint4 tile_rows[];
    __shared__ uint64_t gtab[kGraphSlots];
    __shared__ int32_t eacc[16];
    __shared__ int slot;
    const int n_items = *n_items_p;
    for (;;) {
        const int it = take_item(counter, &slot);
        if (it >= n_items) break;
        const WorkItem w = items[it];
        const GraphJobDev jb = jobs[w.job];
        if (jb.rs == 16)
            graph_tile_item<4>(w, jb, tile_rows, gtab, eacc, one);
        else if (jb.rs == 8)
            graph_tile_item<2>(w, jb, tile_rows, gtab, eacc, one);
        else
            graph_tile_item<1>(w, jb, tile_rows, gtab, eacc, one);
        __syncthreads();  // the next item's first LDS writes wait for this item's last reads
    }
}

// The per-instance graph sweep held in LDS: workgroup t runs tile t (replicas
// [4 W t, + 4 W)) of the job for sweeps [s_begin, s_end), reading and writing its
// columns of the per-instance spins.
template <int W>
__global__ __launch_bounds__(kGraphTileThreads) void k_graph_slab(GraphJobDev jb, int s_begin, int s_end,
                                                                  uint32_t one)
{
    extern __shared__ uint4 tile_rows[];
    __shared__ uint64_t gtab[kGraphSlots];
    __shared__ int32_t eacc[16];
    const WorkItem w{0, (int)blockIdx.x, s_begin, s_end, 0, {0, 0, 0}};
    graph_tile_item<W>(w, jb, tile_rows, gtab, eacc, one);
}

// ---------------------------------------------------------------- biclique tiles

// A tile holds RB x 32 replicas of both sides in LDS, one row per replica:
// side A in columns [0, na_p), side B in [na_p, na_p + nb_p), padding zero.
// Each half-sweep is an MFMA product of the LDS spin rows with the couplings
// streamed from global memory (L2-resident, shared by all tiles of the job),
// followed by the decision epilogue writing the new side into LDS.
constexpr int kRing = 4;  // K-units of J fragments in flight per site block

// 4 x 4 byte transpose across a quad of lanes: lane u holds bytes M[u][0..3]
// and receives M[0..3][u].  Two exchanges (partners u ^ 1, then u ^ 2), each a
// DPP quad permutation and one byte permute.
__device__ __forceinline__ uint32_t quad_transpose(uint32_t d, int u)
{
    // v_perm_b32 selects bytes of {src0:src1} as a 64-bit value: selector byte
    // values 0..3 pick src1 bytes, 4..7 pick src0 bytes
    const uint32_t t = (uint32_t)__builtin_amdgcn_mov_dpp((int)d, 0xB1, 0xF, 0xF, false);  // quad_perm [1,0,3,2]
    // even u: (d0, t0, d2, t2); odd u: (t1, d1, t3, d3); here src0 = t, src1 = d
    const uint32_t d1 = __builtin_amdgcn_perm(t, d, (u & 1) ? 0x03070105u : 0x06020400u);
    const uint32_t t2 = (uint32_t)__builtin_amdgcn_mov_dpp((int)d1, 0x4E, 0xF, 0xF, false);  // quad_perm [2,3,0,1]
    // u < 2: (d1_0, d1_1, t2_0, t2_1); u >= 2: (t2_2, t2_3, d1_2, d1_3)
    return __builtin_amdgcn_perm(t2, d1, (u & 2) ? 0x03020706u : 0x05040100u);
}

// Four dwords of int8 K bytes from one word of two-bit codes: byte i of dword j is
// the code at bits 2 j, 2 j + 1 of byte i (the value J + 1 in {0, 1, 2}).
__device__ __forceinline__ v4i widen_codes(uint32_t x)
{
    return v4i{(int)(x & 0x03030303u), (int)((x >> 2) & 0x03030303u), (int)((x >> 4) & 0x03030303u),
               (int)((x >> 6) & 0x03030303u)};
}

// Sum of the four bytes of x.
__device__ __forceinline__ int byte_sum(uint32_t x)
{
    return (int)((x & 0xFFu) + ((x >> 8) & 0xFFu) + ((x >> 16) & 0xFFu) + (x >> 24));
}

// Biclique tiles with the spins held as bits in LDS: row r holds one bit per site (set = -1), 32 sites per word, side A
// in words [0, na_p / 32), side B after it, with an odd row pitch so that the 32
// rows a fragment read touches sit on distinct banks.  A K step of 32 sites is
// one word per replica, widened in registers to the bytes bit * 2^j (dword j)
// and multiplied on the int8 MFMA with int32 sums by the couplings stored in
// the widened-bit column order and scaled by 2^(3 - j) (Jb, JTb): the sum is
// 8 sum_k J_sk b_k and the field is I = (h + sum_k J) - (acc >> 2), exact.
// A bit row is an eighth of an int8 row, so 128 replicas fit LDS at any side
// length and each coupling fragment feeds RB MFMAs: couplings reach the CU at
// 1 / (32 RB) bytes per multiply-add.  Decisions as in the int8 tiles; the 64
// decisions of a wave for one (replica group, p) form a ballot mask, and the
// words of the 32 replicas of a block are written by one lane each.
template <int RB>
__global__ __launch_bounds__(kBqTileThreads) void k_bq_tiles_bits(const BqJobDev *__restrict__ jobs,
                                                                  const WorkItem *__restrict__ items,
                                                                  const int32_t *__restrict__ n_items_p,
                                                                  int32_t *__restrict__ counter, uint32_t one)
{
    constexpr int RS = 32 * RB;
    extern __shared__ uint4 dyn[];
    __shared__ int32_t eacc[RS];
    __shared__ int slot;
    const int tid = threadIdx.x;
    const int lane = tid & 63, ln = lane & 31, kg = lane >> 5;
    const int wave = tid >> 6;
    const int n_items = *n_items_p;

    for (;;) {
        const int it = take_item(counter, &slot);
        if (it >= n_items) break;
        const WorkItem w = items[it];
        const BqJobDev jb = jobs[w.job];
        const int na = jb.na, nb = jb.nb, na_p = jb.na_p, nb_p = jb.nb_p;
        const int wa = na_p / 32, wb = nb_p / 32;  // spin words of each side in a row
        const int PW = wa + wb, pitch = PW + 1;    // words per row in global memory / in LDS
        uint32_t *sw = reinterpret_cast<uint32_t *>(dyn);
        // decision words after the rows, 8-byte aligned
        uint64_t *Sw = reinterpret_cast<uint64_t *>(sw + ((RS * pitch + 1) & ~1));
        const char *Sb = reinterpret_cast<const char *>(Sw);
        uint32_t *gst = reinterpret_cast<uint32_t *>(jb.state) + (size_t)w.tile * RS * PW;
        const uint32_t rg0 = jb.rq0 + (uint32_t)(w.tile * (RS / 4));

        if (w.init) {
            for (int k = tid; k < RS * pitch; k += kBqTileThreads) sw[k] = 0u;
            __syncthreads();
            // thread (site, replica group): the four replicas' spins of one site
            for (int k = tid; k < (na + nb) * (RS / 4); k += kBqTileThreads) {
                const int g = k % (RS / 4), i = k / (RS / 4);  // site id: A first, then B
                const int col = i < na ? i : na_p + (i - na);
                const Block4 b = philox((uint32_t)i, 0u, rg0 + (uint32_t)g, kDomainInit, jb.k0, jb.k1);
#pragma unroll
                for (int p = 0; p < 4; ++p)
                    if (init_spin(b.w[p]) < 0) atomicOr(&sw[(4 * g + p) * pitch + col / 32], 1u << (col % 32));
            }
        } else {
            for (int k = tid; k < RS * PW; k += kBqTileThreads) {
                const int r = k / PW, c = k % PW;
                sw[r * pitch + c] = gst[(size_t)r * PW + c];
            }
        }
        if (tid < RS) eacc[tid] = 0;

        for (int s = w.s_begin; s < w.s_end; ++s) {
            __syncthreads();
            const uint32_t *trow = jb.table + (size_t)s * jb.width;
            const int top = jb.width - 1;
            for (int e = tid; e <= 2 * top; e += kBqTileThreads) {
                const int I = e - top;
                const uint32_t Tm = load_global<uint32_t>(trow + (I >= 0 ? I : -I));
                Sw[e] = I >= 0 ? (uint64_t)Tm : ((uint64_t)1 << 32) - Tm;
            }
            __syncthreads();
            const uint32_t t = jb.sweep0 + (uint32_t)s;
            const bool last = s + 1 == w.s_end;
#pragma unroll
            for (int side = 0; side < 2; ++side) {
                const int ns_p = side == 0 ? na_p : nb_p;
                const int ns = side == 0 ? na : nb;
                const int ko = side == 0 ? nb_p : na_p;  // coupling bytes per row (the other side)
                const int in_w = side == 0 ? wa : 0;     // word column of the other side
                const int out_w = side == 0 ? 0 : wa;    // word column of this side
                const uint8_t *Jx = reinterpret_cast<const uint8_t *>(side == 0 ? jb.Jb : jb.JTb);
                const int32_t *hs2 = side == 0 ? jb.hA2 : jb.hB2;
                const uint32_t site_base = side == 0 ? 0u : (uint32_t)na;
                // one 32-site block per wave at a time; its coupling fragments stream
                // from global memory through a ring kRing K-units (32 bytes) ahead,
                // which past the end of a block fills with the wave's next block
                const int nku = ko / 32;
                constexpr int kStep = kBqTileThreads / 64;
                const int nblk = ns_p / 32;
                v4i ring[kRing];
                if (wave < nblk) {
                    const uint8_t *br0 = Jx + (size_t)(wave * 32 + ln) * ko + 16 * kg;
#pragma unroll
                    for (int u = 0; u < kRing; ++u) ring[u] = load_global<v4i>(br0 + 32 * min(u, nku - 1));
                }
                for (int blk = wave; blk < nblk; blk += kStep) {
                    const int site = blk * 32 + ln;
                    const uint8_t *br = Jx + (size_t)site * ko + 16 * kg;
                    const uint8_t *bn = blk + kStep < nblk ? br + (size_t)kStep * 32 * ko : br;
                    v16i acc[RB];
#pragma unroll
                    for (int rb = 0; rb < RB; ++rb) acc[rb] = v16i{0};
                    const uint32_t *abase = sw + ln * pitch + in_w;
                    for (int kb = 0; kb < nku; kb += kRing) {
#pragma unroll
                        for (int u = 0; u < kRing; ++u) {
                            const int ku = kb + u;
                            if (ku < nku) {
                                const v4i b = ring[u];
                                const int kn = ku + kRing;
                                ring[u] = load_global<v4i>(kn < nku ? br + 32 * kn : bn + 32 * min(u, nku - 1));
#pragma unroll
                                for (int rb = 0; rb < RB; ++rb) {
                                    const v4i a = widen_bits(abase[rb * 32 * pitch + ku], kg);
                                    acc[rb] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a, b, acc[rb], 0, 0, 0);
                                }
                            }
                        }
                    }
                    // decisions; padding sites take bits that nothing reads (their
                    // couplings and fields are zero and they are never returned)
                    const int h2 = hs2[site];  // field plus coupling sum; site < ns_p
                    const bool site_ok = site < ns;
#pragma unroll
                    for (int rb = 0; rb < RB; ++rb) {
                        uint32_t outw = 0u;
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            const int r4 = rb * 32 + 8 * q + 4 * kg;  // first replica of the group in the tile
                            const Block4 b = philox(site_base + (uint32_t)site, t, rg0 + (uint32_t)(r4 >> 2),
                                                    kDomainSweep, jb.k0, jb.k1);
#pragma unroll
                            for (int p = 0; p < 4; ++p) {
                                const int I = h2 - (acc[rb][4 * q + p] >> 2);  // the accumulator holds 8 sum J b
                                const int Ic = min(max(I, -top), top);
                                const uint64_t S = *static_cast<const uint64_t *>(
                                    __builtin_assume_aligned(Sb + 8 * (Ic + top), 8));
                                const bool neg = (((uint64_t)b.w[p] * one + S) >> 32) != 0;  // new spin -1
                                // energy after the last side-B update: E = -sum_b m_b I_b - sum_a h_a m_a
                                if (side == 1 && last && site_ok) atomicAdd(&eacc[r4 + p], neg ? I : -I);
                                const uint64_t m = __ballot(neg);
                                const int L = 8 * q + p;
                                outw = (uint32_t)lane_write((int)(uint32_t)m, L, (int)outw);
                                outw = (uint32_t)lane_write((int)(uint32_t)(m >> 32), L + 4, (int)outw);
                            }
                        }
                        if (lane < 32) sw[(rb * 32 + lane) * pitch + out_w + blk] = outw;
                    }
                }
                __syncthreads();
            }
        }

        // field part of side A, then the energies and the spins go back to global memory
        for (int k = tid; k < RS * na; k += kBqTileThreads) {
            const int r = k / na, a = k % na;
            const int m = (sw[r * pitch + a / 32] >> (a % 32)) & 1u ? -1 : 1;
            const int v = (int)jb.hA[a] * m;
            if (v != 0) atomicAdd(&eacc[r], -v);
        }
        __syncthreads();
        if (tid < RS) jb.energy[w.tile * RS + tid] = eacc[tid];
        for (int k = tid; k < RS * PW; k += kBqTileThreads) {
            const int r = k / PW, c = k % PW;
            gst[(size_t)r * PW + c] = sw[r * pitch + c];
        }
    }
}

// A tile holds RB x 32 replicas of both sides in LDS, one row per replica:
// side A first, then side B, zero padding.  With int8 operands a row holds one
// byte per site and the half-sweep is the int8 MFMA with int32
// accumulation; the couplings stream as two-bit codes of J + 1 (a quarter of
// the int8 bytes: these tiles are bound by how fast a CU pulls couplings from
// L2), widened to bytes in registers, and the field is the product minus the
// replica's sum over the other side's spins.  Each half-sweep multiplies the LDS rows by the
// couplings streamed from global memory (L2-resident, shared by all tiles of
// the job); each coupling fragment feeds RB MFMAs, so larger tiles stream
// fewer bytes per replica.  The decision epilogue writes the new side into LDS.
template <int RB>
__global__ __launch_bounds__(kBqTileThreads) void k_bq_tiles(const BqJobDev *__restrict__ jobs,
                                                             const WorkItem *__restrict__ items,
                                                             const int32_t *__restrict__ n_items_p,
                                                             int32_t *__restrict__ counter, uint32_t one)
{
    constexpr int RS = 32 * RB;
    extern __shared__ uint4 dyn[];
    __shared__ int32_t eacc[RS];
    __shared__ int32_t mag[RS];  // sum of the other side's spins per replica
    __shared__ int slot;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6, ln = lane & 31, kg = lane >> 5;
    const int n_items = *n_items_p;

    for (;;) {
        const int it = take_item(counter, &slot);
        if (it >= n_items) break;
        const WorkItem w = items[it];
        const BqJobDev jb = jobs[w.job];
        const int na = jb.na, nb = jb.nb, na_p = jb.na_p, nb_p = jb.nb_p;
        const int pa = na_p, pb = nb_p;  // bytes of each side in a row
        const int PR = pa + pb, pitch = PR + 16;
        uint8_t *sp = reinterpret_cast<uint8_t *>(dyn);
        // decision words of the sweep: S(I) = Tm(|I|) for I >= 0, 2^32 - Tm(|I|) for I < 0,
        // I in [-top, top] (RS * pitch is a multiple of 16, so the words are aligned)
        uint64_t *Sw = reinterpret_cast<uint64_t *>(sp + (size_t)RS * pitch);
        const char *Sb = reinterpret_cast<const char *>(Sw);
        uint8_t *gst = jb.state + (size_t)w.tile * RS * PR;
        const uint32_t rg0 = jb.rq0 + (uint32_t)(w.tile * (RS / 4));

        if (w.init) {
            for (int k = tid; k < RS * pitch / 16; k += kBqTileThreads) dyn[k] = make_uint4(0, 0, 0, 0);
            __syncthreads();
            // thread (byte column, replica group): one byte in each of four rows
            for (int k = tid; k < PR * (RS / 4); k += kBqTileThreads) {
                const int g = k % (RS / 4), pi = k / (RS / 4);
                const bool A = pi < pa;
                const int s0 = A ? pi : pi - pa, n = A ? na : nb;
                if (s0 >= n) continue;
                const uint32_t i0 = (uint32_t)(A ? s0 : na + s0);
                const Block4 b0 = philox(i0, 0u, rg0 + (uint32_t)g, kDomainInit, jb.k0, jb.k1);
#pragma unroll
                for (int p = 0; p < 4; ++p) sp[(4 * g + p) * pitch + pi] = (uint8_t)init_spin(b0.w[p]);
            }
        } else {
            for (int k = tid; k < RS * (PR / 16); k += kBqTileThreads) {
                const int r = k / (PR / 16), c16 = k % (PR / 16);
                *reinterpret_cast<uint4 *>(sp + r * pitch + 16 * c16) =
                    *reinterpret_cast<const uint4 *>(gst + (size_t)r * PR + 16 * c16);
            }
        }
        if (tid < RS) eacc[tid] = 0;

        for (int s = w.s_begin; s < w.s_end; ++s) {
            __syncthreads();
            const uint32_t *trow = jb.table + (size_t)s * jb.width;
            const int top = jb.width - 1;
            for (int e = tid; e <= 2 * top; e += kBqTileThreads) {
                const int I = e - top;
                const uint32_t Tm = load_global<uint32_t>(trow + (I >= 0 ? I : -I));
                Sw[e] = I >= 0 ? (uint64_t)Tm : ((uint64_t)1 << 32) - Tm;
            }
            __syncthreads();
            const uint32_t t = jb.sweep0 + (uint32_t)s;
            const bool last = s + 1 == w.s_end;
#pragma unroll
            for (int side = 0; side < 2; ++side) {
                const int ns_p = side == 0 ? na_p : nb_p;
                const int ns = side == 0 ? na : nb;
                const int ko = side == 0 ? pb : pa;         // bytes per coupling row (the other side)
                const int in_col = side == 0 ? pa : 0;      // bytes of the other side (A operand)
                const int out_col = side == 0 ? 0 : pa;     // bytes of this side
                const uint8_t *Jx = reinterpret_cast<const uint8_t *>(side == 0 ? jb.J2 : jb.JT2);
                const int8_t *hs = side == 0 ? jb.hA : jb.hB;
                const uint32_t site_base = side == 0 ? 0u : (uint32_t)na;
                // one 32-site block per wave at a time; its coupling fragments stream
                // from global memory through a ring kRing K-units (32 bytes) ahead.
                // Past the end of a block the ring fills with the first units of the
                // wave's next block, so that they arrive during this block's epilogue.
                const int nku = ko / 32;
                constexpr int kStep = kBqTileThreads / 64;
                const int nblk = ns_p / 32;
                {
                    // the other side's spin sum per replica, padding sites included (their
                    // codes are 1): T threads per row, bytewise
                    // counts of nonzero and of -1 spins (at most 72 per byte for the
                    // row lengths that fit LDS), then a sum over the T lanes
                    constexpr int T = kBqTileThreads / RS;
                    const int r = tid / T, part = tid % T;
                    const uint4 *row = reinterpret_cast<const uint4 *>(sp + r * pitch + in_col);
                    uint32_t nz = 0u, neg = 0u;
#pragma unroll 4
                    for (int d = part; d < ko / 16; d += T) {
                        const uint4 x = row[d];
                        nz += (x.x & 0x01010101u) + (x.y & 0x01010101u) + (x.z & 0x01010101u) + (x.w & 0x01010101u);
                        neg += ((x.x >> 7) & 0x01010101u) + ((x.y >> 7) & 0x01010101u) + ((x.z >> 7) & 0x01010101u) +
                               ((x.w >> 7) & 0x01010101u);
                    }
                    int v = byte_sum(nz) - 2 * byte_sum(neg);
#pragma unroll
                    for (int off = T / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
                    if (part == 0) mag[r] = v;
                    __syncthreads();
                }
                // coupling fragments: [K step][site block] of one word of codes per lane,
                // 64 words per K step and block
                using Frag = uint32_t;
                auto frag_ptr = [&](int blk) -> const uint8_t * {
                    return Jx + 4 * (((size_t)blk * nku * 2 + kg) * 32 + ln);
                };
                constexpr int kUnit = 256;  // bytes from one K step of a fragment to the next
                Frag ring[kRing];
                if (wave < nblk) {
                    const uint8_t *br0 = frag_ptr(wave);
#pragma unroll
                    for (int u = 0; u < kRing; ++u)
                        ring[u] = load_global<Frag>(br0 + (size_t)kUnit * min(u, nku - 1));
                }
                for (int blk = wave; blk < nblk; blk += kStep) {
                    const int site = blk * 32 + ln;
                    const uint8_t *br = frag_ptr(blk);
                    // the next block of this wave, or this one again when there is none
                    const uint8_t *bn = blk + kStep < nblk ? frag_ptr(blk + kStep) : br;
                    v16i acc[RB];
#pragma unroll
                    for (int rb = 0; rb < RB; ++rb) acc[rb] = v16i{0};
                    const uint8_t *abase = sp + ln * pitch + in_col + 16 * kg;
                    for (int kb = 0; kb < nku; kb += kRing) {
#pragma unroll
                        for (int u = 0; u < kRing; ++u) {
                            const int ku = kb + u;
                            if (ku < nku) {
                                const v4i b = widen_codes(ring[u]);
                                // slot u takes unit ku + kRing of this block, or, after this
                                // block's last unit of its residue class, unit u of the next block
                                const int kn = ku + kRing;
                                ring[u] = load_global<Frag>(kn < nku ? br + (size_t)kUnit * kn
                                                                     : bn + (size_t)kUnit * min(u, nku - 1));
#pragma unroll
                                for (int rb = 0; rb < RB; ++rb) {
                                    const v4i a = *reinterpret_cast<const v4i *>(abase + rb * 32 * pitch + 32 * ku);
                                    acc[rb] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a, b, acc[rb], 0, 0, 0);
                                }
                            }
                        }
                    }
                    // decisions: the field F of a replica and site indexes S(F + h)
                    // (clamped to [-top, top]); the sign bits of a group's four
                    // replicas become spin codes, one per byte, transposed across the
                    // lane quad (sites s .. s + 3) so that each lane writes four
                    // consecutive sites of one replica row.
                    // Padding sites may take any value: their couplings and fields are
                    // zero and they are never returned.
                    const int hval = load_global<int8_t>(hs + site);  // site < ns_p: padded fields are zero
                    const bool site_ok = site < ns;
                    const int flo = -top - hval, fhi = top - hval;  // F range whose F + h is in [-top, top]
                    const int base8 = 8 * (hval + top);
                    const int u4 = ln & 3;
                    const int quad_col = out_col + site - u4;
#pragma unroll
                    for (int rb = 0; rb < RB; ++rb) {
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            const int r4 = rb * 32 + 8 * q + 4 * kg;  // first replica of the group in the tile
                            const Block4 b = philox(site_base + (uint32_t)site, t, rg0 + (uint32_t)(r4 >> 2),
                                                    kDomainSweep, jb.k0, jb.k1);
                            uint32_t sgn[4];  // 1: the replica's new spin is -1
#pragma unroll
                            for (int p = 0; p < 4; ++p) {
                                // an exact integer; with codes of J + 1 the product exceeds the
                                // field by the replica's spin sum over the other side
                                const int F = (int)acc[rb][4 * q + p] - mag[r4 + p];
                                const int Fc = min(max(F, flo), fhi);
                                const uint64_t S = *static_cast<const uint64_t *>(
                                    __builtin_assume_aligned(Sb + 8 * Fc + base8, 8));
                                sgn[p] = (uint32_t)(((uint64_t)b.w[p] * one + S) >> 32);
                                // energy after the last side-B update: E = -sum_b m_b I_b - sum_a h_a m_a
                                if (side == 1 && last && site_ok)
                                    atomicAdd(&eacc[r4 + p], (sgn[p] ? 1 : -1) * (F + hval));
                            }
                            const uint32_t lo = __builtin_amdgcn_perm(sgn[1], sgn[0], 0x0C0C0400u);
                            const uint32_t hi = __builtin_amdgcn_perm(sgn[3], sgn[2], 0x0C0C0400u);
                            // sign bit 0 -> +1, 1 -> -1: 0x01 / 0xFF bytes
                            const uint32_t packed = __builtin_amdgcn_perm(0u, 0xFF01u,
                                                                          __builtin_amdgcn_perm(hi, lo, 0x05040100u));
                            const uint32_t x = quad_transpose(packed, u4);  // four sites, one byte each
                            *reinterpret_cast<uint32_t *>(sp + (r4 + u4) * pitch + quad_col) = x;
                        }
                    }
                }
                __syncthreads();
            }
        }

        // field part of side A, then the energies and the spins go back to global memory
        for (int k = tid; k < RS * na; k += kBqTileThreads) {
            const int r = k / na, a = k % na;
            const int m = (int)(int8_t)sp[r * pitch + a];
            const int v = (int)jb.hA[a] * m;
            if (v != 0) atomicAdd(&eacc[r], -v);
        }
        __syncthreads();
        if (tid < RS) jb.energy[w.tile * RS + tid] = eacc[tid];
        for (int k = tid; k < RS * (PR / 16); k += kBqTileThreads) {
            const int r = k / (PR / 16), c16 = k % (PR / 16);
            *reinterpret_cast<uint4 *>(gst + (size_t)r * PR + 16 * c16) =
                *reinterpret_cast<const uint4 *>(sp + r * pitch + 16 * c16);
        }
    }
}

}  // namespace

size_t ea_tile_lds(int64_t N, int rs) { return (size_t)N * rs; }

size_t graph_tile_lds(int64_t N, int rs) { return (size_t)N * rs; }

size_t bq_tile_lds(int rs, int na_p, int nb_p, int width, int mode)
{
    // spin rows, then one 64-bit decision word per field value in [-(width - 1), width - 1]
    size_t rows;
    if (mode == kTileBits)
        rows = sizeof(uint32_t) * (size_t)((rs * ((na_p + nb_p) / 32 + 1) + 1) & ~1);
    else
        rows = (size_t)rs * ((size_t)(na_p + nb_p) + 16);
    return rows + sizeof(uint64_t) * (size_t)(2 * width - 1);
}

template <int W>
static hipError_t graph_slab_launch(const GraphJobDev &jb, int tiles, int s_begin, int s_end, hipStream_t st)
{
    static const hipError_t lds_attr = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_graph_slab<W>),
                                                           hipFuncAttributeMaxDynamicSharedMemorySize,
                                                           160 * 1024 - 4096);
    if (lds_attr != hipSuccess) return lds_attr;
    hipLaunchKernelGGL(k_graph_slab<W>, dim3((unsigned)tiles), dim3(kGraphTileThreads), graph_tile_lds(jb.n, 4 * W),
                       st, jb, s_begin, s_end, 1u);
    return hipGetLastError();
}

hipError_t graph_slab(const GraphJobDev &jb, int tiles, int s_begin, int s_end, hipStream_t st)
{
    if (tiles < 1 || jb.row_stride % 16 != 0 || jb.row_stride < tiles * jb.rs || s_end < s_begin ||
        graph_tile_lds(jb.n, jb.rs) > (size_t)(160 * 1024 - 4096))
        return hipErrorInvalidValue;
    if (jb.rs == 16) return graph_slab_launch<4>(jb, tiles, s_begin, s_end, st);
    if (jb.rs == 8) return graph_slab_launch<2>(jb, tiles, s_begin, s_end, st);
    if (jb.rs == 4) return graph_slab_launch<1>(jb, tiles, s_begin, s_end, st);
    return hipErrorInvalidValue;
}

hipError_t tiles_set_lds_limit()
{
    const int max_lds = 160 * 1024 - 4096;  // leave room for the static shared variables
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_ea_tiles<kEaTileThreads>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, max_lds);
    if (e == hipSuccess)
        e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_ea_tiles<kEaTileThreadsLarge>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, max_lds);
    if (e == hipSuccess)
        e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_graph_tiles),
                                hipFuncAttributeMaxDynamicSharedMemorySize, max_lds);

    const void *bq_kernels[] = {reinterpret_cast<const void *>(&k_bq_tiles_bits<1>),
                                reinterpret_cast<const void *>(&k_bq_tiles_bits<2>),
                                reinterpret_cast<const void *>(&k_bq_tiles_bits<4>),
                                reinterpret_cast<const void *>(&k_bq_tiles<1>),
                                reinterpret_cast<const void *>(&k_bq_tiles<2>)};
    for (const void *k : bq_kernels)
        if (e == hipSuccess) e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, max_lds);
    return e;
}

hipError_t ea_tiles(const EaJobDev *jobs, const WorkItem *items, const int32_t *n_items, int32_t *counter, int grid,
                    size_t lds_bytes, hipStream_t st)
{
    if (lds_bytes > kEaLargeTileLds)
        hipLaunchKernelGGL((k_ea_tiles<kEaTileThreadsLarge>), dim3((unsigned)grid), dim3(kEaTileThreadsLarge),
                           lds_bytes, st, jobs, items, n_items, counter, 1u);
    else
        hipLaunchKernelGGL((k_ea_tiles<kEaTileThreads>), dim3((unsigned)grid), dim3(kEaTileThreads), lds_bytes, st,
                           jobs, items, n_items, counter, 1u);
    return hipGetLastError();
}

hipError_t graph_tiles(const GraphJobDev *jobs, const WorkItem *items, const int32_t *n_items, int32_t *counter,
                       int grid, size_t lds_bytes, hipStream_t st)
{
    hipLaunchKernelGGL(k_graph_tiles, dim3((unsigned)grid), dim3(kGraphTileThreads), lds_bytes, st, jobs, items,
                       n_items, counter, 1u);
    return hipGetLastError();
}

hipError_t bq_tiles(const BqJobDev *jobs, const WorkItem *items, const int32_t *n_items, int32_t *counter, int rs,
                    int mode, int grid, size_t lds_bytes, hipStream_t st)
{
#define PBIT_BQ_TILES(K)                                                                                        \
    hipLaunchKernelGGL(K, dim3((unsigned)grid), dim3(kBqTileThreads), lds_bytes, st, jobs, items, n_items, counter, 1u)
    const int rb = rs == 128 ? 4 : rs == 64 ? 2 : rs == 32 ? 1 : 0;
    if (rb == 0 || (mode != kTileInt8 && mode != kTileBits)) return hipErrorInvalidValue;
    if (mode == kTileBits) {
        if (rb == 4) PBIT_BQ_TILES((k_bq_tiles_bits<4>)); else if (rb == 2) PBIT_BQ_TILES((k_bq_tiles_bits<2>));
        else PBIT_BQ_TILES((k_bq_tiles_bits<1>));
    } else {
        // int8 rows come in 32- and 64-replica tiles (a 128-replica int8 tile spills registers)
        if (rb == 4) return hipErrorInvalidValue;
        if (rb == 2) PBIT_BQ_TILES((k_bq_tiles<2>)); else PBIT_BQ_TILES((k_bq_tiles<1>));
    }
#undef PBIT_BQ_TILES
    return hipGetLastError();
}

}  // namespace pbit
