// ea_kernels.hip — 3D Edwards-Anderson cube (paper Sec. 2) on gfx950.
//
// Device layout: spins int8 [N][Rp], replica fastest, so that the 16 replicas
// a thread updates form one 16-byte load per neighbour and one 16-byte store,
// and a wave's loads of one neighbour row are contiguous.  The checkerboard
// half-sweep (Sec. 1.2.2: the two update groups of a bipartite lattice) reads
// only opposite-colour rows and writes only its own, so each neighbour row is
// fetched once per half-sweep and shared by the six sites around it.
#include <algorithm>

#include "device.h"
#include "internal.h"

namespace pbit {

namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ int wrap_inc(int v, int L) { return v + 1 == L ? 0 : v + 1; }
__device__ __forceinline__ int wrap_dec(int v, int L) { return v == 0 ? L - 1 : v - 1; }

// Random +-1 start: one Philox block gives the 4 replicas of a group.
__global__ __launch_bounds__(kThreads) void k_ea_init(int8_t *__restrict__ spins, int64_t N, int Rp, uint32_t rq0,
                                                      uint32_t k0, uint32_t k1)
{
    const int groups = Rp / 4;
    const int64_t gid = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (gid >= N * groups) return;
    const int g = (int)(gid % groups);
    const uint32_t i = (uint32_t)(gid / groups);
    const Block4 b = philox(i, 0u, rq0 + (uint32_t)g, kDomainInit, k0, k1);
    uint32_t packed = 0;
#pragma unroll
    for (int p = 0; p < 4; ++p) packed |= (uint32_t)(uint8_t)init_spin(b.w[p]) << (8 * p);
    *reinterpret_cast<uint32_t *>(spins + (size_t)i * Rp + 4 * g) = packed;
}

// [R][N] -> [N][Rp] and back, through a 64x64 LDS tile.
template <bool TO_DEVICE>
__global__ __launch_bounds__(kThreads) void k_ea_transpose(const int8_t *__restrict__ src, int8_t *__restrict__ dst,
                                                           int64_t N, int R, int Rp)
{
    __shared__ int8_t tile[64][65];
    const int64_t i0 = (int64_t)blockIdx.x * 64;  // sites
    const int r0 = blockIdx.y * 64;               // replicas
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    if (TO_DEVICE) {
        // read rows r of src[R][N], write rows i of dst[N][Rp]
        for (int rr = ty; rr < 64; rr += 4) {
            const int r = r0 + rr;
            const int64_t i = i0 + tx;
            tile[rr][tx] = (r < R && i < N) ? src[(size_t)r * N + i] : (int8_t)0;
        }
        __syncthreads();
        for (int ii = ty; ii < 64; ii += 4) {
            const int64_t i = i0 + ii;
            const int r = r0 + tx;
            if (i < N && r < Rp) dst[(size_t)i * Rp + r] = tile[tx][ii];
        }
    } else {
        for (int ii = ty; ii < 64; ii += 4) {
            const int64_t i = i0 + ii;
            const int r = r0 + tx;
            tile[tx][ii] = (i < N && r < Rp) ? src[(size_t)i * Rp + r] : (int8_t)0;
        }
        __syncthreads();
        for (int rr = ty; rr < 64; rr += 4) {
            const int r = r0 + rr;
            const int64_t i = i0 + tx;
            if (r < R && i < N) dst[(size_t)r * N + i] = tile[rr][tx];
        }
    }
}

constexpr int kFieldOff = 7;  // |I| <= 6 + |h| <= 7 on the cube
constexpr int kFieldSlots = 2 * kFieldOff + 1;
static_assert(sizeof(EaRow) == kFieldSlots * sizeof(uint64_t), "one decision word per field value");

// Sign mask of bit k of c: 0 or 0xFFFFFFFF.
__device__ __forceinline__ uint32_t bit_mask(uint32_t c, int k) { return (uint32_t)((int32_t)(c << (31 - k)) >> 31); }

// One checkerboard half-sweep.  Block (cbw, spb): x threads walk 16-replica
// chunks, y threads walk the sites of a lattice row; a block covers `ny`
// consecutive rows (y0 .. y0 + ny - 1, z) with y0 = blockIdx.y * ny and
// z = blockIdx.z.  blockIdx.x = chunk-block * nsl + slab: with nsl = 8 the
// slab index equals the XCD a workgroup is dispatched to, so each XCD's L2
// serves one replica slab of the whole lattice and neighbour rows are reused
// there.
//
// Decision: the table in LDS holds, for every field value I, the 64-bit word
// S(I) = Tm for I >= 0 and 2^32 - Tm for I < 0 (EaRow); the heat-bath rule
// (new spin -1 when ~w < Tm for I >= 0, and when w >= Tm for I < 0) is then
// exactly "bit 32 of w + S(I) is set", one v_mad_u64_u32 per update (`one`
// is 1, passed in so that w * one + S is issued as that instruction).
//
// Field, bytewise for four replicas per dword: spin bytes are +1 = 0x01 and
// -1 = 0xFF, so bit 4 of a byte is set exactly for -1, and
// ~(m ^ F) & K (F = all ones for J = -1, K = 0x10 per byte for J != 0) has
// bit 4 set exactly where J m = +1.  Six such terms plus the site's base byte
// give 8 (I + 7) in every byte (at most 112): the LDS byte address of the
// replica's table entry.
template <bool DENSE, bool EARLY_RNG>
__global__ __launch_bounds__(kThreads) void k_ea_halfsweep(int8_t *__restrict__ spins,
                                                           const uint32_t *__restrict__ code, EaRow row, int Lx,
                                                           int Ly, int Lz, int Rp, int colour, int lg_nsl, int cs,
                                                           int ny, uint32_t sweep, uint32_t rq0, uint32_t k0,
                                                           uint32_t k1, uint32_t one)
{
    __shared__ uint64_t tab[kFieldSlots];  // the kernel's only LDS object, so it starts at address 0
    const int tid = threadIdx.x + blockDim.x * threadIdx.y;
    if (tid < kFieldSlots) {
        uint64_t v = row.s[0];
#pragma unroll
        for (int e = 1; e < kFieldSlots; ++e) v = tid == e ? row.s[e] : v;
        tab[tid] = v;
    }
    __syncthreads();

    const int slab = blockIdx.x & ((1 << lg_nsl) - 1);
    const int qs = (blockIdx.x >> lg_nsl) * blockDim.x + threadIdx.x;
    const int q = slab * cs + qs;
    if (qs >= cs || 16 * q >= Rp) return;
    const int z = blockIdx.z;
    const uint32_t rowR = (uint32_t)Lx * (uint32_t)Rp;  // bytes per lattice row
    const uint32_t planeR = rowR * (uint32_t)Ly;         // bytes per plane
    const uint32_t q16 = 16u * (uint32_t)q;
    const uint32_t zR = (uint32_t)z * planeR + q16;
    const uint32_t zpR = (z + 1 == Lz ? 0u : (uint32_t)(z + 1)) * planeR + q16;
    const uint32_t zmR = (z == 0 ? (uint32_t)(Lz - 1) : (uint32_t)(z - 1)) * planeR + q16;
    const int hx = Lx / 2;
    const uint32_t rg4 = rq0 + 4u * (uint32_t)q;  // Philox counter word 2 of this chunk's first group
    const char *tbase = reinterpret_cast<const char *>(tab);

    for (int yy = 0; yy < ny; ++yy) {
        const int y = blockIdx.y * ny + yy;
        const uint32_t yR = (uint32_t)y * rowR;
        const uint32_t base = yR + zR;
        const uint32_t yp = (y + 1 == Ly ? 0u : (uint32_t)(y + 1)) * rowR + zR;
        const uint32_t ym = (y == 0 ? (uint32_t)(Ly - 1) : (uint32_t)(y - 1)) * rowR + zR;
        const uint32_t zp = yR + zpR, zm = yR + zmR;
        const uint32_t siteRow = (uint32_t)Lx * ((uint32_t)y + (uint32_t)Ly * (uint32_t)z);
        const int par = (colour + y + z) & 1;

        for (int kx = threadIdx.y; kx < hx; kx += blockDim.y) {
            const int x = 2 * kx + par;
            const uint32_t xR = (uint32_t)x * (uint32_t)Rp;
            const uint32_t xpR = (x + 1 == Lx ? 0u : (uint32_t)(x + 1)) * (uint32_t)Rp;
            const uint32_t xmR = (x == 0 ? (uint32_t)(Lx - 1) : (uint32_t)(x - 1)) * (uint32_t)Rp;
            const uint32_t offs[6] = {base + xpR, base + xmR, yp + xR, ym + xR, zp + xR, zm + xR};
            const uint32_t i = siteRow + (uint32_t)x;
            const uint32_t c = code[i];
            uint4 v[6];
#pragma unroll
            for (int d = 0; d < 6; ++d) v[d] = *reinterpret_cast<const uint4 *>(spins + offs[d]);
            // the random words do not depend on the loads; EARLY_RNG draws them while the loads
            // are in flight (the scheduling barriers keep the compiler from sinking them)
            Block4 b[4];
            if (EARLY_RNG) {
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int k = 0; k < 4; ++k) b[k] = philox(i, sweep, rg4 + (uint32_t)k, kDomainSweep, k0, k1);
                __builtin_amdgcn_sched_barrier(0);
            }
            uint32_t t[6][4];
#pragma unroll
            for (int d = 0; d < 6; ++d) {
                const uint32_t F = bit_mask(c, kCodeFlipShift + d);
                const uint32_t K = DENSE ? 0x10101010u : (bit_mask(c, d) & 0x10101010u);
                // truth table 0x82: ~(a ^ b) & c
                t[d][0] = __builtin_amdgcn_bitop3_b32(v[d].x, F, K, 0x82);
                t[d][1] = __builtin_amdgcn_bitop3_b32(v[d].y, F, K, 0x82);
                t[d][2] = __builtin_amdgcn_bitop3_b32(v[d].z, F, K, 0x82);
                t[d][3] = __builtin_amdgcn_bitop3_b32(v[d].w, F, K, 0x82);
            }
            const uint32_t pos8 = __builtin_amdgcn_perm(0u, c, 0x03030303u);  // bits 24..31 in every byte
            uint32_t out[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                if (!EARLY_RNG) b[k] = philox(i, sweep, rg4 + (uint32_t)k, kDomainSweep, k0, k1);
                const uint32_t idx = (t[0][k] + t[1][k] + t[2][k]) + (t[3][k] + t[4][k] + t[5][k]) + pos8;
                uint32_t sgn[4];  // 1: the replica's new spin is -1
#pragma unroll
                for (int p = 0; p < 4; ++p) {
                    const uint64_t S = *static_cast<const uint64_t *>(
                        __builtin_assume_aligned(tbase + ((idx >> (8 * p)) & 0xFFu), 8));
                    sgn[p] = (uint32_t)(((uint64_t)b[k].w[p] * one + S) >> 32);
                }
                // gather the four low bytes, then map 0 -> 0x01 and 1 -> 0xFF
                const uint32_t lo = __builtin_amdgcn_perm(sgn[1], sgn[0], 0x0C0C0400u);
                const uint32_t hi = __builtin_amdgcn_perm(sgn[3], sgn[2], 0x0C0C0400u);
                out[k] = __builtin_amdgcn_perm(0u, 0xFF01u, __builtin_amdgcn_perm(hi, lo, 0x05040100u));
            }
            *reinterpret_cast<uint4 *>(spins + base + xR) = make_uint4(out[0], out[1], out[2], out[3]);
        }
    }
}

// The half-sweeps of a small cube, resident in LDS (the stencil's LDS-staged
// form): a workgroup holds 16 replicas (one chunk of the [N][Rp] layout) of the
// whole lattice, 16 bytes per site, and runs a range of sweeps with workgroup
// barriers between the half-sweeps, so that no sweep needs a launch or touches
// HBM.  A thread takes one site at a time with the chunk's 16 replicas, as in
// the streaming kernel (same field bytes, Philox counters and carry decision),
// reading the six neighbour rows from LDS; one 8-byte load from the problem's
// site list gives the site, its periodic-wrap flags and its code.  The decision
// words of a sweep come from its threshold row, loaded one sweep ahead.
constexpr int kSlabThreads = 512;

template <bool DENSE>
__global__ __launch_bounds__(kSlabThreads) void k_ea_slab(int8_t *__restrict__ spins,
                                                        const uint2 *__restrict__ sites,
                                                        const uint32_t *__restrict__ table, int width, int Lx,
                                                        int Ly, int Lz, int Rp, int s_begin, int s_end,
                                                        uint32_t sweep0, uint32_t rq0, uint32_t k0, uint32_t k1,
                                                        uint32_t one)
{
    extern __shared__ uint4 rows[];  // [N]: the chunk's 16 replicas of every site
    __shared__ uint64_t stab[kFieldSlots];
    const int tid = threadIdx.x;
    const int q = blockIdx.x;  // chunk of 16 replicas
    const int plane = Lx * Ly, N = plane * Lz, half = N / 2;
    // neighbour d of site i: i + step[d], or i + step[d] + fix[d] across the boundary
    const int step[6] = {1, -1, Lx, -Lx, plane, -plane};
    const int fix[6] = {-Lx, Lx, -plane, plane, -N, N};
    for (int i = tid; i < N; i += kSlabThreads)
        rows[i] = *reinterpret_cast<const uint4 *>(spins + (size_t)i * Rp + 16 * q);
    const uint32_t rg4 = rq0 + 4u * (uint32_t)q;  // Philox counter word 2 of the chunk's first group
    const char *tb = reinterpret_cast<const char *>(stab);
    const int tix = min(tid >= kFieldOff ? tid - kFieldOff : kFieldOff - tid, width - 1);  // |I| of entry tid
    uint32_t tnext = 0u;
    if (tid < kFieldSlots && s_begin < s_end) tnext = table[(size_t)s_begin * width + tix];
    for (int s = s_begin; s < s_end; ++s) {
        __syncthreads();
        if (tid < kFieldSlots) {
            stab[tid] = tid >= kFieldOff ? (uint64_t)tnext : ((uint64_t)1 << 32) - tnext;
            if (s + 1 < s_end) tnext = table[(size_t)(s + 1) * width + tix];
        }
        __syncthreads();
        const uint32_t t = sweep0 + (uint32_t)s;
        for (int c = 0; c < 2; ++c) {
            for (int j = tid; j < half; j += kSlabThreads) {
                const uint2 e = sites[c * half + j];
                const int i = (int)(e.x & 0xFFFFu);
                const uint32_t wrap = e.x >> 16, w = e.y;
                uint4 v[6];
#pragma unroll
                for (int d = 0; d < 6; ++d) v[d] = rows[i + step[d] + (((wrap >> d) & 1u) ? fix[d] : 0)];
                Block4 b[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) b[r] = philox((uint32_t)i, t, rg4 + (uint32_t)r, kDomainSweep, k0, k1);
                uint32_t tt[6][4];
#pragma unroll
                for (int d = 0; d < 6; ++d) {
                    const uint32_t F = bit_mask(w, kCodeFlipShift + d);
                    const uint32_t K = DENSE ? 0x10101010u : (bit_mask(w, d) & 0x10101010u);
                    tt[d][0] = __builtin_amdgcn_bitop3_b32(v[d].x, F, K, 0x82);  // ~(a ^ b) & c
                    tt[d][1] = __builtin_amdgcn_bitop3_b32(v[d].y, F, K, 0x82);
                    tt[d][2] = __builtin_amdgcn_bitop3_b32(v[d].z, F, K, 0x82);
                    tt[d][3] = __builtin_amdgcn_bitop3_b32(v[d].w, F, K, 0x82);
                }
                const uint32_t pos8 = __builtin_amdgcn_perm(0u, w, 0x03030303u);  // base byte in every byte
                uint32_t out[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const uint32_t idx = (tt[0][r] + tt[1][r] + tt[2][r]) + (tt[3][r] + tt[4][r] + tt[5][r]) + pos8;
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
                rows[i] = make_uint4(out[0], out[1], out[2], out[3]);
            }
            __syncthreads();
        }
    }
    for (int i = tid; i < N; i += kSlabThreads)
        *reinterpret_cast<uint4 *>(spins + (size_t)i * Rp + 16 * q) = rows[i];
}

// From-scratch energy (Eq. 1 with the field): E[r] = -sum_bonds J m_i m_j - sum_i h_i m_i,
// each bond (i, i + e_d) visited once, from its lower-end site i.  With d = 1 where two
// spins differ (bit 1 of the xor of their bytes) and b = 1 where a spin is -1,
// -J m_i m_j = -J + 2 J d and -h m = -h + 2 h b, so
//     E[r] = -(sum J + sum h) + 2 (P[r] - Q[r]),
// P counting the d of bonds with J = +1 and the b of sites with h = +1, Q those with -1.
// A thread counts P and Q bytewise for 16 replicas over kEnergySites sites (at most
// 4 kEnergySites per byte); the workgroup (16 site chunks x 16 replica chunks) sums its
// chunks in LDS and adds one total per replica.
constexpr int kEnergySites = 32;

__global__ __launch_bounds__(kThreads) void k_ea_energy(const int8_t *__restrict__ spins, const int8_t *__restrict__ J,
                                                        const int8_t *__restrict__ h, int Lx, int Ly, int Lz, int Rp,
                                                        int R, int32_t *__restrict__ E)
{
    __shared__ int32_t part[16][256 + 1];
    const int rq = threadIdx.x & 15, sc = threadIdx.x >> 4;
    const int q = blockIdx.y * 16 + rq;                       // chunk of 16 replicas
    const int64_t N = (int64_t)Lx * Ly * Lz;
    const int64_t plane = (int64_t)Lx * Ly;
    const int64_t s0 = ((int64_t)blockIdx.x * 16 + sc) * kEnergySites;
    const int64_t s1 = min(s0 + kEnergySites, N);
    uint32_t P[4] = {0u, 0u, 0u, 0u}, Q[4] = {0u, 0u, 0u, 0u};
    int32_t base = 0;  // -(sum J + sum h) over the chunk's sites
    if (16 * q < Rp) {
        for (int64_t i = s0; i < s1; ++i) {
            const int x = (int)(i % Lx), y = (int)((i / Lx) % Ly), z = (int)(i / plane);
            const int64_t nb[3] = {(x + 1 == Lx ? 0 : x + 1) + (int64_t)Lx * y + plane * z,
                                   x + (int64_t)Lx * (y + 1 == Ly ? 0 : y + 1) + plane * z,
                                   x + (int64_t)Lx * y + plane * (z + 1 == Lz ? 0 : z + 1)};
            const uint4 mi = *reinterpret_cast<const uint4 *>(spins + (size_t)i * Rp + 16 * q);
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const int j = J[d * N + i];
                const uint4 mj = *reinterpret_cast<const uint4 *>(spins + (size_t)nb[d] * Rp + 16 * q);
                const uint32_t mp = j > 0 ? 0x01010101u : 0u, mn = j < 0 ? 0x01010101u : 0u;
                const uint32_t dx = (mi.x ^ mj.x) >> 1, dy = (mi.y ^ mj.y) >> 1, dz = (mi.z ^ mj.z) >> 1,
                               dw = (mi.w ^ mj.w) >> 1;
                P[0] += dx & mp; P[1] += dy & mp; P[2] += dz & mp; P[3] += dw & mp;
                Q[0] += dx & mn; Q[1] += dy & mn; Q[2] += dz & mn; Q[3] += dw & mn;
                base -= j;
            }
            const int hv = h ? h[i] : 0;
            const uint32_t mp = hv > 0 ? 0x01010101u : 0u, mn = hv < 0 ? 0x01010101u : 0u;
            const uint32_t bx = mi.x >> 1, by = mi.y >> 1, bz = mi.z >> 1, bw = mi.w >> 1;
            P[0] += bx & mp; P[1] += by & mp; P[2] += bz & mp; P[3] += bw & mp;
            Q[0] += bx & mn; Q[1] += by & mn; Q[2] += bz & mn; Q[3] += bw & mn;
            base -= hv;
        }
    }
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int p = 0; p < 4; ++p)
            part[sc][16 * rq + 4 * k + p] =
                base + 2 * ((int)((P[k] >> (8 * p)) & 0xFFu) - (int)((Q[k] >> (8 * p)) & 0xFFu));
    __syncthreads();
    const int r = blockIdx.y * 256 + threadIdx.x;
    if (r < R) {
        int32_t e = 0;
#pragma unroll
        for (int c = 0; c < 16; ++c) e += part[c][threadIdx.x];
        atomicAdd(E + r, e);
    }
}

}  // namespace

static inline unsigned blocks_for(int64_t work) { return (unsigned)((work + kThreads - 1) / kThreads); }

hipError_t ea_init(const EaView &p, int8_t *spins, int Rp, uint32_t rq0, Key key, hipStream_t st)
{
    const int64_t work = p.N * (Rp / 4);
    hipLaunchKernelGGL(k_ea_init, dim3(blocks_for(work)), dim3(kThreads), 0, st, spins, p.N, Rp, rq0, key.k0, key.k1);
    return hipGetLastError();
}

hipError_t ea_from_rows(const EaView &p, const int8_t *src_rn, int R, int8_t *spins, int Rp, hipStream_t st)
{
    dim3 grid((unsigned)((p.N + 63) / 64), (unsigned)((Rp + 63) / 64));
    hipLaunchKernelGGL(k_ea_transpose<true>, grid, dim3(kThreads), 0, st, src_rn, spins, p.N, R, Rp);
    return hipGetLastError();
}

hipError_t ea_to_rows(const EaView &p, const int8_t *spins, int Rp, int8_t *dst_rn, int R, hipStream_t st)
{
    dim3 grid((unsigned)((p.N + 63) / 64), (unsigned)((Rp + 63) / 64));
    hipLaunchKernelGGL(k_ea_transpose<false>, grid, dim3(kThreads), 0, st, spins, dst_rn, p.N, R, Rp);
    return hipGetLastError();
}

EaRow ea_row(const uint32_t *trow, int width)
{
    EaRow r;
    for (int e = 0; e < kFieldSlots; ++e) {
        const int I = e - kFieldOff;
        const uint32_t T = trow[std::min(I >= 0 ? I : -I, width - 1)];
        r.s[e] = I >= 0 ? (uint64_t)T : ((uint64_t)1 << 32) - T;
    }
    return r;
}

hipError_t ea_halfsweep(const EaView &p, int8_t *spins, int Rp, int colour, const EaRow &row, uint32_t sweep,
                        uint32_t rq0, Key key, hipStream_t st, int ny, bool early_rng)
{
    if (Rp % 16 != 0) return hipErrorInvalidValue;
    if ((uint64_t)p.N * (uint64_t)Rp >= ((uint64_t)1 << 32)) return hipErrorInvalidValue;  // 32-bit byte offsets
    if (p.Lz > 65535) return hipErrorInvalidValue;                                       // grid z limit
    if (ny <= 0) ny = p.Ly % 2 == 0 ? 2 : 1;  // two rows per workgroup measured best at L = 16 and 32
    if (p.Ly % ny != 0 || p.Ly / ny > 65535) return hipErrorInvalidValue;
    const int C = Rp / 16;                   // 16-replica chunks
    const int lg_nsl = C >= 8 ? 3 : 0;       // 8 replica slabs, one per XCD, when there are enough chunks
    const int nsl = 1 << lg_nsl;
    const int cs = (C + nsl - 1) / nsl;      // chunks per slab
    int cbw = 1;
    while (cbw < cs && cbw < 64) cbw *= 2;
    const int spb = kThreads / cbw;
    const int ncb = (cs + cbw - 1) / cbw;
    dim3 grid((unsigned)(nsl * ncb), (unsigned)(p.Ly / ny), (unsigned)p.Lz), block((unsigned)cbw, (unsigned)spb);
#define PBIT_EA_LAUNCH(D, E)                                                                                     \
    hipLaunchKernelGGL((k_ea_halfsweep<D, E>), grid, block, 0, st, spins, p.code, row, p.Lx, p.Ly, p.Lz, Rp, colour, \
                       lg_nsl, cs, ny, sweep, rq0, key.k0, key.k1, 1u)
    if (p.dense) {
        if (early_rng) PBIT_EA_LAUNCH(true, true); else PBIT_EA_LAUNCH(true, false);
    } else {
        if (early_rng) PBIT_EA_LAUNCH(false, true); else PBIT_EA_LAUNCH(false, false);
    }
#undef PBIT_EA_LAUNCH
    return hipGetLastError();
}

bool ea_slab_fits(const EaView &p) { return p.N <= kEaSlabMaxSites; }

hipError_t ea_slab(const EaView &p, int8_t *spins, int Rp, const uint32_t *table, int width, int s_begin, int s_end,
                   uint32_t sweep0, uint32_t rq0, Key key, hipStream_t st)
{
    if (!ea_slab_fits(p) || !p.slab_sites || Rp % 16 != 0 || width < 1 || s_end < s_begin)
        return hipErrorInvalidValue;
    if (s_end == s_begin) return hipSuccess;
    const size_t lds = sizeof(uint4) * (size_t)p.N;
    static const hipError_t lds_attr = [] {
        const int bytes = (int)sizeof(uint4) * kEaSlabMaxSites;
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_ea_slab<true>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
        if (e == hipSuccess)
            e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_ea_slab<false>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
        return e;
    }();
    if (lds_attr != hipSuccess) return lds_attr;
    const dim3 grid((unsigned)(Rp / 16));
    if (p.dense)
        hipLaunchKernelGGL((k_ea_slab<true>), grid, dim3(kSlabThreads), lds, st, spins,
                           reinterpret_cast<const uint2 *>(p.slab_sites), table, width, p.Lx, p.Ly, p.Lz, Rp, s_begin,
                           s_end, sweep0, rq0, key.k0, key.k1, 1u);
    else
        hipLaunchKernelGGL((k_ea_slab<false>), grid, dim3(kSlabThreads), lds, st, spins,
                           reinterpret_cast<const uint2 *>(p.slab_sites), table, width, p.Lx, p.Ly, p.Lz, Rp, s_begin,
                           s_end, sweep0, rq0, key.k0, key.k1, 1u);
    return hipGetLastError();
}

hipError_t ea_energy(const EaView &p, const int8_t *spins, int Rp, int R, int32_t *E, hipStream_t st)
{
    hipError_t e = fill_i32(E, R, 0, st);
    if (e != hipSuccess) return e;
    // a workgroup: 256 replicas x 16 chunks of kEnergySites sites
    const int64_t sites_per_block = 16 * kEnergySites;
    const int64_t gx = (p.N + sites_per_block - 1) / sites_per_block;
    if ((Rp + 255) / 256 > 65535) return hipErrorInvalidValue;
    dim3 grid((unsigned)gx, (unsigned)((Rp + 255) / 256));
    hipLaunchKernelGGL(k_ea_energy, grid, dim3(kThreads), 0, st, spins, p.J, p.h, p.Lx, p.Ly, p.Lz, Rp, R, E);
    return hipGetLastError();
}

}  // namespace pbit
