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

// Count of negative products J_d m_d, times 2, for the four replicas held in
// the bytes of one dword: spin bytes are +1 (0x01) or -1 (0xFF), so bit 1 of a
// byte is set exactly for -1; masking keeps nonzero couplings and the XOR
// flips the sign of J = -1 bonds.  Byte sums stay <= 12.
__device__ __forceinline__ uint32_t neg2(uint32_t m, uint32_t keep, uint32_t flip)
{
    return (m & keep) ^ flip;
}

// Decision table of one half-sweep, indexed by I + kFieldOff: the minority
// threshold Tm(beta_t, |I|), the mask that turns w into x (~0 for I >= 0),
// and the spin bytes taken on a minority and on a majority outcome.
constexpr int kFieldOff = 7;  // |I| <= 6 + |h| <= 7 on the cube
constexpr int kFieldSlots = 2 * kFieldOff + 1;

__device__ __forceinline__ void build_field_table(uint4 *tab, const uint32_t *__restrict__ trow, int width, int tid)
{
    if (tid < kFieldSlots) {
        const int I = tid - kFieldOff;
        const int a = min(I >= 0 ? I : -I, width - 1);
        const bool pos = I >= 0;
        tab[tid] = make_uint4(trow[a], pos ? 0xFFFFFFFFu : 0u, pos ? 0xFFu : 0x01u, pos ? 0x01u : 0xFFu);
    }
}

// One checkerboard half-sweep.  Block (cbw, spb): x threads walk 16-replica
// chunks, y threads walk the sites of one lattice row (y, z) = (blockIdx.y,
// blockIdx.z).  blockIdx.x = chunk-block * nsl + slab: with nsl = 8 the slab
// index equals the XCD a workgroup is dispatched to, so each XCD's L2 serves
// one replica slab of the whole lattice and neighbour rows are reused there.
__global__ __launch_bounds__(kThreads) void k_ea_halfsweep(int8_t *__restrict__ spins,
                                                           const uint32_t *__restrict__ code,
                                                           const uint32_t *__restrict__ trow, int width, int Lx,
                                                           int Ly, int Lz, int Rp, int colour, int nsl, int cs,
                                                           uint32_t sweep, uint32_t rq0, uint32_t k0, uint32_t k1)
{
    __shared__ uint4 tab[kFieldSlots];
    const int tid = threadIdx.x + blockDim.x * threadIdx.y;
    build_field_table(tab, trow, width, tid);
    __syncthreads();

    const int slab = blockIdx.x % nsl;
    const int qs = (blockIdx.x / nsl) * blockDim.x + threadIdx.x;
    const int q = slab * cs + qs;
    if (qs >= cs || 16 * q >= Rp) return;
    const int y = blockIdx.y, z = blockIdx.z;
    const uint32_t rowR = (uint32_t)Lx * (uint32_t)Rp;                 // bytes per lattice row
    const uint32_t planeR = rowR * (uint32_t)Ly;                        // bytes per plane
    const uint32_t base = (uint32_t)y * rowR + (uint32_t)z * planeR + 16u * (uint32_t)q;
    const uint32_t yp = (y + 1 == Ly ? 0u : (uint32_t)(y + 1)) * rowR + (uint32_t)z * planeR + 16u * (uint32_t)q;
    const uint32_t ym = (y == 0 ? (uint32_t)(Ly - 1) : (uint32_t)(y - 1)) * rowR + (uint32_t)z * planeR + 16u * (uint32_t)q;
    const uint32_t zp = (uint32_t)y * rowR + (z + 1 == Lz ? 0u : (uint32_t)(z + 1)) * planeR + 16u * (uint32_t)q;
    const uint32_t zm = (uint32_t)y * rowR + (z == 0 ? (uint32_t)(Lz - 1) : (uint32_t)(z - 1)) * planeR + 16u * (uint32_t)q;
    const uint32_t siteRow = (uint32_t)Lx * ((uint32_t)y + (uint32_t)Ly * (uint32_t)z);
    const int hx = Lx / 2;
    const int par = (colour + y + z) & 1;
    const uint32_t rg4 = rq0 + 4u * (uint32_t)q;  // Philox counter word 2 of this chunk's first group

    for (int kx = threadIdx.y; kx < hx; kx += blockDim.y) {
        const int x = 2 * kx + par;
        const uint32_t xR = (uint32_t)x * (uint32_t)Rp;
        const uint32_t xpR = (x + 1 == Lx ? 0u : (uint32_t)(x + 1)) * (uint32_t)Rp;
        const uint32_t xmR = (x == 0 ? (uint32_t)(Lx - 1) : (uint32_t)(x - 1)) * (uint32_t)Rp;
        const uint32_t offs[6] = {base + xpR, base + xmR, yp + xR, ym + xR, zp + xR, zm + xR};
        const uint32_t i = siteRow + (uint32_t)x;
        const uint32_t c = code[i];
        uint32_t cnt[4] = {0u, 0u, 0u, 0u};
#pragma unroll
        for (int d = 0; d < 6; ++d) {
            const uint4 v = *reinterpret_cast<const uint4 *>(spins + offs[d]);
            const uint32_t keep = ((c >> d) & 1u) * 0x02020202u;
            const uint32_t flip = ((c >> (kCodeFlipShift + d)) & 1u) * 0x02020202u;
            cnt[0] += neg2(v.x, keep, flip);
            cnt[1] += neg2(v.y, keep, flip);
            cnt[2] += neg2(v.z, keep, flip);
            cnt[3] += neg2(v.w, keep, flip);
        }
        // LDS byte address of the entry for I = base_i (no negative products)
        const int entry0 = ((int)(int8_t)(c >> kCodeBaseShift) + kFieldOff) * (int)sizeof(uint4);
        const char *tbase = reinterpret_cast<const char *>(tab);
        uint32_t out[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const Block4 b = philox(i, sweep, rg4 + (uint32_t)k, kDomainSweep, k0, k1);
            // bytes of cnt are c2 <= 12, so cnt * 16 keeps each 16 c2 <= 192 in its own byte
            const uint32_t off16 = cnt[k] << 4;
            uint32_t packed = 0;
#pragma unroll
            for (int p = 0; p < 4; ++p) {
                const int o = (int)((off16 >> (8 * p)) & 0xFFu);  // 16 c2, with I = base_i - c2
                const uint4 e = *reinterpret_cast<const uint4 *>(tbase + entry0 - o);
                const uint32_t xw = b.w[p] ^ e.y;
                packed |= (xw < e.x ? e.z : e.w) << (8 * p);
            }
            out[k] = packed;
        }
        *reinterpret_cast<uint4 *>(spins + base + xR) = make_uint4(out[0], out[1], out[2], out[3]);
    }
}

// From-scratch energy: E[r] += -sum over a chunk of sites of (bond + field)
// terms.  Each bond (i, i + e_d) is visited once, from its lower-end site i.
__global__ __launch_bounds__(kThreads) void k_ea_energy(const int8_t *__restrict__ spins, const int8_t *__restrict__ J,
                                                        const int8_t *__restrict__ h, int Lx, int Ly, int Lz, int Rp,
                                                        int R, int64_t chunk, int32_t *__restrict__ E)
{
    const int r = blockIdx.x * kThreads + threadIdx.x;
    if (r >= R) return;
    const int64_t N = (int64_t)Lx * Ly * Lz;
    const int64_t plane = (int64_t)Lx * Ly;
    const int64_t s0 = (int64_t)blockIdx.y * chunk;
    const int64_t s1 = min(s0 + chunk, N);
    int32_t e = 0;
    for (int64_t i = s0; i < s1; ++i) {
        const int x = (int)(i % Lx);
        const int y = (int)((i / Lx) % Ly);
        const int z = (int)(i / plane);
        const int mi = spins[(size_t)i * Rp + r];
        const int64_t jx = wrap_inc(x, Lx) + (int64_t)Lx * y + plane * z;
        const int64_t jy = x + (int64_t)Lx * wrap_inc(y, Ly) + plane * z;
        const int64_t jz = x + (int64_t)Lx * y + plane * wrap_inc(z, Lz);
        const int s = J[i] * spins[(size_t)jx * Rp + r] + J[N + i] * spins[(size_t)jy * Rp + r] +
                      J[2 * N + i] * spins[(size_t)jz * Rp + r] + (h ? h[i] : 0);
        e -= mi * s;
    }
    atomicAdd(E + r, e);
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

hipError_t ea_halfsweep(const EaView &p, int8_t *spins, int Rp, int colour, const uint32_t *trow, int width,
                        uint32_t sweep, uint32_t rq0, Key key, hipStream_t st)
{
    if (width < 1 || width > kFieldOff + 1 || Rp % 16 != 0) return hipErrorInvalidValue;
    if ((uint64_t)p.N * (uint64_t)Rp >= ((uint64_t)1 << 32)) return hipErrorInvalidValue;  // 32-bit byte offsets
    if (p.Ly > 65535 || p.Lz > 65535) return hipErrorInvalidValue;                      // grid y / z limits
    const int C = Rp / 16;              // 16-replica chunks
    const int nsl = C >= 8 ? 8 : 1;     // replica slabs, one per XCD when there are enough chunks
    const int cs = (C + nsl - 1) / nsl; // chunks per slab
    int cbw = 1;
    while (cbw < cs && cbw < 64) cbw *= 2;
    const int spb = kThreads / cbw;
    const int ncb = (cs + cbw - 1) / cbw;
    dim3 grid((unsigned)(nsl * ncb), (unsigned)p.Ly, (unsigned)p.Lz), block((unsigned)cbw, (unsigned)spb);
    hipLaunchKernelGGL(k_ea_halfsweep, grid, block, 0, st, spins, p.code, trow, width, p.Lx, p.Ly, p.Lz, Rp, colour,
                       nsl, cs, sweep, rq0, key.k0, key.k1);
    return hipGetLastError();
}

hipError_t ea_energy(const EaView &p, const int8_t *spins, int Rp, int R, int32_t *E, hipStream_t st)
{
    hipError_t e = fill_i32(E, R, 0, st);
    if (e != hipSuccess) return e;
    // 64 sites per block row, more when that would exceed the grid's y limit
    const int64_t chunk = std::max<int64_t>(64, (p.N + 65534) / 65535);
    dim3 grid(blocks_for(R), (unsigned)((p.N + chunk - 1) / chunk));
    hipLaunchKernelGGL(k_ea_energy, grid, dim3(kThreads), 0, st, spins, p.J, p.h, p.Lx, p.Ly, p.Lz, Rp, R, chunk, E);
    return hipGetLastError();
}

}  // namespace pbit
