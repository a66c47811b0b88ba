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

// One checkerboard half-sweep: every site of `colour`, 16 replicas per thread.
__global__ __launch_bounds__(kThreads) void k_ea_halfsweep(int8_t *__restrict__ spins,
                                                           const uint32_t *__restrict__ code,
                                                           const uint32_t *__restrict__ trow, int width, int Lx,
                                                           int Ly, int Lz, int Rp, int colour, uint32_t sweep,
                                                           uint32_t rq0, uint32_t k0, uint32_t k1)
{
    __shared__ uint32_t T[16];
    if (threadIdx.x < width && threadIdx.x < 16) T[threadIdx.x] = trow[threadIdx.x];
    __syncthreads();

    const int chunks = Rp / 16;
    const int64_t half = (int64_t)Lx * Ly * Lz / 2;
    const int64_t gid = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (gid >= half * chunks) return;
    const int q = (int)(gid % chunks);
    const int64_t j = gid / chunks;
    const int hx = Lx / 2;
    const int kx = (int)(j % hx);
    const int64_t row = j / hx;
    const int y = (int)(row % Ly);
    const int z = (int)(row / Ly);
    const int x = 2 * kx + ((colour + y + z) & 1);
    const int64_t plane = (int64_t)Lx * Ly;
    const int64_t i = x + (int64_t)Lx * y + plane * z;
    const int64_t nb[6] = {
        wrap_inc(x, Lx) + (int64_t)Lx * y + plane * z, wrap_dec(x, Lx) + (int64_t)Lx * y + plane * z,
        x + (int64_t)Lx * wrap_inc(y, Ly) + plane * z, x + (int64_t)Lx * wrap_dec(y, Ly) + plane * z,
        x + (int64_t)Lx * y + plane * wrap_inc(z, Lz), x + (int64_t)Lx * y + plane * wrap_dec(z, Lz)};

    const uint32_t c = code[i];
    const int base = (int)(int8_t)(c >> kCodeBaseShift);
    uint32_t cnt[4] = {0u, 0u, 0u, 0u};
#pragma unroll
    for (int d = 0; d < 6; ++d) {
        const uint4 v = *reinterpret_cast<const uint4 *>(spins + (size_t)nb[d] * Rp + 16 * q);
        const uint32_t keep = ((c >> d) & 1u) * 0x02020202u;
        const uint32_t flip = ((c >> (kCodeFlipShift + d)) & 1u) * 0x02020202u;
        cnt[0] += neg2(v.x, keep, flip);
        cnt[1] += neg2(v.y, keep, flip);
        cnt[2] += neg2(v.z, keep, flip);
        cnt[3] += neg2(v.w, keep, flip);
    }
    const int top = width - 1;
    uint32_t out[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const Block4 b = philox((uint32_t)i, sweep, rq0 + 4u * (uint32_t)q + (uint32_t)k, kDomainSweep, k0, k1);
        uint32_t packed = 0;
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            const int I = base - (int)((cnt[k] >> (8 * p)) & 0xFFu);
            const int a = min(I >= 0 ? I : -I, top);
            packed |= (uint32_t)(uint8_t)decide(I, T[a], b.w[p]) << (8 * p);
        }
        out[k] = packed;
    }
    *reinterpret_cast<uint4 *>(spins + (size_t)i * Rp + 16 * q) = make_uint4(out[0], out[1], out[2], out[3]);
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
    if (width < 1 || width > 16 || Rp % 16 != 0) return hipErrorInvalidValue;
    const int64_t work = p.N / 2 * (Rp / 16);
    hipLaunchKernelGGL(k_ea_halfsweep, dim3(blocks_for(work)), dim3(kThreads), 0, st, spins, p.code, trow, width, p.Lx,
                       p.Ly, p.Lz, Rp, colour, sweep, rq0, key.k0, key.k1);
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
