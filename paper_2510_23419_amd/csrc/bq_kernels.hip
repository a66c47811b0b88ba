// bq_kernels.hip — biclique K_{na,nb} (paper Sec. 3) on gfx950.
//
// A biclique half-sweep updates one whole side: the fields of side A for every
// replica are the int8 product F = M_B J^T (replicas x sites), exact in int32
// since |F| <= nb (all neighbours are shared by the whole update group,
// Sec. 1.2.2, which makes the step a dense GEMM).  The product runs on the
// 32x32x32 int8 MFMA; the heat-bath decision is the epilogue.
//
// Device layout: MA [Rp][na_p] and MB [Rp][nb_p], replica-major, so a replica
// row is K-contiguous for the MFMA A operand; J [na_p][nb_p] and its transpose
// JT [nb_p][na_p] are K-contiguous for the B operand.  Padding sites and
// couplings are zero, so they add nothing to any field.
//
// MFMA accumulator layout (32x32 tile, 64 lanes, 16 int32 per lane): lane l
// holds column n = l % 32 and rows m = 8 (j / 4) + 4 (l / 32) + j % 4 for
// j = 0..15.  Rows are replicas and columns are sites, so each lane holds four
// aligned groups of four replicas of one site: exactly the four words of one
// Philox block per group.
#include "device.h"
#include "internal.h"

namespace pbit {

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

constexpr int kThreads = 256;
constexpr int kTileR = 64;  // replicas per workgroup tile
constexpr int kTileS = 64;  // sites per workgroup tile

__global__ __launch_bounds__(kThreads) void k_bq_init(int8_t *__restrict__ MA, int8_t *__restrict__ MB, int na, int nb,
                                                      int na_p, int nb_p, int R, uint32_t rq0, uint32_t k0,
                                                      uint32_t k1)
{
    const int groups = (R + 3) / 4;
    const int64_t gid = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    const int64_t N = (int64_t)na + nb;
    if (gid >= N * groups) return;
    const int g = (int)(gid % groups);
    const int i = (int)(gid / groups);
    const Block4 b = philox((uint32_t)i, 0u, rq0 + (uint32_t)g, kDomainInit, k0, k1);
    for (int p = 0; p < 4; ++p) {
        const int r = 4 * g + p;
        if (r >= R) break;
        const int8_t s = init_spin(b.w[p]);
        if (i < na)
            MA[(size_t)r * na_p + i] = s;
        else
            MB[(size_t)r * nb_p + (i - na)] = s;
    }
}

template <bool TO_DEVICE>
__global__ __launch_bounds__(kThreads) void k_bq_copy(int8_t *__restrict__ rows, int8_t *__restrict__ MA,
                                                      int8_t *__restrict__ MB, int na, int nb, int na_p, int nb_p,
                                                      int R)
{
    const int64_t N = (int64_t)na + nb;
    const int64_t gid = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (gid >= N * R) return;
    const int r = (int)(gid / N);
    const int i = (int)(gid % N);
    int8_t *dev = i < na ? MA + (size_t)r * na_p + i : MB + (size_t)r * nb_p + (i - na);
    if (TO_DEVICE)
        *dev = rows[gid];
    else
        rows[gid] = *dev;
}

// One side's half-sweep (ENERGY = false) or the bond part of the energy
// (ENERGY = true: E[r] -= sum_i m_i F_i for this side).
//   Mo   other side's spins [Rp][Ko]
//   Jx   couplings [Ns_p][Ko]: row i holds J between site i of this side and the other side
//   Ms   this side's spins [Rp][Ns_p]
template <bool ENERGY>
__global__ __launch_bounds__(kThreads) void k_bq_halfsweep(const int8_t *__restrict__ Mo, const int8_t *__restrict__ Jx,
                                                           const int8_t *__restrict__ hs, int8_t *__restrict__ Ms,
                                                           const uint32_t *__restrict__ trow, int width, int Ns,
                                                           int Ns_p, int Ko, int R, uint32_t site_base,
                                                           uint32_t sweep, uint32_t rq0, uint32_t k0, uint32_t k1,
                                                           int32_t *__restrict__ E)
{
    extern __shared__ uint32_t T[];
    if (!ENERGY)
        for (int a = threadIdx.x; a < width; a += kThreads) T[a] = trow[a];
    __syncthreads();

    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int r_base = blockIdx.y * kTileR + 32 * (wave >> 1);
    const int s_base = blockIdx.x * kTileS + 32 * (wave & 1);
    const int kg = lane >> 5;   // which half of the 32-wide K step this lane feeds
    const int ln = lane & 31;

    const int8_t *arow = Mo + (size_t)(r_base + ln) * Ko + 16 * kg;
    const int8_t *brow = Jx + (size_t)(s_base + ln) * Ko + 16 * kg;
    v16i acc = {0};
    for (int k = 0; k < Ko; k += 32) {
        const v4i a = *reinterpret_cast<const v4i *>(arow + k);
        const v4i b = *reinterpret_cast<const v4i *>(brow + k);
        acc = __builtin_amdgcn_mfma_i32_32x32x32_i8(a, b, acc, 0, 0, 0);
    }

    const int site = s_base + ln;
    const int hval = site < Ns ? hs[site] : 0;
    const int top = width - 1;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int r4 = r_base + 8 * q + 4 * kg;  // first replica of this lane's group q
        if (ENERGY) {
#pragma unroll
            for (int p = 0; p < 4; ++p) {
                const int r = r4 + p;
                int32_t v = 0;
                if (site < Ns && r < R) v = -(int32_t)Ms[(size_t)r * Ns_p + site] * acc[4 * q + p];
                // sum over the 32 sites of this half-wave
                for (int off = 16; off > 0; off >>= 1) v += __shfl_xor(v, off, 32);
                if (ln == 0 && r < R) atomicAdd(E + r, v);
            }
        } else {
            const Block4 b =
                philox(site_base + (uint32_t)site, sweep, rq0 + (uint32_t)(r4 >> 2), kDomainSweep, k0, k1);
#pragma unroll
            for (int p = 0; p < 4; ++p) {
                const int r = r4 + p;
                const int I = acc[4 * q + p] + hval;
                const int a = min(I >= 0 ? I : -I, top);
                const int8_t m = decide(I, T[a], b.w[p]);
                if (site < Ns && r < R) Ms[(size_t)r * Ns_p + site] = m;
            }
        }
    }
}

// Field part of the energy: E[r] -= sum_i h_i m_i over both sides.
__global__ __launch_bounds__(kThreads) void k_bq_field_energy(const int8_t *__restrict__ MA,
                                                              const int8_t *__restrict__ MB,
                                                              const int8_t *__restrict__ hA,
                                                              const int8_t *__restrict__ hB, int na_p, int nb_p,
                                                              int R, int32_t *__restrict__ E)
{
    const int r = blockIdx.x;
    if (r >= R) return;
    int32_t e = 0;
    for (int a = threadIdx.x; a < na_p; a += kThreads) e -= hA[a] * MA[(size_t)r * na_p + a];
    for (int b = threadIdx.x; b < nb_p; b += kThreads) e -= hB[b] * MB[(size_t)r * nb_p + b];
    for (int off = 32; off > 0; off >>= 1) e += __shfl_xor(e, off, 64);
    if ((threadIdx.x & 63) == 0) atomicAdd(E + r, e);
}

}  // namespace

static inline unsigned blocks_for(int64_t work) { return (unsigned)((work + kThreads - 1) / kThreads); }

hipError_t bq_init(const BqView &p, int8_t *MA, int8_t *MB, int R, uint32_t rq0, Key key, hipStream_t st)
{
    const int64_t work = ((int64_t)p.na + p.nb) * ((R + 3) / 4);
    hipLaunchKernelGGL(k_bq_init, dim3(blocks_for(work)), dim3(kThreads), 0, st, MA, MB, p.na, p.nb, p.na_p, p.nb_p,
                       R, rq0, key.k0, key.k1);
    return hipGetLastError();
}

hipError_t bq_from_rows(const BqView &p, const int8_t *src_rn, int R, int8_t *MA, int8_t *MB, hipStream_t st)
{
    const int64_t work = ((int64_t)p.na + p.nb) * R;
    hipLaunchKernelGGL(k_bq_copy<true>, dim3(blocks_for(work)), dim3(kThreads), 0, st, const_cast<int8_t *>(src_rn), MA,
                       MB, p.na, p.nb, p.na_p, p.nb_p, R);
    return hipGetLastError();
}

hipError_t bq_to_rows(const BqView &p, const int8_t *MA, const int8_t *MB, int8_t *dst_rn, int R, hipStream_t st)
{
    const int64_t work = ((int64_t)p.na + p.nb) * R;
    hipLaunchKernelGGL(k_bq_copy<false>, dim3(blocks_for(work)), dim3(kThreads), 0, st, dst_rn,
                       const_cast<int8_t *>(MA), const_cast<int8_t *>(MB), p.na, p.nb, p.na_p, p.nb_p, R);
    return hipGetLastError();
}

hipError_t bq_halfsweep(const BqView &p, int side, int8_t *MA, int8_t *MB, int R, int Rp, const uint32_t *trow,
                        int width, uint32_t sweep, uint32_t rq0, Key key, hipStream_t st)
{
    if (Rp % kTileR != 0 || p.na_p % kTileS != 0 || p.nb_p % kTileS != 0 || width < 1) return hipErrorInvalidValue;
    const bool A = side == 0;
    const int Ns_p = A ? p.na_p : p.nb_p;
    dim3 grid((unsigned)(Ns_p / kTileS), (unsigned)(Rp / kTileR));
    const size_t lds = sizeof(uint32_t) * (size_t)width;
    hipLaunchKernelGGL(k_bq_halfsweep<false>, grid, dim3(kThreads), lds, st, A ? MB : MA, A ? p.J : p.JT,
                       A ? p.hA : p.hB, A ? MA : MB, trow, width, A ? p.na : p.nb, Ns_p, A ? p.nb_p : p.na_p, R,
                       A ? 0u : (uint32_t)p.na, sweep, rq0, key.k0, key.k1, (int32_t *)nullptr);
    return hipGetLastError();
}

hipError_t bq_energy(const BqView &p, const int8_t *MA, const int8_t *MB, int R, int Rp, int32_t *E, hipStream_t st)
{
    if (Rp % kTileR != 0) return hipErrorInvalidValue;
    hipError_t e = fill_i32(E, R, 0, st);
    if (e != hipSuccess) return e;
    dim3 grid((unsigned)(p.na_p / kTileS), (unsigned)(Rp / kTileR));
    hipLaunchKernelGGL(k_bq_halfsweep<true>, grid, dim3(kThreads), 0, st, MB, p.J, p.hA, const_cast<int8_t *>(MA),
                       (const uint32_t *)nullptr, 1, p.na, p.na_p, p.nb_p, R, 0u, 0u, 0u, 0u, 0u, E);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_bq_field_energy, dim3((unsigned)R), dim3(kThreads), 0, st, MA, MB, p.hA, p.hB, p.na_p, p.nb_p,
                       R, E);
    return hipGetLastError();
}

}  // namespace pbit
