// bq_slab.hip — the biclique sweep of a small instance with everything in LDS, for
// runs of sweeps in one launch.
//
// A half-sweep of a biclique updates one side from the other (Sec. 3; update
// groups, Sec. 1.2.2): F = J m_other, I = F + h, heat-bath decision.  For sides of
// at most 512 sites the couplings fit in LDS as two-bit codes of J + 1 in both
// orientations (J for side A's fields, J^T for side B's: 64 KiB each at 512 x 512),
// next to the int8 spin rows of 16 replicas.  Replica slices never interact, so a
// workgroup holds one slice and runs a whole chunk of sweeps with workgroup
// barriers only: no launch per half-sweep and no coupling traffic after the
// first load.  Each half-sweep is a v_mfma_i32_16x16x64_i8 product of the spin rows
// (16 replicas x K sites of the other side) with the widened codes (K x 16 sites),
// int32 sums; with codes J + 1 the product exceeds the field by the replica's spin
// sum over the other side, which is subtracted.  The decision is the carry of the
// Philox word plus the 64-bit word S(I) (Tm(|I|) for I >= 0, 2^32 - Tm for I < 0),
// as in the other kernels, with the same counters, so results do not depend on
// the kernel.
//
// Spins stay in the library's int8 biclique layout in global memory (MA [Rp][na_p],
// MB [Rp][nb_p], padding sites zero); the kernel loads a slice at its start and
// stores it at its end.
#include <hip/hip_runtime.h>

#include "bq.h"
#include "device.h"
#include "internal.h"

namespace pbit {

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));

constexpr int kThreads = 1024;  // 16 waves: four per SIMD
constexpr int kWaves = kThreads / 64;
constexpr int kBlkPerWave = 2;  // 16-site blocks per wave and half-sweep: 32 blocks at 512 sites
constexpr int kMaxLds = 160 * 1024 - 4096;

// 4 x 4 byte transpose across a quad of lanes: lane u holds bytes M[u][0..3] and
// receives M[0..3][u] (two DPP quad permutations and two byte permutes).
__device__ __forceinline__ uint32_t quad_transpose4(uint32_t d, int u)
{
    const uint32_t t = (uint32_t)__builtin_amdgcn_mov_dpp((int)d, 0xB1, 0xF, 0xF, false);  // quad_perm [1,0,3,2]
    const uint32_t d1 = __builtin_amdgcn_perm(t, d, (u & 1) ? 0x03070105u : 0x06020400u);
    const uint32_t t2 = (uint32_t)__builtin_amdgcn_mov_dpp((int)d1, 0x4E, 0xF, 0xF, false);  // quad_perm [2,3,0,1]
    return __builtin_amdgcn_perm(t2, d1, (u & 2) ? 0x03020706u : 0x05040100u);
}

// 16 int8 K values from one word of two-bit codes: byte i of dword j is the code at
// bits 8 i + 2 j (K index 4 j + i of the 16).
__device__ __forceinline__ v4i widen16(uint32_t x)
{
    return v4i{(int)(x & 0x03030303u), (int)((x >> 2) & 0x03030303u), (int)((x >> 4) & 0x03030303u),
               (int)((x >> 6) & 0x03030303u)};
}

// Codes of one orientation into LDS: word (kb, s, g) holds J[s][64 kb + 16 g + k] + 1
// for k = 0..15 (k = 4 j + i at bits 8 i + 2 j), words ordered [kb][s][g] so that the
// 64 lanes of an MFMA read 64 consecutive words.  Jrow is [ns_p][ko] int8 (padding 0).
__device__ void stage_codes(const int8_t *__restrict__ Jrow, int ns_p, int ko, uint32_t *codes)
{
    const int nw = (ko / 16) * ns_p;  // words: (ko / 64) K steps x ns_p sites x 4 groups
    for (int wi = threadIdx.x; wi < nw; wi += kThreads) {
        const int g = wi & 3, s = (wi >> 2) % ns_p, kb = (wi >> 2) / ns_p;
        const uint4 v = *reinterpret_cast<const uint4 *>(Jrow + (size_t)s * ko + 64 * kb + 16 * g);
        const uint32_t dw[4] = {v.x, v.y, v.z, v.w};
        uint32_t w = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const uint32_t c = (uint32_t)((int)(int8_t)(dw[j] >> (8 * i)) + 1);  // K index 4 j + i
                // K index k = 4 j' + i' goes to bits 8 i' + 2 j'
                const int k = 4 * j + i;
                w |= c << (8 * (k & 3) + 2 * (k >> 2));
            }
        codes[wi] = w;
    }
}

// Sweeps [s_begin, s_end) of replicas [RS blockIdx.x, + RS) of a small biclique.
//
// RS = 16 fills the MFMA's 16 rows.  RS = 8 gives twice the workgroups for the same
// replicas (a launch of 1024 replicas then uses 128 CUs instead of 64): the rows 8 .. 15
// read a zero row, and the two site blocks of a wave, whose valid rows sit in lanes
// 0 .. 31 of their accumulators, are packed into one register (lanes 32 .. 63 from the
// second block: v_permlane32_swap), so the decision epilogue runs once per wave for
// both blocks instead of twice on half-empty lanes.
template <int RS>
__global__ __launch_bounds__(kThreads) void k_bq_slab(BqView p, int8_t *__restrict__ MA, int8_t *__restrict__ MB,
                                                      int Rp, const uint32_t *__restrict__ table, int width,
                                                      int s_begin, int s_end, uint32_t sweep0, uint32_t rq0,
                                                      uint32_t k0, uint32_t k1, uint32_t one)
{
    static_assert(RS == 16 || RS == 8, "slices of 16 or 8 replicas");
    constexpr int kRows = RS == 16 ? 16 : RS + 1;  // spin rows, plus a zero row for the unused MFMA rows
    extern __shared__ uint4 dyn[];
    // spin sums per replica over side A and over side B, two of each by sweep parity: a
    // half-sweep's decisions read the other side's sum while its epilogue adds up its own
    // side's new spins for the next half-sweep
    __shared__ int32_t magA[2][RS], magB[2][RS];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform: block tests are scalar branches
    const int na = p.na, nb = p.nb, na_p = p.na_p, nb_p = p.nb_p;
    const int pitch = na_p + nb_p + 16;
    // LDS: codes of J (side A's fields, K over side B), codes of J^T, spin rows, decision words
    uint32_t *codesA = reinterpret_cast<uint32_t *>(dyn);
    uint32_t *codesB = codesA + (size_t)na_p * nb_p / 16;
    uint8_t *sp = reinterpret_cast<uint8_t *>(codesB + (size_t)nb_p * na_p / 16);
    // decision words of two sweeps: those of sweep s + 1 are written during sweep s
    uint64_t *Sw2 = reinterpret_cast<uint64_t *>(sp + (size_t)kRows * pitch);
    const int r0 = RS * blockIdx.x;  // first replica of the slice (local to this call)

    stage_codes(p.J, na_p, nb_p, codesA);
    stage_codes(p.JT, nb_p, na_p, codesB);
    for (int k = tid; k < kRows * (pitch / 16); k += kThreads) {
        const int r = k / (pitch / 16), c16 = k % (pitch / 16), c = 16 * c16;
        uint4 v = make_uint4(0, 0, 0, 0);
        if (r < RS) {
            if (c < na_p)
                v = *reinterpret_cast<const uint4 *>(MA + (size_t)(r0 + r) * na_p + c);
            else if (c < na_p + nb_p)
                v = *reinterpret_cast<const uint4 *>(MB + (size_t)(r0 + r) * nb_p + (c - na_p));
        }
        *reinterpret_cast<uint4 *>(sp + r * pitch + c) = v;
    }

    const int top = width - 1;
    const int col = lane & 15, grp = lane >> 4;  // MFMA: row / column lane%16, K group and C rows lane/16
    auto build_words = [&](int s) {
        const uint32_t *trow = table + (size_t)s * width;
        uint64_t *Sw = Sw2 + (size_t)(s & 1) * (2 * top + 1);
        for (int e = tid; e <= 2 * top; e += kThreads) {
            const int I = e - top;
            const uint32_t Tm = trow[I >= 0 ? I : -I];
            Sw[e] = I >= 0 ? (uint64_t)Tm : ((uint64_t)1 << 32) - Tm;
        }
    };
    if (s_begin < s_end) build_words(s_begin);
    __syncthreads();  // the spin rows are in LDS
    // side B's spin sums for the first half-sweep, one wave per replica row; side A's sums
    // start at zero
    if (wave < RS) {
        const uint32_t *row = reinterpret_cast<const uint32_t *>(sp + wave * pitch + na_p);
        int v = 0;
        for (int d = lane; d < nb_p / 4; d += 64) v = __builtin_amdgcn_sdot4((int)row[d], 0x01010101, v, false);
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        if (lane == 0) {
            magB[s_begin & 1][wave] = v;
            magA[s_begin & 1][wave] = 0;
        }
    }
    __syncthreads();  // codes, spins, the first decision words and sums are in LDS
    // A rows: replica row col, or (RS = 8, col >= 8) the zero row
    const int arow_r = col < RS ? col : RS;
    // the replica rows of a lane's accumulator elements: 4 gr + j (RS = 8: the merged
    // register holds rows 0 .. 7 of block wave in lanes 0 .. 31 and of block wave + kWaves
    // in lanes 32 .. 63)
    const int gr = RS == 16 ? grp : (grp & 1);
    // two barriers per sweep, one after each half-sweep (its spins, sums and, after side B,
    // the next sweep's decision words are then complete)
    for (int s = s_begin; s < s_end; ++s) {
        const int par = s & 1;
        const uint32_t t = sweep0 + (uint32_t)s;
        const char *Sb = reinterpret_cast<const char *>(Sw2 + (size_t)par * (2 * top + 1));
        // the sums filled in the next two half-sweeps start at zero (last read a sweep ago)
        if (tid < RS) {
            magB[par ^ 1][tid] = 0;
            magA[par ^ 1][tid] = 0;
        }
#pragma unroll 1
        for (int side = 0; side < 2; ++side) {
            const int ns = side == 0 ? na : nb, ns_p = side == 0 ? na_p : nb_p;
            const int ko = side == 0 ? nb_p : na_p;        // K: sites of the other side
            const int in_col = side == 0 ? na_p : 0;       // the other side's columns
            const int out_col = side == 0 ? 0 : na_p;      // this side's columns
            const uint32_t *codes = side == 0 ? codesA : codesB;
            const int8_t *hs = side == 0 ? p.hA : p.hB;
            const uint32_t site_base = side == 0 ? 0u : (uint32_t)na;
            const int nblk = ns_p / 16;
            // the random words and fields of this lane's sites first: they do not depend on
            // the spins, so they are drawn while the LDS reads below are in flight (RS = 16:
            // one block of four replicas for each of the wave's two site blocks; RS = 8: one
            // for the lane's site in the merged register)
            constexpr int kDraws = RS == 16 ? kBlkPerWave : 1;
            Block4 w[kDraws];
            int hv[kDraws];
#pragma unroll
            for (int q = 0; q < kDraws; ++q) {
                const int blk = wave + kWaves * (RS == 16 ? q : (lane >> 5));
                const int site = blk * 16 + col;
                hv[q] = site < ns_p ? (int)hs[site] : 0;
                w[q] = philox(site_base + (uint32_t)site, t, rq0 + (uint32_t)(blockIdx.x * (RS / 4) + gr),
                              kDomainSweep, k0, k1);
            }
            // the other side's spin sums (side B's of this sweep's parity, side A's just filled)
            const int32_t *mag = side == 0 ? magB[par] : magA[par];
            int32_t *mag_out = side == 0 ? magA[par] : magB[par ^ 1];
            // fields of up to kBlkPerWave 16-site blocks per wave (blocks wave, wave + kWaves)
            v4i acc[kBlkPerWave];
#pragma unroll
            for (int q = 0; q < kBlkPerWave; ++q) acc[q] = v4i{0, 0, 0, 0};
            const uint8_t *arow = sp + arow_r * pitch + in_col + 16 * grp;
            const int nkb = ko / 64;
            // the K loop unrolled to its largest trip count (ko <= 512: 8 steps) under
            // wave-uniform guards: the spin rows then sit at fixed offsets from one
            // address, the code words of step kb at kb * 4 ns_p words from a pointer that
            // advances once per step, and block q's at a fixed offset from block 0's
            const bool one_blk = wave < nblk, two = wave + kWaves < nblk;  // this wave's blocks
            const uint32_t *ck = codes + (wave * 16 + col) * 4 + grp;
            constexpr int kMaxKb = 512 / 64;
            static_assert(kBlkPerWave == 2, "two blocks per wave below");
#pragma unroll
            for (int kb = 0; kb < kMaxKb; ++kb) {
                if (one_blk && kb < nkb) {
                    const v4i a = *reinterpret_cast<const v4i *>(arow + 64 * kb);
                    const uint32_t c0 = ck[0];
                    acc[0] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a, widen16(c0), acc[0], 0, 0, 0);
                    if (two) {
                        const uint32_t c1 = ck[64 * kWaves];
                        acc[1] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a, widen16(c1), acc[1], 0, 0, 0);
                    }
                    ck += (size_t)ns_p * 4;
                }
            }
            // decisions of one site block in a lane: site blk * 16 + col, replicas 4 gr .. 4 gr
            // + 3 (one Philox block); the four bytes are transposed across the lane quad so
            // that each lane writes four consecutive sites of one replica row
            const int u4 = lane & 3;
            auto decide = [&](const v4i &f, int blk, int hval, const Block4 &wq) {
                const int site = blk * 16 + col;
                const int flo = -top - hval, fhi = top - hval;
                const int base8 = 8 * (hval + top);
                uint32_t sgn[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int F = f[j] - mag[4 * gr + j];
                    const int Fc = min(max(F, flo), fhi);
                    const uint64_t S =
                        *static_cast<const uint64_t *>(__builtin_assume_aligned(Sb + 8 * Fc + base8, 8));
                    sgn[j] = (uint32_t)(((uint64_t)wq.w[j] * one + S) >> 32);
                }
                const uint32_t lo = __builtin_amdgcn_perm(sgn[1], sgn[0], 0x0C0C0400u);
                const uint32_t hi = __builtin_amdgcn_perm(sgn[3], sgn[2], 0x0C0C0400u);
                uint32_t packed = __builtin_amdgcn_perm(0u, 0xFF01u, __builtin_amdgcn_perm(hi, lo, 0x05040100u));
                if (site >= ns) packed = 0u;  // padding sites stay zero
                const uint32_t x = quad_transpose4(packed, u4);
                *reinterpret_cast<uint32_t *>(sp + (4 * gr + u4) * pitch + out_col + blk * 16 + (col & ~3)) = x;
                // replica 4 gr + u4's sum over these four sites, then over the block's four
                // site quads (lanes 4 and 8 apart in the row of 16), added once per block
                int ps = __builtin_amdgcn_sdot4((int)x, 0x01010101, 0, false);
                ps += __builtin_amdgcn_update_dpp(0, ps, 0x124, 0xF, 0xF, false);  // row_ror:4
                ps += __builtin_amdgcn_update_dpp(0, ps, 0x128, 0xF, 0xF, false);  // row_ror:8
                if ((col & 12) == 0) atomicAdd(&mag_out[4 * gr + u4], ps);
            };
            if constexpr (RS == 16) {
#pragma unroll
                for (int q = 0; q < kBlkPerWave; ++q)
                    if (wave + kWaves * q < nblk) decide(acc[q], wave + kWaves * q, hv[q], w[q]);
            } else {
                // rows 0 .. 7 of both blocks in one register: lanes 32 .. 63 take lanes 0 .. 31
                // of the second block's accumulator
                v4i m;
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    m[j] = (int)__builtin_amdgcn_permlane32_swap((unsigned)acc[0][j], (unsigned)acc[1][j], false,
                                                                 false)[0];
                const int blk = wave + kWaves * (lane >> 5);
                if (blk < nblk) decide(m, blk, hv[0], w[0]);  // the same on all 16 lanes of a DPP row
            }
            if (side == 1 && s + 1 < s_end) build_words(s + 1);  // published by the next barrier
            __syncthreads();
        }
    }

    for (int k = tid; k < RS * ((na_p + nb_p) / 16); k += kThreads) {
        const int r = k / ((na_p + nb_p) / 16), c = 16 * (k % ((na_p + nb_p) / 16));
        const uint4 v = *reinterpret_cast<const uint4 *>(sp + r * pitch + c);
        if (c < na_p)
            *reinterpret_cast<uint4 *>(MA + (size_t)(r0 + r) * na_p + c) = v;
        else
            *reinterpret_cast<uint4 *>(MB + (size_t)(r0 + r) * nb_p + (c - na_p)) = v;
    }
}

// LDS of a launch: the two code orientations, the spin rows (RS = 8: plus the zero row)
// and the decision words of two sweeps
size_t slab_lds(const BqView &p, int width, int rs)
{
    const int rows = rs == 16 ? 16 : rs + 1;
    return (size_t)2 * p.na_p * p.nb_p / 4 + (size_t)rows * (p.na_p + p.nb_p + 16) +
           2 * sizeof(uint64_t) * (size_t)(2 * width - 1);
}

template <int RS>
hipError_t slab_launch(const BqView &p, int8_t *MA, int8_t *MB, int Rp, const uint32_t *table, int width,
                       int s_begin, int s_end, uint32_t sweep0, uint32_t rq0, Key key, hipStream_t st)
{
    static const hipError_t lds_attr = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_bq_slab<RS>),
                                                           hipFuncAttributeMaxDynamicSharedMemorySize, kMaxLds);
    if (lds_attr != hipSuccess) return lds_attr;
    hipLaunchKernelGGL(k_bq_slab<RS>, dim3((unsigned)(Rp / RS)), dim3(kThreads), slab_lds(p, width, RS), st, p, MA,
                       MB, Rp, table, width, s_begin, s_end, sweep0, rq0, key.k0, key.k1, 1u);
    return hipGetLastError();
}

}  // namespace

int bq_slab_rs(int Rp, int rs)
{
    if (rs == 16 || rs == 8) return Rp % rs == 0 ? rs : 0;
    if (rs != 0) return 0;
    // slices of 16 unless they leave most compute units idle
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        cus = 256;
    return Rp % 16 == 0 && Rp / 16 >= cus ? 16 : 8;
}

bool bq_slab_supported(const BqView &p, int Rp, int width, int rs)
{
    rs = bq_slab_rs(Rp, rs);
    return rs != 0 && p.na_p <= 512 && p.nb_p <= 512 && p.na_p % 64 == 0 && p.nb_p % 64 == 0 && width >= 1 &&
           slab_lds(p, width, rs) <= (size_t)kMaxLds;
}

hipError_t bq_slab(const BqView &p, int8_t *MA, int8_t *MB, int Rp, const uint32_t *table, int width, int s_begin,
                   int s_end, uint32_t sweep0, uint32_t rq0, Key key, hipStream_t st, int rs)
{
    if (!bq_slab_supported(p, Rp, width, rs) || s_end < s_begin) return hipErrorInvalidValue;
    if (bq_slab_rs(Rp, rs) == 16)
        return slab_launch<16>(p, MA, MB, Rp, table, width, s_begin, s_end, sweep0, rq0, key, st);
    return slab_launch<8>(p, MA, MB, Rp, table, width, s_begin, s_end, sweep0, rq0, key, st);
}

}  // namespace pbit
