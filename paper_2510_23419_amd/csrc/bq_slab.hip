// bq_slab.hip — the biclique sweep of a small instance with everything in LDS, for
// runs of sweeps in one launch.
//
// A half-sweep of a biclique updates one side from the other (Sec. 3; update
// groups, Sec. 1.2.2): F = J m_other, I = F + h, heat-bath decision.  For sides of
// at most 512 sites the couplings fit in LDS as two-bit codes in both orientations
// (J for side A's fields, J^T for side B's: 64 KiB each at 512 x 512), next to the
// spin rows of a slice of 16 or 8 replicas.  Replica slices never interact, so a
// workgroup holds one slice and runs a whole chunk of sweeps with workgroup barriers
// only: no launch per half-sweep and no coupling traffic after the first load.
//
// Each half-sweep is a product on the matrix cores, v_mfma_scale_f32_16x16x128_f8f6f4
// with unit scales: the spin rows (16 replicas x K sites of the other side) as fp8
// e4m3 bytes (+1, -1, and 0 on padding sites) times the couplings (K x 16 sites) as
// fp4 e2m1 values (+1, -1, 0), fp32 sums.  Every product and sum is a small integer,
// so the field is exact.  A two-bit code (sign, nonzero) per coupling becomes an fp4
// nibble with one mask: the codes of 16 couplings sit in one word with the bits of the
// first eight at nibble bits 3 and 1 and those of the last eight at bits 2 and 0, so
// the word masked, and the word shifted left by one and masked, are two words of fp4
// values.  The decision is the carry of the Philox word plus the 64-bit word S(I)
// (Tm(|I|) for I >= 0, 2^32 - Tm for I < 0), as in the other kernels, with the same
// counters, so results do not depend on the kernel.
//
// Spins stay in the library's int8 biclique layout in global memory (MA [Rp][na_p],
// MB [Rp][nb_p], padding sites zero); the kernel loads a slice at its start (as fp8)
// and stores it at its end.
#include <hip/hip_runtime.h>

#include "bq.h"
#include "device.h"
#include "internal.h"

namespace pbit {

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v8i __attribute__((ext_vector_type(8)));
typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int kThreads = 1024;  // 16 waves: four per SIMD
constexpr int kWaves = kThreads / 64;
constexpr int kBlkPerWave = 2;  // 16-site blocks per wave and half-sweep: 32 blocks at 512 sites
constexpr int kMaxLds = 160 * 1024 - 4096;
constexpr int kFp8One = 0x38, kFp8MinusOne = 0xB8;  // e4m3 +1, -1
constexpr uint32_t kFp4Mask = 0xAAAAAAAAu;          // sign and exponent-low bit of eight e2m1 nibbles

// 4 x 4 byte transpose across a quad of lanes: lane u holds bytes M[u][0..3] and
// receives M[0..3][u] (two DPP quad permutations and two byte permutes).
__device__ __forceinline__ uint32_t quad_transpose4(uint32_t d, int u)
{
    const uint32_t t = (uint32_t)__builtin_amdgcn_mov_dpp((int)d, 0xB1, 0xF, 0xF, false);  // quad_perm [1,0,3,2]
    const uint32_t d1 = __builtin_amdgcn_perm(t, d, (u & 1) ? 0x03070105u : 0x06020400u);
    const uint32_t t2 = (uint32_t)__builtin_amdgcn_mov_dpp((int)d1, 0x4E, 0xF, 0xF, false);  // quad_perm [2,3,0,1]
    return __builtin_amdgcn_perm(t2, d1, (u & 2) ? 0x03020706u : 0x05040100u);
}

// Codes of one orientation into LDS.  Jrow is [ns_p][ko] int8 (padding 0); K runs to
// ko_pad (a multiple of 128, couplings beyond ko zero).  Word (kb, s, g, h) covers
// J[s][k0 .. k0 + 15], k0 = 128 kb + 32 g + 16 h: for i < 8, bit 4 i + 3 is the sign of
// J[s][k0 + i] and bit 4 i + 1 says it is nonzero; bits 4 i + 2 and 4 i hold the same
// for J[s][k0 + 8 + i].  Words are ordered [kb][s][g][h], so the 64 lanes of an MFMA
// (site s = lane % 16 of a block, K group g = lane / 16) read 64 consecutive pairs.
__device__ void stage_codes(const int8_t *__restrict__ Jrow, int ns_p, int ko, int ko_pad, uint32_t *codes)
{
    const int nw = (ko_pad / 16) * ns_p;
    for (int wi = threadIdx.x; wi < nw; wi += kThreads) {
        const int h = wi & 1, g = (wi >> 1) & 3, s = (wi >> 3) % ns_p, kb = (wi >> 3) / ns_p;
        const int k0 = 128 * kb + 32 * g + 16 * h;
        uint32_t w = 0;
        if (k0 < ko) {  // ko is a multiple of 16: all 16 couplings are in the row, or none
            const uint4 v = *reinterpret_cast<const uint4 *>(Jrow + (size_t)s * ko + k0);
            const uint32_t dw[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                const int J = (int)(int8_t)(dw[k >> 2] >> (8 * (k & 3)));
                const int at = k < 8 ? 4 * k + 1 : 4 * (k - 8);  // nonzero bit; the sign bit is 2 above
                w |= (uint32_t)(J != 0) << at;
                w |= (uint32_t)(J < 0) << (at + 2);
            }
        }
        codes[wi] = w;
    }
}

// fp8 e4m3 bytes of four int8 spins (+1, -1, 0) and back
__device__ __forceinline__ uint32_t int8_to_fp8(uint32_t x)
{
    return (x & 0x01010101u) * (uint32_t)kFp8One | (x & 0x80808080u);
}
__device__ __forceinline__ uint32_t fp8_to_int8(uint32_t y)
{
    const uint32_t nz = (y >> 3) & 0x01010101u, neg = (y >> 7) & 0x01010101u;
    return nz | neg * 0xFEu;
}
__device__ __forceinline__ uint4 int8_to_fp8(uint4 v)
{
    return make_uint4(int8_to_fp8(v.x), int8_to_fp8(v.y), int8_to_fp8(v.z), int8_to_fp8(v.w));
}
__device__ __forceinline__ uint4 fp8_to_int8(uint4 v)
{
    return make_uint4(fp8_to_int8(v.x), fp8_to_int8(v.y), fp8_to_int8(v.z), fp8_to_int8(v.w));
}

// Sweeps [s_begin, s_end) of replicas [RS blockIdx.x, + RS) of a small biclique.
//
// RS = 16 fills the MFMA's 16 rows.  RS = 8 gives twice the workgroups for the same
// replicas (a launch of 1024 replicas then uses 128 CUs instead of 64): the rows 8 .. 15
// read a zero row, and the two site blocks of a wave, whose valid rows sit in lanes
// 0 .. 31 of their accumulators, are packed into one register (lanes 32 .. 63 from the
// second block: v_permlane32_swap), so the decision epilogue runs once per wave for
// both blocks instead of twice on half-empty lanes.
//
// LDS spin rows: side A's sites at [0, pa), side B's at [pa, pa + pb), pa and pb the
// padded sides rounded up to 128 (one MFMA's K), the sites beyond each side zero.
template <int RS>
__global__ __launch_bounds__(kThreads) void k_bq_slab(BqView p, int8_t *__restrict__ MA, int8_t *__restrict__ MB,
                                                      int Rp, const uint32_t *__restrict__ table, int width,
                                                      int s_begin, int s_end, uint32_t sweep0, uint32_t rq0,
                                                      uint32_t k0, uint32_t k1, uint32_t one)
{
    static_assert(RS == 16 || RS == 8, "slices of 16 or 8 replicas");
    constexpr int kRows = RS == 16 ? 16 : RS + 1;  // spin rows, plus a zero row for the unused MFMA rows
    extern __shared__ uint4 dyn[];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform: block tests are scalar branches
    const int na = p.na, nb = p.nb, na_p = p.na_p, nb_p = p.nb_p;
    const int pa = (na_p + 127) & ~127, pb = (nb_p + 127) & ~127;
    const int pitch = pa + pb + 16;
    // LDS: codes of J (side A's fields, K over side B), codes of J^T, spin rows, decision words
    uint32_t *codesA = reinterpret_cast<uint32_t *>(dyn);
    uint32_t *codesB = codesA + (size_t)na_p * pb / 16;
    uint8_t *sp = reinterpret_cast<uint8_t *>(codesB + (size_t)nb_p * pa / 16);
    // decision words of two sweeps: those of sweep s + 1 are written during sweep s
    uint64_t *Sw2 = reinterpret_cast<uint64_t *>(sp + (size_t)kRows * pitch);
    const int r0 = RS * blockIdx.x;  // first replica of the slice (local to this call)

    stage_codes(p.J, na_p, nb_p, pb, codesA);
    stage_codes(p.JT, nb_p, na_p, pa, codesB);
    for (int k = tid; k < kRows * (pitch / 16); k += kThreads) {
        const int r = k / (pitch / 16), c16 = k % (pitch / 16), c = 16 * c16;
        uint4 v = make_uint4(0, 0, 0, 0);
        if (r < RS) {
            if (c < na_p)
                v = int8_to_fp8(*reinterpret_cast<const uint4 *>(MA + (size_t)(r0 + r) * na_p + c));
            else if (c >= pa && c < pa + nb_p)
                v = int8_to_fp8(*reinterpret_cast<const uint4 *>(MB + (size_t)(r0 + r) * nb_p + (c - pa)));
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
    __syncthreads();  // codes, spins and the first decision words are in LDS
    // A rows: replica row col, or (RS = 8, col >= 8) the zero row
    const int arow_r = col < RS ? col : RS;
    // the replica rows of a lane's accumulator elements: 4 gr + j (RS = 8: the merged
    // register holds rows 0 .. 7 of block wave in lanes 0 .. 31 and of block wave + kWaves
    // in lanes 32 .. 63)
    const int gr = RS == 16 ? grp : (grp & 1);
    // one barrier per half-sweep: its spins and, after side B, the next sweep's decision
    // words are then complete
    for (int s = s_begin; s < s_end; ++s) {
        const int par = s & 1;
        const uint32_t t = sweep0 + (uint32_t)s;
        const char *Sb = reinterpret_cast<const char *>(Sw2 + (size_t)par * (2 * top + 1));
#pragma unroll 1
        for (int side = 0; side < 2; ++side) {
            const int ns = side == 0 ? na : nb, ns_p = side == 0 ? na_p : nb_p;
            const int ko = side == 0 ? pb : pa;          // K: sites of the other side, rounded up to 128
            const int in_col = side == 0 ? pa : 0;       // the other side's columns
            const int out_col = side == 0 ? 0 : pa;      // this side's columns
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
            // fields of up to kBlkPerWave 16-site blocks per wave (blocks wave, wave + kWaves)
            v4f acc[kBlkPerWave];
#pragma unroll
            for (int q = 0; q < kBlkPerWave; ++q) acc[q] = v4f{0.f, 0.f, 0.f, 0.f};
            // A operand of K step kb: bytes 0 .. 15 are the row's K 16 grp .. + 15 of the
            // step's 128, bytes 16 .. 31 its K 64 + 16 grp .. + 15; B operand: nibble j of
            // the four words is K 32 grp + j, from the lane's pair of code words
            const uint8_t *arow = sp + arow_r * pitch + in_col + 16 * grp;
            const int nkb = ko / 128;
            // the K loop unrolled to its largest trip count (ko <= 512: 4 steps) under
            // wave-uniform guards
            const bool one_blk = wave < nblk, two = wave + kWaves < nblk;  // this wave's blocks
            const uint2 *ck = reinterpret_cast<const uint2 *>(codes) + (wave * 16 + col) * 4 + grp;
            constexpr int kMaxKb = 512 / 128;
            static_assert(kBlkPerWave == 2, "two blocks per wave below");
#pragma unroll
            for (int kb = 0; kb < kMaxKb; ++kb) {
                if (one_blk && kb < nkb) {
                    const uint4 lo = *reinterpret_cast<const uint4 *>(arow + 128 * kb);
                    const uint4 hi = *reinterpret_cast<const uint4 *>(arow + 128 * kb + 64);
                    const v8i a = v8i{(int)lo.x, (int)lo.y, (int)lo.z, (int)lo.w,
                                      (int)hi.x, (int)hi.y, (int)hi.z, (int)hi.w};
                    const uint2 c0 = ck[0];
                    const v8i b0 = v8i{(int)(c0.x & kFp4Mask), (int)((c0.x << 1) & kFp4Mask),
                                       (int)(c0.y & kFp4Mask), (int)((c0.y << 1) & kFp4Mask), 0, 0, 0, 0};
                    acc[0] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a, b0, acc[0], 0, 4, 0, 127, 0, 127);
                    if (two) {
                        const uint2 c1 = ck[64 * kWaves];
                        const v8i b1 = v8i{(int)(c1.x & kFp4Mask), (int)((c1.x << 1) & kFp4Mask),
                                           (int)(c1.y & kFp4Mask), (int)((c1.y << 1) & kFp4Mask), 0, 0, 0, 0};
                        acc[1] =
                            __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a, b1, acc[1], 0, 4, 0, 127, 0, 127);
                    }
                    ck += (size_t)ns_p * 4;
                }
            }
            // decisions of one site block in a lane: site blk * 16 + col, replicas 4 gr .. 4 gr
            // + 3 (one Philox block); the four bytes are transposed across the lane quad so
            // that each lane writes four consecutive sites of one replica row
            const int u4 = lane & 3;
            auto decide = [&](const v4f &f, int blk, int hval, const Block4 &wq) {
                const int site = blk * 16 + col;
                const int flo = -top - hval, fhi = top - hval;
                const int base8 = 8 * (hval + top);
                uint32_t sgn[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int F = (int)f[j];  // an exact integer
                    const int Fc = min(max(F, flo), fhi);
                    const uint64_t S =
                        *static_cast<const uint64_t *>(__builtin_assume_aligned(Sb + 8 * Fc + base8, 8));
                    sgn[j] = (uint32_t)(((uint64_t)wq.w[j] * one + S) >> 32);
                }
                // byte j: e4m3 +1 (carry 0) or -1 (carry 1)
                const uint32_t lo = __builtin_amdgcn_perm(sgn[1], sgn[0], 0x0C0C0400u);
                const uint32_t hi = __builtin_amdgcn_perm(sgn[3], sgn[2], 0x0C0C0400u);
                uint32_t packed = __builtin_amdgcn_perm(0u, (uint32_t)(kFp8MinusOne << 8 | kFp8One),
                                                        __builtin_amdgcn_perm(hi, lo, 0x05040100u));
                if (site >= ns) packed = 0u;  // padding sites stay zero
                const uint32_t x = quad_transpose4(packed, u4);
                *reinterpret_cast<uint32_t *>(sp + (4 * gr + u4) * pitch + out_col + blk * 16 + (col & ~3)) = x;
            };
            if constexpr (RS == 16) {
#pragma unroll
                for (int q = 0; q < kBlkPerWave; ++q)
                    if (wave + kWaves * q < nblk) decide(acc[q], wave + kWaves * q, hv[q], w[q]);
            } else {
                // rows 0 .. 7 of both blocks in one register: lanes 32 .. 63 take lanes 0 .. 31
                // of the second block's accumulator
                v4f m;
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    m[j] = __uint_as_float(__builtin_amdgcn_permlane32_swap(__float_as_uint(acc[0][j]),
                                                                            __float_as_uint(acc[1][j]), false,
                                                                            false)[0]);
                const int blk = wave + kWaves * (lane >> 5);
                if (blk < nblk) decide(m, blk, hv[0], w[0]);  // uniform over each half of the wave
            }
            if (side == 1 && s + 1 < s_end) build_words(s + 1);  // published by the next barrier
            __syncthreads();
        }
    }

    for (int k = tid; k < RS * ((na_p + nb_p) / 16); k += kThreads) {
        const int r = k / ((na_p + nb_p) / 16), c = 16 * (k % ((na_p + nb_p) / 16));
        if (c < na_p) {
            const uint4 v = *reinterpret_cast<const uint4 *>(sp + r * pitch + c);
            *reinterpret_cast<uint4 *>(MA + (size_t)(r0 + r) * na_p + c) = fp8_to_int8(v);
        } else {
            const uint4 v = *reinterpret_cast<const uint4 *>(sp + r * pitch + pa + (c - na_p));
            *reinterpret_cast<uint4 *>(MB + (size_t)(r0 + r) * nb_p + (c - na_p)) = fp8_to_int8(v);
        }
    }
}

// LDS of a launch: the two code orientations, the spin rows (RS = 8: plus the zero row)
// and the decision words of two sweeps
size_t slab_lds(const BqView &p, int width, int rs)
{
    const int rows = rs == 16 ? 16 : rs + 1;
    const size_t pa = (size_t)(p.na_p + 127) & ~(size_t)127, pb = (size_t)(p.nb_p + 127) & ~(size_t)127;
    return (p.na_p * pb + p.nb_p * pa) / 4 + (size_t)rows * (pa + pb + 16) +
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
