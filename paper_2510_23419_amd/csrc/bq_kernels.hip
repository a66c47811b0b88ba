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
#include "bq.h"

namespace pbit {

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

constexpr int kThreads = 256;
constexpr int kTileR = 64;  // replicas per workgroup tile

// 4 x 4 byte transpose across a lane quad: lane u of the quad holds byte p of
// its dword for replica p; afterwards lane u holds, in byte v, the byte u of
// quad lane v (four consecutive sites of replica u).
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
    const int hval = hs[site];  // site < Ns_p: padded fields are zero
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
            int8_t m[4];
#pragma unroll
            for (int p = 0; p < 4; ++p) {
                const int I = acc[4 * q + p] + hval;
                const int a = min(I >= 0 ? I : -I, top);
                m[p] = decide(I, T[a], b.w[p]);
            }
#pragma unroll
            for (int p = 0; p < 4; ++p)
                if (site < Ns && r4 + p < R) Ms[(size_t)(r4 + p) * Ns_p + site] = m[p];
        }
    }
}

// Tile edge of the DMA-staged half-sweep: 128 replicas x 128 sites per workgroup.
// Four waves each hold a 64 x 64 sub-tile as 2 x 2 MFMA accumulators, so each
// operand fragment read from LDS feeds two MFMAs.
constexpr int kT = 128;

struct Acc4 {
    v16i c00, c01, c10, c11;
};

// ---------------------------------------------------------------- DMA-staged 128 x 128 tiles
//
// The same 128-replica x 128-site tile, with operands staged by the gfx950
// global-to-LDS DMA (global_load_lds_dwordx4: each lane's 16 bytes land at
// LDS base + 16 * lane) into a ring of NS stages of KT K-bytes, so that many
// stages are in flight without occupying registers.  A stage holds 128 rows of
// A (replicas) then 128 rows of B (sites), KT bytes per row (KT = 128: whole
// cache lines); chunk c (K bytes 16c .. 16c + 15) of row r sits at position
// c ^ swz(r), which keeps the 16-byte fragment reads of 8 or 16 consecutive
// rows on distinct banks.  One barrier per stage both publishes stage t + 1
// and frees the slot of stage t - 1 for stage t + NS - 1.
template <int CH>
__device__ __forceinline__ int swz(int r)
{
    return CH == 8 ? ((r ^ (r >> 3)) & 7) : (((r >> 1) ^ (r >> 3)) & 3);
}

// s_waitcnt vmcnt(n) (expcnt and lgkmcnt not waited for)
template <int N>
__device__ __forceinline__ void wait_vm()
{
    static_assert(N >= 0 && N < 64, "vmcnt is a 6-bit field");
    __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4) | (15 << 8));
}

template <int KT, int NS>
struct DmaGeom {
    static constexpr int CH = KT / 16;              // 16-byte chunks per row
    static constexpr int op = kT * KT;              // bytes of one operand per stage
    static constexpr int stage = 2 * op;
    static constexpr int per_wave = CH / 2;         // DMA instructions per operand per wave and stage
    static constexpr int subs = KT / 32;            // MFMA K steps per stage
    static constexpr int ahead = 2 * per_wave * (NS - 2);  // loads allowed in flight after a stage lands
    static constexpr int lds = NS * stage;
    static_assert(ahead < 64, "vmcnt is a 6-bit field");
};

template <int KT, int NS>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_bq_halfsweep_dma(
    const int8_t *__restrict__ Mo, const int8_t *__restrict__ Jx, const int8_t *__restrict__ hs,
    int8_t *__restrict__ Ms, const uint32_t *__restrict__ trow, int width, int Ns_p, int Ko, int tiles_s,
    int xcd_bands, uint32_t site_base, uint32_t sweep, uint32_t rq0, uint32_t k0, uint32_t k1)
{
    using G = DmaGeom<KT, NS>;
    constexpr int CH = G::CH;
    constexpr int kPhxPerStage = G::subs;            // Philox blocks drawn per stage
    constexpr int kPhxStages = 16 / kPhxPerStage;

    extern __shared__ uint4 smem[];
    int8_t *ring = reinterpret_cast<int8_t *>(smem);
    uint32_t *T = reinterpret_cast<uint32_t *>(ring + G::lds);
    for (int a = threadIdx.x; a < width; a += kThreads) T[a] = trow[a];

    int ts, tr;
    if (xcd_bands) {  // tiles_s % 8 == 0: XCD (= block id mod 8) owns tiles_s / 8 site tiles
        const int per = tiles_s / 8;
        const int slot = (int)blockIdx.x / 8;
        ts = ((int)blockIdx.x % 8) * per + slot % per;
        tr = slot / per;
    } else {
        ts = (int)blockIdx.x % tiles_s;
        tr = (int)blockIdx.x / tiles_s;
    }
    const int r0 = tr * kT, s0 = ts * kT;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;

    // DMA sources: wave w fills slots 64 (per_wave w + j) + lane (j < per_wave) of each operand
    // (fixed array bounds: the lambdas below capture these arrays by reference)
    const int8_t *srcA[4], *srcB[4];
    static_assert(G::per_wave <= 4 && G::subs <= 4, "fixed array bounds");
#pragma unroll
    for (int j = 0; j < G::per_wave; ++j) {
        const int S = 64 * (G::per_wave * wave + j) + lane;
        const int r = S / CH, c = (S % CH) ^ swz<CH>(S / CH);
        srcA[j] = Mo + (size_t)(r0 + r) * Ko + 16 * c;
        srcB[j] = Jx + (size_t)(s0 + r) * Ko + 16 * c;
    }
    const int nk = Ko / KT;
    auto issue = [&](int t) {
        int8_t *dA = ring + (t % NS) * G::stage + 1024 * G::per_wave * wave;
        int8_t *dB = dA + G::op;
        const size_t k = (size_t)t * KT;
#pragma unroll
        for (int j = 0; j < G::per_wave; ++j) __builtin_amdgcn_global_load_lds(srcA[j] + k, dA + 1024 * j, 16, 0, 0);
#pragma unroll
        for (int j = 0; j < G::per_wave; ++j) __builtin_amdgcn_global_load_lds(srcB[j] + k, dB + 1024 * j, 16, 0, 0);
    };
    // the threshold row's loads are waited for before any DMA is counted
    wait_vm<0>();
    for (int t = 0; t < NS - 1 && t < nk; ++t) issue(t);

    const int wr = wave >> 1, wc = wave & 1;
    const int ln = lane & 31, kg = lane >> 5;
    // fragment rows of this lane: A rows wr*64 + {0, 32} + ln, B rows wc*64 + {0, 32} + ln
    int offA[2][4], offB[2][4];  // [row block][K step]
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int sub = 0; sub < G::subs; ++sub) {
            const int ra = wr * 64 + 32 * b + ln, rb = wc * 64 + 32 * b + ln;
            offA[b][sub] = KT * ra + 16 * ((2 * sub + kg) ^ swz<CH>(ra));
            offB[b][sub] = G::op + KT * rb + 16 * ((2 * sub + kg) ^ swz<CH>(rb));
        }
    Acc4 acc;
    acc.c00 = acc.c01 = acc.c10 = acc.c11 = v16i{0};
    uint32_t words[16][4];

    // fragments of stage t from LDS and their MFMAs; the MFMAs keep executing
    // while the wave goes on to the barrier and the next stage's reads
    auto compute = [&](int t) {
        const int8_t *st = ring + (t % NS) * G::stage;
#pragma unroll
        for (int sub = 0; sub < G::subs; ++sub) {
            const v4i a0 = *reinterpret_cast<const v4i *>(st + offA[0][sub]);
            const v4i a1 = *reinterpret_cast<const v4i *>(st + offA[1][sub]);
            const v4i b0 = *reinterpret_cast<const v4i *>(st + offB[0][sub]);
            const v4i b1 = *reinterpret_cast<const v4i *>(st + offB[1][sub]);
            acc.c00 = __builtin_amdgcn_mfma_i32_32x32x32_i8(a0, b0, acc.c00, 0, 0, 0);
            acc.c01 = __builtin_amdgcn_mfma_i32_32x32x32_i8(a0, b1, acc.c01, 0, 0, 0);
            acc.c10 = __builtin_amdgcn_mfma_i32_32x32x32_i8(a1, b0, acc.c10, 0, 0, 0);
            acc.c11 = __builtin_amdgcn_mfma_i32_32x32x32_i8(a1, b1, acc.c11, 0, 0, 0);
        }
    };
    auto draw = [&](int blk) {
        // block (bj * 2 + bi) * 4 + q covers site column bj and replica rows bi, q
        const int bj = blk >> 3, bi = (blk >> 2) & 1, q = blk & 3;
        const int site = s0 + wc * 64 + bj * 32 + ln;
        const int r4 = r0 + wr * 64 + bi * 32 + 8 * q + 4 * kg;
        const Block4 b = philox(site_base + (uint32_t)site, sweep, rq0 + (uint32_t)(r4 >> 2), kDomainSweep, k0, k1);
        words[blk][0] = b.w[0];
        words[blk][1] = b.w[1];
        words[blk][2] = b.w[2];
        words[blk][3] = b.w[3];
    };

    // stage 0 landed in every wave (later stages may still be in flight)
    if (nk >= NS - 1) wait_vm<G::ahead>(); else wait_vm<0>();
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");  // LDS written by the DMA: no read may move above here

    // first stages: the Philox draws ride along with the MFMAs
    int t = 0;
#pragma unroll
    for (int u = 0; u < kPhxStages; ++u) {
        if (t < nk) {
            if (t + NS - 1 < nk) issue(t + NS - 1);
            compute(t);
#pragma unroll
            for (int v = 0; v < kPhxPerStage; ++v) draw(kPhxPerStage * u + v);
            if (t + NS - 1 < nk) wait_vm<G::ahead>(); else wait_vm<0>();
            __builtin_amdgcn_s_barrier();
            asm volatile("" ::: "memory");
            ++t;
        } else {
#pragma unroll
            for (int v = 0; v < kPhxPerStage; ++v) draw(kPhxPerStage * u + v);
        }
    }
    // steady state: every stage after this one still has NS - 2 successors in flight
    for (; t + NS - 1 < nk; ++t) {
        issue(t + NS - 1);
        compute(t);
        wait_vm<G::ahead>();
        __builtin_amdgcn_s_barrier();
        asm volatile("" ::: "memory");
    }
    // tail: nothing left to issue
    for (; t < nk; ++t) {
        compute(t);
        wait_vm<0>();
        __builtin_amdgcn_s_barrier();
        asm volatile("" ::: "memory");
    }

    // epilogue: four replicas of a group are packed into one dword, then
    // transposed across the lane quad (sites s .. s + 3) so that each lane
    // stores four consecutive sites of one replica row.  Every store lands
    // inside the padded [Rp][Ns_p] array; padding sites and replicas take
    // values that nothing reads (their couplings and fields are zero).
    const int top = width - 1;
    const int u4 = ln & 3;
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) {
        const int site = s0 + wc * 64 + bj * 32 + ln;
        const int hval = hs[site];  // site < Ns_p: padded fields are zero
        const int quad_col = site - u4;
#pragma unroll
        for (int bi = 0; bi < 2; ++bi) {
            const v16i &c = bi == 0 ? (bj == 0 ? acc.c00 : acc.c01) : (bj == 0 ? acc.c10 : acc.c11);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int blk = (bj * 2 + bi) * 4 + q;
                uint32_t packed = 0;
#pragma unroll
                for (int p = 0; p < 4; ++p) {
                    const int I = c[4 * q + p] + hval;
                    const int a = min(I >= 0 ? I : -I, top);
                    packed |= (uint32_t)(uint8_t)decide(I, T[a], words[blk][p]) << (8 * p);
                }
                const int r4 = r0 + wr * 64 + bi * 32 + 8 * q + 4 * kg;
                *reinterpret_cast<uint32_t *>(Ms + (size_t)(r4 + u4) * Ns_p + quad_col) = quad_transpose(packed, u4);
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


// ---------------------------------------------------------------- spins as bits
//
// Spins are +-1, so a replica fits one bit per site: bit b of spin word w of a
// replica is set when site 32 w + b holds -1.  The words of a side are stored
// by blocks of 128 sites: word w of replica r at ((w / 4) Rp + r) 4 + w % 4, so
// that the 16 bytes of one block of consecutive replicas are contiguous.
// With b_k the bit of site k, m_k = 1 - 2 b_k and the field of a site s is
//     I_s = h_s + sum_k J_sk m_k = (h_s + sum_k J_sk) - 2 sum_k J_sk b_k,
// whose last sum runs on the int8 MFMA with int32 accumulation, the bits
// widened to bytes in registers.  The spins cross from L2 at one eighth of
// the int8 bytes, which is what bounds the int8 tiles of large bicliques.
//
// Widening: lane half g (lanes 32 g .. 32 g + 31) of an MFMA fragment holds 16
// K bytes, dword j byte i at K position 16 g + 4 j + i.  From a spin word w,
// x = w >> 4 g, the dword x & (0x01010101 << j) holds bit 8 i + 4 g + j of w in
// byte i, as the value 0 or 2^j: one AND per dword.  The couplings are stored
// with their columns in that order inside every group of 32 and scaled by
// 2^(3 - j) (Jb, JTb, values in [-8, 8]), so every product is 8 J b and the
// accumulator holds 8 sum_k J_sk b_k exactly.
//
// Tile: 64 sites x RT replicas per workgroup, RT = 256 on large bicliques.  The
// bytes that reach a CU per multiply-add, 1 / RT for the couplings plus 1 / 512
// for the spin bits, bound these tiles there (the L2-to-CU rate of one CU is
// about 20 bytes per clock).  Waves of 32 replicas and all 64 sites (1 x 2 MFMA
// blocks): eight at RT = 256, two per SIMD so that one wave's waits are covered
// by the other's MFMAs (a four-wave form of 64 replicas per wave, 2 x 2 blocks,
// measured about 5 % slower); four at RT = 128 and two at RT = 64, which give
// sides of 1024 and 2048 more workgroups than CUs would get at 256.  The vector
// work stays near 2.5 instructions per MFMA (an MFMA holds the wave's VALU issue
// for about half of its 32 cycles) and the LDS fragment reads under the
// matrix-core time of a stage.
// Stages of KT = 128 or 256 K move by the global-to-LDS DMA into a ring: 64
// coupling rows of KT bytes (chunk c of row r at position c ^ swzb(r)), then the
// RT replicas' 16 bytes (four spin words) per 128-site block of the stage.
//
// Decisions through 64-bit words in LDS, one per clamped field value:
// S(I) = Tm(|I|) for I >= 0, 2^32 - Tm(|I|) for I < 0; the new spin is -1
// exactly when w + S(I) carries into bit 32 (the heat-bath rule with the
// uniform word w), so a lane's decision is one multiply-add and one compare,
// and a wave's 64 decisions form one ballot mask.

constexpr int kBitsST = 64;     // sites per tile
constexpr int kBitsRT = 256;    // replicas per tile of the full-size form; Rp is a multiple of it
constexpr int kBitsBlock = 128; // sites per block of the spin-word layout (four words)
constexpr int kBitsWaves = 8;   // waves per workgroup of the full-size form (32 replicas each, two per SIMD)
constexpr int kBitsMinGroups = 256;  // workgroups (one per CU) below which the default tile shrinks

// KT: K per stage, 128 (an 8-stage ring) or 256 (a 4-stage ring, half the
// barriers per launch, for sides that are multiples of 256).  RT: replicas per
// tile, 32 per wave; tiles of 128 and 64 replicas (four and two waves) give a
// launch more workgroups where sides of 1024 or 2048 would fill only a quarter or
// half of the CUs with 256.
template <int WAVES, int KT, int RT>
struct BitsGeom {
    static constexpr int threads = 64 * WAVES;
    static constexpr int NS = KT == 256 ? 4 : 8;          // stages in the ring
    static constexpr int jbytes = kBitsST * KT;            // coupling rows of one stage
    static constexpr int bbytes = RT * KT / 8;             // spin words of one stage (KT / 128 blocks)
    static constexpr int bblock = 16 * RT;                 // bytes of one 128-site block of the stage's spin words
    static constexpr int stage = jbytes + bbytes;
    static constexpr int j_per_wave = jbytes / 1024 / WAVES;          // 16-byte-lane DMA instructions per wave
    static constexpr int bsz = (bbytes / WAVES) % 1024 == 0 ? 16 : 4; // bytes per lane of the spin-word DMA
    static constexpr int b_per_wave = bbytes / (64 * bsz) / WAVES;
    static constexpr int per_wave = j_per_wave + b_per_wave;
    static constexpr int ahead = per_wave * (NS - 2);
    static constexpr int ring = NS * stage;
    static constexpr int bi = RT / WAVES / 32;  // 32-replica blocks per wave
    static constexpr int waves_per_eu = WAVES >= 8 ? WAVES / 4 : 1;
    static_assert(bi >= 1 && bi * WAVES * 32 == RT, "whole 32-replica blocks per wave");
    static_assert(ahead < 64, "vmcnt is a 6-bit field");
    static_assert(j_per_wave * WAVES * 1024 == jbytes && b_per_wave * WAVES * 64 * bsz == bbytes,
                  "whole DMA instructions");
};

template <int WAVES, int KT, int RT>
__global__ __launch_bounds__(64 * WAVES) __attribute__((amdgpu_waves_per_eu(BitsGeom<WAVES, KT, RT>::waves_per_eu,
                                                                              BitsGeom<WAVES, KT, RT>::waves_per_eu))) void
k_bq_halfsweep_bits(const uint32_t *__restrict__ Mob, const int8_t *__restrict__ Jb, const int32_t *__restrict__ hs2,
                    uint32_t *__restrict__ Msb, const uint32_t *__restrict__ trow, int width, int Ko, int Rp,
                    int tiles_s, int xcd_bands, uint32_t site_base, uint32_t sweep, uint32_t rq0, uint32_t k0,
                    uint32_t k1, uint32_t one)
{
    using G = BitsGeom<WAVES, KT, RT>;
    constexpr int NS = G::NS;
    constexpr int CH = KT / 16;       // 16-byte chunks per coupling row
    constexpr int kSubs = KT / 32;    // K steps per stage
    constexpr int KB = KT / kBitsBlock;  // spin-word blocks per stage
    constexpr int BI = G::bi;         // replica blocks of 32 per wave
    constexpr int RW = 32 * BI;       // replicas per wave

    extern __shared__ uint4 smem[];
    int8_t *ring = reinterpret_cast<int8_t *>(smem);
    uint64_t *Sw = reinterpret_cast<uint64_t *>(ring + G::ring);  // [2 top + 1]
    const int top = width - 1;
    // the threshold row goes to registers now and into the LDS decision words after
    // the K loop, so that its load overlaps the DMA stages instead of preceding them:
    // thread x holds Tm(x + threads k), k < kTv
    constexpr int kTv = (kMaxTableWidth + G::threads - 1) / G::threads;
    uint32_t tv[kTv];
#pragma unroll
    for (int k = 0; k < kTv; ++k) {
        const int x = (int)threadIdx.x + G::threads * k;
        tv[k] = x <= top ? trow[x] : 0u;
    }

    int ts, tr;
    if (xcd_bands) {  // tiles_s % 8 == 0: XCD (= block id mod 8) owns tiles_s / 8 site tiles
        const int per = tiles_s / 8;
        const int slot = (int)blockIdx.x / 8;
        ts = ((int)blockIdx.x % 8) * per + slot % per;
        tr = slot / per;
    } else {
        ts = (int)blockIdx.x % tiles_s;
        tr = (int)blockIdx.x / tiles_s;
    }
    const int r0 = tr * RT, s0 = ts * kBitsST;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform: address math on the SALU

    // DMA sources: wave w fills coupling slots 64 (j_per_wave w + j) + lane (16 bytes
    // each) and spin-word slots 64 (b_per_wave w + j) + lane (bsz bytes each) of each
    // stage, from a wave-uniform base plus a 32-bit lane offset.  Row r of a stage keeps
    // chunk c at position c ^ swzb(r), with a swizzle of r mod 32 only, so that the two
    // site blocks of a fragment read sit at a fixed distance.  Rows of 128 bytes span
    // half the banks: the swizzle spreads 8 even and 8 odd rows; rows of 256 bytes
    // span all of them: it spreads 16 rows.
    auto swzb = [](int r) { return CH == 8 ? ((r ^ ((r >> 3) & 3)) & 7) : (r & 15); };
    uint32_t offJl[4], offBl[4];
    static_assert(G::j_per_wave <= 4 && G::b_per_wave <= 4 && kSubs <= 8, "fixed array bounds");
#pragma unroll
    for (int j = 0; j < G::j_per_wave; ++j) {
        const int S = 64 * (G::j_per_wave * wave + j) + lane;
        const int r = S / CH, c = (S % CH) ^ swzb(S / CH);
        offJl[j] = (uint32_t)(r * Ko + 16 * c);
    }
    // spin words: byte o of a stage's spin area is byte o % bblock of block o / bblock of the
    // stage (its replicas' 16 bytes each, contiguous in the block layout)
#pragma unroll
    for (int j = 0; j < G::b_per_wave; ++j) {
        const uint32_t o = (uint32_t)(G::bsz * (64 * (G::b_per_wave * wave + j) + lane));
        offBl[j] = (o / (uint32_t)G::bblock) * 16u * (uint32_t)Rp + o % (uint32_t)G::bblock;
    }
    const int8_t *Jt0 = Jb + (size_t)s0 * Ko;
    const char *Bt0 = reinterpret_cast<const char *>(Mob + (size_t)r0 * 4);
    const int nk = Ko / KT;
    const int ln = lane & 31, kg = lane >> 5;
    // the fields of this lane's two sites (field plus coupling sum; zero at padding sites),
    // loaded before the DMA so that the stage waits also cover them
    const int h2v[2] = {hs2[s0 + ln], hs2[s0 + 32 + ln]};
    auto issue = [&](int t) {
        int8_t *dJ = ring + (t % NS) * G::stage + 1024 * G::j_per_wave * wave;
        int8_t *dB = ring + (t % NS) * G::stage + G::jbytes + 64 * G::bsz * G::b_per_wave * wave;
        const int8_t *Jt = Jt0 + (size_t)t * KT;
        const char *Bt = Bt0 + (size_t)t * KB * 16 * Rp;
#pragma unroll
        for (int j = 0; j < G::j_per_wave; ++j) __builtin_amdgcn_global_load_lds(Jt + offJl[j], dJ + 1024 * j, 16, 0, 0);
        // size and LDS step as literals: with a template-dependent LDS offset, the
        // compiler's host pass rejects the 16-byte form and silently drops the kernel
#pragma unroll
        for (int j = 0; j < G::b_per_wave; ++j) {
            if constexpr (G::bsz == 16)
                __builtin_amdgcn_global_load_lds(Bt + offBl[j], dB + 1024 * j, 16, 0, 0);
            else
                __builtin_amdgcn_global_load_lds(Bt + offBl[j], dB + 256 * j, 4, 0, 0);
        }
    };
    // the threshold row and field loads above are older than every DMA below, so each
    // wait for a stage also covers them
    for (int t = 0; t < NS - 1 && t < nk; ++t) issue(t);

    // coupling fragment offsets: rows 32 bj + ln, chunk 2 sub + kg; swzb(r) depends on
    // r mod 32 = ln only, so site block bj = 1 sits 32 rows further
    int offJ[8];
#pragma unroll
    for (int sub = 0; sub < kSubs; ++sub) offJ[sub] = KT * ln + 16 * ((2 * sub + kg) ^ swzb(ln));
    const int offB = G::jbytes + 16 * (RW * wave + ln);  // spin words of replica rows RW wave + 32 bi + ln
    v16i acc[BI][2];  // [replica block][site block]
#pragma unroll
    for (int bi = 0; bi < BI; ++bi) acc[bi][0] = acc[bi][1] = v16i{0};
    uint32_t words[8 * BI][4];

    // the fragments of one stage in registers: the next stage's are read from LDS
    // while the MFMAs run on the current one's (a barrier before the reads would
    // otherwise leave the matrix cores idle for the LDS latency at every stage)
    struct Frag {
        v4i w[BI][KB];     // spin words of replica rows 32 bi + ln, one per K step of a block
        v4i b[kSubs][2];   // coupling fragments [K step][site block]
    };
    auto load = [&](int t, Frag &f) {
        const int8_t *st = ring + (t % NS) * G::stage;
        // int vector reads, like every LDS read of the ring: with this access type the
        // compiler adds no wait for all DMA in flight (the stage was waited for, and
        // published by a barrier, before this call)
#pragma unroll
        for (int bi = 0; bi < BI; ++bi)
#pragma unroll
            for (int kb = 0; kb < KB; ++kb)
                f.w[bi][kb] = *reinterpret_cast<const v4i *>(st + offB + G::bblock * kb + 16 * 32 * bi);
#pragma unroll
        for (int sub = 0; sub < kSubs; ++sub)
#pragma unroll
            for (int bj = 0; bj < 2; ++bj)
                f.b[sub][bj] = *reinterpret_cast<const v4i *>(st + offJ[sub] + 32 * KT * bj);
    };
    auto mfmas = [&](const Frag &f) {
#pragma unroll
        for (int sub = 0; sub < kSubs; ++sub)
#pragma unroll
            for (int bi = 0; bi < BI; ++bi) {
                const v4i a = widen_bits((uint32_t)f.w[bi][sub / 4][sub % 4], kg);
#pragma unroll
                for (int bj = 0; bj < 2; ++bj)
                    acc[bi][bj] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a, f.b[sub][bj], acc[bi][bj], 0, 0, 0);
            }
    };
    // an empty statement that takes the fragments as its outputs: called where they are
    // complete, so that the compiler adds no wait for later reads before the MFMAs that
    // use them (it emits no instruction)
    auto settle = [&](Frag &f) {
#pragma unroll
        for (int sub = 0; sub < kSubs; sub += 2)
            asm volatile("" : "+v"(f.b[sub][0]), "+v"(f.b[sub][1]), "+v"(f.b[sub + 1][0]), "+v"(f.b[sub + 1][1]));
#pragma unroll
        for (int bi = 0; bi < BI; ++bi)
#pragma unroll
            for (int kb = 0; kb < KB; ++kb) asm volatile("" : "+v"(f.w[bi][kb]));
    };
    // stage t: refill the ring, publish stage t + 1 and read its fragments, then the
    // MFMAs of stage t.  Every wave's reads of stage t are complete (lgkmcnt 0) before
    // the barrier, so after it no wave reads the slot that the next refill overwrites.
    auto step = [&](int t, Frag &cur, Frag &nxt) {
        if (t + NS - 1 < nk) issue(t + NS - 1);
        __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0): the current fragments are in registers
        settle(cur);
        if (t + 1 < nk) {
            if (t + NS - 1 < nk) wait_vm<G::ahead>(); else wait_vm<0>();
            __builtin_amdgcn_s_barrier();
            asm volatile("" ::: "memory");
            load(t + 1, nxt);
            __builtin_amdgcn_sched_barrier(0);  // the reads go out before the MFMAs, not after
        }
        mfmas(cur);
    };
    auto draw = [&](int blk) {
        // block (bj BI + bi) 4 + q covers site block bj and replica rows 32 bi + 8 q .. of the wave
        const int q = blk & 3, bi = (blk >> 2) % BI, bj = (blk >> 2) / BI;
        const int site = s0 + bj * 32 + ln;
        const int r4 = r0 + RW * wave + bi * 32 + 8 * q + 4 * kg;
        const Block4 b = philox(site_base + (uint32_t)site, sweep, rq0 + (uint32_t)(r4 >> 2), kDomainSweep, k0, k1);
        words[blk][0] = b.w[0];
        words[blk][1] = b.w[1];
        words[blk][2] = b.w[2];
        words[blk][3] = b.w[3];
    };

    if (nk >= NS - 1) wait_vm<G::ahead>(); else wait_vm<0>();
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");  // LDS written by the DMA: no read may move above here
    Frag fa, fb;
    load(0, fa);

    // the first eight stages carry the Philox draws; stage t computes from fa when t
    // is even, from fb when odd
    constexpr int kPhxPerStage = BI, kPhxStages = 8;
    int t = 0;
#pragma unroll
    for (int u = 0; u < kPhxStages; ++u) {
        if (t < nk) {
            if (u & 1)
                step(t, fb, fa);
            else
                step(t, fa, fb);
            ++t;
        }
#pragma unroll
        for (int v = 0; v < kPhxPerStage; ++v) draw(kPhxPerStage * u + v);
    }
    // kPhxStages is even: stage t computes from fa again
    for (; t + 1 < nk; t += 2) {
        step(t, fa, fb);
        step(t + 1, fb, fa);
    }
    if (t < nk) step(t, fa, fb);

    // epilogue: one ballot per (site block, replica block, q, p) gives the new
    // spin bits of 32 sites for two replicas (lane half 0: row 8 q + p of the
    // block, half 1: row 8 q + 4 + p); lane L of out[bj] collects the word of
    // replica row L of the wave for site block bj.  Padding sites and replicas
    // take bits that nothing reads (their couplings and fields are zero).
    // decision words for I = +-x from Tm(x): Tm for I >= 0, 2^32 - Tm for I < 0; built
    // here, where no DMA is in flight, so that waiting for the row costs nothing
#pragma unroll
    for (int k = 0; k < kTv; ++k) {
        const int x = (int)threadIdx.x + G::threads * k;
        if (x <= top) {
            Sw[top + x] = (uint64_t)tv[k];
            Sw[top - x] = ((uint64_t)1 << 32) - tv[k];
        }
    }
    __syncthreads();
    const char *Sb = reinterpret_cast<const char *>(Sw);
    uint32_t out[2] = {0u, 0u};
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) {
        const int h2 = h2v[bj];
#pragma unroll
        for (int bi = 0; bi < BI; ++bi)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int blk = (bj * BI + bi) * 4 + q;
#pragma unroll
                for (int p = 0; p < 4; ++p) {
                    const int I = h2 - (acc[bi][bj][4 * q + p] >> 2);  // the accumulator holds 8 sum J b
                    const int Ic = min(max(I, -top), top);
                    const uint64_t S =
                        *static_cast<const uint64_t *>(__builtin_assume_aligned(Sb + 8 * (Ic + top), 8));
                    const uint64_t m = __ballot((((uint64_t)words[blk][p] * one + S) >> 32) != 0);
                    const int L = bi * 32 + 8 * q + p;
                    out[bj] = (uint32_t)lane_write((int)(uint32_t)m, L, (int)out[bj]);
                    out[bj] = (uint32_t)lane_write((int)(uint32_t)(m >> 32), L + 4, (int)out[bj]);
                }
            }
    }
    // words s0 / 32 and + 1 of replica row RW wave + lane: an aligned pair in a block of four
    if (lane < RW)
        *reinterpret_cast<uint2 *>(Msb + ((size_t)(s0 / kBitsBlock) * Rp + r0 + RW * wave + lane) * 4 + (s0 / 32) % 4) =
            make_uint2(out[0], out[1]);
}

// int8 rows [Rp][cols] <-> spin words by blocks of 128 sites; one thread per word
template <bool PACK>
__global__ __launch_bounds__(kThreads) void k_bq_bits(int8_t *__restrict__ M, uint32_t *__restrict__ Mb, int Rp,
                                                      int cols)
{
    const int64_t k = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    const int nw = cols / 32;
    if (k >= (int64_t)Rp * nw) return;
    const int r = (int)(k / nw), w = (int)(k % nw);
    uint4 *row = reinterpret_cast<uint4 *>(M + (size_t)r * cols + 32 * w);
    uint32_t *word = Mb + ((size_t)(w / 4) * Rp + r) * 4 + w % 4;
    if (PACK) {
        const uint4 v0 = row[0], v1 = row[1];
        const uint32_t d[8] = {v0.x, v0.y, v0.z, v0.w, v1.x, v1.y, v1.z, v1.w};
        uint32_t x = 0;
#pragma unroll
        for (int i = 0; i < 8; ++i)
#pragma unroll
            for (int b = 0; b < 4; ++b) x |= ((d[i] >> (8 * b + 7)) & 1u) << (4 * i + b);  // sign bit of the byte
        *word = x;
    } else {
        const uint32_t x = *word;
        uint32_t d[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const uint32_t y = (x >> (4 * i)) & 0xFu;
            uint32_t v = 0;
#pragma unroll
            for (int b = 0; b < 4; ++b) v |= ((y >> b) & 1u ? 0xFFu : 0x01u) << (8 * b);
            d[i] = v;
        }
        row[0] = make_uint4(d[0], d[1], d[2], d[3]);
        row[1] = make_uint4(d[4], d[5], d[6], d[7]);
    }
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
                        int width, uint32_t sweep, uint32_t rq0, Key key, hipStream_t st, BqVariant variant)
{
    if (Rp % kTileR != 0 || p.na_p % kTileS != 0 || p.nb_p % kTileS != 0 || width < 1 || width > kMaxTableWidth)
        return hipErrorInvalidValue;
    const bool A = side == 0;
    const int Ns_p = A ? p.na_p : p.nb_p, Ko = A ? p.nb_p : p.na_p;
    const int8_t *Mo = A ? MB : MA;
    const int8_t *Jx = A ? p.J : p.JT;
    const int8_t *hs = A ? p.hA : p.hB;
    int8_t *Ms = A ? MA : MB;
    const int Ns = A ? p.na : p.nb;
    const uint32_t site_base = A ? 0u : (uint32_t)p.na;
    static const hipError_t lds_attr = [] {
        // the DMA ring plus the threshold row exceed the default 64 KiB of LDS
        return hipFuncSetAttribute(reinterpret_cast<const void *>(&k_bq_halfsweep_dma<128, 4>),
                                   hipFuncAttributeMaxDynamicSharedMemorySize,
                                   DmaGeom<128, 4>::lds + (int)sizeof(uint32_t) * kMaxTableWidth);
    }();
    if (lds_attr != hipSuccess) return lds_attr;
    if (variant == BqVariant::Dma) {
        if (Ns_p % kT != 0 || Ko % 128 != 0 || Rp % kT != 0) return hipErrorInvalidValue;
        const int tiles_s = Ns_p / kT, tiles_r = Rp / kT;
        const dim3 grid((unsigned)(tiles_s * tiles_r));
        const int bands = tiles_s % 8 == 0 ? 1 : 0;
        const size_t tab = sizeof(uint32_t) * (size_t)width;
        hipLaunchKernelGGL((k_bq_halfsweep_dma<128, 4>), grid, dim3(kThreads), (DmaGeom<128, 4>::lds + tab), st, Mo, Jx,
                           hs, Ms, trow, width, Ns_p, Ko, tiles_s, bands, site_base, sweep, rq0, key.k0, key.k1);
        return hipGetLastError();
    }
    dim3 grid((unsigned)(Ns_p / kTileS), (unsigned)(Rp / kTileR));
    const size_t lds = sizeof(uint32_t) * (size_t)width;
    hipLaunchKernelGGL(k_bq_halfsweep<false>, grid, dim3(kThreads), lds, st, Mo, Jx, hs, Ms, trow, width, Ns, Ns_p,
                       Ko, R, site_base, sweep, rq0, key.k0, key.k1, (int32_t *)nullptr);
    return hipGetLastError();
}

hipError_t bqb_pack(const BqView &p, const int8_t *MA, const int8_t *MB, uint32_t *MAb, uint32_t *MBb, int Rp,
                    hipStream_t st)
{
    if (p.na_p % kBitsBlock || p.nb_p % kBitsBlock) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_bq_bits<true>, dim3(blocks_for((int64_t)Rp * p.na_p / 32)), dim3(kThreads), 0, st,
                       const_cast<int8_t *>(MA), MAb, Rp, p.na_p);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_bq_bits<true>, dim3(blocks_for((int64_t)Rp * p.nb_p / 32)), dim3(kThreads), 0, st,
                       const_cast<int8_t *>(MB), MBb, Rp, p.nb_p);
    return hipGetLastError();
}

hipError_t bqb_unpack(const BqView &p, const uint32_t *MAb, const uint32_t *MBb, int8_t *MA, int8_t *MB, int Rp,
                      hipStream_t st)
{
    if (p.na_p % kBitsBlock || p.nb_p % kBitsBlock) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_bq_bits<false>, dim3(blocks_for((int64_t)Rp * p.na_p / 32)), dim3(kThreads), 0, st, MA,
                       const_cast<uint32_t *>(MAb), Rp, p.na_p);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_bq_bits<false>, dim3(blocks_for((int64_t)Rp * p.nb_p / 32)), dim3(kThreads), 0, st, MB,
                       const_cast<uint32_t *>(MBb), Rp, p.nb_p);
    return hipGetLastError();
}

bool bqb_supported(const BqView &p, int Rp)
{
    return p.Jb && p.na_p % kBitsST == 0 && p.nb_p % kBitsST == 0 && p.na_p % kBitsBlock == 0 &&
           p.nb_p % kBitsBlock == 0 && Rp % kBitsRT == 0;
}

// The replica tile of a launch: `rt` if it is 64, 128 or 256 and divides Rp, else 256
// where that gives at least kBitsMinGroups workgroups and 128 elsewhere (measured at
// R = 1024: 128 is fastest at n = 1024 and 2048, 256 at 4096; the tuner times all three)
static int bits_rt(int tiles_s, int Rp, int rt)
{
    if ((rt == 64 || rt == 128 || rt == 256) && Rp % rt == 0) return rt;
    if (Rp % 256 == 0 && (int64_t)tiles_s * (Rp / 256) >= kBitsMinGroups) return 256;
    return Rp % 128 == 0 ? 128 : 64;
}

template <int WAVES, int KT, int RT>
static hipError_t bits_launch(const uint32_t *Mob, const int8_t *Jb, const int32_t *hs2, uint32_t *Msb,
                              const uint32_t *trow, int width, int Ko, int Rp, int tiles_s, uint32_t site_base,
                              uint32_t sweep, uint32_t rq0, Key key, hipStream_t st)
{
    using G = BitsGeom<WAVES, KT, RT>;
    static const hipError_t lds_attr = hipFuncSetAttribute(
        reinterpret_cast<const void *>(&k_bq_halfsweep_bits<WAVES, KT, RT>), hipFuncAttributeMaxDynamicSharedMemorySize,
        G::ring + (int)sizeof(uint64_t) * (2 * kMaxTableWidth - 1));
    if (lds_attr != hipSuccess) return lds_attr;
    const int bands = tiles_s % 8 == 0 ? 1 : 0;
    const size_t tab = sizeof(uint64_t) * (size_t)(2 * width - 1);
    const dim3 grid((unsigned)(tiles_s * (Rp / RT)));
    hipLaunchKernelGGL((k_bq_halfsweep_bits<WAVES, KT, RT>), grid, dim3(G::threads), G::ring + tab, st, Mob, Jb, hs2,
                       Msb, trow, width, Ko, Rp, tiles_s, bands, site_base, sweep, rq0, key.k0, key.k1, 1u);
    return hipGetLastError();
}

hipError_t bqb_halfsweep(const BqView &p, int side, uint32_t *MAb, uint32_t *MBb, int Rp, const uint32_t *trow,
                         int width, uint32_t sweep, uint32_t rq0, Key key, hipStream_t st, int rt)
{
    if (!bqb_supported(p, Rp) || width < 1 || width > kMaxTableWidth) return hipErrorInvalidValue;
    const bool A = side == 0;
    const int Ns_p = A ? p.na_p : p.nb_p, Ko = A ? p.nb_p : p.na_p;
    const uint32_t *Mob = A ? MBb : MAb;
    const int8_t *Jb = A ? p.Jb : p.JTb;
    const int32_t *hs2 = A ? p.hA2 : p.hB2;
    uint32_t *Msb = A ? MAb : MBb;
    const uint32_t site_base = A ? 0u : (uint32_t)p.na;
    const int tiles_s = Ns_p / kBitsST;
    // two waves cannot take a 256-deep stage (its DMA needs more than four 16-byte
    // loads per lane), so 64-replica tiles always stage 128
    switch (bits_rt(tiles_s, Rp, rt)) {
    case 256:
        return Ko % 256 == 0 ? bits_launch<kBitsWaves, 256, 256>(Mob, Jb, hs2, Msb, trow, width, Ko, Rp, tiles_s,
                                                                  site_base, sweep, rq0, key, st)
                             : bits_launch<kBitsWaves, 128, 256>(Mob, Jb, hs2, Msb, trow, width, Ko, Rp, tiles_s,
                                                                  site_base, sweep, rq0, key, st);
    case 128:
        return Ko % 256 == 0 ? bits_launch<4, 256, 128>(Mob, Jb, hs2, Msb, trow, width, Ko, Rp, tiles_s, site_base,
                                                         sweep, rq0, key, st)
                             : bits_launch<4, 128, 128>(Mob, Jb, hs2, Msb, trow, width, Ko, Rp, tiles_s, site_base,
                                                         sweep, rq0, key, st);
    default:
        return bits_launch<2, 128, 64>(Mob, Jb, hs2, Msb, trow, width, Ko, Rp, tiles_s, site_base, sweep, rq0, key,
                                       st);
    }
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
