// ea_mfma.hip — the cube half-sweep with the fields on the int8 matrix cores.
//
// A checkerboard half-sweep updates the N/2 sites of one colour from the six
// neighbours of the other colour (Sec. 2; update groups, Sec. 1.2.2).  Number
// the sites of each colour by class position j: x = 2 (j mod Lx/2) + parity,
// lattice row j div (Lx/2).  Then 32 consecutive positions of colour c (two
// lattice rows when Lx = 32) have all their neighbours inside a few blocks of
// 32 consecutive positions of colour 1 - c: the same rows, the rows before and
// after them, and the same rows one plane up and down.  With the spins of
// colour 1 - c held as bytes b = 1 for -1 and 0 for +1, the fields of 32 sites
// for 32 replicas are
//     I = (h + sum_d J_d) - 2 sum_blocks (B_block^T b_block),
// where B_block[k][n] is the coupling between in-position k of the block and
// out-position n (zero unless they are neighbours).  Each block is one
// v_mfma_i32_32x32x32_i8 with the 32 replicas as rows, the block's 32 positions
// as K and the 32 out-positions as columns; the sums are exact in int32.  The
// coupling fragments hold -16 B and the accumulator starts at 8 (h + sum J + 7),
// so the sum is 8 (I + 7) = the LDS byte address of the decision word S(I): the
// vector ALU is left with the random words and the carry of w + S(I), which is
// the new spin byte b (the heat-bath rule with the Philox word w, as in the
// other kernels), stored as it is.
//
// Device layout of this path: spins as bytes b in {0, 1}, tile-major: for each
// colour, replica tile of 32 and position tile of 32, one 1 KiB block of 32 rows
// (replicas) x 32 bytes (positions), [2][Rp / 32][N / 64][32][32]; Rp a multiple
// of 128.  An MFMA operand is then one contiguous 1 KiB read, and the results of a
// tile fill one 1 KiB block.  The couplings are prepared once per problem: for
// every colour and tile of 32 out-positions the list of K blocks, and for every
// position its (block, K index, -16 J) entries, at most six; each wave writes its
// tile's MFMA B fragments (64 lanes x 16 bytes per block, mostly zeros) from these
// entries into LDS and reads them back once.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <numeric>
#include <vector>

#include "device.h"
#include "internal.h"

namespace pbit {

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

constexpr int kThreads = 256;
constexpr int kFieldOff = 7;
constexpr int kFieldSlots = 2 * kFieldOff + 1;
constexpr int kXcds = 8;  // MI355X: workgroup i runs on XCD i mod 8

// Byte offset of (colour c, replica r, class position j): RT replica tiles, T position tiles.
__device__ __forceinline__ size_t eam_off(int c, int r, int j, int RT, int T)
{
    return ((((size_t)c * RT + (r >> 5)) * T + (j >> 5)) << 10) + ((r & 31) << 5) + (j & 31);
}

// Global site index of class position j of colour c.
__device__ __forceinline__ int site_of(int c, int j, int hx, int Lx, int Ly)
{
    const int row = j / hx, kx = j - row * hx;
    const int y = row % Ly, z = row / Ly;
    return 2 * kx + ((c + y + z) & 1) + Lx * row;
}

// Random start: thread (colour, replica group, position) writes the four replicas' bytes.
__global__ __launch_bounds__(kThreads) void k_eam_init(uint8_t *__restrict__ S, int N2, int Rp, int hx, int Lx,
                                                       int Ly, uint32_t rq0, uint32_t k0, uint32_t k1)
{
    const int64_t gid = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    const int groups = Rp / 4;
    if (gid >= (int64_t)2 * N2 * groups) return;
    const int j = (int)(gid % N2);
    const int64_t rest = gid / N2;
    const int g = (int)(rest % groups), c = (int)(rest / groups);
    const int i = site_of(c, j, hx, Lx, Ly);
    const Block4 b = philox((uint32_t)i, 0u, rq0 + (uint32_t)g, kDomainInit, k0, k1);
#pragma unroll
    for (int p = 0; p < 4; ++p)
        S[eam_off(c, 4 * g + p, j, Rp / 32, N2 / 32)] = init_spin(b.w[p]) < 0 ? (uint8_t)1 : (uint8_t)0;
}

// [R][N] +-1 rows <-> the tile-major bytes of this path (padding replicas start at +1).
template <bool TO_DEVICE>
__global__ __launch_bounds__(kThreads) void k_eam_copy(int8_t *__restrict__ rows, uint8_t *__restrict__ S, int N2,
                                                       int R, int Rp, int hx, int Lx, int Ly)
{
    const int64_t gid = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (gid >= (int64_t)2 * N2 * Rp) return;
    const int j = (int)(gid % N2);
    const int64_t rest = gid / N2;
    const int r = (int)(rest % Rp), c = (int)(rest / Rp);
    const int64_t N = 2 * (int64_t)N2;
    const int i = site_of(c, j, hx, Lx, Ly);
    const size_t o = eam_off(c, r, j, Rp / 32, N2 / 32);
    if (TO_DEVICE) {
        S[o] = r < R && rows[(size_t)r * N + i] < 0 ? (uint8_t)1 : (uint8_t)0;
    } else if (r < R) {
        rows[(size_t)r * N + i] = S[o] ? (int8_t)-1 : (int8_t)1;
    }
}

// E[r] = -sum_{i of colour 1} m_i sum_d J_d m_{nb_d(i)} - sum_i h_i m_i: every bond has
// exactly one end of colour 1.  Block (position chunk, replica r0 + blockIdx.y): 256
// positions of colour 1 (their bonds) and of both colours (their fields).
__global__ __launch_bounds__(kThreads) void k_eam_energy(const uint8_t *__restrict__ S, const uint32_t *__restrict__ code,
                                                         int N2, int Rp, int hx, int Lx, int Ly, int Lz, int r0,
                                                         int32_t *__restrict__ E)
{
    const int r = r0 + (int)blockIdx.y;
    const int j = blockIdx.x * kThreads + threadIdx.x;
    const int RT = Rp / 32, T = N2 / 32;
    int e = 0;
    if (j < N2) {
        for (int c = 0; c < 2; ++c) {
            const int i = site_of(c, j, hx, Lx, Ly);
            const uint32_t w = code[i];
            const int nnz = __builtin_popcount(w & 63u);
            const int hv = (int)(int8_t)(w >> kCodeBaseShift) - nnz;
            const int m = S[eam_off(c, r, j, RT, T)] ? -1 : 1;
            e -= hv * m;
            if (c == 1) {
                const int x = i % Lx, y = (i / Lx) % Ly, z = i / (Lx * Ly);
                const int xs[6] = {x + 1 == Lx ? 0 : x + 1, x == 0 ? Lx - 1 : x - 1, x, x, x, x};
                const int ys[6] = {y, y, y + 1 == Ly ? 0 : y + 1, y == 0 ? Ly - 1 : y - 1, y, y};
                const int zs[6] = {z, z, z, z, z + 1 == Lz ? 0 : z + 1, z == 0 ? Lz - 1 : z - 1};
                int f = 0;
#pragma unroll
                for (int d = 0; d < 6; ++d) {
                    if (!((w >> d) & 1u)) continue;
                    const int J = ((w >> (kCodeFlipShift + d)) & 1u) ? -1 : 1;
                    const int jn = (xs[d] >> 1) + hx * (ys[d] + Ly * zs[d]);
                    f += J * (S[eam_off(0, r, jn, RT, T)] ? -1 : 1);
                }
                e -= m * f;
            }
        }
    }
    for (int off = 32; off > 0; off >>= 1) e += __shfl_xor(e, off, 64);
    __shared__ int32_t part[kThreads / 64];
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = e;
    __syncthreads();
    if (threadIdx.x == 0) atomicAdd(E + r, part[0] + part[1] + part[2] + part[3]);
}

// One half-sweep.  A wave (a unit of work) takes one tile of 32 out-positions of
// colour c and RTW tiles of 32 replicas: its coupling fragments (one per K block)
// are built once, then for every replica tile the spin fragments of the K blocks,
// NB MFMAs, and the decisions.  Lane l holds out-position l % 32; accumulator
// element 4 q + i of lane l is replica 8 q + 4 (l / 32) + i of the tile, so a lane's
// elements 4q .. 4q + 3 are the four replicas of one Philox block.
//
// The units are split over the 8 XCDs (workgroup i runs on XCD i mod 8) so that
// each XCD's L2 holds one part of the spins: gx = gcd(groups, 8) parts of the
// replica-tile groups times 8 / gx ranges of position tiles (a range reads the
// planes next to it from its neighbours' ranges).  Inside an XCD the units run
// group by group, tile by tile.
template <int NB, int RTW>
__global__ __launch_bounds__(kThreads) void k_eam_halfsweep(uint8_t *__restrict__ S, const int32_t *__restrict__ tiles,
                                                            const int2 *__restrict__ pos,
                                                            const v4i *__restrict__ bonds, EaRow row, int T, int RT,
                                                            int colour, int gx, uint32_t sweep, uint32_t rq0, uint32_t k0, uint32_t k1,
                                                            uint32_t one)
{
    __shared__ uint64_t tab[kFieldSlots];
    __shared__ v4i fragbuf[kThreads / 64][NB][64];  // each wave's B fragments
    const int tid = threadIdx.x;
    if (tid < kFieldSlots) {
        uint64_t v = row.s[0];
#pragma unroll
        for (int e = 1; e < kFieldSlots; ++e) v = tid == e ? row.s[e] : v;
        tab[tid] = v;
    }
    __syncthreads();
    const int x = (int)(blockIdx.x % kXcds), px = kXcds / gx;
    const int xr = x % gx, xp = x / gx, gpx = RT / RTW / gx;  // replica part, tile range, groups per part
    const int t_lo = (int)((int64_t)T * xp / px), nt = (int)((int64_t)T * (xp + 1) / px) - t_lo;
    const int u = __builtin_amdgcn_readfirstlane((int)(blockIdx.x / kXcds) * (kThreads / 64) + (tid >> 6));
    if (u >= gpx * nt) return;
    const int t = t_lo + u % nt, rg = xr * gpx + u / nt;
    const int lane = tid & 63, n = lane & 31, g = lane >> 5;
    const int c = colour;
    // tile record: the NB block starts (positions of colour 1 - c)
    const int32_t *tr = tiles + (size_t)(c * T + t) * 16;
    int blk[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) blk[b] = __builtin_amdgcn_readfirstlane(tr[1 + b]);
    // B fragments: zero this wave's LDS copy, write the bonds of out-position n (lanes
    // n and n + 32 take three entries each; entry: block, K index k, -16 J at lane
    // n + 32 (k / 16), byte k % 16 of the block's fragment), read the fragments back
    const int wv = tid >> 6;
    const v4i ent = bonds[(size_t)c * (32 * T) + 32 * t + n];
#pragma unroll
    for (int b = 0; b < NB; ++b) fragbuf[wv][b][lane] = v4i{0, 0, 0, 0};
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    char *fb = reinterpret_cast<char *>(&fragbuf[wv][0][0]);
#pragma unroll
    for (int e = 0; e < 3; ++e) {
        const int w16 = 3 * g + e;  // entry index 0..5
        const uint32_t word = (uint32_t)ent[w16 >> 1] >> (16 * (w16 & 1));
        const int b = (int)(word & 7u), k = (int)((word >> 3) & 31u);
        const int8_t v = (int8_t)(word >> 8);
        if (v != 0) fb[((b * 64) + n + 32 * (k >> 4)) * 16 + (k & 15)] = v;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    v4i B[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) B[b] = fragbuf[wv][b][lane];
    const int2 pm = pos[(size_t)c * (32 * T) + 32 * t + n];  // site, 8 (h + sum J + 7)
    v16i cinit;
#pragma unroll
    for (int e = 0; e < 16; ++e) cinit[e] = pm.y;
    const char *tb = reinterpret_cast<const char *>(tab);
    const uint8_t *Sin = S + ((size_t)(1 - c) * RT * T << 10);
    uint8_t *Sout = S + ((size_t)c * RT * T << 10);
    const int a_off = 32 * n + 16 * g;   // A fragment: row n, K bytes 16 g .. 16 g + 15
    const int s_off = 128 * g + n;       // result element (q, i): row 8 q + 4 g + i, column n
    // Pipelined over the replica tiles, with two sets of spin fragments: step rt
    // issues the loads of tile rt + 2 (before the stores of tile rt, so that waiting
    // for them never waits for those stores), makes the decisions and stores of tile
    // rt, then runs the MFMAs of tile rt + 1 with the random words of tile rt + 1
    // drawn between them, so that the vector ALU works while the dependent MFMAs run.
    v4i A0[NB], A1[NB];
    Block4 w[4];
    auto load = [&](v4i(&A)[NB], int rtile) {
        const uint8_t *in = Sin + ((size_t)rtile * T << 10) + a_off;
#pragma unroll
        for (int b = 0; b < NB; ++b) A[b] = *reinterpret_cast<const v4i *>(in + ((size_t)blk[b] << 5));
    };
    auto draw = [&](int rtile) {
#pragma unroll
        for (int q = 0; q < 4; ++q)
            w[q] = philox((uint32_t)pm.x, sweep, rq0 + (uint32_t)(8 * rtile + 2 * q + g), kDomainSweep, k0, k1);
    };
    auto fields = [&](const v4i(&A)[NB]) {
        v16i f = __builtin_amdgcn_mfma_i32_32x32x32_i8(A[0], B[0], cinit, 0, 0, 0);
#pragma unroll
        for (int b = 1; b < NB; ++b) f = __builtin_amdgcn_mfma_i32_32x32x32_i8(A[b], B[b], f, 0, 0, 0);
        return f;
    };
    const int rt0 = rg * RTW;
    load(A0, rt0);
    load(A1, rt0 + 1);
    draw(rt0);
    v16i acc = fields(A0);
    // cur holds tile rt + 1's fragments, nxt is free
    auto step = [&](int rt, v4i(&cur)[NB], v4i(&nxt)[NB]) {
        __builtin_amdgcn_sched_barrier(0);
        // past the last tile: the last tile again (in bounds, and without a branch here)
        load(nxt, rt0 + min(rt + 2, RTW - 1));
        __builtin_amdgcn_sched_barrier(0);
        uint8_t *out = Sout + (((size_t)(rt0 + rt) * T + t) << 10) + s_off;
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                // acc = 8 (I + 7): the byte address of S(I) in the table
                const uint64_t Sd = *static_cast<const uint64_t *>(__builtin_assume_aligned(tb + acc[4 * q + i], 8));
                const uint32_t b1 = (uint32_t)(((uint64_t)w[q].w[i] * one + Sd) >> 32);  // 1: the new spin is -1
                out[32 * (8 * q + i)] = (uint8_t)b1;
            }
        __builtin_amdgcn_sched_barrier(0);
        if (rt + 1 < RTW) {
            acc = fields(cur);
            draw(rt0 + rt + 1);
            // one MFMA, then a share of the Philox rounds, NB times
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
                __builtin_amdgcn_sched_group_barrier(0x002, 144 / NB, 0);
            }
        }
    };
#pragma unroll 1
    for (int rt = 0; rt < RTW; rt += 2) {
        step(rt, A1, A0);
        step(rt + 1, A0, A1);
    }
}

}  // namespace

// ---- host: the tiles and coupling fragments of a cube ------------------------

bool ea_mfma_build(int Lx, int Ly, int Lz, const int8_t *J, const int8_t *h, EaMfmaHost &out)
{
    const int64_t N = (int64_t)Lx * Ly * Lz, N2 = N / 2, hx = Lx / 2;
    if (N2 % 32 != 0 || N2 > (1 << 26)) return false;
    const int n_tiles = (int)(N2 / 32);
    auto pos_of = [&](int x, int y, int z) { return (int64_t)(x >> 1) + hx * (y + (int64_t)Ly * z); };
    std::vector<std::vector<int>> blocks((size_t)2 * n_tiles);
    int nb = 0;
    // per colour and tile: the distinct blocks its out-positions' neighbours fall in
    for (int c = 0; c < 2; ++c)
        for (int t = 0; t < n_tiles; ++t) {
            std::vector<int> &bl = blocks[(size_t)c * n_tiles + t];
            for (int n = 0; n < 32; ++n) {
                const int64_t j = 32 * (int64_t)t + n, rowi = j / hx, kx = j % hx;
                const int y = (int)(rowi % Ly), z = (int)(rowi / Ly), x = (int)(2 * kx + ((c + y + z) & 1));
                const int xs[6] = {(x + 1) % Lx, (x + Lx - 1) % Lx, x, x, x, x};
                const int ys[6] = {y, y, (y + 1) % Ly, (y + Ly - 1) % Ly, y, y};
                const int zs[6] = {z, z, z, z, (z + 1) % Lz, (z + Lz - 1) % Lz};
                for (int d = 0; d < 6; ++d) {
                    const int blk = (int)(32 * (pos_of(xs[d], ys[d], zs[d]) / 32));
                    if (std::find(bl.begin(), bl.end(), blk) == bl.end()) bl.push_back(blk);
                }
            }
            std::sort(bl.begin(), bl.end());
            nb = std::max(nb, (int)bl.size());
        }
    if (nb > kEaMfmaMaxBlocks) return false;
    nb = std::max(nb, 3);  // the kernel is instantiated for 3 to 8 blocks; extra blocks carry zero couplings
    out.nb = nb;
    out.n_tiles = n_tiles;
    out.tiles.assign((size_t)2 * n_tiles * 16, 0);
    out.bonds.assign((size_t)2 * N2 * 8, 0);
    out.pos.assign((size_t)2 * N2 * 2, 0);
    for (int c = 0; c < 2; ++c)
        for (int t = 0; t < n_tiles; ++t) {
            const size_t ti = (size_t)c * n_tiles + t;
            std::vector<int> bl = blocks[ti];
            while ((int)bl.size() < nb) bl.push_back(bl[0]);  // padding blocks carry zero couplings
            int32_t *rec = &out.tiles[ti * 16];
            for (int b = 0; b < nb; ++b) rec[1 + b] = bl[(size_t)b];
            for (int n = 0; n < 32; ++n) {
                const int64_t j = 32 * (int64_t)t + n, rowi = j / hx, kx = j % hx;
                const int y = (int)(rowi % Ly), z = (int)(rowi / Ly), x = (int)(2 * kx + ((c + y + z) & 1));
                const int64_t i = x + (int64_t)Lx * rowi;
                // the six bonds of site i: +x, -x, +y, -y, +z, -z (two bonds between a pair when a side is 2)
                const int xs[6] = {(x + 1) % Lx, (x + Lx - 1) % Lx, x, x, x, x};
                const int ys[6] = {y, y, (y + 1) % Ly, (y + Ly - 1) % Ly, y, y};
                const int zs[6] = {z, z, z, z, (z + 1) % Lz, (z + Lz - 1) % Lz};
                const int64_t im[3] = {xs[1] + (int64_t)Lx * (y + (int64_t)Ly * z),
                                       x + (int64_t)Lx * (ys[3] + (int64_t)Ly * z),
                                       x + (int64_t)Lx * (y + (int64_t)Ly * zs[5])};
                const int8_t Jd[6] = {J[i], J[im[0]], J[N + i], J[N + im[1]], J[2 * N + i], J[2 * N + im[2]]};
                int base = h ? h[i] : 0;
                // entries (block, K index, -16 J), bonds to the same neighbour merged (at most two
                // bonds join a pair, when a side is 2: |value| <= 32)
                int eb[6], ek[6], ev[6], ne = 0;
                for (int d = 0; d < 6; ++d) {
                    base += Jd[d];
                    if (Jd[d] == 0) continue;
                    const int64_t jn = pos_of(xs[d], ys[d], zs[d]);
                    const int b = (int)(std::find(bl.begin(), bl.end(), (int)(32 * (jn / 32))) - bl.begin());
                    const int k = (int)(jn % 32);
                    int e = 0;
                    while (e < ne && (eb[e] != b || ek[e] != k)) ++e;
                    if (e == ne) {
                        eb[ne] = b;
                        ek[ne] = k;
                        ev[ne++] = 0;
                    }
                    ev[e] -= 16 * Jd[d];
                }
                uint16_t *rec16 = &out.bonds[((size_t)c * N2 + j) * 8];
                for (int e = 0; e < ne; ++e)
                    rec16[e] = (uint16_t)(eb[e] | ek[e] << 3 | (uint32_t)(uint8_t)(int8_t)ev[e] << 8);
                out.pos[((size_t)c * N2 + j) * 2] = (int32_t)i;
                out.pos[((size_t)c * N2 + j) * 2 + 1] = 8 * (base + kFieldOff);
            }
        }
    return true;
}

// ---- launchers ---------------------------------------------------------------

static inline unsigned blocks_for(int64_t work) { return (unsigned)((work + kThreads - 1) / kThreads); }

hipError_t eam_init(const EaView &p, uint8_t *S, int Rp, uint32_t rq0, Key key, hipStream_t st)
{
    const int N2 = (int)(p.N / 2);
    hipLaunchKernelGGL(k_eam_init, dim3(blocks_for((int64_t)2 * N2 * (Rp / 4))), dim3(kThreads), 0, st, S, N2, Rp,
                       p.Lx / 2, p.Lx, p.Ly, rq0, key.k0, key.k1);
    return hipGetLastError();
}

hipError_t eam_from_rows(const EaView &p, const int8_t *src, int R, uint8_t *S, int Rp, hipStream_t st)
{
    const int N2 = (int)(p.N / 2);
    hipLaunchKernelGGL(k_eam_copy<true>, dim3(blocks_for((int64_t)2 * N2 * Rp)), dim3(kThreads), 0, st,
                       const_cast<int8_t *>(src), S, N2, R, Rp, p.Lx / 2, p.Lx, p.Ly);
    return hipGetLastError();
}

hipError_t eam_to_rows(const EaView &p, const uint8_t *S, int Rp, int8_t *dst, int R, hipStream_t st)
{
    const int N2 = (int)(p.N / 2);
    hipLaunchKernelGGL(k_eam_copy<false>, dim3(blocks_for((int64_t)2 * N2 * Rp)), dim3(kThreads), 0, st, dst,
                       const_cast<uint8_t *>(S), N2, R, Rp, p.Lx / 2, p.Lx, p.Ly);
    return hipGetLastError();
}

hipError_t eam_energy(const EaView &p, const uint8_t *S, int Rp, int R, int32_t *E, hipStream_t st)
{
    hipError_t e = fill_i32(E, R, 0, st);
    if (e != hipSuccess) return e;
    const int N2 = (int)(p.N / 2);
    // at most 65535 replicas per launch (grid y)
    for (int r0 = 0; r0 < R; r0 += 65535) {
        hipLaunchKernelGGL(k_eam_energy, dim3(blocks_for(N2), (unsigned)std::min(65535, R - r0)), dim3(kThreads), 0,
                           st, S, p.code, N2, Rp, p.Lx / 2, p.Lx, p.Ly, p.Lz, r0, E);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t eam_halfsweep(const EaView &p, uint8_t *S, int Rp, int colour, const EaRow &row, uint32_t sweep,
                         uint32_t rq0, Key key, hipStream_t st)
{
    if (!p.mfma_tiles || Rp % kEaMfmaRPad != 0) return hipErrorInvalidValue;
    const int T = p.mfma_n_tiles, RT = Rp / 32;
    // replica tiles per unit (each unit loads its coupling fragments once): the most
    // that still leaves 16 units (four waves per SIMD) per CU, at least 4
    int rtw = 4;
    for (int w : {16, 8})
        if (RT % w == 0 && (int64_t)T * (RT / w) >= 16 * 256) {
            rtw = w;
            break;
        }
    const int groups = RT / rtw, gx = std::gcd(groups, kXcds), px = kXcds / gx;
    const int most = (groups / gx) * ((T + px - 1) / px);  // units of the busiest XCD
    const dim3 grid((unsigned)(kXcds * ((most + 3) / 4)));
#define PBIT_EAM(NB, W)                                                                                          \
    hipLaunchKernelGGL((k_eam_halfsweep<NB, W>), grid, dim3(kThreads), 0, st, S, p.mfma_tiles, p.mfma_pos,        \
                       reinterpret_cast<const v4i *>(p.mfma_bonds), row, T, RT, colour, gx, sweep,                \
                       rq0, key.k0, key.k1, 1u)
#define PBIT_EAM_W(NB)              \
    if (rtw == 16) PBIT_EAM(NB, 16); \
    else if (rtw == 8) PBIT_EAM(NB, 8); \
    else PBIT_EAM(NB, 4);
    switch (p.mfma_nb) {
    case 3: PBIT_EAM_W(3); break;
    case 4: PBIT_EAM_W(4); break;
    case 5: PBIT_EAM_W(5); break;
    case 6: PBIT_EAM_W(6); break;
    case 7: PBIT_EAM_W(7); break;
    case 8: PBIT_EAM_W(8); break;
    default: return hipErrorInvalidValue;
    }
#undef PBIT_EAM_W
#undef PBIT_EAM
    return hipGetLastError();
}

}  // namespace pbit
