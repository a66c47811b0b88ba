// internal.h — declarations shared by the host runtime and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

namespace pbit {

// Per-site coupling code of a periodic cube.  Directions d = 0..5 are
// +x, -x, +y, -y, +z, -z.  Bit d: J != 0 on that bond; bit 6 + d: J == -1;
// bits 16..23: nnz(J) + h as a signed byte, so that the local field is
//   I = (nnz + h) - 2 * #{d : J_d m_d = -1};
// bits 24..31: 8 (7 - nnz(J) + h), so that
//   8 (I + 7) = 16 #{d : J_d m_d = +1} + bits 24..31.
constexpr int kCodeFlipShift = 6;
constexpr int kCodeBaseShift = 16;
constexpr int kCodePosShift = 24;

struct EaView {
    int Lx, Ly, Lz;
    int64_t N;
    const uint32_t *code;  // [N]
    const int8_t *J;       // [3][N] as given (for from-scratch energies)
    const int8_t *h;       // [N] or null
    bool dense;            // every coupling is nonzero
    // for lattices the LDS-resident kernel takes: per colour c and class position j
    // (x = 2 (j mod Lx/2) + parity, row j / (Lx/2)), the pair {site | wrap flags of
    // the +x, -x, +y, -y, +z, -z neighbours << 16, site code}, [2][N / 2]; else null
    const uint32_t *slab_sites;
    // the matrix-core half-sweep (ea_mfma.hip), where the cube's shape allows it: per
    // colour and tile of 32 class positions a 16-word record (first coupling fragment,
    // then the K block starts), per colour and position {site, 8 (h + sum J + 7)}, and
    // the B fragments (64 lanes x 16 bytes each); null where not built
    const int32_t *mfma_tiles;
    const int2 *mfma_pos;
    const void *mfma_bonds;
    int mfma_nb;       // K blocks per tile
    int mfma_n_tiles;  // tiles per colour
};

constexpr int kEaMfmaMaxBlocks = 8;
struct EaMfmaHost {
    int nb = 0, n_tiles = 0;
    std::vector<int32_t> tiles;  // [2][n_tiles][16]
    std::vector<int32_t> pos;    // [2][N / 2][2]
    std::vector<uint16_t> bonds; // [2][N / 2][8]: per position up to 6 (block, K index, -16 J) entries
};
// Builds the tiles of the matrix-core half-sweep; false where the shape does not allow it
// (N / 2 not a multiple of 32, or a tile whose neighbours span more than kEaMfmaMaxBlocks blocks).
bool ea_mfma_build(int Lx, int Ly, int Lz, const int8_t *J, const int8_t *h, EaMfmaHost &out);

// General sparse graph with k colour classes (greedy colouring by default).
constexpr int kGraphMaxDegree = 127;  // bytewise counts of negative products stay below 256

struct GraphView {
    int n, n_bonds, n_colours, max_degree;
    // sites are numbered by position: grouped by colour, ascending inside a class
    const int32_t *class_start;  // host [n_colours + 1]: class c holds positions class_start[c] .. class_start[c+1]
    const int32_t *site_meta;    // device [n][4] by position: site id, first and end adjacency entry,
                                 // nnz(J) + h (in [-1, kGraphMaxDegree + 1])
    const uint32_t *adj;         // device [2 n_bonds] in position order: neighbour << 2 | bit 0 J != 0, bit 1 J == -1
    const int32_t *bi, *bj;      // device bond list
    const int8_t *bJ;
    const int8_t *h;             // device [n] or null
    const int32_t *class_start_dev;  // device copy of class_start (the batched tiles read it)
};

constexpr int kEaRPad = 16;   // replica padding of the cube spin matrix (one dwordx4 per thread)

struct Key {
    uint32_t k0, k1;
};

// ---- EA launchers; spins are device [N][Rp] (replica fastest) ------------
hipError_t ea_init(const EaView &p, int8_t *spins, int Rp, uint32_t rq0, Key key, hipStream_t st);
hipError_t ea_from_rows(const EaView &p, const int8_t *src_rn, int R, int8_t *spins, int Rp, hipStream_t st);
hipError_t ea_to_rows(const EaView &p, const int8_t *spins, int Rp, int8_t *dst_rn, int R, hipStream_t st);
// Decision words of one sweep for the cube: S(I) for I = -7 .. 7 (Tm for
// I >= 0, 2^32 - Tm for I < 0), passed to the half-sweep by value.
struct EaRow {
    uint64_t s[15];
};
EaRow ea_row(const uint32_t *host_trow, int width);
// ny: lattice rows per workgroup (0 = choose); early_rng: draw the random words before the field
// Sweeps [s_begin, s_end) of a cube of at most kEaSlabMaxSites sites held in LDS,
// 16 replicas per workgroup; table row s is sweep s, its absolute index sweep0 + s.
constexpr int kEaSlabMaxSites = 8192;
bool ea_slab_fits(const EaView &p);
hipError_t ea_slab(const EaView &p, int8_t *spins, int Rp, const uint32_t *table, int width, int s_begin, int s_end,
                   uint32_t sweep0, uint32_t rq0, Key key, hipStream_t st);
hipError_t ea_halfsweep(const EaView &p, int8_t *spins, int Rp, int colour, const EaRow &row, uint32_t sweep,
                        uint32_t rq0, Key key, hipStream_t st, int ny = 0, bool early_rng = true);
hipError_t ea_energy(const EaView &p, const int8_t *spins, int Rp, int R, int32_t *E, hipStream_t st);

// ---- the matrix-core cube path: spins as bytes b (1 = -1), tile-major [2][Rp / 32][N / 64][32][32]
// (colour, replica tile, position tile, replica, position), Rp a multiple of 128
constexpr int kEaMfmaRPad = 128;
hipError_t eam_init(const EaView &p, uint8_t *S, int Rp, uint32_t rq0, Key key, hipStream_t st);
hipError_t eam_from_rows(const EaView &p, const int8_t *src, int R, uint8_t *S, int Rp, hipStream_t st);
hipError_t eam_to_rows(const EaView &p, const uint8_t *S, int Rp, int8_t *dst, int R, hipStream_t st);
hipError_t eam_energy(const EaView &p, const uint8_t *S, int Rp, int R, int32_t *E, hipStream_t st);
hipError_t eam_halfsweep(const EaView &p, uint8_t *S, int Rp, int colour, const EaRow &row, uint32_t sweep,
                         uint32_t rq0, Key key, hipStream_t st);

// ---- general graphs; spins are device [N][Rp] like the cube ----------------
hipError_t graph_halfsweep(const GraphView &g, int colour, int8_t *spins, int Rp, const uint32_t *trow, int width,
                           uint32_t sweep, uint32_t rq0, Key key, hipStream_t st);
hipError_t graph_energy(const GraphView &g, const int8_t *spins, int Rp, int R, int32_t *E, hipStream_t st);

// ---- misc ---------------------------------------------------------------
hipError_t fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t st);
hipError_t widen_i32_i64(const int32_t *src, int64_t *dst, int64_t n, hipStream_t st);
// *hit = sweep if min_r E[r] <= target and *hit is still INT32_MAX
hipError_t check_target(const int32_t *E, int R, int64_t target, int32_t sweep, int32_t *hit, hipStream_t st);

}  // namespace pbit
