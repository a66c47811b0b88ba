// batch.h — device descriptors of the persistent batched sweep (many jobs in
// one launch).  A job is one anneal (problem, schedule, replicas, seed).  It is
// cut into replica tiles that never need each other: a cube tile is 4, 8 or 16
// replicas of the whole lattice, a biclique tile is 32, 64 or 128 replicas of
// both sides.
// A work item advances one tile over a range of sweeps; a persistent kernel
// pulls items from a queue until the queue is empty.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pbit {

struct EaJobDev {
    const uint2 *sites;     // [2][N / 2] class position -> {site | wrap flags << 16, code}
    const uint32_t *table;  // [S][width] thresholds, row s = local sweep s
    int8_t *state;          // [tiles][N][rs]: spins of a tile, replica fastest (rs = 4, 8 or 16)
    int32_t *energy;        // [tiles * rs]: energies after the tile's last item
    int Lx, Ly, Lz, width;
    int rs;                 // replicas per tile: 4, 8 or 16
    int dense;              // 1: every coupling is nonzero
    uint32_t sweep0;        // absolute index of local sweep 0
    uint32_t rq0;           // global replica group of tile 0 (replica_offset / 4)
    uint32_t k0, k1;        // Philox key
};

struct BqJobDev {
    const int8_t *J, *JT;     // int8 couplings [na_p][nb_p], [nb_p][na_p]
    const int8_t *Jb, *JTb;   // couplings in the widened-bit column order, scaled (bit tiles)
    const int32_t *hA2, *hB2; // field plus coupling sum per site (bit tiles)
    const uint32_t *J2, *JT2; // J + 1 as two-bit codes in fragment order (int8 tiles)
    const int8_t *hA, *hB;    // [na_p], [nb_p]
    const uint32_t *table;    // [S][width]
    uint8_t *state;           // [tiles][RS][row]: row r = side A then side B, as int8 (na_p + nb_p
                              // bytes, the default) or bits ((na_p + nb_p) / 8 bytes)
    int32_t *energy;        // [tiles * RS]
    int na, nb, na_p, nb_p, width;
    uint32_t sweep0, rq0, k0, k1;
};

struct GraphJobDev {
    const int4 *meta;          // [n] by class position: site, first and end adjacency entry, nnz + h
    const uint32_t *adj;       // adjacency words in position order: neighbour << 2 | J != 0 | (J == -1) << 1
    const int32_t *class_start;  // [n_colours + 1] class boundaries in position order
    const int32_t *bi, *bj;    // bond list (for energies)
    const int8_t *bJ;
    const int8_t *h;           // [n] or null
    const uint32_t *table;     // [S][width] thresholds, row s = local sweep s
    int8_t *state;             // [tiles][n][rs]: spins of a tile, replica fastest (rs = 4, 8 or 16)
    int32_t *energy;           // [tiles * rs]
    int n, n_bonds, n_colours, width, rs;
    uint32_t sweep0, rq0, k0, k1;
    // 0: the layout above; else the bytes from one site's row to the next in a [n][row_stride]
    // matrix whose columns [rs t, + rs) are tile t (the per-instance spins, row_stride = Rp)
    int row_stride = 0;
};

struct WorkItem {
    int32_t job;      // index into the job array of the item's kind
    int32_t tile;
    int32_t s_begin;  // local sweeps [s_begin, s_end)
    int32_t s_end;
    int32_t init;     // 1: draw the tile's random start before the first sweep
    int32_t pad[3];
};

constexpr int kEaTileThreads = 512;
// cube tiles with more than this many bytes of LDS rows run one workgroup per CU, as
// kEaTileThreadsLarge threads (ea_tiles picks the form from the launch's LDS bytes)
constexpr int kEaTileThreadsLarge = 1024;
constexpr size_t kEaLargeTileLds = 80 * 1024;
constexpr int kGraphTileThreads = 512;
constexpr int kBqTileThreads = 512;

// Launch a persistent kernel over `n_items` items; `counter` (device int,
// zeroed by the caller) hands out item indices.
hipError_t ea_tiles(const EaJobDev *jobs, const WorkItem *items, const int32_t *n_items, int32_t *counter,
                    int grid, size_t lds_bytes, hipStream_t st);
// operand modes of the biclique tiles
constexpr int kTileInt8 = 0, kTileBits = 2;
hipError_t bq_tiles(const BqJobDev *jobs, const WorkItem *items, const int32_t *n_items, int32_t *counter,
                    int rs, int mode, int grid, size_t lds_bytes, hipStream_t st);

hipError_t graph_tiles(const GraphJobDev *jobs, const WorkItem *items, const int32_t *n_items, int32_t *counter,
                       int grid, size_t lds_bytes, hipStream_t st);
// The per-instance graph sweep held in LDS: sweeps [s_begin, s_end) of tiles [0, tiles) of
// job `jb` (row_stride set: the spins stay in the per-instance [n][Rp] layout), one
// workgroup per tile, no work queue.  jb.energy receives each replica's energy.
hipError_t graph_slab(const GraphJobDev &jb, int tiles, int s_begin, int s_end, hipStream_t st);

// LDS a tile kernel needs for the given job shape.
size_t ea_tile_lds(int64_t N, int rs);  // rs = 4, 8 or 16 replicas
size_t graph_tile_lds(int64_t N, int rs);
size_t bq_tile_lds(int rs, int na_p, int nb_p, int width, int mode);
hipError_t tiles_set_lds_limit();

}  // namespace pbit
