// bq.h — biclique problem view and launchers (declarations shared by the
// host runtime and the biclique kernels).
#pragma once

#include "internal.h"

namespace pbit {

struct BqView {
    int na, nb;      // real side sizes
    int na_p, nb_p;  // padded to kBqPad (extra couplings and spins are zero)
    const int8_t *J;   // [na_p][nb_p]
    const int8_t *JT;  // [nb_p][na_p]
    const int8_t *hA;  // [na_p]
    const int8_t *hB;  // [nb_p]
    // for the kernels on spin bits: the couplings with the columns of every group of
    // 32 in the order the widened bits take, scaled by 2^(3 - j) for the bit's
    // position j in its byte lane, [na_p][nb_p] and [nb_p][na_p], and each site's
    // field plus its coupling sum
    const int8_t *Jb;
    const int8_t *JTb;
    const int32_t *hA2;  // [na_p]
    const int32_t *hB2;  // [nb_p]
    // for the batched int8 tiles: J + 1 (padding included) as two-bit codes, 16 per word,
    // in MFMA fragment order (see load_biclique), [na_p * nb_p / 16] and [nb_p * na_p / 16]
    const uint32_t *J2;
    const uint32_t *JT2;
};

constexpr int kBqPad = 64;       // site padding of small biclique sides (MFMA K and N tiles)
constexpr int kBqPadLarge = 128; // site padding of sides with at least kBqLargeSide sites
constexpr int kBqLargeSide = 512;
constexpr int kBqRPad = 128;     // replica padding of biclique spin matrices (MFMA M tile)
constexpr int kMaxTableWidth = 4096;  // threshold-row entries a biclique kernel stages in LDS (16 KiB)

// ---- biclique launchers; spins are device MA [Rp][na_p], MB [Rp][nb_p] -----
// Kernel variants of a biclique half-sweep.  Small: 64 x 64 tiles straight from
// global memory (any padding); Dma: 128 x 128 tiles with K stages of 128 bytes
// moved by the global-to-LDS DMA into a ring of 4 stages (sides padded to 128,
// Rp a multiple of 128); Bits: tiles of 64 sites x 256, 128 or 64 replicas on spins
// held as bits, widened for the int8 MFMA (bqb_*; sides padded to 128, Rp a multiple
// of 256); Slab: sides of
// at most 512 sites, couplings and 16- or 8-replica slices held in LDS for runs of
// sweeps in one launch (bq_slab).
enum class BqVariant : int { Auto = 0, Small = 1, Dma = 2, Bits = 3, Slab = 4 };
// The LDS-resident form for small sides: sweeps [s_begin, s_end) (table rows), absolute
// index sweep0 + s, of all Rp replicas (Rp / rs workgroups of rs-replica slices) on MA / MB
// in place.  rs is 16 or 8; 0 picks 16 when that gives a workgroup to every compute unit,
// else 8.  bq_slab_rs returns the slice that a launch with rs uses (0: none fits Rp).
int bq_slab_rs(int Rp, int rs);
bool bq_slab_supported(const BqView &p, int Rp, int width, int rs = 0);
hipError_t bq_slab(const BqView &p, int8_t *MA, int8_t *MB, int Rp, const uint32_t *table, int width, int s_begin,
                   int s_end, uint32_t sweep0, uint32_t rq0, Key key, hipStream_t st, int rs = 0);
hipError_t bq_init(const BqView &p, int8_t *MA, int8_t *MB, int R, uint32_t rq0, Key key, hipStream_t st);
hipError_t bq_from_rows(const BqView &p, const int8_t *src_rn, int R, int8_t *MA, int8_t *MB, hipStream_t st);
hipError_t bq_to_rows(const BqView &p, const int8_t *MA, const int8_t *MB, int8_t *dst_rn, int R, hipStream_t st);
hipError_t bq_halfsweep(const BqView &p, int side, int8_t *MA, int8_t *MB, int R, int Rp, const uint32_t *trow,
                        int width, uint32_t sweep, uint32_t rq0, Key key, hipStream_t st, BqVariant variant);
hipError_t bq_energy(const BqView &p, const int8_t *MA, const int8_t *MB, int R, int Rp, int32_t *E, hipStream_t st);

// ---- the same with spins held as bits (set = -1), 32 sites per word, by blocks of 128 sites:
// word w of replica r at ((w / 4) Rp + r) 4 + w % 4 of MAb (na_p / 32 words per replica) or MBb
bool bqb_supported(const BqView &p, int Rp);
hipError_t bqb_pack(const BqView &p, const int8_t *MA, const int8_t *MB, uint32_t *MAb, uint32_t *MBb, int Rp,
                    hipStream_t st);
hipError_t bqb_unpack(const BqView &p, const uint32_t *MAb, const uint32_t *MBb, int8_t *MA, int8_t *MB, int Rp,
                      hipStream_t st);
// rt: replicas per tile, 64, 128 or 256; 0 (or a value that does not divide Rp): 256
// where that gives at least 256 workgroups, else 128
hipError_t bqb_halfsweep(const BqView &p, int side, uint32_t *MAb, uint32_t *MBb, int Rp, const uint32_t *trow,
                         int width, uint32_t sweep, uint32_t rq0, Key key, hipStream_t st, int rt = 0);

}  // namespace pbit
