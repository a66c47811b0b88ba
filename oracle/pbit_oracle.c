/*
 * pbit_oracle.c — plain, single-threaded CPU reference of the simulated p-bit
 * Ising-machine sweep.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle that the HIP library is
 * checked against.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load it; the library never calls it and shares no
 * code with it.
 *
 * What it computes (paper: "Probabilistic Computing Optimization of Complex
 * Spin-Glass Topologies", arXiv 2510.23419):
 *
 *   energy   E(m) = - sum_{bonds (i,j)} J_ij m_i m_j - sum_i h_i m_i
 *            (Sec. 1.1.1, Eq. 1, read with the minus sign and a field term so
 *            that the heat-bath rule below samples exp(-beta E); m_i = +-1)
 *   field    I_i = sum_{j in N(i)} J_ij m_j + h_i          (Sec. 1.2.1, Eq. 3)
 *   update   m_i = sgn(tanh(beta I_i) - u),  u uniform on (-1, 1)
 *            (Sec. 1.2.1, Eq. 2, read with tanh and a per-iteration beta,
 *            Sec. 1.3.1)
 *   groups   the spins of one colour class are updated together; classes are
 *            visited in ascending colour id (Sec. 1.2.2, update groups)
 *   anneal   one sweep = every colour class once; beta is constant within a
 *            sweep and follows a caller-given schedule (Sec. 1.3.1); replicas
 *            are independent runs (Sec. 1.3.3).
 *
 * Integer form of the update.  u is drawn as u = (w + 1/2) / 2^31 - 1 from a
 * uint32 w.  With a = |I| the minority probability is
 *     q(beta, a) = (1 - tanh(beta a)) / 2 = 1 / (1 + exp(2 beta a)),
 * and the threshold  Tm = round-half-down(q * 2^32)  is evaluated in IEEE
 * binary64 as  Tm = ceil(ldexp(1.0 / (1.0 + exp((2.0 * beta) * a)), 32) - 0.5).
 * With s = +1 if I >= 0 else -1 and x = ~w if I >= 0 else w, the new spin is
 * -s if x < Tm and s otherwise.
 *
 * Randomness.  Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random
 * numbers: as easy as 1, 2, 3", SC'11), key = (seed mod 2^32, seed >> 32),
 * counter = (spin id, absolute sweep index, global replica >> 2, domain).
 * Domain 0 draws the updates, domain 1 (sweep 0) the random initial spins.
 * Word (global replica & 3) of the 4-word output is the replica's draw, so
 * every (spin, sweep, replica) uses exactly one word.  The initial spin is +1
 * if that word is below 2^31 and -1 otherwise.
 *
 * The oracle works on a general bond list with an explicit colouring, so the
 * cubic lattice and the biclique are two ways of building its input.  It keeps
 * each replica's energy incrementally (dE = -(m_new - m_old) I_i) and checks
 * it against a from-scratch evaluation after every traced sweep and at the end.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_OK 0
#define ORACLE_E_ARG (-1)
#define ORACLE_E_COLOURING (-2)
#define ORACLE_E_NOMEM (-4)
#define ORACLE_E_ENERGY_DRIFT (-100)

/* ---- Philox4x32-10, written from the SC'11 description ------------------ */

void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u; /* round multipliers */
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u; /* Weyl key increments */
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)M0 * (uint64_t)x0;
        uint64_t p1 = (uint64_t)M1 * (uint64_t)x2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y1 = lo1;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        uint32_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
        k0 += W0; k1 += W1;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* One uniform word for (spin, sweep, replica, domain). */
static uint32_t draw(uint64_t seed, uint32_t spin, uint32_t sweep, uint32_t replica, uint32_t domain)
{
    uint32_t ctr[4] = {spin, sweep, replica >> 2, domain};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t out[4];
    oracle_philox4x32_10(ctr, key, out);
    return out[replica & 3u];
}

/* ---- threshold of the heat-bath decision -------------------------------- */

uint32_t oracle_minority_threshold(double beta, int32_t a)
{
    double q = 1.0 / (1.0 + exp((2.0 * beta) * (double)a));
    return (uint32_t)ceil(ldexp(q, 32) - 0.5);
}

/* new spin from field I, threshold table row, and the uniform word w */
static int8_t decide(int32_t I, const uint32_t *row, uint32_t w)
{
    int32_t a = I >= 0 ? I : -I;
    int8_t s = I >= 0 ? 1 : -1;
    uint32_t x = I >= 0 ? ~w : w;
    return (x < row[a]) ? (int8_t)-s : s;
}

/* ---- energy -------------------------------------------------------------- */

static int64_t energy_one(int32_t n, int32_t n_bonds, const int32_t *bi, const int32_t *bj,
                          const int8_t *bJ, const int8_t *h, const int8_t *m)
{
    int64_t e = 0;
    for (int32_t b = 0; b < n_bonds; ++b)
        e -= (int64_t)bJ[b] * m[bi[b]] * m[bj[b]];
    if (h)
        for (int32_t i = 0; i < n; ++i)
            e -= (int64_t)h[i] * m[i];
    return e;
}

int oracle_energy(int32_t n, int32_t n_bonds, const int32_t *bi, const int32_t *bj, const int8_t *bJ,
                  const int8_t *h, const int8_t *spins, int32_t R, int64_t *energy_out)
{
    if (n <= 0 || n_bonds < 0 || R < 0 || !spins || !energy_out) return ORACLE_E_ARG;
    for (int32_t r = 0; r < R; ++r)
        energy_out[r] = energy_one(n, n_bonds, bi, bj, bJ, h, spins + (size_t)r * n);
    return ORACLE_OK;
}

/* ---- anneal -------------------------------------------------------------- */

int oracle_anneal(int32_t n, int32_t n_bonds, const int32_t *bi, const int32_t *bj, const int8_t *bJ,
                  const int8_t *h, const uint8_t *colour, int32_t n_colours,
                  const double *beta, int32_t n_sweeps, int32_t sweep_offset,
                  int32_t R, int32_t replica_offset, uint64_t seed,
                  const int8_t *init_spins, const int32_t *order,
                  int8_t *spins_out, int64_t *energy_out,
                  int32_t trace_every, int64_t *energy_trace, int8_t *spin_trace)
{
    if (n <= 0 || n_bonds < 0 || n_colours < 1 || n_sweeps < 0 || sweep_offset < 0 || R < 0 ||
        replica_offset < 0 || trace_every < 0 || !colour || !spins_out || !energy_out)
        return ORACLE_E_ARG;
    if (n_sweeps > 0 && !beta) return ORACLE_E_ARG;
    for (int32_t s = 0; s < n_sweeps; ++s)
        if (!(beta[s] >= 0.0) || isinf(beta[s])) return ORACLE_E_ARG;
    for (int32_t i = 0; i < n; ++i)
        if (colour[i] >= n_colours) return ORACLE_E_COLOURING;

    /* adjacency lists from the bond list; every bond joins two colour classes */
    int32_t *deg = calloc((size_t)n + 1, sizeof *deg);
    if (!deg) return ORACLE_E_NOMEM;
    for (int32_t b = 0; b < n_bonds; ++b) {
        if (bi[b] < 0 || bi[b] >= n || bj[b] < 0 || bj[b] >= n) { free(deg); return ORACLE_E_ARG; }
        if (colour[bi[b]] == colour[bj[b]]) { free(deg); return ORACLE_E_COLOURING; }
        deg[bi[b] + 1]++;
        deg[bj[b] + 1]++;
    }
    for (int32_t i = 0; i < n; ++i) deg[i + 1] += deg[i];
    int32_t *nb = malloc(sizeof(int32_t) * (size_t)(2 * (size_t)n_bonds + 1));
    int8_t *nJ = malloc((size_t)2 * n_bonds + 1);
    int32_t *fill = malloc(sizeof(int32_t) * (size_t)n);
    if (!nb || !nJ || !fill) { free(deg); free(nb); free(nJ); free(fill); return ORACLE_E_NOMEM; }
    memcpy(fill, deg, sizeof(int32_t) * (size_t)n);
    for (int32_t b = 0; b < n_bonds; ++b) {
        nb[fill[bi[b]]] = bj[b]; nJ[fill[bi[b]]++] = bJ[b];
        nb[fill[bj[b]]] = bi[b]; nJ[fill[bj[b]]++] = bJ[b];
    }
    free(fill);

    /* largest possible |I|: sum of |J| over neighbours plus |h| */
    int32_t amax = 0;
    for (int32_t i = 0; i < n; ++i) {
        int32_t a = h ? abs(h[i]) : 0;
        for (int32_t k = deg[i]; k < deg[i + 1]; ++k) a += abs(nJ[k]);
        if (a > amax) amax = a;
    }

    /* threshold table, one row per sweep of this call */
    size_t width = (size_t)amax + 1;
    uint32_t *table = malloc(sizeof(uint32_t) * width * (size_t)(n_sweeps > 0 ? n_sweeps : 1));
    int8_t *m = malloc((size_t)n);
    if (!table || !m) { free(deg); free(nb); free(nJ); free(table); free(m); return ORACLE_E_NOMEM; }
    for (int32_t s = 0; s < n_sweeps; ++s)
        for (int32_t a = 0; a <= amax; ++a)
            table[(size_t)s * width + a] = oracle_minority_threshold(beta[s], a);

    int rc = ORACLE_OK;
    int32_t n_snap = trace_every > 0 ? n_sweeps / trace_every : 0;
    for (int32_t r = 0; r < R && rc == ORACLE_OK; ++r) {
        uint32_t rg = (uint32_t)replica_offset + (uint32_t)r;  /* global replica index, 32 bits */
        if (init_spins) {
            memcpy(m, init_spins + (size_t)r * n, (size_t)n);
        } else {
            for (int32_t i = 0; i < n; ++i)
                m[i] = draw(seed, (uint32_t)i, 0u, rg, 1u) < 0x80000000u ? 1 : -1;
        }
        int64_t e = energy_one(n, n_bonds, bi, bj, bJ, h, m);
        for (int32_t s = 0; s < n_sweeps; ++s) {
            uint32_t t = (uint32_t)sweep_offset + (uint32_t)s;  /* absolute sweep, 32 bits */
            const uint32_t *row = table + (size_t)s * width;
            for (int32_t c = 0; c < n_colours; ++c) {
                for (int32_t k = 0; k < n; ++k) {
                    int32_t i = order ? order[k] : k;
                    if (colour[i] != c) continue;
                    int32_t I = h ? h[i] : 0;
                    for (int32_t q = deg[i]; q < deg[i + 1]; ++q) I += nJ[q] * m[nb[q]];
                    int8_t mn = decide(I, row, draw(seed, (uint32_t)i, t, rg, 0u));
                    e -= (int64_t)(mn - m[i]) * I;
                    m[i] = mn;
                }
            }
            if (trace_every > 0 && (s + 1) % trace_every == 0) {
                int32_t k = (s + 1) / trace_every - 1;
                if (k < n_snap) {
                    if (e != energy_one(n, n_bonds, bi, bj, bJ, h, m)) { rc = ORACLE_E_ENERGY_DRIFT; break; }
                    if (energy_trace) energy_trace[(size_t)k * R + r] = e;
                    if (spin_trace) memcpy(spin_trace + ((size_t)k * R + r) * n, m, (size_t)n);
                }
            }
        }
        if (rc == ORACLE_OK && e != energy_one(n, n_bonds, bi, bj, bJ, h, m)) rc = ORACLE_E_ENERGY_DRIFT;
        memcpy(spins_out + (size_t)r * n, m, (size_t)n);
        energy_out[r] = e;
    }
    free(deg); free(nb); free(nJ); free(table); free(m);
    return rc;
}
