// Host-side code under AddressSanitizer and UndefinedBehaviorSanitizer: the
// library's host-only entry points (threshold table, greedy colouring, error
// strings) and the C oracle, on ordinary, edge and invalid inputs.  Built with
// g++/gcc -fsanitize=address,undefined by the test that runs it; any sanitizer
// report aborts with a nonzero status.  Prints "sanitize ok" on success.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <vector>

#include "../../include/pbit.h"

extern "C" {
void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
uint32_t oracle_minority_threshold(double beta, int32_t a);
int oracle_energy(int32_t n, int32_t n_bonds, const int32_t *bi, const int32_t *bj, const int8_t *bJ,
                  const int8_t *h, const int8_t *spins, int32_t R, int64_t *energy_out);
int oracle_anneal(int32_t n, int32_t n_bonds, const int32_t *bi, const int32_t *bj, const int8_t *bJ,
                  const int8_t *h, const uint8_t *colour, int32_t n_colours, const double *beta, int32_t n_sweeps,
                  int32_t sweep_offset, int32_t R, int32_t replica_offset, uint64_t seed, const int8_t *init_spins,
                  const int32_t *order, int8_t *spins_out, int64_t *energy_out, int32_t trace_every,
                  int64_t *energy_trace, int8_t *spin_trace);
}

#define CHECK(c)                                                              \
    do {                                                                      \
        if (!(c)) {                                                           \
            std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
            std::exit(2);                                                     \
        }                                                                     \
    } while (0)

int main()
{
    std::mt19937_64 rng(2510);
    // threshold tables: every width up to the biclique limit, edge betas, threads
    for (int S : {0, 1, 7, 3000}) {
        for (int A : {0, 1, 6, 229, 4095}) {
            std::vector<double> beta((size_t)S);
            for (int s = 0; s < S; ++s) beta[(size_t)s] = (s % 5 == 0) ? 0.0 : 0.05 + 20.0 * (double)s / (S + 1);
            std::vector<uint32_t> out((size_t)S * (A + 1) + 1, 0xDEADBEEFu);
            CHECK(pbit_threshold_table(beta.data(), S, A, out.data()) == PBIT_OK);
            CHECK(out[(size_t)S * (A + 1)] == 0xDEADBEEFu);  // nothing written past the table
            for (int s = 0; s < S; ++s)
                for (int a = 0; a <= A; a += 17)
                    CHECK(out[(size_t)s * (A + 1) + a] == oracle_minority_threshold(beta[(size_t)s], a));
        }
    }
    const double bad[3] = {0.5, NAN, -1.0};
    uint32_t tab[8];
    CHECK(pbit_threshold_table(bad, 2, 3, tab) == PBIT_E_RANGE);
    CHECK(std::strlen(pbit_last_error()) > 0);
    CHECK(pbit_threshold_table(bad + 2, 1, 3, tab) == PBIT_E_RANGE);
    CHECK(pbit_threshold_table(nullptr, 2, 3, tab) == PBIT_E_ARG);
    CHECK(pbit_threshold_table(bad, -1, 3, tab) == PBIT_E_ARG);
    CHECK(std::strstr(pbit_version(), "gfx950") != nullptr);

    // greedy colouring: random graphs (degrees up to the 256-colour limit), empty, invalid
    for (int trial = 0; trial < 40; ++trial) {
        const int n = 1 + (int)(rng() % 300), m = (int)(rng() % (4 * n + 1));
        std::vector<int32_t> bi, bj;
        for (int b = 0; b < m; ++b) {
            const int32_t i = (int32_t)(rng() % n), j = (int32_t)(rng() % n);
            if (i != j) {
                bi.push_back(i);
                bj.push_back(j);
            }
        }
        std::vector<uint8_t> colour((size_t)n, 0xFF);
        int32_t nc = -1;
        CHECK(pbit_greedy_colouring(n, (int32_t)bi.size(), bi.data(), bj.data(), colour.data(), &nc) == PBIT_OK);
        for (size_t b = 0; b < bi.size(); ++b) CHECK(colour[(size_t)bi[b]] != colour[(size_t)bj[b]]);
        for (int i = 0; i < n; ++i) CHECK(colour[(size_t)i] < nc);
    }
    {
        const int n = 300;  // K_300 needs 300 colours: refused
        std::vector<int32_t> bi, bj;
        for (int i = 0; i < n; ++i)
            for (int j = i + 1; j < n; ++j) {
                bi.push_back(i);
                bj.push_back(j);
            }
        std::vector<uint8_t> colour((size_t)n);
        int32_t nc = 0;
        CHECK(pbit_greedy_colouring(n, (int32_t)bi.size(), bi.data(), bj.data(), colour.data(), &nc) ==
              PBIT_E_UNSUPPORTED);
        const int32_t si[1] = {0}, sj[1] = {0}, oi[1] = {0}, oj[1] = {5};
        CHECK(pbit_greedy_colouring(3, 1, si, sj, colour.data(), &nc) == PBIT_E_ARG);  // self-loop
        CHECK(pbit_greedy_colouring(3, 1, oi, oj, colour.data(), &nc) == PBIT_E_ARG);  // out of range
        CHECK(pbit_greedy_colouring(0, 0, nullptr, nullptr, colour.data(), &nc) == PBIT_OK && nc == 0);
    }

    // the oracle: Philox, energies and anneals on random coloured graphs, with traces,
    // offsets, given spins and invalid arguments
    uint32_t ctr[4] = {1, 2, 3, 4}, key[2] = {5, 6}, out4[4];
    oracle_philox4x32_10(ctr, key, out4);
    for (int trial = 0; trial < 12; ++trial) {
        const int n = 2 + (int)(rng() % 40), R = 1 + (int)(rng() % 9), S = (int)(rng() % 30);
        std::vector<int32_t> bi, bj;
        std::vector<int8_t> bJ, h((size_t)n);
        std::vector<uint8_t> colour((size_t)n);
        for (int i = 0; i < n; ++i) {
            colour[(size_t)i] = (uint8_t)(i % 3);
            h[(size_t)i] = (int8_t)((int)(rng() % 3) - 1);
        }
        for (int b = 0; b < 3 * n; ++b) {
            const int32_t i = (int32_t)(rng() % n), j = (int32_t)(rng() % n);
            if (colour[(size_t)i] == colour[(size_t)j]) continue;
            bi.push_back(i);
            bj.push_back(j);
            bJ.push_back((int8_t)((int)(rng() % 3) - 1));
        }
        std::vector<double> beta((size_t)S);
        for (int s = 0; s < S; ++s) beta[(size_t)s] = 0.1 * s;
        std::vector<int8_t> spins((size_t)R * n), strace((size_t)R * n * (S + 1));
        std::vector<int64_t> en((size_t)R), etrace((size_t)R * (S + 1));
        const int every = S > 0 ? 1 + (int)(rng() % 3) : 0;
        CHECK(oracle_anneal(n, (int32_t)bi.size(), bi.data(), bj.data(), bJ.data(), h.data(), colour.data(), 3,
                            beta.data(), S, 4, R, 8, rng(), nullptr, nullptr, spins.data(), en.data(), every,
                            etrace.data(), strace.data()) == 0);
        // counters past 31 bits: absolute sweeps from 2^31 - 3, replicas from 2^31 - 64
        std::vector<int8_t> spins_hi((size_t)R * n);
        std::vector<int64_t> en_hi((size_t)R);
        CHECK(oracle_anneal(n, (int32_t)bi.size(), bi.data(), bj.data(), bJ.data(), h.data(), colour.data(), 3,
                            beta.data(), S, 2147483645, R, 2147483584, rng(), nullptr, nullptr, spins_hi.data(),
                            en_hi.data(), 0, nullptr, nullptr) == 0);
        std::vector<int64_t> en2((size_t)R);
        CHECK(oracle_energy(n, (int32_t)bi.size(), bi.data(), bj.data(), bJ.data(), h.data(), spins.data(), R,
                            en2.data()) == 0);
        CHECK(en == en2);
        CHECK(oracle_anneal(n, (int32_t)bi.size(), bi.data(), bj.data(), bJ.data(), h.data(), colour.data(), 3,
                            beta.data(), S, 0, R, 0, 1, spins.data(), nullptr, spins.data(), en.data(), 0, nullptr,
                            nullptr) == 0);
        colour[0] = 7;  // out of range colour: refused
        CHECK(oracle_anneal(n, (int32_t)bi.size(), bi.data(), bj.data(), bJ.data(), h.data(), colour.data(), 3,
                            beta.data(), S, 0, R, 0, 1, nullptr, nullptr, spins.data(), en.data(), 0, nullptr,
                            nullptr) != 0);
    }
    std::printf("sanitize ok\n");
    return 0;
}
