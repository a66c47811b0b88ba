// host.cpp — the host-only part of libpbit: error messages, the FP64
// threshold table and the greedy colouring.  It includes no HIP header, so it
// also builds with a plain C++ compiler (the sanitizer checks build it that way).
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <string>
#include <thread>
#include <vector>

#include "../../include/pbit.h"
#include "host.h"

using namespace pbit;

// ---------------------------------------------------------------- errors

static thread_local std::string g_last_error;

namespace pbit {

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

}  // namespace pbit

extern "C" const char *pbit_last_error(void) { return g_last_error.c_str(); }

extern "C" const char *pbit_version(void) { return "pbit-mi355x 0.1 (gfx950)"; }

// ---------------------------------------------------------------- threshold table

namespace pbit {

// Tm(beta, a): the minority probability 1 / (1 + exp(2 beta a)) of the p-bit
// law (Sec. 1.2.1, Eq. 2 read with tanh and beta), scaled to 2^32 and rounded
// half-down, in IEEE binary64.
uint32_t minority_threshold(double beta, int a)
{
    const double q = 1.0 / (1.0 + std::exp((2.0 * beta) * (double)a));
    return (uint32_t)std::ceil(std::ldexp(q, 32) - 0.5);
}

// Width of the per-sweep rows actually needed: |I| never exceeds amax, and
// beyond the first a at which every row is 0 all entries are 0 (Tm is
// non-increasing in a), so the kernel clamps |I| to width - 1.  Tm is also
// non-increasing in beta for a >= 1 (every step of its evaluation is monotone),
// so the row of the smallest beta is the last to reach 0.
int table_width(const double *beta, int S, int amax)
{
    if (S <= 0) return 1;
    double bmin = beta[0];
    for (int s = 1; s < S; ++s) bmin = std::min(bmin, beta[s]);
    int a = 0;
    while (a <= amax && minority_threshold(bmin, a) != 0u) ++a;
    return std::min(a, amax) + 1;
}

// Rows of the table; large tables (a biclique schedule: thousands of sweeps by
// hundreds of field values, one exp each) are split over up to 16 host threads.
void build_table(const double *beta, int S, int width, uint32_t *out, int max_threads)
{
    auto rows = [=](int s0, int s1) {
        for (int s = s0; s < s1; ++s)
            for (int a = 0; a < width; ++a) out[(size_t)s * width + a] = minority_threshold(beta[s], a);
    };
    const size_t cells = (size_t)S * width;
    const int nt = (int)std::min<size_t>({(size_t)std::max(max_threads, 1), (size_t)16,
                                          (size_t)std::max(1u, std::thread::hardware_concurrency()),
                                          cells >> 15, (size_t)std::max(S, 1)});
    if (nt < 2) {
        rows(0, S);
        return;
    }
    std::vector<std::thread> pool;
    pool.reserve((size_t)nt - 1);
    for (int t = 1; t < nt; ++t) {
        const int s0 = (int)((int64_t)S * t / nt), s1 = (int)((int64_t)S * (t + 1) / nt);
        try {
            pool.emplace_back(rows, s0, s1);
        } catch (...) {
            rows(s0, s1);  // no thread: this one does the rows
        }
    }
    rows(0, (int)((int64_t)S / nt));
    for (std::thread &th : pool) th.join();
}

}  // namespace pbit

extern "C" int pbit_threshold_table(const double *beta, int32_t S, int32_t A, uint32_t *out)
{
    if (S < 0 || A < 0 || (S > 0 && (!beta || !out))) return fail(PBIT_E_ARG, "pbit_threshold_table: bad arguments");
    for (int s = 0; s < S; ++s)
        if (!(beta[s] >= 0.0) || std::isinf(beta[s]))
            return fail(PBIT_E_RANGE, "pbit_threshold_table: beta[%d] must be finite and >= 0", s);
    build_table(beta, S, A + 1, out);
    return PBIT_OK;
}

namespace pbit {

// Greedy colouring (Sec. 1.2.2): vertices in ascending order take the
// smallest colour none of their already coloured neighbours has.
int greedy_colouring(int n, int n_bonds, const int32_t *bi, const int32_t *bj, uint8_t *colour, int *n_colours)
{
    std::vector<int32_t> start((size_t)n + 1, 0), nbr((size_t)2 * n_bonds);
    for (int b = 0; b < n_bonds; ++b) {
        ++start[(size_t)bi[b] + 1];
        ++start[(size_t)bj[b] + 1];
    }
    for (int i = 0; i < n; ++i) start[(size_t)i + 1] += start[i];
    std::vector<int32_t> fill(start.begin(), start.end() - 1);
    for (int b = 0; b < n_bonds; ++b) {
        nbr[(size_t)fill[bi[b]]++] = bj[b];
        nbr[(size_t)fill[bj[b]]++] = bi[b];
    }
    std::vector<int> seen(257, -1);
    int used = 0;
    for (int v = 0; v < n; ++v) {
        for (int e = start[v]; e < start[(size_t)v + 1]; ++e) {
            const int u = nbr[(size_t)e];
            if (u < v) seen[colour[u]] = v;
        }
        int c = 0;
        while (seen[c] == v) ++c;
        if (c > 255) return fail(PBIT_E_UNSUPPORTED, "greedy colouring needs more than 256 colours");
        colour[v] = (uint8_t)c;
        used = std::max(used, c + 1);
    }
    *n_colours = n > 0 ? used : 0;
    return PBIT_OK;
}

}  // namespace pbit

extern "C" int pbit_greedy_colouring(int32_t n, int32_t n_bonds, const int32_t *bond_i, const int32_t *bond_j,
                                     uint8_t *colour, int32_t *n_colours)
{
    try {
        if (n < 0 || n_bonds < 0 || !colour || !n_colours || (n_bonds > 0 && (!bond_i || !bond_j)))
            return fail(PBIT_E_ARG, "pbit_greedy_colouring: bad arguments");
        for (int b = 0; b < n_bonds; ++b)
            if (bond_i[b] < 0 || bond_i[b] >= n || bond_j[b] < 0 || bond_j[b] >= n || bond_i[b] == bond_j[b])
                return fail(PBIT_E_ARG, "pbit_greedy_colouring: bad bond %d", b);
        int nc = 0;
        int rc = greedy_colouring(n, n_bonds, bond_i, bond_j, colour, &nc);
        *n_colours = nc;
        return rc;
    } catch (...) {
        return fail(PBIT_E_NOMEM, "pbit_greedy_colouring: host allocation failed");
    }
}

