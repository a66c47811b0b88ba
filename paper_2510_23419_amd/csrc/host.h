// host.h — host-only helpers of libpbit (no HIP types): error reporting, the
// FP64 minority-threshold table and the greedy colouring.
#pragma once

#include <stdint.h>

namespace pbit {

int fail(int code, const char *fmt, ...);
uint32_t minority_threshold(double beta, int a);
int table_width(const double *beta, int S, int amax);
void build_table(const double *beta, int S, int width, uint32_t *out, int max_threads = 16);
int greedy_colouring(int n, int n_bonds, const int32_t *bi, const int32_t *bj, uint8_t *colour, int *n_colours);

}  // namespace pbit
