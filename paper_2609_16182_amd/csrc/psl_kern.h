// psl_kern.h -- host-side launchers of libpsl's kernels.
#pragma once
#include <hip/hip_runtime.h>

#include "psl_dev.h"

namespace psl {

// ----- primitives.hip ------------------------------------------------------
// Exclusive prefix sum of in[0..n) into out (in == out allowed); the total
// is written to *total (device pointer) when total != nullptr. ws must hold
// scan_ws_ints(n) ints.
size_t scan_ws_ints(int64_t n);
void scan_excl(const int32_t* in, int32_t* out, int64_t n, int32_t* total, int32_t* ws, hipStream_t s);

// One stable counting-sort pass by the digit (key >> shift) & (2^bits - 1),
// bits <= 8. vals_in == nullptr means value = index. ws: radix_ws_ints(n).
size_t radix_ws_ints(int64_t n);
void radix_pass(const uint32_t* keys_in, const int32_t* vals_in, uint32_t* keys_out, int32_t* vals_out,
                int64_t n, int shift, int bits, int32_t* ws, hipStream_t s);

// The same pass moving a payload of a row index and a value with each key;
// rows_in == nullptr takes row rowid1[p + 1] for item p. Buffers must not
// alias. ws: radix_ws_ints(n).
void radix_pass_payload(const uint32_t* keys_in, const int32_t* rows_in, const int32_t* rowid1,
                        const double* vals_in, uint32_t* keys_out, int32_t* rows_out, double* vals_out, int64_t n,
                        int shift, int bits, int32_t* ws, hipStream_t s);

// out[i] = v (32-bit words)
void fill_i32(int32_t* out, int32_t v, int64_t n, hipStream_t s);

// Canonical pairwise tree sum of x[0..n) into *out (device), ws: pairwise_ws_doubles(n).
size_t pairwise_ws_doubles(int64_t n);
void pairwise_sum(const double* x, int64_t n, double* out, double* ws, hipStream_t s);

// out[k] = +0-canonical (off[k] + canonical pairwise sum of x[seg[k]..seg[k+1]))
// for k < K; the tree of every segment starts at the segment's first element.
// seg is given on the device and on the host; segments of more than
// 2048 * 2048 elements are summed by pairwise_sum (ws: pairwise_ws_doubles + 1).
void segmented_pairwise_sum(const double* x, const int32_t* seg_dev, const int32_t* seg_host, int K,
                            const double* off, double* out, double* ws, hipStream_t s);

}  // namespace psl
