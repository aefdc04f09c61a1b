// Device primitives shared by the HIP sources (scan, radix sort, fills).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace tdp {
// Exclusive prefix sum of in[0..n) into out (may alias in); n = min(cap, *d_n)
// when d_n is given.  *d_total (optional) receives the sum.  tmp needs
// scan_tmp_size(cap) ints.
void scan_exclusive(const int32_t *in, int32_t *out, int cap, const int32_t *d_n, int32_t *d_total,
                    int32_t *tmp, hipStream_t s);
int scan_tmp_size(int cap);
// Stable sort of 64-bit keys (low `bits` bits, a multiple of 8) carrying
// 32-bit values; the result is left in k0/v0.  hist needs sort_hist_size(cap)
// ints; scan_tmp needs scan_tmp_size(sort_hist_size(cap)).
void radix_sort(uint64_t *k0, uint32_t *v0, uint64_t *k1, uint32_t *v1, int cap, const int32_t *d_n, int bits,
                int32_t *hist, int32_t *scan_tmp, hipStream_t s);
int sort_hist_size(int cap);
void fill_i32(int32_t *p, int n, int32_t v, hipStream_t s);
// xy[i] = (x[i], y[i]): one 8-byte gather per random position lookup; where
// a coordinate is NaN or infinite, *bad = gen (if bad is given)
void pack_xy(const float *x, const float *y, float2 *xy, int n, hipStream_t s, int32_t *bad = nullptr,
             int32_t gen = 0);

// order-preserving maps from floating point to unsigned integers
__host__ __device__ __forceinline__ uint64_t order_key(float f) {
  uint32_t u = __builtin_bit_cast(uint32_t, f);
  return (uint64_t)((u & 0x80000000u) ? ~u : (u | 0x80000000u));
}
__host__ __device__ __forceinline__ uint64_t order_key(double f) {
  uint64_t u = __builtin_bit_cast(uint64_t, f);
  return (u & 0x8000000000000000ull) ? ~u : (u | 0x8000000000000000ull);
}
}  // namespace tdp
