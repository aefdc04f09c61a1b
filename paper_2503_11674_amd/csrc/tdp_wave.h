// Wavefront (64-lane) helpers: segmented reductions over contiguous lane
// ranges [head, tail].  Every lane of the wave must call them (they shuffle);
// the result is the same for every lane of a segment and is computed in a
// fixed order, so it does not depend on timing.
#pragma once

#include <hip/hip_runtime.h>

#include "tdp_internal.h"

namespace tdp {

// {arrival, transition} of a driver, one load in the forward gathers
template <typename T> struct vec2_of;
template <> struct vec2_of<float> { using type = float2; };
template <> struct vec2_of<double> { using type = double2; };
template <typename T> using V2 = typename vec2_of<T>::type;
template <typename T>
__device__ __forceinline__ V2<T> v2(T a, T b) {
  V2<T> w;
  w.x = a;
  w.y = b;
  return w;
}

template <typename T> __device__ __forceinline__ T pos_inf();
template <> __device__ __forceinline__ float pos_inf<float>() { return __builtin_huge_valf(); }
template <> __device__ __forceinline__ double pos_inf<double>() { return __builtin_huge_val(); }

__device__ __forceinline__ int wave_lane() { return threadIdx.x & 63; }

// Segmented reductions over the 64 lanes of a wave (segment [head, tail],
// the result broadcast to every lane).  These shuffle forms combine lane L
// with lane L - d for d = 1, 2, 4, ..., so the order of the operations
// depends only on the offsets within the segment: the same segment gives the
// same bits wherever it sits in a wave (a batched graph's chunks equal its
// instances' bitwise).  Every lane of the wave must call them.
template <typename T>
__device__ __forceinline__ T seg_sum(T v, int lane, int head, int tail) {
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    T u = __shfl_up(v, d, 64);
    if (lane - d >= head) v += u;
  }
  return __shfl(v, tail, 64);
}

template <typename T>
__device__ __forceinline__ T seg_max(T v, int lane, int head, int tail) {
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    T u = __shfl_up(v, d, 64);
    if (lane - d >= head) v = u > v ? u : v;
  }
  return __shfl(v, tail, 64);
}

template <typename T>
__device__ __forceinline__ T seg_min(T v, int lane, int head, int tail) {
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    T u = __shfl_up(v, d, 64);
    if (lane - d >= head) v = u < v ? u : v;
  }
  return __shfl(v, tail, 64);
}

// The same reductions with DPP lane moves (no LDS traffic, a fraction of the
// shuffles' cost): shifts by 1, 2, 4 and 8 within rows of 16 lanes, then
// the last lane of rows 0 / 2 into rows 1 / 3, then lane 31 into rows 2 and
// 3.  A lane takes a value only from lanes of its own segment, so after the
// six steps lane L holds op over [head, L]; one shuffle broadcasts the tail
// lane's.  The association follows the row boundaries, so a sum's rounding
// depends on where the segment sits: for values that are not compared
// across layouts.  Every lane of the wave must call them.
template <int CTRL>
__device__ __forceinline__ int dpp_move(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}

template <int CTRL, typename T>
__device__ __forceinline__ T dpp_move_t(T v) {
  static_assert(sizeof(T) == 4, "32-bit lanes");
  return __builtin_bit_cast(T, dpp_move<CTRL>(__builtin_bit_cast(int, v)));
}

template <typename T, typename Op>
__device__ __forceinline__ T seg_scan_dpp(T v, int lane, int head, Op op) {
  const int r = lane & 15, row = lane >> 4;
  T u;
  u = dpp_move_t<0x111>(v);  // row_shr:1
  if (r >= 1 && lane - 1 >= head) v = op(v, u);
  u = dpp_move_t<0x112>(v);  // row_shr:2
  if (r >= 2 && lane - 2 >= head) v = op(v, u);
  u = dpp_move_t<0x114>(v);  // row_shr:4
  if (r >= 4 && lane - 4 >= head) v = op(v, u);
  u = dpp_move_t<0x118>(v);  // row_shr:8
  if (r >= 8 && lane - 8 >= head) v = op(v, u);
  u = dpp_move_t<0x142>(v);  // row_bcast:15, taken by rows 1 and 3
  if ((row & 1) && (lane & ~15) - 1 >= head) v = op(v, u);
  u = dpp_move_t<0x143>(v);  // row_bcast:31, taken by rows 2 and 3
  if (row >= 2 && 31 >= head) v = op(v, u);
  return v;
}

template <typename T>
__device__ __forceinline__ T seg_sum_dpp(T v, int lane, int head, int tail) {
  return __shfl(seg_scan_dpp(v, lane, head, [](T a, T b) { return a + b; }), tail, 64);
}

template <typename T>
__device__ __forceinline__ T seg_max_dpp(T v, int lane, int head, int tail) {
  return __shfl(seg_scan_dpp(v, lane, head, [](T a, T b) { return b > a ? b : a; }), tail, 64);
}

template <typename T>
__device__ __forceinline__ T seg_min_dpp(T v, int lane, int head, int tail) {
  return __shfl(seg_scan_dpp(v, lane, head, [](T a, T b) { return b < a ? b : a; }), tail, 64);
}

// For segments of at most WM lanes: every lane fetches the values of lanes
// head .. head + WM - 1 of its own segment (clamped to the tail, so a short
// segment repeats its last value) with independent shuffles, which the
// hardware overlaps: one cross-lane latency instead of a dependent chain of
// log2(64) steps.  Every lane of the wave must call it.
template <int WM, typename T>
__device__ __forceinline__ void seg_fetch(T v, int head, int tail, T (&u)[WM]) {
#pragma unroll
  for (int j = 0; j < WM; ++j) u[j] = __shfl(v, min(head + j, tail), 64);
}

// maximum of u[] and the first index that attains it (0 when none does)
template <int WM, typename T>
__device__ __forceinline__ T max_first(const T (&u)[WM], int &arg) {
  T m = u[0];
#pragma unroll
  for (int j = 1; j < WM; ++j) m = u[j] > m ? u[j] : m;
  arg = 0;
#pragma unroll
  for (int j = WM - 1; j >= 0; --j) arg = u[j] == m ? j : arg;
  return m;
}

__device__ __forceinline__ int wave_max_int(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    int u = __shfl_xor(v, o, 64);
    v = u > v ? u : v;
  }
  return v;
}

// KM consecutive list entries at a KM-aligned index, moved 16 bytes at a
// time where the list's size allows (the arrays come 256-byte aligned)
template <int KM, typename V>
__device__ __forceinline__ void load_list(const V *__restrict__ p, V (&out)[KM]) {
  if constexpr ((KM * sizeof(V)) % 16 == 0) {
    const int4 *q = reinterpret_cast<const int4 *>(p);
#pragma unroll
    for (int i = 0; i < (int)(KM * sizeof(V) / 16); ++i) {
      const int4 w = q[i];
      __builtin_memcpy(&out[i * (16 / sizeof(V))], &w, 16);
    }
  } else {
#pragma unroll
    for (int j = 0; j < KM; ++j) out[j] = p[j];
  }
}

template <int KM, typename V>
__device__ __forceinline__ void store_list(V *__restrict__ p, const V (&in)[KM]) {
  if constexpr ((KM * sizeof(V)) % 16 == 0) {
    int4 *q = reinterpret_cast<int4 *>(p);
#pragma unroll
    for (int i = 0; i < (int)(KM * sizeof(V) / 16); ++i) {
      int4 w;
      __builtin_memcpy(&w, &in[i * (16 / sizeof(V))], 16);
      q[i] = w;
    }
  } else {
#pragma unroll
    for (int j = 0; j < KM; ++j) p[j] = in[j];
  }
}

// the library's table image (LutView::flat4) copied into LDS by the whole
// workgroup; every thread of the workgroup must call it
__device__ __forceinline__ void stage_lut(const LutView &L, float *s_lut) {
  // two float4 loads in flight per thread before their LDS writes (one
  // memory latency for the usual table sizes)
  float4 *dst = (float4 *)s_lut;
  const int n4 = L.n4, bd = blockDim.x;
  for (int i = threadIdx.x; i < n4; i += 2 * bd) {
    const int i1 = i + bd;
    const float4 v0 = L.flat4[i];
    const float4 v1 = i1 < n4 ? L.flat4[i1] : make_float4(0.f, 0.f, 0.f, 0.f);
    dst[i] = v0;
    if (i1 < n4) dst[i1] = v1;
  }
  __syncthreads();
}

// the library's tables staged in LDS: [slew axes][load axes][delay][slew]
template <typename T>
__device__ __forceinline__ void lut_lds(const float *__restrict__ s_lut, int nt, int ns, int nl, int type, T s,
                                        T l, T &d_out, T &s_out) {
  const float *sa = s_lut + type * ns;
  const float *la = s_lut + nt * ns + type * nl;
  const T s0 = (T)sa[0], s1 = (T)sa[ns - 1], l0 = (T)la[0], l1 = (T)la[nl - 1];
  s = s < s0 ? s0 : (s > s1 ? s1 : s);
  l = l < l0 ? l0 : (l > l1 ? l1 : l);
  // the interval is the last one whose left end is <= the value
  int i = 0, j = 0;
  for (int q = 1; q <= ns - 2; ++q) i += ((T)sa[q] <= s);
  for (int q = 1; q <= nl - 2; ++q) j += ((T)la[q] <= l);
  const T tau = (s - (T)sa[i]) / ((T)sa[i + 1] - (T)sa[i]);
  const T ups = (l - (T)la[j]) / ((T)la[j + 1] - (T)la[j]);
  const float *D = s_lut + nt * (ns + nl);
  const float *S = D + nt * ns * nl;
  const int base = (type * ns + i) * nl + j;
  const T w00 = (1 - tau) * (1 - ups), w10 = tau * (1 - ups), w01 = (1 - tau) * ups, w11 = tau * ups;
  d_out = w00 * (T)D[base] + w10 * (T)D[base + nl] + w01 * (T)D[base + 1] + w11 * (T)D[base + nl + 1];
  s_out = w00 * (T)S[base] + w10 * (T)S[base + nl] + w01 * (T)S[base + 1] + w11 * (T)S[base + nl + 1];
}

}  // namespace tdp
