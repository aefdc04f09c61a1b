// Device primitives: exclusive scan and a stable LSD radix sort.
//
// Both take a host capacity `cap` (sizes the grid) and an optional device
// count `d_n` (the live length, read on the device) so that callers never
// have to read a count back to the host; this keeps every call capturable in
// a hipGraph.  Results are deterministic: no floating-point atomics, integer
// counts only.
#include "tdp_prims.h"

namespace tdp {

constexpr int SCAN_BLOCK = 256;
constexpr int SCAN_ITEMS = 16;  // four int4 per thread
constexpr int SCAN_TILE = SCAN_BLOCK * SCAN_ITEMS;

// a thread's SCAN_ITEMS consecutive values starting at base (16-byte
// aligned): vector loads for a full run, element loads in the ragged tail
__device__ __forceinline__ void load_items(const int32_t *in, int base, int n, int (&v)[SCAN_ITEMS]) {
  if (base + SCAN_ITEMS <= n) {
    const int4 *p = (const int4 *)(in + base);
#pragma unroll
    for (int q = 0; q < SCAN_ITEMS / 4; ++q) {
      const int4 x = p[q];
      v[4 * q] = x.x;
      v[4 * q + 1] = x.y;
      v[4 * q + 2] = x.z;
      v[4 * q + 3] = x.w;
    }
  } else {
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i) v[i] = base + i < n ? in[base + i] : 0;
  }
}

__device__ __forceinline__ void store_items(int32_t *out, int base, int n, const int (&v)[SCAN_ITEMS]) {
  if (base + SCAN_ITEMS <= n) {
    int4 *p = (int4 *)(out + base);
#pragma unroll
    for (int q = 0; q < SCAN_ITEMS / 4; ++q) p[q] = make_int4(v[4 * q], v[4 * q + 1], v[4 * q + 2], v[4 * q + 3]);
  } else {
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i)
      if (base + i < n) out[base + i] = v[i];
  }
}

__device__ __forceinline__ int live_count(int cap, const int32_t *d_n) {
  if (!d_n) return cap;
  int n = *d_n;
  return n < cap ? (n < 0 ? 0 : n) : cap;
}

// inclusive scan of one value per thread across a 256-thread block
__device__ __forceinline__ int block_inclusive_scan(int v, int *sh /*[4]*/) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    int u = __shfl_up(v, o, 64);
    if (lane >= o) v += u;
  }
  if (lane == 63) sh[wid] = v;
  __syncthreads();
  int add = 0;
  for (int w = 0; w < wid; ++w) add += sh[w];
  __syncthreads();
  return v + add;
}

__global__ void __launch_bounds__(SCAN_BLOCK) k_scan_reduce(const int32_t *__restrict__ in, int cap,
                                                             const int32_t *d_n, int32_t *__restrict__ part) {
  __shared__ int sh[4];
  const int n = live_count(cap, d_n);
  const int base = blockIdx.x * SCAN_TILE + threadIdx.x * SCAN_ITEMS;
  int v[SCAN_ITEMS];
  load_items(in, base, n, v);
  int s = 0;
#pragma unroll
  for (int i = 0; i < SCAN_ITEMS; ++i) s += v[i];
  int incl = block_inclusive_scan(s, sh);
  if (threadIdx.x == SCAN_BLOCK - 1) part[blockIdx.x] = incl;
}

// one block: exclusive scan of the per-tile sums in place, total to *d_total
__global__ void __launch_bounds__(SCAN_BLOCK) k_scan_partials(int32_t *__restrict__ part, int nparts,
                                                               int32_t *d_total) {
  __shared__ int sh[4];
  __shared__ int block_total;
  int carry = 0;
  for (int b0 = 0; b0 < nparts; b0 += SCAN_BLOCK) {
    int i = b0 + threadIdx.x;
    int v = i < nparts ? part[i] : 0;
    int incl = block_inclusive_scan(v, sh);
    if (i < nparts) part[i] = carry + incl - v;
    if (threadIdx.x == SCAN_BLOCK - 1) block_total = incl;
    __syncthreads();
    carry += block_total;
    __syncthreads();
  }
  if (threadIdx.x == 0 && d_total) *d_total = carry;
}

// (in and out may be the same array: a thread reads its items before it
// writes them and no other thread touches them)
__global__ void __launch_bounds__(SCAN_BLOCK) k_scan_down(const int32_t *in, int cap, const int32_t *d_n,
                                                           const int32_t *__restrict__ part, int32_t *out) {
  __shared__ int sh[4];
  const int n = live_count(cap, d_n);
  const int base = blockIdx.x * SCAN_TILE + threadIdx.x * SCAN_ITEMS;
  int v[SCAN_ITEMS];
  load_items(in, base, n, v);
  int s = 0;
#pragma unroll
  for (int i = 0; i < SCAN_ITEMS; ++i) s += v[i];
  int incl = block_inclusive_scan(s, sh);
  int run = part[blockIdx.x] + incl - s;
#pragma unroll
  for (int i = 0; i < SCAN_ITEMS; ++i) {
    const int x = v[i];
    v[i] = run;
    run += x;
  }
  store_items(out, base, n, v);
}

// Second pass without a separate scan of the tile sums: every tile adds up
// the sums of the tiles before it itself (a few thousand integers from L2),
// which saves a launch; the last live tile writes the total.
__global__ void __launch_bounds__(SCAN_BLOCK) k_scan_down_sum(const int32_t *in, int cap, const int32_t *d_n,
                                                               const int32_t *__restrict__ part, int32_t *out,
                                                               int32_t *d_total) {
  __shared__ int sh[4];
  __shared__ int offset;
  const int n = live_count(cap, d_n);
  const int tiles = n > 0 ? (n + SCAN_TILE - 1) / SCAN_TILE : 1;
  if ((int)blockIdx.x >= tiles) return;
  int acc = 0;
  for (int i = threadIdx.x; i < (int)blockIdx.x; i += SCAN_BLOCK) acc += part[i];
  acc = block_inclusive_scan(acc, sh);
  if (threadIdx.x == SCAN_BLOCK - 1) offset = acc;
  __syncthreads();
  const int base = blockIdx.x * SCAN_TILE + threadIdx.x * SCAN_ITEMS;
  int v[SCAN_ITEMS];
  load_items(in, base, n, v);
  int s = 0;
#pragma unroll
  for (int i = 0; i < SCAN_ITEMS; ++i) s += v[i];
  const int incl = block_inclusive_scan(s, sh);
  int run = offset + incl - s;
#pragma unroll
  for (int i = 0; i < SCAN_ITEMS; ++i) {
    const int x = v[i];
    v[i] = run;
    run += x;
  }
  store_items(out, base, n, v);
  if (d_total && (int)blockIdx.x == tiles - 1 && threadIdx.x == SCAN_BLOCK - 1) *d_total = offset + incl;
}

int scan_tmp_size(int cap) { return (cap + SCAN_TILE - 1) / SCAN_TILE + 1; }

void scan_exclusive(const int32_t *in, int32_t *out, int cap, const int32_t *d_n, int32_t *d_total,
                    int32_t *tmp, hipStream_t s) {
  if (cap <= 0) {
    hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(SCAN_BLOCK), 0, s, tmp, 0, d_total);
    return;
  }
  int nb = (cap + SCAN_TILE - 1) / SCAN_TILE;
  hipLaunchKernelGGL(k_scan_reduce, dim3(nb), dim3(SCAN_BLOCK), 0, s, in, cap, d_n, tmp);
  if (nb <= 8192) {
    hipLaunchKernelGGL(k_scan_down_sum, dim3(nb), dim3(SCAN_BLOCK), 0, s, in, cap, d_n, tmp, out, d_total);
    return;
  }
  hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(SCAN_BLOCK), 0, s, tmp, nb, d_total);
  hipLaunchKernelGGL(k_scan_down, dim3(nb), dim3(SCAN_BLOCK), 0, s, in, cap, d_n, tmp, out);
}

// ------------------------------------------------------------------ sort
constexpr int RS_BLOCK = 256;
constexpr int RS_ITEMS = 8;
constexpr int RS_TILE = RS_BLOCK * RS_ITEMS;

__device__ __forceinline__ uint32_t digit_of(uint64_t k, int shift) { return (uint32_t)(k >> shift) & 0xFFu; }

// tiles are counted from the live length, so the histogram and its scan cover
// only live tiles; the count of histogram entries goes to *hist_n
__global__ void k_rs_size(int cap, const int32_t *d_n, int32_t *__restrict__ hist_n) {
  const int n = live_count(cap, d_n);
  *hist_n = 256 * ((n + RS_TILE - 1) / RS_TILE);
}

__global__ void __launch_bounds__(RS_BLOCK) k_rs_hist(const uint64_t *__restrict__ keys, int cap,
                                                       const int32_t *d_n, int shift, int32_t *__restrict__ hist) {
  __shared__ int cnt[256];
  const int n = live_count(cap, d_n);
  const int ntiles = (n + RS_TILE - 1) / RS_TILE;
  if ((int)blockIdx.x >= ntiles) return;
  cnt[threadIdx.x] = 0;
  __syncthreads();
  const int base = blockIdx.x * RS_TILE;
  // every key of the thread is requested before the first count
  uint32_t dg[RS_ITEMS];
#pragma unroll
  for (int j = 0; j < RS_ITEMS; ++j) {
    const int i = base + j * RS_BLOCK + threadIdx.x;
    dg[j] = i < n ? digit_of(keys[i], shift) : 256u;
  }
#pragma unroll
  for (int j = 0; j < RS_ITEMS; ++j)
    if (dg[j] < 256u) atomicAdd(&cnt[dg[j]], 1);
  __syncthreads();
  hist[threadIdx.x * ntiles + blockIdx.x] = cnt[threadIdx.x];
}

__global__ void __launch_bounds__(RS_BLOCK) k_rs_scatter(const uint64_t *__restrict__ kin,
                                                          const uint32_t *__restrict__ vin, int cap,
                                                          const int32_t *d_n, int shift,
                                                          const int32_t *__restrict__ offs,
                                                          uint64_t *__restrict__ kout, uint32_t *__restrict__ vout) {
  __shared__ int run[256];
  __shared__ int wcnt[4][256];
  const int n = live_count(cap, d_n);
  const int ntiles = (n + RS_TILE - 1) / RS_TILE;
  if ((int)blockIdx.x >= ntiles) return;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  run[tid] = offs[tid * ntiles + blockIdx.x];
  wcnt[0][tid] = wcnt[1][tid] = wcnt[2][tid] = wcnt[3][tid] = 0;
  __syncthreads();
  const int base = blockIdx.x * RS_TILE;
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  // every key and value of the thread is requested before the ranking
  uint64_t kk[RS_ITEMS];
  uint32_t vv[RS_ITEMS];
#pragma unroll
  for (int j = 0; j < RS_ITEMS; ++j) {
    const int i = base + j * RS_BLOCK + tid;
    kk[j] = i < n ? kin[i] : 0ull;
    vv[j] = i < n ? vin[i] : 0u;
  }
#pragma unroll
  for (int j = 0; j < RS_ITEMS; ++j) {
    const int i = base + j * RS_BLOCK + tid;
    const bool valid = i < n;
    const uint64_t k = kk[j];
    const uint32_t v = vv[j];
    uint32_t d = digit_of(k, shift);
    uint64_t m = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      uint64_t bal = __ballot((d >> b) & 1u);
      m &= ((d >> b) & 1u) ? bal : ~bal;
    }
    int rank = __popcll(m & lt);
    int tot = __popcll(m);
    bool leader = valid && rank == 0;
    if (leader) wcnt[wid][d] = tot;
    __syncthreads();
    if (valid) {
      int off = run[d] + rank;
      for (int w = 0; w < wid; ++w) off += wcnt[w][d];
      kout[off] = k;
      vout[off] = v;
    }
    __syncthreads();
    run[tid] += wcnt[0][tid] + wcnt[1][tid] + wcnt[2][tid] + wcnt[3][tid];
    wcnt[0][tid] = wcnt[1][tid] = wcnt[2][tid] = wcnt[3][tid] = 0;
    __syncthreads();
  }
}

int sort_hist_size(int cap) { return 256 * ((cap + RS_TILE - 1) / RS_TILE) + 1; }

// Sorts (keys, vals) by the key bits [0, bits) (a multiple of 8); the result
// ends in k0/v0.  k1/v1 are ping-pong buffers of the same capacity.
void radix_sort(uint64_t *k0, uint32_t *v0, uint64_t *k1, uint32_t *v1, int cap, const int32_t *d_n, int bits,
                int32_t *hist, int32_t *scan_tmp, hipStream_t s) {
  if (cap <= 0) return;
  const int ntiles = (cap + RS_TILE - 1) / RS_TILE;
  int32_t *hist_n = hist + 256 * ntiles;  // the extra slot of sort_hist_size
  hipLaunchKernelGGL(k_rs_size, dim3(1), dim3(1), 0, s, cap, d_n, hist_n);
  uint64_t *ka = k0, *kb = k1;
  uint32_t *va = v0, *vb = v1;
  for (int shift = 0; shift < bits; shift += 8) {
    hipLaunchKernelGGL(k_rs_hist, dim3(ntiles), dim3(RS_BLOCK), 0, s, ka, cap, d_n, shift, hist);
    scan_exclusive(hist, hist, 256 * ntiles, hist_n, nullptr, scan_tmp, s);
    hipLaunchKernelGGL(k_rs_scatter, dim3(ntiles), dim3(RS_BLOCK), 0, s, ka, va, cap, d_n, shift, hist, kb, vb);
    std::swap(ka, kb);
    std::swap(va, vb);
  }
  // an odd number of passes leaves the result in k1/v1
  if (ka != k0) {
    hipMemcpyAsync(k0, ka, sizeof(uint64_t) * cap, hipMemcpyDeviceToDevice, s);
    hipMemcpyAsync(v0, va, sizeof(uint32_t) * cap, hipMemcpyDeviceToDevice, s);
  }
}

// ------------------------------------------------------ packed positions
__global__ void k_pack_xy(const float *__restrict__ x, const float *__restrict__ y, float2 *__restrict__ xy, int n,
                          int32_t *__restrict__ bad, int32_t gen) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float a = x[i], b = y[i];
  xy[i] = make_float2(a, b);
  // every writer stores the same value, so no atomic is needed
  if (bad && !(__builtin_isfinite(a) && __builtin_isfinite(b))) *bad = gen;
}
void pack_xy(const float *x, const float *y, float2 *xy, int n, hipStream_t s, int32_t *bad, int32_t gen) {
  if (n > 0) hipLaunchKernelGGL(k_pack_xy, dim3((n + 255) / 256), dim3(256), 0, s, x, y, xy, n, bad, gen);
}

// ---------------------------------------------------------- small fills
__global__ void k_fill_i32(int32_t *p, int n, int32_t v) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}
void fill_i32(int32_t *p, int n, int32_t v, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_fill_i32, dim3((n + 255) / 256), dim3(256), 0, s, p, n, v);
}

}  // namespace tdp
