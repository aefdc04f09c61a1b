// The placement loop around the hot path: a bin-density penalty with its
// gradient, and one step of Nesterov's method (the paper's placer minimises
// wirelength + lambda * density (Eq. 1) + beta * PP (Eq. 6) with
// DREAMPlace's Nesterov optimiser; Sec. IV).
//
// Density: the die is cut into gx x gy bins of bw x bh, bin (i, j) at
// j * gx + i.  Cell c spreads its area a_c as a Gaussian centred on its
// position with standard deviations (bw, bh), integrated over each bin, over
// the (2R+1)^2 bins around the bin holding it (its indices clamped into the
// grid); mass the window puts off the die is reflected back in at the edges
// (mirror images, the Neumann boundary of an electrostatic density):
//   D(i, j) = sum_c a_c Wx_c(i) Wy_c(j),   Wx_c(i) = sum of Phi(upper) -
// Phi(lower) at the standardised edges of the window bins that fold onto i.  value = sum_b max(0, D_b - cap)^2 with
// cap = target * bw * bh, overflow = sum_b max(0, D_b - cap) / sum_c a_c.
//
// One evaluation: cells are sorted by bin (stable radix sort); each sorted
// cell writes its 2(2R+1) window weights (x weights times its area); each bin
// then gathers, in a fixed order, the weights of the cells in the bins whose
// windows reach it (a crowded bin with a whole workgroup); the gradient is a
// gather per cell over its window's overflow.  No floating-point atomics:
// results are bitwise reproducible.
// A cell's bin is decided in double precision (its position minus the
// grid origin, over the bin size), so that the decision does not depend on
// the rounding of a single-precision quotient.
#include "tdp_impl.h"
#include "tdp_prims.h"

namespace tdp {

static inline int nbk(long long n, int b) { return n > 0 ? (int)((n + b - 1) / b) : 1; }

constexpr int DN_BLOCK = 256;
constexpr int DN_PARTS = 1024;  // partial sums per reduction (fixed grid)

__device__ __forceinline__ int dn_bin(float v, float v0, float w, int g, float &frac) {
  const double q = ((double)v - (double)v0) / (double)w;
  double f = floor(q);
  f = !(f >= 0.0) ? 0.0 : (f > (double)(g - 1) ? (double)(g - 1) : f);  // NaN -> bin 0: never out of the grid
  frac = (float)(q - f);  // position inside the bin in bin widths (outside [0, 1) when clamped)
  return (int)f;
}

// Phi(hi) - Phi(lo) for hi >= lo, from complementary error functions on the
// side where both are small (no cancellation between two values near 1)
__device__ __forceinline__ float gauss_mass(float lo, float hi) {
  const float s = 0.70710678118654752f;  // 1 / sqrt(2)
  if (lo >= 0.f) return 0.5f * (erfcf(lo * s) - erfcf(hi * s));
  if (hi <= 0.f) return 0.5f * (erfcf(-hi * s) - erfcf(-lo * s));
  return 1.f - 0.5f * (erfcf(hi * s) + erfcf(-lo * s));
}

__device__ __forceinline__ float gauss_pdf(float z) { return 0.39894228040143268f * expf(-0.5f * z * z); }

// Weight and its derivative (per unit of position) for grid bin i of a cell
// at fraction f of window bin b: the window bins u = b - R .. b + R that fold
// onto i (u itself inside the grid; u < 0 onto -1 - u, u >= g onto
// 2g - 1 - u, repeatedly), summed in window order.  Cells whose window lies
// inside the grid take the single direct term.
__device__ __forceinline__ void axis_weight(int b, float f, int g, int R, int i, float inv_w, float &wt,
                                            float &dt) {
  if (b - R >= 0 && b + R < g) {
    const float lo = (float)(i - b) - f, hi = lo + 1.f;
    wt = gauss_mass(lo, hi);
    dt = (gauss_pdf(lo) - gauss_pdf(hi)) * inv_w;
    return;
  }
  wt = 0.f;
  dt = 0.f;
  for (int k = 0; k <= 2 * R; ++k) {
    int v = b - R + k;
    for (int r = 0; r < 64 && (v < 0 || v >= g); ++r) v = v < 0 ? -1 - v : 2 * g - 1 - v;
    if (v != i) continue;
    const float lo = (float)(k - R) - f, hi = lo + 1.f;
    wt += gauss_mass(lo, hi);
    dt += (gauss_pdf(lo) - gauss_pdf(hi)) * inv_w;
  }
}

__global__ void __launch_bounds__(DN_BLOCK) k_dn_keys(int n, const float *__restrict__ x, const float *__restrict__ y,
                                                       DensityGrid gr, uint64_t *__restrict__ key,
                                                       uint32_t *__restrict__ val) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  float fx, fy;
  const int bx = dn_bin(x[c], gr.x0, gr.bw, gr.gx, fx);
  const int by = dn_bin(y[c], gr.y0, gr.bh, gr.gy, fy);
  key[c] = (uint64_t)by * (uint64_t)gr.gx + (uint64_t)bx;
  val[c] = (uint32_t)c;
}

// start[b] = first sorted position with key >= b, for b in [0, G]: a binary
// search per bin (balanced however crowded the bins are)
__global__ void __launch_bounds__(DN_BLOCK) k_dn_starts(int n, int G, const uint64_t *__restrict__ key,
                                                         int32_t *__restrict__ start) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b > G) return;
  int lo = 0, hi = n;  // the answer lies in [lo, hi]
  while (lo < hi) {
    const int mid = lo + ((hi - lo) >> 1);
    if (key[mid] < (uint64_t)b) lo = mid + 1;
    else hi = mid;
  }
  start[b] = lo;
}

// weights of sorted cell s: w[k * n + s] = a_c Wx(k - R), w[(K + k) * n + s] = Wy(k - R), K = 2R + 1
__global__ void __launch_bounds__(DN_BLOCK) k_dn_weights(int n, const uint32_t *__restrict__ order,
                                                          const float *__restrict__ x, const float *__restrict__ y,
                                                          const float *__restrict__ area, DensityGrid gr,
                                                          float *__restrict__ w) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const int c = (int)order[s];
  float fx, fy;
  const int bx = dn_bin(x[c], gr.x0, gr.bw, gr.gx, fx);
  const int by = dn_bin(y[c], gr.y0, gr.bh, gr.gy, fy);
  const float a = area[c];
  const int K = 2 * gr.R + 1;
  for (int k = 0; k < K; ++k) {
    const int i = bx - gr.R + k, j = by - gr.R + k;
    float wt = 0.f, dt;
    if (i >= 0 && i < gr.gx) axis_weight(bx, fx, gr.gx, gr.R, i, 1.f, wt, dt);
    w[(size_t)k * n + s] = a * wt;
    wt = 0.f;
    if (j >= 0 && j < gr.gy) axis_weight(by, fy, gr.gy, gr.R, j, 1.f, wt, dt);
    w[(size_t)(K + k) * n + s] = wt;
  }
}

__device__ __forceinline__ void block_sum2(double &a, double &b) {
  __shared__ double sa[DN_BLOCK], sb[DN_BLOCK];
  sa[threadIdx.x] = a;
  sb[threadIdx.x] = b;
  __syncthreads();
  for (int o = DN_BLOCK / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      sa[threadIdx.x] += sa[threadIdx.x + o];
      sb[threadIdx.x] += sb[threadIdx.x + o];
    }
    __syncthreads();
  }
  a = sa[0];
  b = sb[0];
}

// Bin gathers.  Keys are row-major (by * gx + bx), so the cells of the bins
// [i - R, i + R] of one row are one contiguous range of the sorted order: a
// bin's window is 2R+1 ranges.  A bin whose window holds at most DN_HEAVY
// cells sums them in one thread (rows in order, cells in sorted order); a
// crowded bin is listed and summed by a whole workgroup (cells dealt to
// threads by position, a fixed-order tree over the threads).  Either way the
// sum depends on the data alone: results are bitwise reproducible.
constexpr int DN_HEAVY = 512;

__device__ __forceinline__ void window_row(const DensityGrid &gr, const int32_t *__restrict__ start, int i, int sj,
                                           int &s0, int &s1) {
  const int lo = sj * gr.gx + (i - gr.R > 0 ? i - gr.R : 0);
  const int hi = sj * gr.gx + (i + gr.R < gr.gx - 1 ? i + gr.R : gr.gx - 1);
  s0 = start[lo];
  s1 = start[hi + 1];
}

// the product a_c Wx_c(i) Wy_c(j) of sorted cell s in row sj = j - dj
__device__ __forceinline__ double dn_term(const DensityGrid &gr, const uint64_t *__restrict__ key,
                                          const float *__restrict__ w, int n, int K, int i, int sj, int dj, int s) {
  const int di = i - (int)(key[s] - (uint64_t)sj * (uint64_t)gr.gx);
  return (double)(w[(size_t)(di + gr.R) * n + s] * w[(size_t)(K + dj + gr.R) * n + s]);
}

__global__ void __launch_bounds__(DN_BLOCK) k_dn_bins(int n, DensityGrid gr, const int32_t *__restrict__ start,
                                                       const uint64_t *__restrict__ key, const float *__restrict__ w,
                                                       float *__restrict__ map, int32_t *__restrict__ heavy,
                                                       int32_t *__restrict__ n_heavy) {
  const int G = gr.gx * gr.gy, R = gr.R, K = 2 * R + 1;
  const int b = blockIdx.x * DN_BLOCK + threadIdx.x;
  if (b >= G) return;
  const int i = b % gr.gx, j = b / gr.gx;
  int cnt = 0;
  for (int dj = -R; dj <= R; ++dj) {
    const int sj = j - dj;
    if (sj < 0 || sj >= gr.gy) continue;
    int s0, s1;
    window_row(gr, start, i, sj, s0, s1);
    cnt += s1 - s0;
  }
  if (cnt > DN_HEAVY) {
    heavy[atomicAdd(n_heavy, 1)] = b;  // summed by k_dn_heavy
    return;
  }
  // rows in order; within a row, source bins (and so cells) in sorted
  // order, each bin's x-weight column fixed by its offset from bin i
  double d = 0.0;
  for (int dj = -R; dj <= R; ++dj) {
    const int sj = j - dj;
    if (sj < 0 || sj >= gr.gy) continue;
    const float *wy = w + (size_t)(K + dj + R) * n;
    const int lo = i - R > 0 ? i - R : 0, hi = i + R < gr.gx - 1 ? i + R : gr.gx - 1;
    int s0 = start[sj * gr.gx + lo];
    for (int si = lo; si <= hi; ++si) {
      const int s1 = start[sj * gr.gx + si + 1];
      const float *wx = w + (size_t)(i - si + R) * n;
      for (int s = s0; s < s1; ++s) d += (double)(wx[s] * wy[s]);
      s0 = s1;
    }
  }
  map[b] = (float)d;
}

__device__ __forceinline__ double block_sum1(double a) {
  double unused = 0.0;
  block_sum2(a, unused);
  return a;
}

// one workgroup per listed bin (grid-stride over the list)
__global__ void __launch_bounds__(DN_BLOCK) k_dn_heavy(int n, DensityGrid gr, const int32_t *__restrict__ start,
                                                        const uint64_t *__restrict__ key, const float *__restrict__ w,
                                                        const int32_t *__restrict__ heavy,
                                                        const int32_t *__restrict__ n_heavy, float *__restrict__ map) {
  const int R = gr.R, K = 2 * R + 1;
  const int nh = *n_heavy;
  for (int h = blockIdx.x; h < nh; h += gridDim.x) {
    const int b = heavy[h];
    const int i = b % gr.gx, j = b / gr.gx;
    double d = 0.0;
    for (int dj = -R; dj <= R; ++dj) {
      const int sj = j - dj;
      if (sj < 0 || sj >= gr.gy) continue;
      int s0, s1;
      window_row(gr, start, i, sj, s0, s1);
      for (int s = s0 + (int)threadIdx.x; s < s1; s += DN_BLOCK) d += dn_term(gr, key, w, n, K, i, sj, dj, s);
    }
    d = block_sum1(d);
    if (threadIdx.x == 0) map[b] = (float)d;
    __syncthreads();  // the reduction's shared arrays are reused by the next bin
  }
}

// sums of o^2 and o over the finished map, o = max(0, D - cap); the block's
// go to part[blk], part[DN_PARTS + blk]
__global__ void __launch_bounds__(DN_BLOCK) k_dn_reduce(DensityGrid gr, const float *__restrict__ map,
                                                         double *__restrict__ part) {
  const int G = gr.gx * gr.gy;
  const float cap = gr.target * gr.bw * gr.bh;
  double so2 = 0.0, so = 0.0;
  for (int b = blockIdx.x * DN_BLOCK + threadIdx.x; b < G; b += DN_PARTS * DN_BLOCK) {
    const float df = map[b];
    const double o = df > cap ? (double)df - (double)cap : 0.0;
    so2 += o * o;
    so += o;
  }
  block_sum2(so2, so);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = so2;
    part[DN_PARTS + blockIdx.x] = so;
  }
}

__global__ void __launch_bounds__(DN_BLOCK) k_dn_final(const double *__restrict__ part, double inv_area,
                                                        double *value, double *overflow) {
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < DN_PARTS; i += DN_BLOCK) {
    a += part[i];
    b += part[DN_PARTS + i];
  }
  block_sum2(a, b);
  if (threadIdx.x == 0) {
    if (value) *value = a;
    if (overflow) *overflow = b * inv_area;
  }
}

// gradient of the penalty on movable cells: += scale * d value / d (x, y).
// The window's weights and derivatives are evaluated once per axis (2R+1
// each, in registers: R is a template parameter); the window sum is then
//   d/dx = 2 a sum_j Wy(j) sum_i Wx'(i) o(i, j),  d/dy likewise.
// Threads take the cells in bin order, so that a wave's windows overlap and
// share the map's cache lines.
template <int R>
__global__ void __launch_bounds__(DN_BLOCK) k_dn_grad(int n, const uint32_t *__restrict__ order,
                                                       const float *__restrict__ x, const float *__restrict__ y,
                                                       const float *__restrict__ area,
                                                       const uint8_t *__restrict__ fixed, DensityGrid gr,
                                                       const float *__restrict__ map, float scale,
                                                       float *__restrict__ gx, float *__restrict__ gy) {
  constexpr int K = 2 * R + 1;
  const int si = blockIdx.x * blockDim.x + threadIdx.x;
  if (si >= n) return;
  const int c = (int)order[si];
  if (fixed[c]) return;
  float fx, fy;
  const int bx = dn_bin(x[c], gr.x0, gr.bw, gr.gx, fx);
  const int by = dn_bin(y[c], gr.y0, gr.bh, gr.gy, fy);
  const float cap = gr.target * gr.bw * gr.bh;
  float wx[K], dx[K], wy[K], dy[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int i = bx - R + k, j = by - R + k;
    wx[k] = dx[k] = wy[k] = dy[k] = 0.f;
    if (i >= 0 && i < gr.gx) axis_weight(bx, fx, gr.gx, R, i, 1.f / gr.bw, wx[k], dx[k]);
    if (j >= 0 && j < gr.gy) axis_weight(by, fy, gr.gy, R, j, 1.f / gr.bh, wy[k], dy[k]);
  }
  float ax = 0.f, ay = 0.f;
#pragma unroll
  for (int kj = 0; kj < K; ++kj) {
    const int j = by - R + kj;
    if (j < 0 || j >= gr.gy) continue;
    float sx = 0.f, sy = 0.f;
#pragma unroll
    for (int ki = 0; ki < K; ++ki) {
      const int i = bx - R + ki;
      if (i < 0 || i >= gr.gx) continue;
      const float o = map[j * gr.gx + i] - cap;
      if (o <= 0.f) continue;
      sx += o * dx[ki];
      sy += o * wx[ki];
    }
    ax += sx * wy[kj];
    ay += sy * dy[kj];
  }
  const float k2 = 2.f * area[c] * scale;
  gx[c] += k2 * ax;
  gy[c] += k2 * ay;
}

template <int R>
static void launch_grad(int n, const uint32_t *order, const float *x, const float *y, const float *area,
                        const uint8_t *fixed, const DensityGrid &gr, const float *map, float scale, float *gx,
                        float *gy, hipStream_t s) {
  hipLaunchKernelGGL(k_dn_grad<R>, dim3(nbk(n, DN_BLOCK)), dim3(DN_BLOCK), 0, s, n, order, x, y, area, fixed, gr, map,
                     scale, gx, gy);
}

void density_impl(tdp_graph g, const float *x, const float *y, float scale, double *value, double *overflow,
                  float *gx, float *gy, float *map_out, hipStream_t s) {
  const int n = g->topo.N;
  const DensityGrid &gr = g->dn;
  const int G = gr.gx * gr.gy;
  prof_begin(g, TDP_STAGE_DENSITY, s);
  if (n > 0) {
    hipLaunchKernelGGL(k_dn_keys, dim3(nbk(n, DN_BLOCK)), dim3(DN_BLOCK), 0, s, n, x, y, gr, g->dn_k0, g->dn_v0);
    radix_sort(g->dn_k0, g->dn_v0, g->dn_k1, g->dn_v1, n, nullptr, g->dn_key_bits, g->dn_hist, g->dn_scan, s);
    hipLaunchKernelGGL(k_dn_weights, dim3(nbk(n, DN_BLOCK)), dim3(DN_BLOCK), 0, s, n, (const uint32_t *)g->dn_v0,
                       x, y, (const float *)g->dn_area, gr, g->dn_w);
  }
  hipLaunchKernelGGL(k_dn_starts, dim3(nbk((long long)G + 1, DN_BLOCK)), dim3(DN_BLOCK), 0, s, n, G,
                     (const uint64_t *)g->dn_k0, g->dn_start);
  float *map = map_out ? map_out : g->dn_map;
  fill_i32(g->dn_nheavy, 1, 0, s);
  hipLaunchKernelGGL(k_dn_bins, dim3(nbk(G, DN_BLOCK)), dim3(DN_BLOCK), 0, s, n, gr, (const int32_t *)g->dn_start,
                     (const uint64_t *)g->dn_k0, (const float *)g->dn_w, map, g->dn_heavy, g->dn_nheavy);
  hipLaunchKernelGGL(k_dn_heavy, dim3(DN_PARTS), dim3(DN_BLOCK), 0, s, n, gr, (const int32_t *)g->dn_start,
                     (const uint64_t *)g->dn_k0, (const float *)g->dn_w, (const int32_t *)g->dn_heavy,
                     (const int32_t *)g->dn_nheavy, map);
  hipLaunchKernelGGL(k_dn_reduce, dim3(DN_PARTS), dim3(DN_BLOCK), 0, s, gr, (const float *)map, g->dn_part);
  hipLaunchKernelGGL(k_dn_final, dim3(1), dim3(DN_BLOCK), 0, s, (const double *)g->dn_part,
                     g->dn_total_area > 0 ? 1.0 / g->dn_total_area : 0.0, value, overflow);
  if (gx && gy && n > 0) {
    const float *area = g->dn_area;
    const uint8_t *fixed = g->topo.cell_fixed;
    const uint32_t *order = g->dn_v0;  // cell ids in bin order (this call's sort)
    switch (gr.R) {
      case 0: launch_grad<0>(n, order, x, y, area, fixed, gr, map, scale, gx, gy, s); break;
      case 1: launch_grad<1>(n, order, x, y, area, fixed, gr, map, scale, gx, gy, s); break;
      case 2: launch_grad<2>(n, order, x, y, area, fixed, gr, map, scale, gx, gy, s); break;
      case 3: launch_grad<3>(n, order, x, y, area, fixed, gr, map, scale, gx, gy, s); break;
      case 4: launch_grad<4>(n, order, x, y, area, fixed, gr, map, scale, gx, gy, s); break;
      case 5: launch_grad<5>(n, order, x, y, area, fixed, gr, map, scale, gx, gy, s); break;
      case 6: launch_grad<6>(n, order, x, y, area, fixed, gr, map, scale, gx, gy, s); break;
      case 7: launch_grad<7>(n, order, x, y, area, fixed, gr, map, scale, gx, gy, s); break;
      default: launch_grad<8>(n, order, x, y, area, fixed, gr, map, scale, gx, gy, s); break;
    }
  }
  prof_end(g, TDP_STAGE_DENSITY, s);
}

// ---------------------------------------------------------------- Nesterov
// One step on the 2n coordinates of the graph's cells (frozen: fixed cells):
//   q = gradient / max(1, pdiv_c);  alpha = |v - vp| / |q - gp| (alpha0 on
//   the first step or when that is not a positive number);
//   u' = clamp(v - alpha q);  v' = clamp(u' + coef (u' - u));
//   then vp = v, gp = q, u = u', v = v'.
__global__ void __launch_bounds__(DN_BLOCK) k_nest_norms(int n, const uint8_t *__restrict__ fixed,
                                                          const float *__restrict__ pdiv, const float *__restrict__ gx,
                                                          const float *__restrict__ gy, const float *__restrict__ vx,
                                                          const float *__restrict__ vy, const float *__restrict__ vpx,
                                                          const float *__restrict__ vpy, const float *__restrict__ gpx,
                                                          const float *__restrict__ gpy, double *__restrict__ part) {
  double dv = 0.0, dg = 0.0;
  for (int c = blockIdx.x * DN_BLOCK + threadIdx.x; c < n; c += DN_PARTS * DN_BLOCK) {
    if (fixed[c]) continue;
    const float p = pdiv[c] > 1.f ? pdiv[c] : 1.f;
    const double ex = (double)vx[c] - (double)vpx[c], ey = (double)vy[c] - (double)vpy[c];
    const double qx = (double)(gx[c] / p) - (double)gpx[c], qy = (double)(gy[c] / p) - (double)gpy[c];
    dv += ex * ex + ey * ey;
    dg += qx * qx + qy * qy;
  }
  block_sum2(dv, dg);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = dv;
    part[DN_PARTS + blockIdx.x] = dg;
  }
}

__global__ void __launch_bounds__(DN_BLOCK) k_nest_alpha(const double *__restrict__ part, double alpha0, int first,
                                                          double *__restrict__ alpha) {
  double dv = 0.0, dg = 0.0;
  for (int i = threadIdx.x; i < DN_PARTS; i += DN_BLOCK) {
    dv += part[i];
    dg += part[DN_PARTS + i];
  }
  block_sum2(dv, dg);
  if (threadIdx.x == 0) {
    double a = alpha0;
    if (!first && dg > 0.0) {
      const double r = sqrt(dv) / sqrt(dg);
      if (r > 0.0 && isfinite(r)) a = r;
    }
    *alpha = a;
  }
}

__global__ void __launch_bounds__(DN_BLOCK) k_nest_update(int n, const uint8_t *__restrict__ fixed,
                                                           const float *__restrict__ pdiv, const float *__restrict__ gx,
                                                           const float *__restrict__ gy, float *__restrict__ vx,
                                                           float *__restrict__ vy, float *__restrict__ ux,
                                                           float *__restrict__ uy, float *__restrict__ vpx,
                                                           float *__restrict__ vpy, float *__restrict__ gpx,
                                                           float *__restrict__ gpy, float coef,
                                                           const double *__restrict__ alpha, float xlo, float xhi,
                                                           float ylo, float yhi) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  const float x = vx[c], yv = vy[c];
  if (fixed[c]) {
    vpx[c] = x;
    vpy[c] = yv;
    gpx[c] = 0.f;
    gpy[c] = 0.f;
    return;
  }
  const float p = pdiv[c] > 1.f ? pdiv[c] : 1.f;
  const float qx = gx[c] / p, qy = gy[c] / p;
  const float a = (float)*alpha;
  const float nux = fminf(fmaxf(x - a * qx, xlo), xhi), nuy = fminf(fmaxf(yv - a * qy, ylo), yhi);
  const float nvx = fminf(fmaxf(nux + coef * (nux - ux[c]), xlo), xhi);
  const float nvy = fminf(fmaxf(nuy + coef * (nuy - uy[c]), ylo), yhi);
  vpx[c] = x;
  vpy[c] = yv;
  gpx[c] = qx;
  gpy[c] = qy;
  ux[c] = nux;
  uy[c] = nuy;
  vx[c] = nvx;
  vy[c] = nvy;
}

void nesterov_impl(tdp_graph g, const float *gx, const float *gy, const float *pdiv, float *vx, float *vy, float *ux,
                   float *uy, float *vpx, float *vpy, float *gpx, float *gpy, double coef, double alpha0, int first,
                   float xlo, float xhi, float ylo, float yhi, double *alpha_out, hipStream_t s) {
  const int n = g->topo.N;
  const uint8_t *fixed = g->topo.cell_fixed;
  double *alpha = alpha_out ? alpha_out : g->nest_alpha;
  hipLaunchKernelGGL(k_nest_norms, dim3(DN_PARTS), dim3(DN_BLOCK), 0, s, n, fixed, pdiv, gx, gy,
                     (const float *)vx, (const float *)vy, (const float *)vpx, (const float *)vpy,
                     (const float *)gpx, (const float *)gpy, g->nest_part);
  hipLaunchKernelGGL(k_nest_alpha, dim3(1), dim3(DN_BLOCK), 0, s, (const double *)g->nest_part, alpha0, first, alpha);
  if (n > 0)
    hipLaunchKernelGGL(k_nest_update, dim3(nbk(n, DN_BLOCK)), dim3(DN_BLOCK), 0, s, n, fixed, pdiv, gx, gy, vx, vy, ux,
                       uy, vpx, vpy, gpx, gpy, (float)coef, (const double *)alpha, xlo, xhi, ylo, yhi);
}

// sum over cells of |a_c| + |b_c| (an L1 norm of a gradient), fixed order
__global__ void __launch_bounds__(DN_BLOCK) k_abs_parts(int n, const float *__restrict__ a,
                                                         const float *__restrict__ b, double *__restrict__ part) {
  double s = 0.0, unused = 0.0;
  for (int c = blockIdx.x * DN_BLOCK + threadIdx.x; c < n; c += DN_PARTS * DN_BLOCK)
    s += (double)fabsf(a[c]) + (double)fabsf(b[c]);
  block_sum2(s, unused);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void __launch_bounds__(DN_BLOCK) k_abs_final(const double *__restrict__ part, double *out) {
  double s = 0.0, unused = 0.0;
  for (int i = threadIdx.x; i < DN_PARTS; i += DN_BLOCK) s += part[i];
  block_sum2(s, unused);
  if (threadIdx.x == 0) *out = s;
}

void abs_sum_impl(tdp_graph g, const float *a, const float *b, double *out, hipStream_t s) {
  hipLaunchKernelGGL(k_abs_parts, dim3(DN_PARTS), dim3(DN_BLOCK), 0, s, g->topo.N, a, b, g->nest_part);
  hipLaunchKernelGGL(k_abs_final, dim3(1), dim3(DN_BLOCK), 0, s, (const double *)g->nest_part, out);
}

int density_parts() { return DN_PARTS; }

}  // namespace tdp
