// Differentiable objectives: a log-sum-exp smoothed TNS with its adjoint, and
// weighted-average wirelength.  Both give gradients on cell positions with a
// fixed summation order per cell (terms per pin computed per net, then
// gathered over the cell's own pins; no floating-point atomics).
//
// Smoothed TNS (not in the paper; this is its definition here): cell-arc
// delays and start-point arrivals are frozen from the last timing update, net
// delays follow the positions (the library's net model as a function of L,
// the Manhattan length).
//   sink t:          A(t) = A(drv) + dnet(t)
//   comb output o:   A(o) = m + g ln sum_j exp((a_j - m)/g), a_j = A(in_j) + d_arc(in_j)
//   endpoint e:      s(e) = (period - setup) - A(e)
//   value:           -g * sum_e softplus(-s(e)/g)
// The adjoint runs the levels top-down: dv/dA(e) = -sigmoid(-s(e)/g); an
// output passes its adjoint to input j in proportion to softmax_j(a/g); a
// driver collects the adjoints of its sinks (per level over the net chunks,
// as the required-time pass runs).  dv/d dnet(t) is the adjoint at
// t, and on a star net d dnet/dX_s = dnet'(L) sign(X_s - X_t) = -d dnet/dX_t
// (the spanning-tree model differentiates through its tree).  The net delays
// and the per-pin terms come from the net kernels of tdp_tree.hip.
//
// Weighted-average wirelength (the smoothed WL of Eq. 1): per net and axis,
// sum x e^{x/g} / sum e^{x/g} - sum x e^{-x/g} / sum e^{-x/g}, with the
// exponents shifted by the net's max and min.
#include "tdp_impl.h"
#include "tdp_prims.h"
#include "tdp_wave.h"

namespace tdp {

static inline int nb(long long n, int b) { return n > 0 ? (int)((n + b - 1) / b) : 1; }

template <typename T>
__device__ __forceinline__ T sgn(T v) {
  return (T)((v > (T)0) - (v < (T)0));
}

template <typename T>
__global__ void k_st_start(Topo tp, const T *__restrict__ at, T *__restrict__ sa) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v < tp.n_start) sa[v] = at[v];
}

// one level's combinational cells on the forward chunks, a lane per input
// (each cell a segment): the input's arrival, then the cell's log-sum-exp
// over its inputs by segment reductions
template <typename T>
__global__ void __launch_bounds__(256) k_st_fwd(Topo tp, int ch0, int ch1, T gam, const T *__restrict__ dnl,
                                                 const T *__restrict__ darc, T *__restrict__ sa) {
  const int lane = wave_lane();
  const int chunk = ch0 + blockIdx.x * 4 + (threadIdx.x >> 6);
  if (chunk >= ch1) return;
  const int4 rec = tp.fw_rec[chunk * CHUNK + lane];
  const int t = rec.x;
  const int head = rec.w & 63, tail = (rec.w >> 8) & 63;
  const bool valid = t >= 0;
  T a = -pos_inf<T>();
  if (valid) {
    const T ai = sa[rec.y] + dnl[t];
    sa[tp.M + t] = ai;
    a = ai + darc[t];
  }
  const T m = seg_max(a, lane, head, tail);
  const T sum = seg_sum(valid ? exp((a - m) / gam) : (T)0, lane, head, tail);
  if (valid && lane == head) sa[tp.n_start + rec.z] = m + gam * log(sum);
}

// endpoint values and adjoint seeds; per-block partial sums of the value
template <typename T>
__global__ void __launch_bounds__(256) k_st_end(Topo tp, const double *__restrict__ inst_req, T gam,
                                                 const T *__restrict__ dnl,
                                                 T *__restrict__ sa, T *__restrict__ adj,
                                                 double *__restrict__ part) {
  __shared__ double sh[256];
  double acc = 0.0;
  for (int f = blockIdx.x * blockDim.x + threadIdx.x; f < tp.E; f += gridDim.x * blockDim.x) {
    const int t = tp.A + f;
    const T a = sa[tp.snk_drv[t]] + dnl[t];
    sa[tp.M + t] = a;
    const T z = (a - (T)inst_req[tp.ff_inst[f]]) / gam;  // -slack / g
    const T sp = (z > 0 ? z : (T)0) + log1p(exp(-fabs(z)));
    acc += (double)(-gam * sp);
    adj[tp.M + t] = -(T)1 / ((T)1 + exp(-z));
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// The adjoint of one level's nets (drivers at that level, top-down), a lane
// per net pin: a combinational-input sink takes its cell output's adjoint
// times its softmax weight (the output's level is higher, so it is final), an
// endpoint keeps the seed the endpoint kernel wrote; the driver collects its
// sinks' (a segment sum).
template <typename T>
__global__ void __launch_bounds__(256) k_st_bwd(Topo tp, int ch0, int ch1, T gam, const T *__restrict__ darc,
                                                 const T *__restrict__ sa, T *__restrict__ adj) {
  const int lane = wave_lane();
  const int chunk = ch0 + blockIdx.x * 4 + (threadIdx.x >> 6);
  if (chunk >= ch1) return;
  const int4 rec = tp.nm_rec[chunk * CHUNK + lane];
  const int p = rec.x, vo = rec.z;
  const int head = rec.w & 63, tail = (rec.w >> 8) & 63;
  T a = 0;
  if (p >= 0 && lane != head) {
    if (vo >= 0) {
      a = adj[vo] * exp((sa[p] + darc[p - tp.M] - sa[vo]) / gam);
      adj[p] = a;
    } else {
      a = adj[p];
    }
  }
  a = seg_sum(a, lane, head, tail);
  if (p >= 0 && lane == head) adj[p] = a;
}

// the same for nets wider than a chunk, one thread per net
template <typename T>
__global__ void k_st_bwd_big(Topo tp, int i0, int i1, T gam, const T *__restrict__ darc, const T *__restrict__ sa,
                             T *__restrict__ adj) {
  const int i = i0 + blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= i1) return;
  const int v = tp.big_net[i];
  T ab = 0;
  for (int k = tp.net_ptr[v]; k < tp.net_ptr[v + 1]; ++k) {
    const int t = tp.net_sink[k];
    const int p = tp.M + t;
    T a;
    if (t < tp.A) {
      const int vo = tp.n_start + tp.snk_comb[t];
      a = adj[vo] * exp((sa[p] + darc[t] - sa[vo]) / gam);
      adj[p] = a;
    } else {
      a = adj[p];
    }
    ab += a;
  }
  adj[v] = ab;
}

// gradient per cell: the sum of its pins' gradients (its output pin, then its
// input pins), which the net kernels computed per pin
template <typename T>
__global__ void __launch_bounds__(256) k_st_grad(Topo tp, const T *__restrict__ gp, const double *__restrict__ gout,
                                                  float *__restrict__ gx, float *__restrict__ gy) {
  const int cell = blockIdx.x * blockDim.x + threadIdx.x;
  if (cell >= tp.N || tp.cell_fixed[cell]) return;
  const int ci = tp.cell_int[cell];
  int v, t0, t1;
  if (ci >= 0) {
    v = tp.n_start + ci;
    t0 = tp.comb_inptr[ci];
    t1 = tp.comb_inptr[ci + 1];
  } else {
    const int f = -ci - 1;
    v = tp.n_pi + f;
    t0 = tp.A + f;
    t1 = t0 + 1;
  }
  T ax = gp[v], ay = gp[tp.P + v];
  for (int t = t0; t < t1; ++t) {
    ax += gp[tp.M + t];
    ay += gp[tp.P + tp.M + t];
  }
  const T go = (T)*gout;
  gx[cell] += (float)(go * ax);
  gy[cell] += (float)(go * ay);
}

__global__ void __launch_bounds__(256) k_sum_parts2(int n, const double *__restrict__ part, double *__restrict__ out) {
  __shared__ double sh[256];
  double a = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) a += part[i];
  sh[threadIdx.x] = a;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sh[0];
}

constexpr int RED_BLOCKS = 512;

template <typename T>
void stns_fwd_impl(tdp_graph g, const float *x, const float *y, float gamma, double *val, hipStream_t s) {
  const Topo &tp = g->topo;
  prof_begin(g, TDP_STAGE_STNS, s);
  const T gam = (T)gamma;
  st_net_fwd_impl<T>(g, x, y, (T *)g->st_dnet, s);
  if (tp.n_start > 0)
    hipLaunchKernelGGL(k_st_start<T>, dim3(nb(tp.n_start, 256)), dim3(256), 0, s, tp, (const T *)g->at,
                       (T *)g->st_at);
  for (int l = 1; l <= tp.D; ++l) {
    const int ch0 = g->lv.fw_lvl[l - 1], ch1 = g->lv.fw_lvl[l];
    if (ch1 > ch0)
      hipLaunchKernelGGL(k_st_fwd<T>, dim3(nb(ch1 - ch0, 4)), dim3(256), 0, s, tp, ch0, ch1, gam,
                         (const T *)g->st_dnet, (const T *)g->darc, (T *)g->st_at);
  }
  hipLaunchKernelGGL(k_st_end<T>, dim3(RED_BLOCKS), dim3(256), 0, s, tp, g->d_inst_req, gam, (const T *)g->st_dnet,
                     (T *)g->st_at, (T *)g->st_adj, g->red_loss);
  hipLaunchKernelGGL(k_sum_parts2, dim3(1), dim3(256), 0, s, RED_BLOCKS, g->red_loss, val);
  g->st_gamma = gamma;
  g->st_x = x;
  g->st_y = y;
  g->stns_ready = true;
  prof_end(g, TDP_STAGE_STNS, s);
}

template <typename T>
void stns_bwd_impl(tdp_graph g, const double *gout, float *gx, float *gy, hipStream_t s) {
  const Topo &tp = g->topo;
  prof_begin(g, TDP_STAGE_STNS, s);
  const T gam = (T)g->st_gamma;
  for (int l = tp.D; l >= 0; --l) {
    const int ch0 = g->lv.nm_lvl[l], ch1 = g->lv.nm_lvl[l + 1];
    if (ch1 > ch0)
      hipLaunchKernelGGL(k_st_bwd<T>, dim3(nb(ch1 - ch0, 4)), dim3(256), 0, s, tp, ch0, ch1, gam,
                         (const T *)g->darc, (const T *)g->st_at, (T *)g->st_adj);
    const int b0 = g->lv.big_lvl[l], b1 = g->lv.big_lvl[l + 1];
    if (b1 > b0)
      hipLaunchKernelGGL(k_st_bwd_big<T>, dim3(nb(b1 - b0, 64)), dim3(64), 0, s, tp, b0, b1, gam,
                         (const T *)g->darc, (const T *)g->st_at, (T *)g->st_adj);
  }
  st_net_grad_impl<T>(g, g->st_x, g->st_y, (const T *)g->st_adj, s);
  hipLaunchKernelGGL(k_st_grad<T>, dim3(nb(tp.N, 256)), dim3(256), 0, s, tp, (const T *)g->st_gp, gout, gx, gy);
  prof_end(g, TDP_STAGE_STNS, s);
}

// ------------------------------------------------------------------- WA
// Coordinates enter relative to the net's max (the e^{x/g} side) and min (the
// e^{-x/g} side): d = x - max <= 0, e = x - min >= 0, so the weighted means
// and the (x - mean) terms stay small numbers in single precision.
//   WA = (max - min) + sum d a / sum a - sum e b / sum b,  a = e^{d/g}, b = e^{-e/g}
//   dWA/dx = a/sum a (1 + (d - sum d a / sum a)/g) - b/sum b (1 - (e - sum e b / sum b)/g)

// one axis for one lane of a chunked net; returns the net's WA on that axis.
// A pin's coordinate is (cell position c) + (offset o); differences are taken
// as (c_i - c_m) + (o_i - o_m), which keeps them exact to within the rounding
// of the result instead of carrying the rounding of c + o at die scale.
__device__ __forceinline__ float wa_lane(float c, float o, bool valid, int lane, int head, int tail, float ig,
                                         float &grad) {
  const float X = c + o;
  const float mx = seg_max_dpp(valid ? X : -3.0e38f, lane, head, tail);
  const float mn = seg_min_dpp(valid ? X : 3.0e38f, lane, head, tail);
  const int am = seg_min_dpp((valid && X == mx) ? lane : 64, lane, head, tail) & 63;
  const int an = seg_min_dpp((valid && X == mn) ? lane : 64, lane, head, tail) & 63;
  const float cm = __shfl(c, am, 64), om = __shfl(o, am, 64);
  const float cn = __shfl(c, an, 64), on = __shfl(o, an, 64);
  const float d = valid ? (c - cm) + (o - om) : 0.f, e = valid ? (c - cn) + (o - on) : 0.f;
  // exponents are <= 0 (d <= 0 <= e); the hardware exponential (2^(x log2 e))
  // has a relative error of about |x| 2^-24 plus a few units in the last
  // place, and terms with large |x| are negligible in the sums
  const float a = valid ? __expf(d * ig) : 0.f, b = valid ? __expf(-e * ig) : 0.f;
  const float sa = seg_sum_dpp(a, lane, head, tail), sda = seg_sum_dpp(a * d, lane, head, tail);
  const float sb = seg_sum_dpp(b, lane, head, tail), seb = seg_sum_dpp(b * e, lane, head, tail);
  const float ra = valid ? 1.f / sa : 0.f, rb = valid ? 1.f / sb : 0.f;  // sa, sb >= 1 (the extreme pin's term)
  const float fp = sda * ra, fm = seb * rb;
  grad = valid ? a * ra * (1.f + (d - fp) * ig) - b * rb * (1.f - (e - fm) * ig) : 0.f;
  return valid ? ((cm - cn) + (om - on)) + fp - fm : 0.f;
}

// chunked nets: value partials and the gradient of each pin (internal pin order)
// cxy (optional): the cell coordinates of every slot, gathered by the last
// timing update; otherwise they are gathered here from xy
__global__ void __launch_bounds__(256) k_wa_net(Topo tp, const float2 *__restrict__ xy,
                                                 const float2 *__restrict__ cxy, float gam,
                                                 float *__restrict__ gpin, double *__restrict__ part) {
  __shared__ double sh[256];
  double acc = 0.0;
  const float ig = 1.0f / gam;
  const int lane = wave_lane();
  const int stride = gridDim.x * 4;
  // each chunk's inputs are loaded one chunk ahead, before the current
  // chunk's stores: a wave's loads retire after its earlier stores, so a
  // load issued after them would wait for them
  auto fetch = [&](int chunk, int4 &rec, float2 &q, float &ox, float &oy) {
    const int k = chunk * CHUNK + lane;
    rec = tp.nm_rec[k];
    q = cxy ? cxy[k] : (rec.y >= 0 ? xy[rec.y] : make_float2(0.f, 0.f));
    ox = tp.nm_ox[k];
    oy = tp.nm_oy[k];
  };
  int chunk = blockIdx.x * 4 + (threadIdx.x >> 6);
  int4 nrec = make_int4(-1, -1, -1, 0);
  float2 nq = make_float2(0.f, 0.f);
  float nox = 0.f, noy = 0.f;
  if (chunk < tp.n_nm_chunks) fetch(chunk, nrec, nq, nox, noy);
  for (; chunk < tp.n_nm_chunks; chunk += stride) {
    const int4 rec = nrec;
    const float2 q = nq;
    const float ox = nox, oy = noy;
    if (chunk + stride < tp.n_nm_chunks) fetch(chunk + stride, nrec, nq, nox, noy);
    const int p = rec.x;
    const int head = rec.w & 63, tail = (rec.w >> 8) & 63;
    const bool valid = p >= 0;
    float gxp, gyp;
    const float wx = wa_lane(q.x, ox, valid, lane, head, tail, ig, gxp);
    const float wy = wa_lane(q.y, oy, valid, lane, head, tail, ig, gyp);
    if (valid) {
      gpin[2 * p] = gxp;
      gpin[2 * p + 1] = gyp;
      if (lane == head) acc += (double)wx + (double)wy;
    }
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// nets wider than a chunk: one thread per net, same arithmetic
__global__ void __launch_bounds__(64) k_wa_big(Topo tp, const float2 *__restrict__ xy, float gam,
                                                float *__restrict__ gpin, double *__restrict__ part) {
  __shared__ double sh[64];
  double acc = 0.0;
  const float ig = 1.0f / gam;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < tp.n_big; i += gridDim.x * blockDim.x) {
    const int v = tp.big_net[i];
    const int b = tp.net_ptr[v], e = tp.net_ptr[v + 1];
    const int dc = tp.drv_cell[v];
    for (int axis = 0; axis < 2; ++axis) {
      const float *so = axis ? tp.snk_oy : tp.snk_ox;
      auto pc = [&](int cell) { return axis ? xy[cell].y : xy[cell].x; };
      const float pd = (dc >= 0 ? pc(dc) : 0.f) + (axis ? tp.drv_oy[v] : tp.drv_ox[v]);
      float mx = pd, mn = pd;
      for (int k = b; k < e; ++k) {
        const int t = tp.net_sink[k];
        const float q = pc(tp.snk_cell[t]) + so[t];
        mx = fmaxf(mx, q);
        mn = fminf(mn, q);
      }
      float sa = 0.f, sda = 0.f, sb = 0.f, seb = 0.f;
      for (int k = b - 1; k < e; ++k) {
        const float q = k < b ? pd : pc(tp.snk_cell[tp.net_sink[k]]) + so[tp.net_sink[k]];
        const float d = q - mx, ee = q - mn;
        const float a = expf(d * ig), bb = expf(-ee * ig);
        sa += a; sda += a * d; sb += bb; seb += bb * ee;
      }
      const float fp = sda / sa, fm = seb / sb;
      acc += (double)((mx - mn) + fp - fm);
      for (int k = b - 1; k < e; ++k) {
        const int t = k < b ? -1 : tp.net_sink[k];
        const float q = k < b ? pd : pc(tp.snk_cell[t]) + so[t];
        const float d = q - mx, ee = q - mn;
        const float a = expf(d * ig), bb = expf(-ee * ig);
        const float gr = a / sa * (1.f + (d - fp) * ig) - bb / sb * (1.f - (ee - fm) * ig);
        gpin[2 * (k < b ? v : tp.M + t) + axis] = gr;
      }
    }
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 32; o > 0; o >>= 1) {
    if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ void __launch_bounds__(256) k_wa_cell(Topo tp, const float *__restrict__ gpin, float *__restrict__ gx,
                                                  float *__restrict__ gy) {
  const int cell = blockIdx.x * blockDim.x + threadIdx.x;
  if (cell >= tp.N || tp.cell_fixed[cell]) return;
  const int ci = tp.cell_int[cell];
  int v, t0, t1;
  if (ci >= 0) {
    v = tp.n_start + ci;
    t0 = tp.comb_inptr[ci];
    t1 = tp.comb_inptr[ci + 1];
  } else {
    const int f = -ci - 1;
    v = tp.n_pi + f;
    t0 = tp.A + f;
    t1 = t0 + 1;
  }
  float ax = gpin[2 * v], ay = gpin[2 * v + 1];
  for (int t = t0; t < t1; ++t) {
    ax += gpin[2 * (tp.M + t)];
    ay += gpin[2 * (tp.M + t) + 1];
  }
  gx[cell] += ax;
  gy[cell] += ay;
}

void wa_impl(tdp_graph g, const float *x, const float *y, float gamma, double *wl, float *gx, float *gy,
             hipStream_t s) {
  const Topo &tp = g->topo;
  prof_begin(g, TDP_STAGE_WA, s);
  constexpr int WB = RED_BLOCKS * 4, BB = 64;  // partial slots: chunked nets, then big nets
  // x == nullptr: the positions of the last timing update, whose cell
  // coordinates per slot it already gathered
  const float2 *xy = g->xy, *cxy = g->cxy_nm;
  if (x) {
    pack_xy(x, y, g->xy_wa, tp.N, s);
    xy = g->xy_wa;
    cxy = nullptr;
  }
  hipLaunchKernelGGL(k_wa_net, dim3(WB), dim3(256), 0, s, tp, xy, cxy, gamma, g->wa_gpin, g->red_wa);
  hipLaunchKernelGGL(k_wa_big, dim3(BB), dim3(64), 0, s, tp, xy, gamma, g->wa_gpin, g->red_wa + WB);
  hipLaunchKernelGGL(k_sum_parts2, dim3(1), dim3(256), 0, s, WB + BB, g->red_wa, wl);
  hipLaunchKernelGGL(k_wa_cell, dim3(nb(tp.N, 256)), dim3(256), 0, s, tp, g->wa_gpin, gx, gy);
  prof_end(g, TDP_STAGE_WA, s);
}

template void stns_fwd_impl<float>(tdp_graph, const float *, const float *, float, double *, hipStream_t);
template void stns_fwd_impl<double>(tdp_graph, const float *, const float *, float, double *, hipStream_t);
template void stns_bwd_impl<float>(tdp_graph, const double *, float *, float *, hipStream_t);
template void stns_bwd_impl<double>(tdp_graph, const double *, float *, float *, hipStream_t);

}  // namespace tdp
