// Rise / fall timing: both transitions of every pin (a fuller timing model
// around the paper's, whose timer times both; Sec. II-B), with
// report_timing_endpoint(n, 1) on it (Sec. III-B).
//
// A cell type's arcs are positive unate (an input rise causes an output
// rise, a fall a fall), negative unate (rise -> fall, fall -> rise) or
// non-unate (either causes either).  The library's tables give the output
// rise, the rise / fall extension the output fall.  A net passes a
// transition through with the same delay either way.
//
//   forward    one launch per level, one thread per combinational cell: its
//              sinks take their drivers' arrivals plus the net delay; for each
//              output transition x, the maximum over (input j, input
//              transition y that causes x) of arrival + table delay, the first
//              (j, y) attaining it (j ascending, rise first) and the worst
//              output transition; the arc delays are kept for the backward
//              pass
//   endpoint   per D pin: both slacks, the worse one is the endpoint's;
//              WNS / TNS / count by the single-transition reduction
//   backward   one launch per level from the top: a cell output's required
//              time per transition is the minimum over its sinks; each input
//              transition y then takes the minimum over the outputs x it
//              causes of (required x - arc delay); start points last
//   paths      the n worst endpoints (or the violated ones) ordered by
//              (slack, pin), cut to K; each path ends in its endpoint's worse
//              transition (rise on a tie) and follows the critical (input,
//              transition) back to a start point
//
// Per-pin arrays are [2 * pin + transition] in the device's pin order.
#include "tdp_impl.h"
#include "tdp_prims.h"
#include "tdp_walk.h"
#include "tdp_wave.h"

namespace tdp {

namespace {

inline int nb(long long n, int b) { return n > 0 ? (int)((n + b - 1) / b) : 1; }

__device__ __forceinline__ bool causes(int unate, int y, int x) { return unate == 2 || ((unate == 0) == (y == x)); }

template <typename T>
__global__ void k_rf_start(Topo tp, LutView Lr, LutView Lf, T in_slew, T clk_slew, const T *__restrict__ load,
                           T *__restrict__ at, T *__restrict__ slew) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= tp.n_start) return;
  if (v < tp.n_pi) {
    at[2 * v] = at[2 * v + 1] = (T)0;
    slew[2 * v] = slew[2 * v + 1] = in_slew;
    return;
  }
  const int ty = tp.ff_type[v - tp.n_pi];
  T a, so;
  lut_pair<T>(Lr, ty, clk_slew, load[v], a, so);
  at[2 * v] = a;
  slew[2 * v] = so;
  lut_pair<T>(Lf, ty, clk_slew, load[v], a, so);
  at[2 * v + 1] = a;
  slew[2 * v + 1] = so;
}

// cells [c0, c1) of one level
template <typename T>
__global__ void __launch_bounds__(256) k_rf_forward(Topo tp, LutView Lr, LutView Lf, int net_model,
                                                    const int32_t *__restrict__ unate, int c0, int c1,
                                                    const T *__restrict__ load, const T *__restrict__ dnet,
                                                    T *__restrict__ at, T *__restrict__ slew,
                                                    T *__restrict__ darc4, int32_t *__restrict__ crit) {
  const int c = c0 + blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= c1) return;
  const int o = tp.n_start + c;
  const int ty = tp.comb_type[c], un = unate[ty];
  const T ld = load[o];
  const int b = tp.comb_inptr[c], e = tp.comb_inptr[c + 1];
  T best[2] = {-pos_inf<T>(), -pos_inf<T>()}, so[2] = {(T)0, (T)0};
  int arg[2] = {-1, -1};
  for (int t = b; t < e; ++t) {
    const int s = tp.snk_drv[t];
    const T dn = dnet[t];
    const int p = tp.M + t;
    for (int y = 0; y < 2; ++y) {
      const T ain = at[2 * s + y] + dn;
      const T sin = sink_slew<T>(net_model, slew[2 * s + y], dn);
      at[2 * p + y] = ain;
      slew[2 * p + y] = sin;
      for (int x = 0; x < 2; ++x) {
        if (!causes(un, y, x)) continue;
        T d, os;
        lut_pair<T>(x == 0 ? Lr : Lf, ty, sin, ld, d, os);
        darc4[4 * t + 2 * x + y] = d;
        if (ain == -pos_inf<T>()) continue;
        const T a = ain + d;
        if (a > best[x]) {
          best[x] = a;
          arg[x] = 2 * (t - b) + y;
        }
        if (os > so[x]) so[x] = os;
      }
    }
  }
  for (int x = 0; x < 2; ++x) {
    at[2 * o + x] = best[x];
    slew[2 * o + x] = so[x];
    crit[2 * c + x] = arg[x];
  }
}

// D pins: arrivals, required times, the endpoint's (worse) slack
template <typename T>
__global__ void k_rf_endpoint(Topo tp, int net_model, const double *__restrict__ inst_req, const T *__restrict__ dnet,
                              T *__restrict__ at, T *__restrict__ slew, T *__restrict__ rat,
                              T *__restrict__ ep_slack) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= tp.E) return;
  const int t = tp.A + f, p = tp.M + t, s = tp.snk_drv[t];
  const T dn = dnet[t], req = (T)inst_req[tp.ff_inst[f]];
  T worst = pos_inf<T>();
  for (int y = 0; y < 2; ++y) {
    const T a = at[2 * s + y] + dn;
    at[2 * p + y] = a;
    slew[2 * p + y] = sink_slew<T>(net_model, slew[2 * s + y], dn);
    rat[2 * p + y] = req;
    if (a != -pos_inf<T>()) {
      const T sl = req - a;
      worst = sl < worst ? sl : worst;
    }
  }
  ep_slack[f] = worst;
}

// required time of driver v per transition: minimum over its sinks
template <typename T>
__device__ __forceinline__ void rf_driver_required(const Topo &tp, int v, const T *__restrict__ dnet,
                                                   T *__restrict__ rat) {
  T r[2] = {pos_inf<T>(), pos_inf<T>()};
  for (int k = tp.net_ptr[v]; k < tp.net_ptr[v + 1]; ++k) {
    const int t = tp.net_sink[k];
    const int p = tp.M + t;
    for (int y = 0; y < 2; ++y) {
      const T rt = rat[2 * p + y];
      if (rt == pos_inf<T>()) continue;
      const T q = rt - dnet[t];
      r[y] = q < r[y] ? q : r[y];
    }
  }
  rat[2 * v] = r[0];
  rat[2 * v + 1] = r[1];
}

template <typename T>
__global__ void __launch_bounds__(256) k_rf_backward(Topo tp, const int32_t *__restrict__ unate, int c0, int c1,
                                                     const T *__restrict__ dnet, const T *__restrict__ darc4,
                                                     T *__restrict__ rat) {
  const int c = c0 + blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= c1) return;
  const int o = tp.n_start + c;
  rf_driver_required<T>(tp, o, dnet, rat);
  const T ro[2] = {rat[2 * o], rat[2 * o + 1]};
  const int un = unate[tp.comb_type[c]];
  for (int t = tp.comb_inptr[c]; t < tp.comb_inptr[c + 1]; ++t) {
    const int p = tp.M + t;
    for (int y = 0; y < 2; ++y) {
      T r = pos_inf<T>();
      for (int x = 0; x < 2; ++x) {
        if (!causes(un, y, x) || ro[x] == pos_inf<T>()) continue;
        const T q = ro[x] - darc4[4 * t + 2 * x + y];
        r = q < r ? q : r;
      }
      rat[2 * p + y] = r;
    }
  }
}

template <typename T>
__global__ void k_rf_backward_start(Topo tp, const T *__restrict__ dnet, T *__restrict__ rat) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= tp.n_start) return;
  rf_driver_required<T>(tp, v, dnet, rat);
}

template <typename T>
__global__ void k_rf_export(Topo tp, const T *__restrict__ at, const T *__restrict__ rat,
                            const T *__restrict__ slew, double *__restrict__ o_at, double *__restrict__ o_rat,
                            double *__restrict__ o_slack, double *__restrict__ o_slew) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= tp.P) return;
  const int q = tp.ext_pin_int[p];
  for (int y = 0; y < 2; ++y) {
    const double a = (double)at[2 * q + y], r = (double)rat[2 * q + y];
    if (o_at) o_at[2 * p + y] = a;
    if (o_rat) o_rat[2 * p + y] = r;
    if (o_slew) o_slew[2 * p + y] = (double)slew[2 * q + y];
    if (o_slack) o_slack[2 * p + y] = (r == __builtin_huge_val() || a == -__builtin_huge_val()) ? __builtin_huge_val()
                                                                                              : r - a;
  }
}

// selected endpoints, ordered by slack (stable on the flip-flop index order of
// the compacted list, which is the pin order)
template <typename T>
__global__ void k_rf_sel_keys(const int32_t *__restrict__ d_nsel, const int32_t *__restrict__ sel,
                              const T *__restrict__ ep_slack, uint64_t *__restrict__ keys,
                              uint32_t *__restrict__ vals) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= *d_nsel) return;
  const int f = sel[i];
  keys[i] = sizeof(T) == 4 ? (order_key((float)ep_slack[f]) & 0xFFFFFFFFull) : order_key((double)ep_slack[f]);
  vals[i] = (uint32_t)f;
}

// endpoint f's path: its worse transition at the D pin, then critical
// (input, transition) pairs back to a start point
template <typename T>
__device__ __forceinline__ int rf_end_transition(const Topo &tp, int f, const T *__restrict__ at) {
  const int p = tp.M + tp.A + f;
  return at[2 * p] >= at[2 * p + 1] ? 0 : 1;  // equal slacks: rise
}

template <typename T>
__global__ void k_rf_path_len(Topo tp, int K, const int32_t *__restrict__ d_nsel, const uint32_t *__restrict__ order,
                              const T *__restrict__ at, const int32_t *__restrict__ crit, int32_t *__restrict__ len,
                              int32_t *__restrict__ d_num_paths) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int m = min(*d_nsel, K);
  if (i == 0) *d_num_paths = m;
  if (i >= m) return;
  const int f = (int)order[i];
  int y = rf_end_transition<T>(tp, f, at);
  int t = tp.A + f, n = 0;
  for (;;) {
    n += 2;
    const int s = tp.snk_drv[t];
    if (s < tp.n_start) break;
    const int c = s - tp.n_start, cr = crit[2 * c + y];
    if (cr < 0) break;
    t = tp.comb_inptr[c] + (cr >> 1);
    y = cr & 1;
  }
  len[i] = n;
}

template <typename T>
__global__ void k_rf_walk(Topo tp, const int32_t *__restrict__ d_num_paths, const uint32_t *__restrict__ order,
                          const T *__restrict__ at, const T *__restrict__ ep_slack, const int32_t *__restrict__ crit,
                          const int32_t *__restrict__ path_ptr, int32_t *__restrict__ path_pins,
                          int32_t *__restrict__ path_int, uint8_t *__restrict__ path_tran,
                          int32_t *__restrict__ path_ep, int32_t *__restrict__ path_epi,
                          int32_t *__restrict__ path_rank, T *__restrict__ path_slack, int32_t *__restrict__ slot_out,
                          int32_t *__restrict__ err, int pin_cap) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= *d_num_paths) return;
  const int f = (int)order[i];
  const int lo = path_ptr[i], hi = path_ptr[i + 1];
  if (lo < 0 || hi > pin_cap || hi - lo < 2) {
    atomicOr(err, 1);
    return;
  }
  int y = rf_end_transition<T>(tp, f, at);
  int t = tp.A + f, w = hi - 1;
  for (;;) {
    const int s = tp.snk_drv[t];
    if (w - 1 < lo) {
      atomicOr(err, 1);
      return;
    }
    path_pins[w] = tp.snk_ext[t];
    path_int[w] = tp.M + t;
    path_tran[w] = (uint8_t)y;
    path_pins[w - 1] = tp.drv_ext[s];
    path_int[w - 1] = s;
    path_tran[w - 1] = (uint8_t)y;
    w -= 2;
    if (s < tp.n_start) break;
    const int c = s - tp.n_start, cr = crit[2 * c + y];
    if (cr < 0) break;
    t = tp.comb_inptr[c] + (cr >> 1);
    y = cr & 1;
  }
  if (w != lo - 1) atomicOr(err, 1);
  path_ep[i] = tp.snk_ext[tp.A + f];
  path_epi[i] = f;
  path_rank[i] = 0;
  path_slack[i] = ep_slack[f];
  slot_out[i] = i;
}

__global__ void k_rf_nslots(const int32_t *__restrict__ d_num_paths, int32_t *__restrict__ d_nslots) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *d_nslots = *d_num_paths;
}

}  // namespace

template <typename T>
void rf_update_impl(tdp_graph g, const float *x, const float *y, hipStream_t s) {
  const Topo &tp = g->topo;
  netpass_impl<T>(g, x, y, s);
  LutView Lf = g->lut;
  Lf.delay = g->rf_delay_fall;
  Lf.slew = g->rf_slew_fall;
  T *at = (T *)g->rf_at, *sl = (T *)g->rf_slew, *rat = (T *)g->rf_rat, *darc4 = (T *)g->rf_darc4;
  if (tp.n_start > 0)
    hipLaunchKernelGGL(k_rf_start<T>, dim3(nb(tp.n_start, 256)), dim3(256), 0, s, tp, g->lut, Lf, (T)g->input_slew,
                       (T)g->clock_slew, (const T *)g->load, at, sl);
  for (int l = 1; l <= tp.D; ++l) {
    const int c0 = g->lv.lvl[l - 1], c1 = g->lv.lvl[l];
    if (c1 > c0)
      hipLaunchKernelGGL(k_rf_forward<T>, dim3(nb(c1 - c0, 256)), dim3(256), 0, s, tp, g->lut, Lf, g->lut.net_model,
                         g->rf_unate, c0, c1, (const T *)g->load, (const T *)g->dnet, at, sl, darc4, g->rf_crit);
  }
  if (tp.E > 0)
    hipLaunchKernelGGL(k_rf_endpoint<T>, dim3(nb(tp.E, 256)), dim3(256), 0, s, tp, g->lut.net_model, g->d_inst_req,
                       (const T *)g->dnet, at, sl, rat, (T *)g->ep_slack);
  ep_reduce_impl<T>(g, s);
  for (int l = tp.D; l >= 1; --l) {
    const int c0 = g->lv.lvl[l - 1], c1 = g->lv.lvl[l];
    if (c1 > c0)
      hipLaunchKernelGGL(k_rf_backward<T>, dim3(nb(c1 - c0, 256)), dim3(256), 0, s, tp, g->rf_unate, c0, c1,
                         (const T *)g->dnet, (const T *)darc4, rat);
  }
  if (tp.n_start > 0)
    hipLaunchKernelGGL(k_rf_backward_start<T>, dim3(nb(tp.n_start, 256)), dim3(256), 0, s, tp, (const T *)g->dnet,
                       rat);
}

template <typename T>
void rf_export_impl(tdp_graph g, double *at, double *rat, double *slack, double *slew, hipStream_t s) {
  hipLaunchKernelGGL(k_rf_export<T>, dim3(nb(g->topo.P, 256)), dim3(256), 0, s, g->topo, (const T *)g->rf_at,
                     (const T *)g->rf_rat, (const T *)g->rf_slew, at, rat, slack, slew);
}

template <typename T>
void rf_extract_impl(tdp_graph g, int n, int K, hipStream_t s) {
  const Topo &tp = g->topo;
  select_stage<T>(g, n, s);
  hipLaunchKernelGGL(k_rf_sel_keys<T>, dim3(nb(tp.E, 256)), dim3(256), 0, s, g->d_nsel, g->sel_list,
                     (const T *)g->ep_slack, g->sort_k0, g->sort_v0);
  radix_sort(g->sort_k0, g->sort_v0, g->sort_k1, g->sort_v1, tp.E, g->d_nsel, sizeof(T) == 4 ? 32 : 64,
             g->sort_hist, g->scan_tmp, s);
  const int cap = std::min(K, g->max_out);
  hipLaunchKernelGGL(k_rf_path_len<T>, dim3(nb(cap, 256)), dim3(256), 0, s, tp, cap, g->d_nsel, g->sort_v0,
                     (const T *)g->rf_at, g->rf_crit, g->out_len, g->d_num_paths);
  scan_exclusive(g->out_len, g->path_ptr, g->max_out, g->d_num_paths, nullptr, g->scan_tmp, s);
  ptr_tail(g->d_num_paths, g->out_len, g->path_ptr, s);
  hipLaunchKernelGGL(k_rf_walk<T>, dim3(nb(cap, 256)), dim3(256), 0, s, tp, g->d_num_paths, g->sort_v0,
                     (const T *)g->rf_at, (const T *)g->ep_slack, g->rf_crit, g->path_ptr, g->path_pins, g->path_int,
                     g->rf_path_tran, g->path_ep, g->path_epi, g->path_rank, (T *)g->path_slack, g->slot_out, g->d_err,
                     g->pin_cap);
  hipLaunchKernelGGL(k_rf_nslots, dim3(1), dim3(1), 0, s, g->d_num_paths, g->d_nslots);
}

template void rf_update_impl<float>(tdp_graph, const float *, const float *, hipStream_t);
template void rf_update_impl<double>(tdp_graph, const float *, const float *, hipStream_t);
template void rf_export_impl<float>(tdp_graph, double *, double *, double *, double *, hipStream_t);
template void rf_export_impl<double>(tdp_graph, double *, double *, double *, double *, hipStream_t);
template void rf_extract_impl<float>(tdp_graph, int, int, hipStream_t);
template void rf_extract_impl<double>(tdp_graph, int, int, hipStream_t);

}  // namespace tdp
