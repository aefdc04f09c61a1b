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
//   forward    one launch per level, one lane per combinational input (the
//              forward chunks): sinks take their drivers' arrivals plus the
//              net delay; for each
//              output transition x, the maximum over (input j, input
//              transition y that causes x) of arrival + table delay, the first
//              (j, y) attaining it (j ascending, rise first) and the worst
//              output transition; the arc delays are kept for the backward
//              pass
//   endpoint   per D pin: both slacks, the worse one is the endpoint's;
//              WNS / TNS / count by the single-transition reduction
//   backward   one launch per level from the top, one lane per pin of the
//              nets driven at that level (the net chunks): an input
//              transition y of a sink's cell takes the minimum over the
//              outputs x it causes of (required x - arc delay), and the
//              driver's required time per transition is the minimum over its
//              sinks of (required - net delay); start points last
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

// One level of the forward pass on the forward chunks: one lane per
// combinational input (a cell's inputs on consecutive lanes), both
// transitions' tables staged in LDS, and the cell's maxima by segmented
// reductions over its lanes.  Candidate (j, y) of an
// output transition carries the index 2 j + y; among equal arrivals the
// smallest index wins (j ascending, rise first), as in the per-cell loop.
template <typename T>
__global__ void __launch_bounds__(256) k_rf_forward_chunks(Topo tp, LutView Lr, LutView Lf, int net_model,
                                                           const int32_t *__restrict__ unate, int ch0, int ch1,
                                                           const T *__restrict__ load, const T *__restrict__ dnet,
                                                           T *__restrict__ at, T *__restrict__ slew,
                                                           T *__restrict__ darc4, int32_t *__restrict__ crit) {
  extern __shared__ float4 s_rf4[];
  float *s_r = (float *)s_rf4, *s_f = (float *)(s_rf4 + Lr.n4);
  const int lane = wave_lane();
  const int chunk = ch0 + blockIdx.x * 4 + (threadIdx.x >> 6);
  const int4 rec = tp.fw_rec[(chunk < ch1 ? chunk : ch1 - 1) * CHUNK + lane];
  const int t = rec.x, s = rec.y, c = rec.z;
  const int head = rec.w & 63, tail = (rec.w >> 8) & 63;
  const bool valid = t >= 0 && chunk < ch1;
  T a2[2] = {(T)0, (T)0}, w2[2] = {(T)0, (T)0}, dn = 0, ld = 0;
  int ty = 0;
  if (valid) {
    a2[0] = at[2 * s];
    a2[1] = at[2 * s + 1];
    w2[0] = slew[2 * s];
    w2[1] = slew[2 * s + 1];
    dn = dnet[t];
    ld = load[tp.n_start + c];
    ty = tp.comb_type[c];
  }
  stage_lut(Lr, s_r);
  stage_lut(Lf, s_f);
  if (chunk >= ch1) return;
  const int un = valid ? unate[ty] : 0;
  const int j = lane - head;
  // this lane's best candidate per output transition and its worst
  // output transition
  T cand[2] = {-pos_inf<T>(), -pos_inf<T>()}, osx[2] = {(T)0, (T)0};
  int cidx[2] = {1 << 20, 1 << 20};
  if (valid) {
    const int p = tp.M + t;
    T ain[2], sin[2];
#pragma unroll
    for (int y = 0; y < 2; ++y) {
      ain[y] = a2[y] + dn;
      sin[y] = sink_slew<T>(net_model, w2[y], dn);
    }
    at[2 * p] = ain[0];
    at[2 * p + 1] = ain[1];
    slew[2 * p] = sin[0];
    slew[2 * p + 1] = sin[1];
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int x = 0; x < 2; ++x) {
        if (!causes(un, y, x)) continue;
        T d, os;
        lut_lds<T>(x == 0 ? s_r : s_f, Lr.nt, Lr.ns, Lr.nl, ty, sin[y], ld, d, os);
        darc4[4 * t + 2 * x + y] = d;
        if (ain[y] == -pos_inf<T>()) continue;
        const T a = ain[y] + d;
        if (a > cand[x]) {  // y ascending: a tie keeps the rise
          cand[x] = a;
          cidx[x] = 2 * j + y;
        }
        if (os > osx[x]) osx[x] = os;
      }
  }
#pragma unroll
  for (int x = 0; x < 2; ++x) {
    const T best = seg_max(cand[x], lane, head, tail);
    const T so = seg_max(osx[x], lane, head, tail);
    const int arg = seg_min((valid && cand[x] == best && best != -pos_inf<T>()) ? cidx[x] : (1 << 20), lane, head,
                            tail);
    if (valid && lane == head) {
      const int o = tp.n_start + c;
      at[2 * o + x] = best;
      slew[2 * o + x] = so;
      crit[2 * c + x] = arg < (1 << 20) ? arg : -1;
    }
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

// required times of an input pin's two transitions from its cell output's
// and the arc delays [x][y]
template <typename T>
__device__ __forceinline__ void rf_input_required(int un, const T (&ro)[2], const T (&da)[4], T (&r)[2]) {
#pragma unroll
  for (int y = 0; y < 2; ++y) {
    r[y] = pos_inf<T>();
#pragma unroll
    for (int x = 0; x < 2; ++x) {
      if (!causes(un, y, x) || ro[x] == pos_inf<T>()) continue;
      const T q = ro[x] - da[2 * x + y];
      r[y] = q < r[y] ? q : r[y];
    }
  }
}

// One level of the backward pass on the net chunks: one lane per pin of a
// net driven at this level.  A sink that is a combinational input takes its
// required times from its cell's output (a later level, already done) and
// the arc delays; a D pin's are the endpoint's.  The driver's are the
// minimum over its sinks of required - net delay.
template <typename T>
__global__ void __launch_bounds__(256) k_rf_backward_chunks(Topo tp, const int32_t *__restrict__ unate, int ch0,
                                                            int ch1, const T *__restrict__ dnet_nm,
                                                            const T *__restrict__ darc4, T *__restrict__ rat) {
  const int lane = wave_lane();
  const int chunk = ch0 + blockIdx.x * 4 + (threadIdx.x >> 6);
  if (chunk >= ch1) return;
  const int k = chunk * CHUNK + lane;
  const int4 rec = tp.nm_rec[k];
  const int p = rec.x, vo = rec.z;
  const int head = rec.w & 63, tail = (rec.w >> 8) & 63;
  const bool sink = p >= 0 && lane != head;
  const int t = p - tp.M;
  T q[2] = {pos_inf<T>(), pos_inf<T>()};
  if (sink) {
    const T dn = dnet_nm[k];
    T r[2];
    if (vo >= 0) {  // a combinational input
      const T ro[2] = {rat[2 * vo], rat[2 * vo + 1]};
      T da[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) da[i] = darc4[4 * t + i];
      rf_input_required<T>(unate[tp.comb_type[vo - tp.n_start]], ro, da, r);
      rat[2 * p] = r[0];
      rat[2 * p + 1] = r[1];
    } else {
      r[0] = rat[2 * p];
      r[1] = rat[2 * p + 1];
    }
#pragma unroll
    for (int y = 0; y < 2; ++y)
      if (r[y] != pos_inf<T>()) q[y] = r[y] - dn;
  }
  const T r0 = seg_min(q[0], lane, head, tail), r1 = seg_min(q[1], lane, head, tail);
  if (p >= 0 && lane == head) {
    rat[2 * p] = r0;
    rat[2 * p + 1] = r1;
  }
}

// nets too wide for one chunk: one thread per net, the same arithmetic
template <typename T>
__global__ void k_rf_backward_big(Topo tp, const int32_t *__restrict__ unate, int i0, int i1,
                                  const T *__restrict__ dnet, const T *__restrict__ darc4, T *__restrict__ rat) {
  const int i = i0 + blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= i1) return;
  const int v = tp.big_net[i];
  T q[2] = {pos_inf<T>(), pos_inf<T>()};
  for (int kk = tp.net_ptr[v]; kk < tp.net_ptr[v + 1]; ++kk) {
    const int t = tp.net_sink[kk];
    const int p = tp.M + t;
    T r[2];
    if (t < tp.A) {
      const int c = tp.snk_comb[t], vo = tp.n_start + c;
      const T ro[2] = {rat[2 * vo], rat[2 * vo + 1]};
      T da[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) da[j] = darc4[4 * t + j];
      rf_input_required<T>(unate[tp.comb_type[c]], ro, da, r);
      rat[2 * p] = r[0];
      rat[2 * p + 1] = r[1];
    } else {
      r[0] = rat[2 * p];
      r[1] = rat[2 * p + 1];
    }
#pragma unroll
    for (int y = 0; y < 2; ++y)
      if (r[y] != pos_inf<T>()) {
        const T qq = r[y] - dnet[t];
        q[y] = qq < q[y] ? qq : q[y];
      }
  }
  rat[2 * v] = q[0];
  rat[2 * v + 1] = q[1];
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
  // the fall tables' view: the same axes, its own image for the LDS staging
  LutView Lf = g->lut;
  Lf.slew_axis = (const float *)g->rf_flat;
  Lf.load_axis = (const float *)g->rf_flat + (size_t)g->lut.nt * g->lut.ns;
  Lf.delay = g->rf_delay_fall;
  Lf.slew = g->rf_slew_fall;
  Lf.flat4 = g->rf_flat;
  T *at = (T *)g->rf_at, *sl = (T *)g->rf_slew, *rat = (T *)g->rf_rat, *darc4 = (T *)g->rf_darc4;
  if (tp.n_start > 0)
    hipLaunchKernelGGL(k_rf_start<T>, dim3(nb(tp.n_start, 256)), dim3(256), 0, s, tp, g->lut, Lf, (T)g->input_slew,
                       (T)g->clock_slew, (const T *)g->load, at, sl);
  for (int l = 1; l <= tp.D; ++l) {
    const int ch0 = g->lv.fw_lvl[l - 1], ch1 = g->lv.fw_lvl[l];
    if (ch1 > ch0)
      hipLaunchKernelGGL(k_rf_forward_chunks<T>, dim3(nb(ch1 - ch0, 4)), dim3(256), 2 * sizeof(float4) * g->lut.n4,
                         s, tp, g->lut, Lf, g->lut.net_model, g->rf_unate, ch0, ch1, (const T *)g->load,
                         (const T *)g->dnet, at, sl, darc4, g->rf_crit);
  }
  if (tp.E > 0)
    hipLaunchKernelGGL(k_rf_endpoint<T>, dim3(nb(tp.E, 256)), dim3(256), 0, s, tp, g->lut.net_model, g->d_inst_req,
                       (const T *)g->dnet, at, sl, rat, (T *)g->ep_slack);
  ep_reduce_impl<T>(g, s);
  // from the last level's nets down to the start points' (level 0)
  for (int l = tp.D; l >= 0; --l) {
    const int ch0 = g->lv.nm_lvl[l], ch1 = g->lv.nm_lvl[l + 1];
    if (ch1 > ch0)
      hipLaunchKernelGGL(k_rf_backward_chunks<T>, dim3(nb(ch1 - ch0, 4)), dim3(256), 0, s, tp, g->rf_unate, ch0, ch1,
                         (const T *)g->dnet_nm, (const T *)darc4, rat);
    const int b0 = g->lv.big_lvl[l], b1 = g->lv.big_lvl[l + 1];
    if (b1 > b0)
      hipLaunchKernelGGL(k_rf_backward_big<T>, dim3(nb(b1 - b0, 64)), dim3(64), 0, s, tp, g->rf_unate, b0, b1,
                         (const T *)g->dnet, (const T *)darc4, rat);
  }
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
