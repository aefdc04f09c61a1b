// Early (hold) analysis: the other half of an early/late timer, on the net
// delays and loads of the last timing update.  Start points arrive as in the
// late sweep; a sink arrives at its driver's early arrival plus the net
// delay, with the transition the net model gives a sink from its driver's
// early transition; a combinational output takes the minimum over its
// inputs of (input arrival + table delay at the input's early transition and
// the output's load), and the minimum of the table transitions (best case).
// At a D pin the hold check (ideal clock) is: hold slack = early arrival -
// hold time.  WHS / THS / count are over every D pin of the graph.
//
// One launch per level over the same 64-lane input chunks as the late sweep:
// a lane per combinational input, the cell's minima as segmented reductions.
// Reductions are fixed-order: results are bitwise reproducible.
#include "tdp_impl.h"
#include "tdp_wave.h"

namespace tdp {

static inline int nbe(long long n, int b) { return n > 0 ? (int)((n + b - 1) / b) : 1; }

constexpr int EA_BLOCK = 256;
constexpr int EA_PARTS = 512;

template <typename T>
__global__ void __launch_bounds__(EA_BLOCK) k_early_start(Topo tp, const V2<T> *__restrict__ as, V2<T> *__restrict__ es) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v < tp.n_start) es[v] = as[v];
}

template <typename T>
__global__ void __launch_bounds__(EA_BLOCK) k_early_level(Topo tp, LutView L, int ch0, int ch1,
                                                           const T *__restrict__ load, const T *__restrict__ dnet,
                                                           V2<T> *__restrict__ es, T *__restrict__ at_snk,
                                                           T *__restrict__ darc) {
  const int lane = wave_lane();
  const int chunk = ch0 + blockIdx.x * (EA_BLOCK / 64) + (threadIdx.x >> 6);
  if (chunk >= ch1) return;
  const int4 rec = tp.fw_rec[chunk * CHUNK + lane];
  const int t = rec.x, s = rec.y, c = rec.z;
  const int head = rec.w & 63, tail = (rec.w >> 8) & 63;
  const bool valid = t >= 0;
  T a = pos_inf<T>(), o = pos_inf<T>();
  if (valid) {
    const T ld = load[tp.n_start + c];
    const V2<T> w = es[s];
    const T dn = dnet[t];
    const T a_in = w.x + dn;
    T d;
    lut_pair<T>(L, (rec.w >> 16) & 255, sink_slew<T>(L.net_model, w.y, dn), ld, d, o);
    at_snk[t] = a_in;
    darc[t] = d;
    a = a_in + d;
  }
  const T best = seg_min(a, lane, head, tail);
  const T so = seg_min(o, lane, head, tail);
  if (valid && lane == head) es[tp.n_start + c] = v2<T>(best, so);
}

// D pins: early arrival and hold slack; per-block partials of
// {min slack, sum of negative slacks, count of negative slacks}
template <typename T>
__global__ void __launch_bounds__(EA_BLOCK) k_early_end(Topo tp, const V2<T> *__restrict__ es,
                                                         const T *__restrict__ dnet, T hold, T *__restrict__ at_snk,
                                                         double *__restrict__ part) {
  __shared__ double s_min[EA_BLOCK], s_sum[EA_BLOCK], s_cnt[EA_BLOCK];
  double mn = 0.0, sm = 0.0, ct = 0.0;
  for (int f = blockIdx.x * EA_BLOCK + threadIdx.x; f < tp.E; f += EA_PARTS * EA_BLOCK) {
    const int t = tp.A + f;
    const T a = es[tp.snk_drv[t]].x + dnet[t];
    at_snk[t] = a;
    const T h = a - hold;
    if (h < (T)0) {
      mn = fmin(mn, (double)h);
      sm += (double)h;
      ct += 1.0;
    }
  }
  s_min[threadIdx.x] = mn;
  s_sum[threadIdx.x] = sm;
  s_cnt[threadIdx.x] = ct;
  __syncthreads();
  for (int k = EA_BLOCK / 2; k > 0; k >>= 1) {
    if (threadIdx.x < k) {
      s_min[threadIdx.x] = fmin(s_min[threadIdx.x], s_min[threadIdx.x + k]);
      s_sum[threadIdx.x] += s_sum[threadIdx.x + k];
      s_cnt[threadIdx.x] += s_cnt[threadIdx.x + k];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[blockIdx.x] = s_min[0];
    part[EA_PARTS + blockIdx.x] = s_sum[0];
    part[2 * EA_PARTS + blockIdx.x] = s_cnt[0];
  }
}

__global__ void k_early_final(const double *__restrict__ part, double *__restrict__ summary) {
  if (threadIdx.x != 0) return;
  double mn = 0.0, sm = 0.0, ct = 0.0;
  for (int i = 0; i < EA_PARTS; ++i) {
    mn = fmin(mn, part[i]);
    sm += part[EA_PARTS + i];
    ct += part[2 * EA_PARTS + i];
  }
  summary[0] = mn;
  summary[1] = sm;
  summary[2] = ct;
}

template <typename T>
__global__ void __launch_bounds__(EA_BLOCK) k_early_export(Topo tp, int net_model, const V2<T> *__restrict__ es,
                                                            const T *__restrict__ at_snk, const T *__restrict__ darc,
                                                            const T *__restrict__ dnet, T hold, double *o_at,
                                                            double *o_slew, double *o_darc, double *o_hold) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= tp.P) return;
  const int i = tp.ext_pin_int[p];
  const bool sink = i >= tp.M;
  const int t = i - tp.M;
  if (o_at) o_at[p] = (double)(sink ? at_snk[t] : es[i].x);
  if (o_slew) o_slew[p] = (double)(sink ? sink_slew<T>(net_model, es[tp.snk_drv[t]].y, dnet[t]) : es[i].y);
  if (o_darc) o_darc[p] = (sink && t < tp.A) ? (double)darc[t] : 0.0;
  if (o_hold) o_hold[p] = (sink && t >= tp.A) ? (double)(at_snk[t] - hold) : (double)pos_inf<T>();
}

template <typename T>
void early_impl(tdp_graph g, float hold, hipStream_t s) {
  const Topo &tp = g->topo;
  V2<T> *es = (V2<T> *)g->ea_as;
  T *at_snk = (T *)g->ea_at, *darc = (T *)g->ea_darc;
  if (tp.n_start > 0)
    hipLaunchKernelGGL(k_early_start<T>, dim3(nbe(tp.n_start, EA_BLOCK)), dim3(EA_BLOCK), 0, s, tp,
                       (const V2<T> *)g->drv_as, es);
  for (int l = 1; l <= tp.D; ++l) {
    const int ch0 = g->lv.fw_lvl[l - 1], ch1 = g->lv.fw_lvl[l];
    if (ch1 > ch0)
      hipLaunchKernelGGL(k_early_level<T>, dim3(nbe(ch1 - ch0, EA_BLOCK / 64)), dim3(EA_BLOCK), 0, s, tp, g->lut,
                         ch0, ch1, (const T *)g->load, (const T *)g->dnet, es, at_snk, darc);
  }
  hipLaunchKernelGGL(k_early_end<T>, dim3(EA_PARTS), dim3(EA_BLOCK), 0, s, tp, (const V2<T> *)es,
                     (const T *)g->dnet, (T)hold, at_snk, g->ea_part);
  hipLaunchKernelGGL(k_early_final, dim3(1), dim3(64), 0, s, (const double *)g->ea_part, g->ea_summary);
}

template <typename T>
void early_export_impl(tdp_graph g, double *at, double *slew, double *darc, double *hold_slack, hipStream_t s) {
  const Topo &tp = g->topo;
  hipLaunchKernelGGL(k_early_export<T>, dim3(nbe(tp.P, EA_BLOCK)), dim3(EA_BLOCK), 0, s, tp, g->lut.net_model,
                     (const V2<T> *)g->ea_as, (const T *)g->ea_at, (const T *)g->ea_darc, (const T *)g->dnet,
                     (T)g->ea_hold, at, slew, darc, hold_slack);
}

int early_parts() { return EA_PARTS; }

template void early_impl<float>(tdp_graph, float, hipStream_t);
template void early_impl<double>(tdp_graph, float, hipStream_t);
template void early_export_impl<float>(tdp_graph, double *, double *, double *, double *, hipStream_t);
template void early_export_impl<double>(tdp_graph, double *, double *, double *, double *, hipStream_t);

}  // namespace tdp
