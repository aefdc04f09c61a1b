// Declarations shared by the kernel files and the entry points.
#pragma once

#include <algorithm>

#include "tdp_internal.h"

namespace tdp {

// stage timing with HIP events on the caller's stream
inline void prof_begin(tdp_graph g, int stage, hipStream_t s) {
  if (!g->prof.on || !((g->prof.mask >> stage) & 1)) return;
  hipEvent_t a = g->prof.take();
  if (!a) return;
  hipEventRecord(a, s);
  g->prof.open[stage] = a;
}
inline void prof_end(tdp_graph g, int stage, hipStream_t s) {
  if (!g->prof.on || !g->prof.open[stage]) return;
  hipEvent_t b = g->prof.take();
  if (!b) return;
  hipEventRecord(b, s);
  g->prof.marks.push_back({stage, g->prof.open[stage], b});
  g->prof.open[stage] = nullptr;
}

template <typename T> void netpass_impl(tdp_graph g, const float *x, const float *y, hipStream_t s);
// spanning-tree net model, one thread per net: the net delays of every net
// (list null) or of the n nets listed, and the trees' lengths
template <typename T>
void tree_net_impl(tdp_graph g, const TreeBuf &b, const float *x, const float *y, T *dnet, const int32_t *list,
                   int n, hipStream_t s);
// the smoothed TNS's net delays at positions (x, y), in the graph's net model
template <typename T>
void st_net_fwd_impl(tdp_graph g, const float *x, const float *y, T *dnl, hipStream_t s);
// the smoothed TNS's gradient per pin and axis (into st_gp) from the adjoint
// of the net delays, at the positions of the last st_net_fwd_impl call (its
// packed copy; x and y serve the nets wider than a chunk)
template <typename T>
void st_net_grad_impl(tdp_graph g, const float *x, const float *y, const T *adj, hipStream_t s);
// WNS / TNS / violated count per instance from the endpoint slacks
template <typename T> void ep_reduce_impl(tdp_graph g, hipStream_t s);
template <typename T> void rf_update_impl(tdp_graph g, const float *x, const float *y, hipStream_t s);
template <typename T>
void rf_export_impl(tdp_graph g, double *at, double *rat, double *slack, double *slew, hipStream_t s);
template <typename T> void rf_extract_impl(tdp_graph g, int n, int K, hipStream_t s);
template <typename T> void sta_arrivals_impl(tdp_graph g, const float *x, const float *y, hipStream_t s);
template <typename T>
void sta_arrivals_incremental_impl(tdp_graph g, const float *x, const float *y, const int32_t *cells, int n,
                                   hipStream_t s);
void inc_maps(tdp_graph g, hipStream_t s);
template <typename T> void sta_required_impl(tdp_graph g, hipStream_t s);
template <typename T>
void sta_export_impl(tdp_graph g, double *at, double *rat, double *slack, double *slew, double *dnet,
                     double *load, double *darc, hipStream_t s);
void sta_export_crit(tdp_graph g, int32_t *out, hipStream_t s);
template <typename T> void extract_impl(tdp_graph g, int n, int k, int K, float slack_limit, hipStream_t s);
template <typename T> void select_stage(tdp_graph g, int n, hipStream_t s);
template <typename T> void search_stage(tdp_graph g, int k, float slack_limit, hipStream_t s);
template <typename T> void slot_sort_stage(tdp_graph g, int k, hipStream_t s);
void ptr_tail(const int32_t *d_num_paths, const int32_t *len, int32_t *ptr, hipStream_t s);
// report_timing(K)'s node store and its sort / scan scratch: the graph's own
// (allocated by the first call) or carved from the fixed device array of the
// no-allocation entry point
struct GtStore {
  int cap = 0;  // nodes
  void *gt_cost = nullptr, *gt_key = nullptr, *gt_theta = nullptr;
  int32_t *gt_dev = nullptr, *gt_par = nullptr, *gt_ep = nullptr, *gt_cells = nullptr, *gt_nd = nullptr;
  int32_t *gt_cnt = nullptr, *gt_off = nullptr, *gt_start = nullptr, *gt_end = nullptr, *gt_misc = nullptr;
  uint64_t *gt_k0 = nullptr, *gt_k1 = nullptr;
  uint32_t *gt_v0 = nullptr, *gt_v1 = nullptr;
  int32_t *gt_hist = nullptr, *gt_scan = nullptr;
};
// node capacity report_timing(K) uses for graph g
int report_node_cap(const tdp_graph_s *g);
// report_timing(K); returns a status (it synchronises on s)
template <typename T> tdp_status report_impl(tdp_graph g, const GtStore &st, int K, float slack_limit, hipStream_t s);
template <typename T> void pairs_update_impl(tdp_graph g, int rule, float w0, float w1, hipStream_t s);
void pairs_rebuild(tdp_graph g, hipStream_t s);
void pairs_compact(tdp_graph g, hipStream_t s);
template <typename T>
void p2p_fwd_impl(tdp_graph g, int kind, const float *x, const float *y, double *loss, hipStream_t s);
template <typename T>
void p2p_bwd_impl(tdp_graph g, int kind, const float *x, const float *y, const double *gout, float *gx, float *gy,
                  hipStream_t s);
template <typename T>
void stns_fwd_impl(tdp_graph g, const float *x, const float *y, float gamma, double *val, hipStream_t s);
template <typename T> void stns_bwd_impl(tdp_graph g, const double *gout, float *gx, float *gy, hipStream_t s);
void wa_impl(tdp_graph g, const float *x, const float *y, float gamma, double *wl, float *gx, float *gy,
             hipStream_t s);
void density_impl(tdp_graph g, const float *x, const float *y, float scale, double *value, double *overflow,
                  float *gx, float *gy, float *map_out, hipStream_t s);
void nesterov_impl(tdp_graph g, const float *gx, const float *gy, const float *pdiv, float *vx, float *vy, float *ux,
                   float *uy, float *vpx, float *vpy, float *gpx, float *gpy, double coef, double alpha0, int first,
                   float xlo, float xhi, float ylo, float yhi, double *alpha_out, hipStream_t s);
void abs_sum_impl(tdp_graph g, const float *a, const float *b, double *out, hipStream_t s);
int density_parts();
template <typename T> void early_impl(tdp_graph g, float hold, hipStream_t s);
template <typename T>
void early_export_impl(tdp_graph g, double *at, double *slew, double *darc, double *hold_slack, hipStream_t s);
int early_parts();

}  // namespace tdp
