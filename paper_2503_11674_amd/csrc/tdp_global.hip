// report_timing(K) on the device: the K worst paths over the whole design
// (Sec. III-B, Table I), however many fall on one endpoint.
//
// Every path is a node of its endpoint's deviation tree (a path's parent is
// itself without its upstream-most deviation; its children add one deviation
// on the critical chain above that point), and a child's slack is never below
// its parent's.  So, given a bound theta on the K-th smallest slack, the
// answer is the K smallest of the nodes with slack <= theta, and those form
// a top part of every tree that a breadth-first expansion finds exactly:
//
//   bound      the per-endpoint search (k = max_k at the K worst endpoints)
//              yields real paths; the K-th smallest of their slacks is an
//              upper bound on the true K-th slack
//   expand     rounds of count / scan / emit over the frontier; a node's
//              children within the bound come from its chain start's list
//              of cheapest deviations when that list is known to hold them
//              all, otherwise from a walk up the critical chain
//   refine     if the node store overflows, the K-th smallest slack among
//              the stored nodes (real paths again) is a tighter bound, and
//              the expansion restarts under it
//   order      sort by (instance, slack), cut to K, walk, rank per endpoint
//
// Node order is fixed by the rounds (scan positions, list / chain order), so
// equal slacks come out in the same order on every run.  The call reads a
// counter back to the host per round and so synchronises its stream.
#include "tdp_impl.h"
#include "tdp_prims.h"
#include "tdp_walk.h"

namespace tdp {

namespace {

inline int nb(long long n, int b) { return n > 0 ? (int)((n + b - 1) / b) : 1; }

tdp_status gt_fail(tdp_graph g, tdp_status st, const char *msg) {
  g->last_error = msg;
  return st;
}

template <typename T>
struct Nodes {
  T *cost, *key;           // deviation cost sum; path slack = endpoint slack + cost
  int32_t *dev, *par;      // upstream-most deviation (sink pin, -1 at a root); parent node
  int32_t *ep, *cells, *ndev;  // endpoint (flip-flop index); cells on the path; deviation count
};

template <typename T>
struct Ctx {
  const T *at, *darc, *side_cost, *ep_slack, *theta;
  const int32_t *crit, *side_pin, *cdep;
  T limit;
};

// per instance: the K-th smallest slack among the per-endpoint candidates
// (sorted by (instance, slack); unfound slots are +inf and sort last), or
// +inf when fewer than K were found
template <typename T>
__global__ void k_gt_theta0(int num_inst, int k, int K, const int32_t *__restrict__ inst_nsel,
                            const int32_t *__restrict__ inst_nvalid, const uint32_t *__restrict__ perm,
                            const T *__restrict__ slot_key, T *__restrict__ theta) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  int s = 0;
  for (int i = 0; i < num_inst; ++i) {
    theta[i] = inst_nvalid[i] >= K ? slot_key[perm[s + K - 1]] : inf_of<T>();
    s += inst_nsel[i] * k;
  }
}

template <typename T>
__global__ void k_gt_root_flags(Topo tp, const T *__restrict__ ep_slack, const T *__restrict__ theta, T limit,
                                int32_t *__restrict__ flag) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= tp.E) return;
  const T s = ep_slack[f];
  flag[f] = (s < inf_of<T>() && s <= theta[tp.ff_inst[f]] && s < limit) ? 1 : 0;
}

// the roots: each endpoint's critical path
template <typename T>
__global__ void k_gt_roots(Topo tp, const int32_t *__restrict__ flag, const int32_t *__restrict__ pos,
                           const T *__restrict__ ep_slack, const int32_t *__restrict__ cdep, int cap, Nodes<T> nd) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= tp.E || !flag[f]) return;
  const int i = pos[f];
  if (i >= cap) return;
  nd.cost[i] = (T)0;
  nd.key[i] = ep_slack[f];
  nd.dev[i] = -1;
  nd.par[i] = -1;
  nd.ep[i] = f;
  nd.cells[i] = cdep[tp.snk_drv[tp.A + f]];
  nd.ndev[i] = 0;
}

// Children of node i within the bound: one more deviation on the critical
// chain from its chain start u up to the start point.  The chain start's list
// of its KM cheapest deviations is ascending, so the children are a prefix
// of it, unless every entry is within the bound: the list may then be cut
// short, and the chain is walked instead (deviation cost = the cell output's
// arrival minus the input's arrival through its arc, as the lists compute
// it).  With EMIT the children go to slots out, out + 1, ... below cap.
template <typename T, int KM, bool EMIT>
__device__ int gt_children(const Topo &tp, const Ctx<T> &cx, const Nodes<T> &nd, int i, int out, int cap) {
  const int f = nd.ep[i], dv = nd.dev[i];
  const int u = dv < 0 ? tp.snk_drv[tp.A + f] : tp.snk_drv[dv];
  if (u < tp.n_start) return 0;
  const T cost = nd.cost[i];
  const T se = cx.ep_slack[f], th = cx.theta[tp.ff_inst[f]], lim = cx.limit;
  int cells = 0, ndv = 0;
  if constexpr (EMIT) {
    cells = nd.cells[i];
    ndv = nd.ndev[i];
  }
  auto put = [&](int o, int t, T cc) {
    if (o >= cap) return;
    nd.cost[o] = cc;
    nd.key[o] = se + cc;
    nd.dev[o] = t;
    nd.par[o] = i;
    nd.ep[o] = f;
    nd.cells[o] = cells + 1 - cx.cdep[tp.n_start + tp.snk_comb[t]] + cx.cdep[tp.snk_drv[t]];
    nd.ndev[o] = ndv + 1;
  };
  if constexpr (KM > 1) {
    const size_t lb = (size_t)(u - tp.n_start) * KM;
    int j = 0;
    for (; j < KM; ++j) {
      const T d = cx.side_cost[lb + j];
      if (!(d < inf_of<T>())) break;
      const T key = se + (cost + d);
      if (!(key <= th && key < lim)) break;
    }
    if (j < KM) {
      if constexpr (EMIT)
        for (int q = 0; q < j; ++q) put(out + q, cx.side_pin[lb + q], cost + cx.side_cost[lb + q]);
      return j;
    }
  }
  int n = 0;
  for (int v = u; v >= tp.n_start;) {
    const int c = v - tp.n_start;
    const T best = cx.at[v];
    const int b = tp.comb_inptr[c], e = tp.comb_inptr[c + 1], cr = b + cx.crit[c];
    for (int t = b; t < e; ++t) {
      if (t == cr) continue;
      const T a = cx.at[tp.M + t] + cx.darc[t];
      const T cc = cost + (best - a);
      const T key = se + cc;
      if (key <= th && key < lim) {
        if constexpr (EMIT) put(out + n, t, cc);
        ++n;
      }
    }
    v = tp.snk_drv[cr];
  }
  return n;
}

template <typename T, int KM>
__global__ void __launch_bounds__(256) k_gt_count(Topo tp, Ctx<T> cx, Nodes<T> nd, int fb, int n,
                                                   int32_t *__restrict__ cnt) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  cnt[j] = gt_children<T, KM, false>(tp, cx, nd, fb + j, 0, 0);
}

template <typename T, int KM>
__global__ void __launch_bounds__(256) k_gt_emit(Topo tp, Ctx<T> cx, Nodes<T> nd, int fb, int n, int fe, int cap,
                                                  const int32_t *__restrict__ off) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  gt_children<T, KM, true>(tp, cx, nd, fb + j, fe + off[j], cap);
}

// sort keys of nodes [0, n): (instance, slack) in single precision, slack
// alone in double precision (one instance)
template <typename T>
__global__ void k_gt_keys(Topo tp, int n, const int32_t *__restrict__ ep, const T *__restrict__ key,
                          uint64_t *__restrict__ keys, uint32_t *__restrict__ vals) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  if constexpr (sizeof(T) == 4)
    keys[j] = ((uint64_t)tp.ff_inst[ep[j]] << 32) | (order_key((float)key[j]) & 0xFFFFFFFFull);
  else
    keys[j] = order_key((double)key[j]);
  vals[j] = (uint32_t)j;
}

// per instance: its range [start, end) in the sorted keys (both 0 if empty)
__global__ void k_gt_segments(int n, int f32, const uint64_t *__restrict__ keys, int32_t *__restrict__ start,
                              int32_t *__restrict__ end) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const int inst = f32 ? (int)(keys[j] >> 32) : 0;
  if (j == 0 || (f32 ? (int)(keys[j - 1] >> 32) : 0) != inst) start[inst] = j;
  if (j == n - 1 || (f32 ? (int)(keys[j + 1] >> 32) : 0) != inst) end[inst] = j + 1;
}

// after an overflow: the K-th smallest stored slack of an instance that
// stored at least K nodes bounds its K-th slack; misc[2] = 1 when a bound
// went down
template <typename T>
__global__ void k_gt_refine(int num_inst, int K, const int32_t *__restrict__ start, const int32_t *__restrict__ end,
                            const uint32_t *__restrict__ perm, const T *__restrict__ key, T *__restrict__ theta,
                            int32_t *__restrict__ misc) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  int moved = 0;
  for (int i = 0; i < num_inst; ++i) {
    if (end[i] - start[i] < K) continue;
    const T t = key[perm[start[i] + K - 1]];
    if (t < theta[i]) {
      theta[i] = t;
      moved = 1;
    }
  }
  misc[2] = moved;
}

// per instance: paths kept and their first output index
__global__ void k_gt_bases(int num_inst, int K, const int32_t *__restrict__ start, const int32_t *__restrict__ end,
                           int32_t *__restrict__ outb, int32_t *__restrict__ kept, int32_t *__restrict__ d_num_paths,
                           int32_t *__restrict__ d_nslots) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  int o = 0;
  for (int i = 0; i < num_inst; ++i) {
    const int c = end[i] - start[i];
    const int kp = c < K ? c : K;
    outb[i] = o;
    kept[i] = kp;
    o += kp;
  }
  *d_num_paths = o;
  *d_nslots = o;
}

// output index of each kept node; the pair update visits paths through
// slot_out, here the identity
template <typename T>
__global__ void k_gt_index(int n, int f32, const uint64_t *__restrict__ keys, const uint32_t *__restrict__ perm,
                           const int32_t *__restrict__ start, const int32_t *__restrict__ outb,
                           const int32_t *__restrict__ kept, const int32_t *__restrict__ cells,
                           int32_t *__restrict__ out_slot, int32_t *__restrict__ out_len,
                           int32_t *__restrict__ slot_out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const int inst = f32 ? (int)(keys[j] >> 32) : 0;
  const int rho = j - start[inst];
  if (rho >= kept[inst]) return;
  const int q = outb[inst] + rho;
  const int node = (int)perm[j];
  out_slot[q] = node;
  out_len[q] = 2 * cells[node] + 2;
  slot_out[q] = q;
}

template <typename T>
__global__ void __launch_bounds__(128) k_walk_nodes(Topo tp, const int32_t *__restrict__ d_num_paths,
                                                     const int32_t *__restrict__ out_slot, Nodes<T> nd,
                                                     const int4 *__restrict__ hop4, const int32_t *__restrict__ path_ptr,
                                                     int32_t *__restrict__ path_pins, int32_t *__restrict__ path_int,
                                                     int32_t *__restrict__ path_ep, int32_t *__restrict__ path_epi,
                                                     T *__restrict__ path_slack, int32_t *__restrict__ err,
                                                     int pin_cap) {
  __shared__ int32_t stage[128 * WALK_ROW];
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  // every lane stays to the end: the wave shares the walk's flush points
  bool live = q < *d_num_paths;
  int node = 0, f = 0, lo = 0, hi = 0;
  if (live) {
    node = out_slot[q];
    f = nd.ep[node];
    lo = path_ptr[q];
    hi = path_ptr[q + 1];
    if (lo < 0 || hi > pin_cap || hi - lo < 2) {
      atomicOr(err, 1);
      live = false;
    }
  }
  LinkDevs ds;
  ds.dev = nd.dev;
  ds.par = nd.par;
  ds.node = node;
  ds.nd = live ? nd.ndev[node] : 0;
  ds.used = 0;
  ds.nb = 0;
  ds.bi = 0;
  RevWriter w{path_pins, path_int, stage + threadIdx.x * WALK_ROW, live ? hi - 1 : -1, live ? lo : 0, live ? hi : 0};
  const bool ok = walk_path(tp, hop4, w, f, live, [&]() { return ds.next(); });
  if (!live) return;
  if (!ok) atomicOr(err, 1);
  path_ep[q] = tp.snk_ext[tp.A + f];
  path_epi[q] = f;
  path_slack[q] = nd.key[node];
}

// rank of each path among the paths of its endpoint, in output order: sort
// (endpoint, output index), then rank = position - start of the endpoint's run
__global__ void k_gt_rank_keys(const int32_t *__restrict__ d_num_paths, const int32_t *__restrict__ path_epi,
                               uint64_t *__restrict__ keys, uint32_t *__restrict__ vals) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= *d_num_paths) return;
  keys[q] = (uint64_t)(uint32_t)path_epi[q];
  vals[q] = (uint32_t)q;
}

__global__ void k_gt_rank_heads(const int32_t *__restrict__ d_num_paths, const uint64_t *__restrict__ keys,
                                int32_t *__restrict__ head) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= *d_num_paths) return;
  head[j] = (j == 0 || keys[j] != keys[j - 1]) ? 1 : 0;
}

// run id of position j = heads before j + head(j) - 1
__global__ void k_gt_rank_starts(const int32_t *__restrict__ d_num_paths, const int32_t *__restrict__ head,
                                 const int32_t *__restrict__ before, int32_t *__restrict__ run_start) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= *d_num_paths) return;
  if (head[j]) run_start[before[j]] = j;
}

__global__ void k_gt_rank_write(const int32_t *__restrict__ d_num_paths, const int32_t *__restrict__ head,
                                const int32_t *__restrict__ before, const int32_t *__restrict__ run_start,
                                const uint32_t *__restrict__ vals, int32_t *__restrict__ path_rank) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= *d_num_paths) return;
  const int run = before[j] + head[j] - 1;
  path_rank[vals[j]] = j - run_start[run];
}

template <typename T, int KM>
void expand_round(tdp_graph g, const GtStore &st, const Ctx<T> &cx, const Nodes<T> &nd, int fb, int n, int fe,
                  hipStream_t s) {
  const Topo &tp = g->topo;
  hipLaunchKernelGGL((k_gt_count<T, KM>), dim3(nb(n, 256)), dim3(256), 0, s, tp, cx, nd, fb, n, st.gt_cnt);
  scan_exclusive(st.gt_cnt, st.gt_off, n, nullptr, st.gt_misc, st.gt_scan, s);
  hipLaunchKernelGGL((k_gt_emit<T, KM>), dim3(nb(n, 256)), dim3(256), 0, s, tp, cx, nd, fb, n, fe, st.cap,
                     st.gt_off);
}

template <typename T>
void expand(tdp_graph g, const GtStore &st, const Ctx<T> &cx, const Nodes<T> &nd, int fb, int n, int fe,
            hipStream_t s) {
  switch (g->side_k) {
    case 1: expand_round<T, 1>(g, st, cx, nd, fb, n, fe, s); break;
    case 2: expand_round<T, 2>(g, st, cx, nd, fb, n, fe, s); break;
    case 4: expand_round<T, 4>(g, st, cx, nd, fb, n, fe, s); break;
    case 8: expand_round<T, 8>(g, st, cx, nd, fb, n, fe, s); break;
    case 16: expand_round<T, 16>(g, st, cx, nd, fb, n, fe, s); break;
    default: expand_round<T, 32>(g, st, cx, nd, fb, n, fe, s); break;
  }
}

bool read_i32(const int32_t *d, int32_t *h, hipStream_t s) {
  return hipStreamSynchronize(s) == hipSuccess && hipMemcpy(h, d, 4, hipMemcpyDeviceToHost) == hipSuccess;
}

// sort nodes [0, n) by (instance, slack) into gt_k0 / gt_v0 and find each
// instance's range
template <typename T>
void sort_nodes(tdp_graph g, const GtStore &st, const Nodes<T> &nd, int n, hipStream_t s) {
  const Topo &tp = g->topo;
  hipLaunchKernelGGL(k_gt_keys<T>, dim3(nb(n, 256)), dim3(256), 0, s, tp, n, nd.ep, nd.key, st.gt_k0, st.gt_v0);
  radix_sort(st.gt_k0, st.gt_v0, st.gt_k1, st.gt_v1, n, nullptr, sizeof(T) == 4 ? g->key_bits32 : 64, st.gt_hist,
             st.gt_scan, s);
  fill_i32(st.gt_start, tp.num_inst, 0, s);
  fill_i32(st.gt_end, tp.num_inst, 0, s);
  hipLaunchKernelGGL(k_gt_segments, dim3(nb(n, 256)), dim3(256), 0, s, n, sizeof(T) == 4 ? 1 : 0, st.gt_k0,
                     st.gt_start, st.gt_end);
}

}  // namespace

template <typename T>
tdp_status report_impl(tdp_graph g, const GtStore &st, int K, float slack_limit, hipStream_t s) {
  const Topo &tp = g->topo;
  const int cap = st.cap;
  Nodes<T> nd{(T *)st.gt_cost, (T *)st.gt_key, st.gt_dev, st.gt_par, st.gt_ep, st.gt_cells, st.gt_nd};
  Ctx<T> cx{(const T *)g->at, (const T *)g->darc, (const T *)g->side_cost, (const T *)g->ep_slack,
            (const T *)st.gt_theta, g->crit, g->side_pin, g->cdep, (T)slack_limit};
  int total = 0;
  if (K > 0 && tp.E > 0) {
    // bound from the per-endpoint search at the K worst endpoints
    const int k = g->max_k;
    select_stage<T>(g, K, s);
    search_stage<T>(g, k, slack_limit, s);
    slot_sort_stage<T>(g, k, s);
    hipLaunchKernelGGL(k_gt_theta0<T>, dim3(1), dim3(1), 0, s, tp.num_inst, k, K, g->inst_nsel, g->inst_nvalid,
                       g->sort_v0, (const T *)g->slot_key, (T *)st.gt_theta);
    constexpr int kMaxRestarts = 64;
    for (int attempt = 0;; ++attempt) {
      if (attempt == kMaxRestarts)
        return gt_fail(g, TDP_E_CAPACITY, "report_timing: too many paths share the K-th slack for the node store");
      hipLaunchKernelGGL(k_gt_root_flags<T>, dim3(nb(tp.E, 256)), dim3(256), 0, s, tp, (const T *)g->ep_slack,
                         (const T *)st.gt_theta, (T)slack_limit, g->sel_flag);
      scan_exclusive(g->sel_flag, g->sel_pos, tp.E, nullptr, st.gt_misc + 1, g->scan_tmp, s);
      hipLaunchKernelGGL(k_gt_roots<T>, dim3(nb(tp.E, 256)), dim3(256), 0, s, tp, g->sel_flag, g->sel_pos,
                         (const T *)g->ep_slack, g->cdep, cap, nd);
      int32_t nroots = 0;
      if (!read_i32(st.gt_misc + 1, &nroots, s)) return gt_fail(g, TDP_E_DEVICE, "report_timing: count copy failed");
      bool over = nroots > cap;
      int fb = 0, fe = over ? cap : nroots;
      while (!over && fb < fe) {
        const int n = fe - fb;
        expand<T>(g, st, cx, nd, fb, n, fe, s);
        int32_t add = 0;
        if (!read_i32(st.gt_misc, &add, s)) return gt_fail(g, TDP_E_DEVICE, "report_timing: count copy failed");
        if ((long long)fe + add > cap) {
          over = true;
          fe = cap;
          break;
        }
        fb = fe;
        fe += add;
      }
      total = fe;
      if (!over) break;
      // the store is full of real paths: tighten the bound and start again
      sort_nodes<T>(g, st, nd, cap, s);
      hipLaunchKernelGGL(k_gt_refine<T>, dim3(1), dim3(1), 0, s, tp.num_inst, K, st.gt_start, st.gt_end, st.gt_v0,
                         (const T *)st.gt_key, (T *)st.gt_theta, st.gt_misc);
      int32_t moved = 0;
      if (!read_i32(st.gt_misc + 2, &moved, s)) return gt_fail(g, TDP_E_DEVICE, "report_timing: count copy failed");
      if (!moved)
        return gt_fail(g, TDP_E_CAPACITY, "report_timing: more paths share the K-th slack than the node store holds");
    }
  }
  // order, cut to K per instance, walk
  if (total > 0) {
    sort_nodes<T>(g, st, nd, total, s);
  } else {
    fill_i32(st.gt_start, tp.num_inst, 0, s);
    fill_i32(st.gt_end, tp.num_inst, 0, s);
  }
  hipLaunchKernelGGL(k_gt_bases, dim3(1), dim3(1), 0, s, tp.num_inst, K, st.gt_start, st.gt_end, g->inst_outb,
                     g->inst_kept, g->d_num_paths, g->d_nslots);
  if (total > 0)
    hipLaunchKernelGGL(k_gt_index<T>, dim3(nb(total, 256)), dim3(256), 0, s, total, sizeof(T) == 4 ? 1 : 0,
                       st.gt_k0, st.gt_v0, st.gt_start, g->inst_outb, g->inst_kept, st.gt_cells, g->out_slot,
                       g->out_len, g->slot_out);
  scan_exclusive(g->out_len, g->path_ptr, g->max_out, g->d_num_paths, nullptr, g->scan_tmp, s);
  ptr_tail(g->d_num_paths, g->out_len, g->path_ptr, s);
  hipLaunchKernelGGL(k_walk_nodes<T>, dim3(nb(g->max_out, 128)), dim3(128), 0, s, tp, g->d_num_paths, g->out_slot,
                     nd, (const int4 *)g->hop4, g->path_ptr, g->path_pins, g->path_int, g->path_ep, g->path_epi,
                     (T *)g->path_slack, g->d_err, g->pin_cap);
  // ranks per endpoint (the node store is free again: its arrays serve as scratch)
  const int mo = g->max_out;
  hipLaunchKernelGGL(k_gt_rank_keys, dim3(nb(mo, 256)), dim3(256), 0, s, g->d_num_paths, g->path_epi, st.gt_k0,
                     st.gt_v0);
  radix_sort(st.gt_k0, st.gt_v0, st.gt_k1, st.gt_v1, mo, g->d_num_paths, 32, st.gt_hist, st.gt_scan, s);
  hipLaunchKernelGGL(k_gt_rank_heads, dim3(nb(mo, 256)), dim3(256), 0, s, g->d_num_paths, st.gt_k0, st.gt_cnt);
  scan_exclusive(st.gt_cnt, st.gt_off, mo, g->d_num_paths, nullptr, st.gt_scan, s);
  hipLaunchKernelGGL(k_gt_rank_starts, dim3(nb(mo, 256)), dim3(256), 0, s, g->d_num_paths, st.gt_cnt, st.gt_off,
                     st.gt_dev);
  hipLaunchKernelGGL(k_gt_rank_write, dim3(nb(mo, 256)), dim3(256), 0, s, g->d_num_paths, st.gt_cnt, st.gt_off,
                     st.gt_dev, st.gt_v0, g->path_rank);
  return TDP_OK;
}

template tdp_status report_impl<float>(tdp_graph, const GtStore &, int, float, hipStream_t);
template tdp_status report_impl<double>(tdp_graph, const GtStore &, int, float, hipStream_t);

}  // namespace tdp
