// report_timing_endpoint(n, k) on the device (Sec. III-B, Table I).
//
// A path into endpoint e is described by its deviations from the
// arrival-time tree: walking back from e along critical inputs, a deviation
// takes a non-critical input j of a cell instead.  The path's slack is the
// endpoint's slack plus the sum of its deviation costs
//     delta(j) = AT(out) - (AT(in_j) + d_arc(in_j)) >= 0,
// so the k worst paths at e are the k cheapest deviation sets.  Every path has
// a unique parent (itself without its upstream-most deviation) and its children
// add one deviation on the critical chain above that point, so the cheapest
// paths come out of a best-first expansion.  The forward sweep already keeps,
// for every cell, the max_k cheapest deviations along its critical chain, so a
// pop needs one list read, not a chain walk.
//
//   k_sel_*        endpoints of each instance in (slack, pin id) order; the
//                  first n, or the violated ones (n < 0)
//   k_search       one thread per selected endpoint: best-first expansion
//                  with a register-resident candidate list; writes, per path
//                  slot, its slack, its deviation, its parent slot and its pin
//                  count (from the critical-chain depths)
//   ordering       stable radix sort of the slots by (instance, slack); per
//                  instance cut to K; prefix sum of the pin counts
//   k_walk         one thread per output path: follow critical inputs and
//                  the deviations from the endpoint back to the start point,
//                  writing the pins in place from the end.
#include "tdp_impl.h"
#include "tdp_prims.h"
#include "tdp_walk.h"
#include "tdp_wave.h"

namespace tdp {

// ------------------------------------------------------------- selection
template <typename T>
__global__ void k_sel_keys(Topo tp, const T *__restrict__ ep_slack, uint64_t *__restrict__ keys,
                           uint32_t *__restrict__ vals) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= tp.E) return;
  keys[f] = ((uint64_t)tp.ff_inst[f] << 32) | (order_key((float)ep_slack[f]) & 0xFFFFFFFFull);
  vals[f] = f;
}

// flags of the first n endpoints of each instance in sorted order; the
// double-precision tie-break is settled by a second key pass in sel_by_rank
template <typename T>
__global__ void k_sel_first_n(Topo tp, const int32_t *__restrict__ ep_base, const uint64_t *__restrict__ keys,
                              const uint32_t *__restrict__ perm, const T *__restrict__ ep_slack, int n,
                              int32_t *__restrict__ flag) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= tp.E) return;
  const int inst = (int)(keys[j] >> 32);
  const int rank = j - ep_base[inst];
  const int f = perm[j];
  flag[f] = (rank < n && ep_slack[f] < inf_of<T>()) ? 1 : 0;
}

template <typename T>
__global__ void k_sel_violated(Topo tp, const T *__restrict__ ep_slack, int32_t *__restrict__ flag) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= tp.E) return;
  flag[f] = ep_slack[f] < (T)0 ? 1 : 0;
}

__global__ void k_sel_compact(Topo tp, const int32_t *__restrict__ flag, const int32_t *__restrict__ pos,
                              int32_t *__restrict__ list) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= tp.E) return;
  if (flag[f]) list[pos[f]] = f;
}

// per instance: first selected index and count (endpoint ranges are
// contiguous per instance, so the scan positions give both)
__global__ void k_sel_counts(int num_inst, int E, const int32_t *__restrict__ ep_base, const int32_t *__restrict__ pos,
                             const int32_t *__restrict__ d_nsel, int32_t *__restrict__ inst_selb,
                             int32_t *__restrict__ inst_nsel) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= num_inst) return;
  const int b = ep_base[i] < E ? pos[ep_base[i]] : *d_nsel;
  const int e = ep_base[i + 1] < E ? pos[ep_base[i + 1]] : *d_nsel;
  inst_selb[i] = b;
  inst_nsel[i] = e - b;
}

// per instance: number of paths found (sum of the per-endpoint counts)
__global__ void __launch_bounds__(256) k_valid_counts(const int32_t *__restrict__ inst_selb,
                                                       const int32_t *__restrict__ inst_nsel,
                                                       const int32_t *__restrict__ npop,
                                                       int32_t *__restrict__ inst_nvalid) {
  __shared__ int sh[256];
  const int i = blockIdx.x;
  const int b = inst_selb[i], n = inst_nsel[i];
  int acc = 0;
  for (int q = threadIdx.x; q < n; q += 256) acc += npop[b + q];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) inst_nvalid[i] = sh[0];
}

// --------------------------------------------------------------- search
template <typename T, int KM>
__global__ void __launch_bounds__(64) k_search(Topo tp, int k, T slack_limit, const int32_t *__restrict__ d_nsel,
                                                const int32_t *__restrict__ sel, const T *__restrict__ ep_slack,
                                                const int32_t *__restrict__ cdep, const T *__restrict__ side_cost,
                                                const int32_t *__restrict__ side_pin, T *__restrict__ slot_key,
                                                int32_t *__restrict__ slot_dev, int32_t *__restrict__ slot_par,
                                                int32_t *__restrict__ slot_len, int32_t *__restrict__ slot_cells,
                                                int32_t *__restrict__ npop_out) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= *d_nsel) return;
  const int f = sel[q];
  const T se = ep_slack[f];
  const size_t base = (size_t)q * k;
  // candidate list, ascending by (cost, creation order)
  T cc[KM];
  int32_t cdv[KM], cpr[KM];
#pragma unroll
  for (int j = 0; j < KM; ++j) {
    cc[j] = inf_of<T>();
    cdv[j] = -1;
    cpr[j] = -1;
  }
  cc[0] = 0;
  int npop = 0;
  const int eroot = tp.snk_drv[tp.A + f];
  // the slots found, kept in registers and written after the search: the
  // loads of each round then never wait behind the stores of the last one
  // (a wave's memory operations retire in order)
  T okey[KM];
  int32_t odev[KM], opar[KM], ocells[KM];
#pragma unroll
  for (int r = 0; r < KM; ++r) {
    okey[r] = inf_of<T>();
    odev[r] = -1;
    opar[r] = -1;
    ocells[r] = 0;
  }
#pragma unroll
  for (int r = 0; r < KM; ++r) {
    if (r >= k || !(cc[0] < inf_of<T>())) break;
    const T cost = cc[0];
    const int dev = cdv[0], par = cpr[0];
#pragma unroll
    for (int j = 0; j + 1 < KM; ++j) {
      cc[j] = cc[j + 1];
      cdv[j] = cdv[j + 1];
      cpr[j] = cpr[j + 1];
    }
    cc[KM - 1] = inf_of<T>();
    cdv[KM - 1] = -1;
    cpr[KM - 1] = -1;
    const T sk = se + cost;
    if (!(sk < slack_limit)) break;
    int u, cells;
    if (dev < 0) {
      u = eroot;
      cells = cdep[u];
    } else {
      u = tp.snk_drv[dev];
      const int dc = tp.snk_comb[dev];
      int pc = 0;
#pragma unroll
      for (int j = 0; j < KM; ++j) pc = j == par ? ocells[j] : pc;
      cells = pc + 1 - cdep[tp.n_start + dc] + cdep[u];
    }
    okey[r] = sk;
    odev[r] = dev;
    opar[r] = par;
    ocells[r] = cells;
    ++npop;
    if (r + 1 == k || u < tp.n_start) continue;
    // children: one more deviation on the critical chain above u
    const size_t lb = (size_t)(u - tp.n_start) * KM;
    T dl[KM];
    int32_t pl[KM];
    load_list<KM>(side_cost + lb, dl);
    load_list<KM>(side_pin + lb, pl);
#pragma unroll
    for (int j = 0; j < KM; ++j) {
      const T d = dl[j];
      const int32_t p = pl[j];
      if (!(d < inf_of<T>())) break;
      // insert behind every candidate of equal cost (they were created earlier)
      T c = cost + d;
      int32_t pd = p, pp = r;
      bool moving = false;
#pragma unroll
      for (int i = 0; i < KM; ++i) {
        const bool go = moving || c < cc[i];
        const T oc = cc[i];
        const int32_t od = cdv[i], op = cpr[i];
        cc[i] = go ? c : oc;
        cdv[i] = go ? pd : od;
        cpr[i] = go ? pp : op;
        c = go ? oc : c;
        pd = go ? od : pd;
        pp = go ? op : pp;
        moving = go;
      }
    }
  }
#pragma unroll
  for (int r = 0; r < KM; ++r) {
    if (r >= k) break;
    const bool found = r < npop;
    slot_key[base + r] = found ? okey[r] : inf_of<T>();
    slot_dev[base + r] = found ? odev[r] : -1;
    slot_par[base + r] = found ? opar[r] : -1;
    slot_cells[base + r] = found ? ocells[r] : 0;
    slot_len[base + r] = found ? 2 * ocells[r] + 2 : 0;
  }
  npop_out[q] = npop;
}

// ------------------------------------------------------------- ordering
template <typename T>
__global__ void k_slot_keys(Topo tp, int k, const int32_t *__restrict__ d_nsel, const int32_t *__restrict__ sel,
                            const T *__restrict__ slot_key, int32_t *__restrict__ d_nslots,
                            uint64_t *__restrict__ keys, uint32_t *__restrict__ vals, int64_t cap) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n = (int64_t)(*d_nsel) * k;
  if (i == 0) *d_nslots = (int32_t)n;
  if (i >= n || i >= cap) return;
  const int f = sel[i / k];
  uint64_t kk;
  if constexpr (sizeof(T) == 4) kk = ((uint64_t)tp.ff_inst[f] << 32) | (order_key((float)slot_key[i]) & 0xFFFFFFFFull);
  else kk = order_key((double)slot_key[i]);
  keys[i] = kk;
  vals[i] = (uint32_t)i;
}

// per instance: start of its slot segment, start of its output range, paths kept
__global__ void k_path_bases(int num_inst, int k, int K, const int32_t *__restrict__ inst_nsel,
                             const int32_t *__restrict__ inst_nvalid, int32_t *__restrict__ seg,
                             int32_t *__restrict__ outb, int32_t *__restrict__ kept, int32_t *__restrict__ d_num_paths) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  int s = 0, o = 0;
  for (int i = 0; i < num_inst; ++i) {
    seg[i] = s;
    outb[i] = o;
    const int kp = inst_nvalid[i] < K ? inst_nvalid[i] : K;
    kept[i] = kp;
    s += inst_nsel[i] * k;
    o += kp;
  }
  *d_num_paths = o;
}

template <typename T>
__global__ void k_path_index(Topo tp, int k, const int32_t *__restrict__ d_nslots, const uint32_t *__restrict__ perm,
                             const int32_t *__restrict__ sel, const int32_t *__restrict__ seg,
                             const int32_t *__restrict__ outb, const int32_t *__restrict__ kept,
                             const int32_t *__restrict__ slot_len, int32_t *__restrict__ out_slot,
                             int32_t *__restrict__ out_len, int32_t *__restrict__ slot_out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= *d_nslots) return;
  const int slot = perm[j];
  const int f = sel[slot / k];
  const int inst = tp.ff_inst[f];
  const int rho = j - seg[inst];
  if (rho < kept[inst]) {
    const int q = outb[inst] + rho;
    out_slot[q] = slot;
    out_len[q] = slot_len[slot];
    slot_out[slot] = q;
  } else {
    slot_out[slot] = -1;
  }
}

// ----------------------------------------------------------------- walk
template <typename T>
__global__ void __launch_bounds__(128) k_walk(Topo tp, int k, const int32_t *__restrict__ d_num_paths,
                                               const int32_t *__restrict__ out_slot, const int32_t *__restrict__ sel,
                                               const int32_t *__restrict__ slot_dev, const int32_t *__restrict__ slot_par,
                                               const T *__restrict__ slot_key, const int4 *__restrict__ hop4,
                                               const int32_t *__restrict__ path_ptr, int32_t *__restrict__ path_pins,
                                               int32_t *__restrict__ path_int, int32_t *__restrict__ path_ep,
                                               int32_t *__restrict__ path_epi, int32_t *__restrict__ path_rank,
                                               T *__restrict__ path_slack, int32_t *__restrict__ err, int pin_cap) {
  __shared__ int32_t stage[128 * WALK_ROW];
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  // every lane stays to the end: the wave shares the walk's flush points
  bool live = q < *d_num_paths;
  int slot = 0, r = 0, f = 0, lo = 0, hi = 0;
  int devs[TDP_MAX_K];
  int nd = 0;
  if (live) {
    slot = out_slot[q];
    const int qs = slot / k;
    r = slot - qs * k;
    const int base = qs * k;
    f = sel[qs];
    // deviations, upstream-most first (the walk meets them last to first)
    for (int a = r; a >= 0 && nd < TDP_MAX_K;) {
      const int d = slot_dev[base + a];
      if (d < 0) break;
      devs[nd++] = d;
      a = slot_par[base + a];
    }
    lo = path_ptr[q];
    hi = path_ptr[q + 1];
    if (lo < 0 || hi > pin_cap || hi - lo < 2) {  // only after a failed update
      atomicOr(err, 1);
      live = false;
    }
  }
  int di = nd - 1;
  RevWriter w{path_pins, path_int, stage + threadIdx.x * WALK_ROW, live ? hi - 1 : -1, live ? lo : 0, live ? hi : 0};
  const bool ok = walk_path(tp, hop4, w, f, live, [&]() { return di >= 0 ? devs[di--] : -1; });
  if (!live) return;
  if (!ok) atomicOr(err, 1);
  const int et = tp.A + f;
  path_ep[q] = tp.snk_ext[et];
  path_epi[q] = f;
  path_rank[q] = r;
  path_slack[q] = slot_key[slot];
}

// path_ptr[num_paths] = path_ptr[num_paths-1] + len (the scan is exclusive)
__global__ void k_ptr_tail(const int32_t *__restrict__ d_num_paths, const int32_t *__restrict__ len,
                           int32_t *__restrict__ ptr) {
  const int n = *d_num_paths;
  ptr[n] = n > 0 ? ptr[n - 1] + len[n - 1] : 0;
}

// ------------------------------------------------------------- launcher
static inline int nb(long long n, int b) { return n > 0 ? (int)((n + b - 1) / b) : 1; }

template <typename T, int KM>
static void launch_search(tdp_graph g, int k, T limit, hipStream_t s) {
  const Topo &tp = g->topo;
  hipLaunchKernelGGL((k_search<T, KM>), dim3(nb(tp.E, 64)), dim3(64), 0, s, tp, k, limit, g->d_nsel, g->sel_list,
                     (const T *)g->ep_slack, g->cdep, (const T *)g->side_cost, g->side_pin, (T *)g->slot_key,
                     g->slot_dev, g->slot_par, g->slot_len, g->slot_cells, g->sel_npop);
}

// endpoints of each instance: the first n in (slack, pin) order, or the
// violated ones (n < 0); fills sel_list, d_nsel, inst_selb, inst_nsel
template <typename T>
void select_stage(tdp_graph g, int n, hipStream_t s) {
  const Topo &tp = g->topo;
  const int E = tp.E;
  if (n < 0) {
    hipLaunchKernelGGL(k_sel_violated<T>, dim3(nb(E, 256)), dim3(256), 0, s, tp, (const T *)g->ep_slack,
                       g->sel_flag);
  } else {
    hipLaunchKernelGGL(k_sel_keys<T>, dim3(nb(E, 256)), dim3(256), 0, s, tp, (const T *)g->ep_slack, g->sort_k0,
                       g->sort_v0);
    radix_sort(g->sort_k0, g->sort_v0, g->sort_k1, g->sort_v1, E, nullptr, g->key_bits32, g->sort_hist,
               g->scan_tmp, s);
    hipLaunchKernelGGL(k_sel_first_n<T>, dim3(nb(E, 256)), dim3(256), 0, s, tp, g->d_ep_base, g->sort_k0,
                       g->sort_v0, (const T *)g->ep_slack, n, g->sel_flag);
  }
  scan_exclusive(g->sel_flag, g->sel_pos, E, nullptr, g->d_nsel, g->scan_tmp, s);
  hipLaunchKernelGGL(k_sel_compact, dim3(nb(E, 256)), dim3(256), 0, s, tp, g->sel_flag, g->sel_pos, g->sel_list);
  hipLaunchKernelGGL(k_sel_counts, dim3(nb(tp.num_inst, 64)), dim3(64), 0, s, tp.num_inst, E, g->d_ep_base,
                     g->sel_pos, g->d_nsel, g->inst_selb, g->inst_nsel);
}

// up to k paths per selected endpoint, in slots q * k + r; per instance the
// number found (inst_nvalid)
template <typename T>
void search_stage(tdp_graph g, int k, float slack_limit, hipStream_t s) {
  const T limit = (T)slack_limit;
  switch (g->side_k) {
    case 1: launch_search<T, 1>(g, k, limit, s); break;
    case 2: launch_search<T, 2>(g, k, limit, s); break;
    case 4: launch_search<T, 4>(g, k, limit, s); break;
    case 8: launch_search<T, 8>(g, k, limit, s); break;
    case 16: launch_search<T, 16>(g, k, limit, s); break;
    default: launch_search<T, 32>(g, k, limit, s); break;
  }
  hipLaunchKernelGGL(k_valid_counts, dim3(g->topo.num_inst), dim3(256), 0, s, g->inst_selb, g->inst_nsel,
                     g->sel_npop, g->inst_nvalid);
}

// slots sorted by (instance, path slack), stable: sort_v0 holds the slot
// order, sort_k0 the keys
template <typename T>
void slot_sort_stage(tdp_graph g, int k, hipStream_t s) {
  const int cap = g->slot_cap;
  hipLaunchKernelGGL(k_slot_keys<T>, dim3(nb(cap, 256)), dim3(256), 0, s, g->topo, k, g->d_nsel, g->sel_list,
                     (const T *)g->slot_key, g->d_nslots, g->sort_k0, g->sort_v0, (int64_t)cap);
  radix_sort(g->sort_k0, g->sort_v0, g->sort_k1, g->sort_v1, cap, g->d_nslots,
             sizeof(T) == 4 ? g->key_bits32 : 64, g->sort_hist, g->scan_tmp, s);
}

void ptr_tail(const int32_t *d_num_paths, const int32_t *len, int32_t *ptr, hipStream_t s) {
  hipLaunchKernelGGL(k_ptr_tail, dim3(1), dim3(1), 0, s, d_num_paths, len, ptr);
}

template <typename T>
void extract_impl(tdp_graph g, int n, int k, int K, float slack_limit, hipStream_t s) {
  const Topo &tp = g->topo;
  prof_begin(g, TDP_STAGE_SELECT, s);
  select_stage<T>(g, n, s);
  prof_end(g, TDP_STAGE_SELECT, s);
  prof_begin(g, TDP_STAGE_SEARCH, s);
  search_stage<T>(g, k, slack_limit, s);
  prof_end(g, TDP_STAGE_SEARCH, s);
  // ordering
  prof_begin(g, TDP_STAGE_ORDER, s);
  const int cap = g->slot_cap;
  slot_sort_stage<T>(g, k, s);
  hipLaunchKernelGGL(k_path_bases, dim3(1), dim3(1), 0, s, tp.num_inst, k, K, g->inst_nsel, g->inst_nvalid,
                     g->inst_seg, g->inst_outb, g->inst_kept, g->d_num_paths);
  hipLaunchKernelGGL(k_path_index<T>, dim3(nb(cap, 256)), dim3(256), 0, s, tp, k, g->d_nslots, g->sort_v0,
                     g->sel_list, g->inst_seg, g->inst_outb, g->inst_kept, g->slot_len, g->out_slot, g->out_len, g->slot_out);
  scan_exclusive(g->out_len, g->path_ptr, g->max_out, g->d_num_paths, nullptr, g->scan_tmp, s);
  ptr_tail(g->d_num_paths, g->out_len, g->path_ptr, s);
  prof_end(g, TDP_STAGE_ORDER, s);
  // walk
  prof_begin(g, TDP_STAGE_WALK, s);
  hipLaunchKernelGGL(k_walk<T>, dim3(nb(g->max_out, 128)), dim3(128), 0, s, tp, k, g->d_num_paths, g->out_slot,
                     g->sel_list, g->slot_dev, g->slot_par, (const T *)g->slot_key, (const int4 *)g->hop4,
                     g->path_ptr, g->path_pins, g->path_int, g->path_ep, g->path_epi, g->path_rank,
                     (T *)g->path_slack, g->d_err, g->pin_cap);
  prof_end(g, TDP_STAGE_WALK, s);
}

template void extract_impl<float>(tdp_graph, int, int, int, float, hipStream_t);
template void extract_impl<double>(tdp_graph, int, int, int, float, hipStream_t);
template void select_stage<float>(tdp_graph, int, hipStream_t);
template void select_stage<double>(tdp_graph, int, hipStream_t);
template void search_stage<float>(tdp_graph, int, float, hipStream_t);
template void search_stage<double>(tdp_graph, int, float, hipStream_t);
template void slot_sort_stage<float>(tdp_graph, int, hipStream_t);
template void slot_sort_stage<double>(tdp_graph, int, hipStream_t);

}  // namespace tdp
