// Pin-pair set P, weights (Eq. 9) and the pin-to-pin loss (Eqs. 8, 10).
//
// Pairs are the net arcs (driver, sink) of the extracted paths; a sink pin has
// one driver, so the sink names the pair and P is a dense per-sink array.
//
// Eq. 9 takes the paths in order: a pair not in P enters with w0, a pair in P
// gains w1 * slack / WNS.  The sum over one round does not depend on the order
// except for which occurrence inserts the pair, so the device form is
//   new pair:      w = w0 + w1 * (sum of slack/WNS - first occurrence's)
//   existing pair: w = w  + w1 * (sum of slack/WNS)
// where "first" is the smallest output index.  The sums are accumulated as
// 2^-32 fixed point in 64-bit integer atomics, so the result is independent of
// thread timing; a second pass, run by the first occurrence, applies the
// update and clears the accumulators.
//
// The loss uses a compact pair list (ascending sink id) and, for the gradient,
// a per-cell incidence list in a fixed order so that every cell sums its terms
// in the same order on every run (no floating-point atomics).
#include "tdp_impl.h"
#include "tdp_prims.h"

namespace tdp {

constexpr double FIX_ONE = 4294967296.0;  // 2^32

template <typename T>
__device__ __forceinline__ bool pair_contrib(int rule, T slack, double wns, unsigned long long &v) {
  if (rule == 0) {
    if (!(wns < 0.0) || !((double)slack < 0.0)) return false;
    v = (unsigned long long)llrint((double)slack / wns * FIX_ONE);
    return true;
  }
  const double sc = fabs(wns) > 1.0 ? fabs(wns) : 1.0;
  v = (unsigned long long)llrint(exp(-(double)slack / sc) * FIX_ONE);
  return true;
}

// one wavefront per path: its lanes take the path's sinks
template <typename T>
__global__ void __launch_bounds__(256) k_pairs_acc(Topo tp, int rule, const int32_t *__restrict__ d_num_paths,
                                                    const int32_t *__restrict__ path_ptr,
                                                    const int32_t *__restrict__ path_int,
                                                    const int32_t *__restrict__ path_epi,
                                                    const T *__restrict__ path_slack,
                                                    const double *__restrict__ summary,
                                                    unsigned long long *__restrict__ acc, int32_t *__restrict__ first) {
  const int lane = threadIdx.x & 63;
  const int nw = gridDim.x * (blockDim.x >> 6);
  const int n = *d_num_paths;
  for (int q = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); q < n; q += nw) {
    const double wns = summary[4 * tp.ff_inst[path_epi[q]]];
    unsigned long long v;
    if (!pair_contrib<T>(rule, path_slack[q], wns, v)) continue;
    const int b = path_ptr[q], e = path_ptr[q + 1];
    for (int i = b + 1 + 2 * lane; i < e; i += 128) {
      const int t = path_int[i] - tp.M;
      if (t < 0 || t >= tp.S) continue;
      atomicAdd(&acc[t], v);
      atomicMin(&first[t], q);
    }
  }
}

// Same sums, aggregated per block first: a block takes a run of consecutive
// slots, i.e. the k paths of a few endpoints, which share most of their pins,
// merges its occurrences in an LDS hash table with integer atomics, and sends
// one global atomic per distinct pin.  The first occurrence is still the
// smallest output index, whatever order the paths are visited in.  The
// block's paths are not walked one after another: their descriptors (range,
// contribution) are loaded for all of them at once, and the threads then
// take the concatenation of their sink occurrences in equal shares, so the
// dependent loads are paid once per block rather than once per path.
constexpr int HASH_BITS = 11;
constexpr int HASH_SLOTS = 1 << HASH_BITS;  // 24 KB of LDS: several workgroups per CU
constexpr int ACC_MAX_PATHS = 64;           // paths per workgroup at most

template <typename T>
__global__ void __launch_bounds__(256) k_pairs_acc_lds(Topo tp, int rule, int per_block,
                                                        const int32_t *__restrict__ d_nslots,
                                                        const int32_t *__restrict__ slot_out,
                                                        const int32_t *__restrict__ path_ptr,
                                                        const int32_t *__restrict__ path_int,
                                                        const int32_t *__restrict__ path_epi,
                                                        const T *__restrict__ path_slack,
                                                        const double *__restrict__ summary,
                                                        const uint8_t *__restrict__ in_p,
                                                        unsigned long long *__restrict__ acc,
                                                        int32_t *__restrict__ first) {
  __shared__ int32_t hkey[HASH_SLOTS];
  __shared__ unsigned long long hacc[HASH_SLOTS];
  __shared__ int32_t hfirst[HASH_SLOTS];
  __shared__ unsigned long long s_v[ACC_MAX_PATHS];
  __shared__ int32_t s_b[ACC_MAX_PATHS], s_q[ACC_MAX_PATHS], s_pre[ACC_MAX_PATHS + 1];
  const int n = *d_nslots;
  const int j0 = blockIdx.x * per_block;
  if (j0 >= n) return;  // whole block: the grid is sized for the slot capacity
  const int np = min(n - j0, per_block);
  for (int i = threadIdx.x; i < HASH_SLOTS; i += blockDim.x) {
    hkey[i] = -1;
    hacc[i] = 0ull;
    hfirst[i] = 0x7fffffff;
  }
  // path descriptors: first sink position, number of sinks (every second pin
  // after the start point), contribution
  int cnt = 0;
  if ((int)threadIdx.x < np) {
    const int q = slot_out[j0 + threadIdx.x];
    unsigned long long v = 0ull;
    if (q >= 0) {
      const int b = path_ptr[q], e = path_ptr[q + 1];
      const T sl = path_slack[q];
      const double wns = summary[4 * tp.ff_inst[path_epi[q]]];
      if (pair_contrib<T>(rule, sl, wns, v)) {
        cnt = (e - b) / 2;
        s_b[threadIdx.x] = b + 1;
        s_q[threadIdx.x] = q;
        s_v[threadIdx.x] = v;
      }
    }
  }
  // inclusive scan of the counts over the first wave (np <= 64)
  if (threadIdx.x < 64) {
    int c = cnt;
    for (int o = 1; o < 64; o <<= 1) {
      const int u = __shfl_up(c, o, 64);
      if ((int)threadIdx.x >= o) c += u;
    }
    s_pre[threadIdx.x + 1] = c;
    if (threadIdx.x == 0) s_pre[0] = 0;
  }
  __syncthreads();
  const int total = s_pre[np];
  for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
    // the path holding occurrence idx: the last r with s_pre[r] <= idx
    int lo = 0, hi = np - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (s_pre[mid] <= idx) lo = mid;
      else hi = mid - 1;
    }
    const int t = path_int[s_b[lo] + 2 * (idx - s_pre[lo])] - tp.M;
    if (t < 0 || t >= tp.S) continue;
    const unsigned long long v = s_v[lo];
    const int q = s_q[lo];
    unsigned h = ((unsigned)t * 2654435761u) >> (32 - HASH_BITS);
    for (int probe = 0; probe < HASH_SLOTS; ++probe) {
      const int k = atomicCAS(&hkey[h], -1, t);
      if (k == -1 || k == t) {
        atomicAdd(&hacc[h], v);
        atomicMin(&hfirst[h], q);
        break;
      }
      h = (h + 1) & (HASH_SLOTS - 1);
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < HASH_SLOTS; i += blockDim.x) {
    const int t = hkey[i];
    if (t >= 0) {
      atomicAdd(&acc[t], hacc[i]);
      // the first occurrence matters only to a pair that Eq. 9 inserts
      if (rule != 0 || !in_p[t]) atomicMin(&first[t], hfirst[i]);
    }
  }
}

// every sink pin: apply this round's sum to the pairs it touched (the first
// occurrence inserts under Eq. 9), clear the accumulators, flag P's members
template <typename T>
__global__ void k_pairs_apply(Topo tp, int rule, float w0, float w1, int max_out, const int32_t *__restrict__ path_epi,
                              const T *__restrict__ path_slack, const double *__restrict__ summary,
                              unsigned long long *__restrict__ acc, int32_t *__restrict__ first,
                              float *__restrict__ w, uint8_t *__restrict__ in_p, int32_t *__restrict__ flag) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= tp.S) return;
  const int q = first[t];
  const unsigned long long sum = acc[t];
  // a pair already in P (Eq. 9) only sums; its first occurrence is not kept
  const bool member = rule == 0 && in_p[t];
  if (member && sum != 0ull) {
    w[t] = (float)((double)w[t] + (double)w1 * ((double)sum / FIX_ONE));
    acc[t] = 0ull;
  } else if (!member && q >= 0 && q < max_out) {
    const double wns = summary[4 * tp.ff_inst[path_epi[q]]];
    unsigned long long v = 0;
    pair_contrib<T>(rule, path_slack[q], wns, v);
    if (rule == 0) {  // inserted by its first occurrence, which adds no weight
      w[t] = (float)((double)w0 + (double)w1 * ((double)(sum - v) / FIX_ONE));
      in_p[t] = 1;
    } else {
      w[t] = (float)((double)sum / FIX_ONE);
      in_p[t] = 1;
    }
    acc[t] = 0ull;
    first[t] = 0x7fffffff;
  }
  flag[t] = in_p[t] ? 1 : 0;
}

// stateless rule: drop the previous round's pairs
__global__ void k_pairs_clear_list(const int32_t *__restrict__ d_npairs, const int32_t *__restrict__ pair_sink,
                                   float *__restrict__ w, uint8_t *__restrict__ in_p) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= *d_npairs) return;
  const int t = pair_sink[q];
  w[t] = 0.f;
  in_p[t] = 0;
}

__global__ void k_pairs_flags(int S, const uint8_t *__restrict__ in_p, int32_t *__restrict__ flag) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < S) flag[t] = in_p[t] ? 1 : 0;
}

// compact list + per-pair loss record + incidence counts per cell
__global__ void k_pairs_records(Topo tp, const uint8_t *__restrict__ in_p, const int32_t *__restrict__ pos,
                                const float *__restrict__ w, int32_t *__restrict__ pair_sink,
                                int32_t *__restrict__ pair_cs, int32_t *__restrict__ pair_ct,
                                float *__restrict__ pair_dox, float *__restrict__ pair_doy,
                                float *__restrict__ pair_w, int32_t *__restrict__ cell_cnt) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= tp.S || !in_p[t]) return;
  const int q = pos[t];
  const int s = tp.snk_drv[t];
  const int cs = tp.drv_cell[s], ct = tp.snk_cell[t];
  pair_sink[q] = t;
  pair_cs[q] = cs;
  pair_ct[q] = ct;
  pair_dox[q] = tp.drv_ox[s] - tp.snk_ox[t];
  pair_doy[q] = tp.drv_oy[s] - tp.snk_oy[t];
  pair_w[q] = w[t];
  if (!tp.cell_fixed[ct]) atomicAdd(&cell_cnt[ct], 1);
  if (cs >= 0 && !tp.cell_fixed[cs]) atomicAdd(&cell_cnt[cs], 1);
}

__global__ void k_cell_flags(int N, const int32_t *__restrict__ cnt, int32_t *__restrict__ flag) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c < N) flag[c] = cnt[c] > 0 ? 1 : 0;
}

__global__ void k_cell_touched(int N, const int32_t *__restrict__ cnt, const int32_t *__restrict__ tpos,
                               int32_t *__restrict__ touched) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c < N && cnt[c] > 0) touched[tpos[c]] = c;
}

// incidences of pair q, first pass: a slot in each of its two cells' lists
// (arbitrary order within a list) holding only the key that orders the list,
// 2q at the sink's cell and 2q + 1 at the driver's
__global__ void k_inc_fill(Topo tp, const int32_t *__restrict__ d_npairs, const int32_t *__restrict__ pair_cs,
                           const int32_t *__restrict__ pair_ct, const int32_t *__restrict__ cell_ptr,
                           int32_t *__restrict__ cell_cur, int32_t *__restrict__ inc_key) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= *d_npairs) return;
  const int cs = pair_cs[q], ct = pair_ct[q];
  if (!tp.cell_fixed[ct]) inc_key[cell_ptr[ct] + atomicAdd(&cell_cur[ct], 1)] = 2 * q;
  if (cs >= 0 && !tp.cell_fixed[cs]) inc_key[cell_ptr[cs] + atomicAdd(&cell_cur[cs], 1)] = 2 * q + 1;
}

// second pass, one thread per slot: the slot's place in its cell's list is
// the number of smaller keys in the list (keys are distinct), so every list
// ends up in key order whatever order the first pass filled it in; writes
// the incidence there (the other cell, -1 for a port; this pin's offset
// minus the other pin's; the weight) and resets the cell's counters.  Only
// loads precede the stores, so no load waits behind a store.
__global__ void k_inc_rank(const int32_t *__restrict__ cell_ptr, int N, const int32_t *__restrict__ inc_key,
                           const int32_t *__restrict__ pair_cs, const int32_t *__restrict__ pair_ct,
                           const float *__restrict__ pair_dox, const float *__restrict__ pair_doy,
                           const float *__restrict__ pair_w, int32_t *__restrict__ cell_cnt,
                           int32_t *__restrict__ cell_cur, int32_t *__restrict__ inc_other,
                           float *__restrict__ inc_dx, float *__restrict__ inc_dy, float *__restrict__ inc_w) {
  const int total = cell_ptr[N];
  for (int a = blockIdx.x * blockDim.x + threadIdx.x; a < total; a += gridDim.x * blockDim.x) {
    const int key = inc_key[a];
    const int q = key >> 1;
    const bool drv = key & 1;  // this cell drives the pair
    const int cs = pair_cs[q], ct = pair_ct[q];
    const int c = drv ? cs : ct;
    const int b = cell_ptr[c], e = cell_ptr[c + 1];
    int rank = 0;
    for (int z = b; z < e; ++z) rank += inc_key[z] < key;
    const float dox = pair_dox[q], doy = pair_doy[q];
    const int d = b + rank;
    inc_other[d] = drv ? ct : cs;
    inc_dx[d] = drv ? dox : -dox;
    inc_dy[d] = drv ? doy : -doy;
    inc_w[d] = pair_w[q];
    if (rank == 0) {
      cell_cnt[c] = 0;
      cell_cur[c] = 0;
    }
  }
}

// ------------------------------------------------------------------ loss
constexpr int LOSS_BLOCKS = 512;

// Pair distance losses: KIND 0 is PP's quadratic term (Eqs. 8, 10); 1 and 2
// are the Manhattan and linear Euclidean distances Sec. III-C compares it
// with.  pair_term is w * f(dx, dy); pair_grad the derivative of that term
// with respect to the first pin's coordinates (the second pin's is its
// negative).
template <typename T, int KIND>
__device__ __forceinline__ T pair_term(T w, T dx, T dy) {
  if constexpr (KIND == 0) return w * (dx * dx + dy * dy);
  else if constexpr (KIND == 1) return w * (fabs(dx) + fabs(dy));
  else return w * sqrt(dx * dx + dy * dy);
}
template <typename T>
__device__ __forceinline__ T sgn_of(T v) {
  return (T)((v > (T)0) - (v < (T)0));
}
template <typename T, int KIND>
__device__ __forceinline__ void pair_grad(T w, T dx, T dy, T &gx, T &gy) {
  if constexpr (KIND == 0) {
    gx = (T)2 * w * dx;
    gy = (T)2 * w * dy;
  } else if constexpr (KIND == 1) {
    gx = w * sgn_of(dx);
    gy = w * sgn_of(dy);
  } else {
    const T len = sqrt(dx * dx + dy * dy);
    gx = len > (T)0 ? w * dx / len : (T)0;
    gy = len > (T)0 ? w * dy / len : (T)0;
  }
}

// each pair's term in the graph's precision T, summed in double
template <typename T, int KIND>
__global__ void __launch_bounds__(256) k_p2p_fwd(const int32_t *__restrict__ d_npairs,
                                                  const int32_t *__restrict__ pair_cs,
                                                  const int32_t *__restrict__ pair_ct,
                                                  const float *__restrict__ pair_dox,
                                                  const float *__restrict__ pair_doy,
                                                  const float *__restrict__ pair_w, const float *__restrict__ x,
                                                  const float *__restrict__ y, double *__restrict__ part) {
  __shared__ double sh[256];
  const int n = *d_npairs;
  double acc = 0.0;
  for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < n; q += gridDim.x * blockDim.x) {
    const int cs = pair_cs[q], ct = pair_ct[q];
    const T xs = cs >= 0 ? (T)x[cs] : (T)0, ys = cs >= 0 ? (T)y[cs] : (T)0;
    const T dx = xs - (T)x[ct] + (T)pair_dox[q];
    const T dy = ys - (T)y[ct] + (T)pair_doy[q];
    acc += (double)pair_term<T, KIND>((T)pair_w[q], dx, dy);
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ void __launch_bounds__(256) k_sum_parts(int n, const double *__restrict__ part, double *__restrict__ out) {
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

template <typename T, int KIND>
__global__ void __launch_bounds__(256) k_p2p_bwd(const int32_t *__restrict__ d_ntouched,
                                                  const int32_t *__restrict__ touched,
                                                  const int32_t *__restrict__ cell_ptr,
                                                  const int32_t *__restrict__ inc_other,
                                                  const float *__restrict__ inc_dx, const float *__restrict__ inc_dy,
                                                  const float *__restrict__ inc_w, const float *__restrict__ x,
                                                  const float *__restrict__ y, const double *__restrict__ gout,
                                                  float *__restrict__ gx, float *__restrict__ gy) {
  const int n = *d_ntouched;
  const T g = (T)*gout;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const int c = touched[i];
    const T xc = (T)x[c], yc = (T)y[c];
    T ax = 0, ay = 0;
    for (int a = cell_ptr[c]; a < cell_ptr[c + 1]; ++a) {
      const int o = inc_other[a];
      const T xo = o >= 0 ? (T)x[o] : (T)0, yo = o >= 0 ? (T)y[o] : (T)0;
      T gx1, gy1;
      pair_grad<T, KIND>((T)inc_w[a], xc - xo + (T)inc_dx[a], yc - yo + (T)inc_dy[a], gx1, gy1);
      ax += gx1;
      ay += gy1;
    }
    gx[c] += (float)(g * ax);
    gy[c] += (float)(g * ay);
  }
}

// ------------------------------------------------------------- launchers
static inline int nb(long long n, int b) { return n > 0 ? (int)((n + b - 1) / b) : 1; }

template <typename T>
void pairs_update_impl(tdp_graph g, int rule, float w0, float w1, hipStream_t s) {
  const Topo &tp = g->topo;
  prof_begin(g, TDP_STAGE_PAIRS, s);
  if (rule == 1 && g->pairs_built)
    hipLaunchKernelGGL(k_pairs_clear_list, dim3(nb(tp.S, 256)), dim3(256), 0, s, g->d_npairs, g->pair_sink, g->pw,
                       g->pin_p);
  // a path has at most depth + 1 sinks; keep a block's occurrences within
  // 80 % of the hash table, otherwise fall back to plain global atomics
  const int per_block = std::min(ACC_MAX_PATHS, (HASH_SLOTS * 4 / 5) / (tp.D + 1));
  if (per_block >= 1)
    hipLaunchKernelGGL(k_pairs_acc_lds<T>, dim3(nb(std::max(g->slot_cap, g->max_out), per_block)), dim3(256), 0, s, tp, rule, per_block,
                       g->d_nslots, g->slot_out, g->path_ptr, g->path_int, g->path_epi, (const T *)g->path_slack,
                       g->summary, g->pin_p, g->pacc, g->pfirst);
  else
    hipLaunchKernelGGL(k_pairs_acc<T>, dim3(std::min(2048, nb(g->max_out, 4))), dim3(256), 0, s, tp, rule,
                       g->d_num_paths, g->path_ptr, g->path_int, g->path_epi, (const T *)g->path_slack, g->summary,
                       g->pacc, g->pfirst);
  hipLaunchKernelGGL(k_pairs_apply<T>, dim3(nb(tp.S, 256)), dim3(256), 0, s, tp, rule, w0, w1, g->max_out,
                     g->path_epi, (const T *)g->path_slack, g->summary, g->pacc, g->pfirst, g->pw, g->pin_p,
                     g->pflag);
  pairs_compact(g, s);
  prof_end(g, TDP_STAGE_PAIRS, s);
}

void pairs_rebuild(tdp_graph g, hipStream_t s) {
  const Topo &tp = g->topo;
  hipLaunchKernelGGL(k_pairs_flags, dim3(nb(tp.S, 256)), dim3(256), 0, s, tp.S, g->pin_p, g->pflag);
  pairs_compact(g, s);
}

// pflag holds the membership flags; build the pair list and the per-cell lists
void pairs_compact(tdp_graph g, hipStream_t s) {
  const Topo &tp = g->topo;
  scan_exclusive(g->pflag, g->pflag, tp.S, nullptr, g->d_npairs, g->scan_tmp, s);
  hipLaunchKernelGGL(k_pairs_records, dim3(nb(tp.S, 256)), dim3(256), 0, s, tp, g->pin_p, g->pflag, g->pw,
                     g->pair_sink, g->pair_cs, g->pair_ct, g->pair_dox, g->pair_doy, g->pair_w, g->cell_cnt);
  // cell_ptr = exclusive scan of counts; touched list = compaction of cells with any
  scan_exclusive(g->cell_cnt, g->cell_ptr, tp.N, nullptr, g->cell_ptr + tp.N, g->scan_tmp, s);
  hipLaunchKernelGGL(k_cell_flags, dim3(nb(tp.N, 256)), dim3(256), 0, s, tp.N, g->cell_cnt, g->cell_flag);
  scan_exclusive(g->cell_flag, g->cell_flag, tp.N, nullptr, g->d_ntouched, g->scan_tmp, s);
  hipLaunchKernelGGL(k_cell_touched, dim3(nb(tp.N, 256)), dim3(256), 0, s, tp.N, g->cell_cnt, g->cell_flag,
                     g->touched);
  hipLaunchKernelGGL(k_inc_fill, dim3(nb(tp.S, 256)), dim3(256), 0, s, tp, g->d_npairs, g->pair_cs, g->pair_ct,
                     g->cell_ptr, g->cell_cur, g->inc_key);
  hipLaunchKernelGGL(k_inc_rank, dim3(1024), dim3(256), 0, s, g->cell_ptr, tp.N, g->inc_key, g->pair_cs, g->pair_ct,
                     g->pair_dox, g->pair_doy, g->pair_w, g->cell_cnt, g->cell_cur, g->inc_other, g->inc_dx,
                     g->inc_dy, g->inc_w);
  g->pairs_built = true;
}

template <typename T, int KIND>
static void launch_pair_fwd(tdp_graph g, const float *x, const float *y, hipStream_t s) {
  hipLaunchKernelGGL((k_p2p_fwd<T, KIND>), dim3(LOSS_BLOCKS), dim3(256), 0, s, g->d_npairs, g->pair_cs, g->pair_ct,
                     g->pair_dox, g->pair_doy, g->pair_w, x, y, g->red_loss);
}

template <typename T>
void p2p_fwd_impl(tdp_graph g, int kind, const float *x, const float *y, double *loss, hipStream_t s) {
  prof_begin(g, TDP_STAGE_P2P_FWD, s);
  if (kind == 1) launch_pair_fwd<T, 1>(g, x, y, s);
  else if (kind == 2) launch_pair_fwd<T, 2>(g, x, y, s);
  else launch_pair_fwd<T, 0>(g, x, y, s);
  hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(256), 0, s, LOSS_BLOCKS, g->red_loss, loss);
  prof_end(g, TDP_STAGE_P2P_FWD, s);
}

template <typename T, int KIND>
static void launch_pair_bwd(tdp_graph g, const float *x, const float *y, const double *gout, float *gx, float *gy,
                            hipStream_t s) {
  hipLaunchKernelGGL((k_p2p_bwd<T, KIND>), dim3(LOSS_BLOCKS * 2), dim3(256), 0, s, g->d_ntouched, g->touched,
                     g->cell_ptr, g->inc_other, g->inc_dx, g->inc_dy, g->inc_w, x, y, gout, gx, gy);
}

template <typename T>
void p2p_bwd_impl(tdp_graph g, int kind, const float *x, const float *y, const double *gout, float *gx, float *gy,
                  hipStream_t s) {
  prof_begin(g, TDP_STAGE_P2P_BWD, s);
  if (kind == 1) launch_pair_bwd<T, 1>(g, x, y, gout, gx, gy, s);
  else if (kind == 2) launch_pair_bwd<T, 2>(g, x, y, gout, gx, gy, s);
  else launch_pair_bwd<T, 0>(g, x, y, gout, gx, gy, s);
  prof_end(g, TDP_STAGE_P2P_BWD, s);
}

template void pairs_update_impl<float>(tdp_graph, int, float, float, hipStream_t);
template void pairs_update_impl<double>(tdp_graph, int, float, float, hipStream_t);
template void p2p_fwd_impl<float>(tdp_graph, int, const float *, const float *, double *, hipStream_t);
template void p2p_fwd_impl<double>(tdp_graph, int, const float *, const float *, double *, hipStream_t);
template void p2p_bwd_impl<float>(tdp_graph, int, const float *, const float *, const double *, float *, float *,
                                  hipStream_t);
template void p2p_bwd_impl<double>(tdp_graph, int, const float *, const float *, const double *, float *, float *,
                                   hipStream_t);

}  // namespace tdp
