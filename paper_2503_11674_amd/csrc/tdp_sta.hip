// Static timing analysis kernels (Sec. II-B, Eqs. 2-4; net delay Eq. 7).
//
// One update is:
//   net pass   every net as a segment of a 64-lane chunk (driver lane, then
//              its sinks): pin positions, the RC delay into each sink
//              (kappa * L^2 with L Manhattan, or the sink's Elmore delay),
//              the driver's load (star model, a segmented sum); start points
//              get arrival and transition.
//   forward    one launch per level; one lane per combinational input pin,
//              a cell's inputs adjacent: arrival = segmented max over inputs of
//              (driver arrival + net delay + table delay at the input's
//              transition, under the Elmore model the driver's degraded by the
//              wire, and the output load), output transition =
//              segmented max of the table transitions, the critical input =
//              lowest lane attaining the max; the cell's head lane writes the
//              output and, with deviation lists on, merges the cell's own
//              deviations into the critical driver's list.
//   endpoint   slack at every D pin; WNS / TNS / count per instance in a
//              fixed-order two-level reduction.
//   backward   one launch per level from the top; one lane per net pin:
//              required time of a driver = segmented min over its sinks of
//              (sink required time - net delay); the driver lane then gives
//              its cell's inputs their required time (output's minus the arc
//              delay) and slack.
// Tables live in LDS for the forward sweep.  Nets with more than 63 sinks
// take a one-thread-per-net path.
#include "tdp_impl.h"
#include "tdp_prims.h"
#include "tdp_wave.h"
#include "tdp_tree.h"

namespace tdp {

// published words of the dataflow sweeps (relaxed device-scope atomics; a
// consumer polls one word, so no fences are needed)
constexpr uint64_t W_EMPTY = ~0ull;
constexpr uint32_t R_EMPTY = ~0u;

__device__ __forceinline__ uint64_t pub_ld(const uint64_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t pub_ld(const uint32_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void pub_st(uint64_t *p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void pub_st(uint32_t *p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t pack2(float lo, float hi) {
  return (uint64_t)__float_as_uint(lo) | ((uint64_t)__float_as_uint(hi) << 32);
}

// Poll *p until it differs from `empty`, with one short sleep between polls
// (a longer back-off delays the frontier by the sleep).  The wait is
// bounded: after `limit` polls (or once another wave has given up) it sets
// bit 2 of *err and returns `empty`, so every wave always finishes.
template <typename U>
__device__ __forceinline__ U wait_pub(const U *p, U empty, int32_t *err, int limit) {
  U v = pub_ld(p);
  int it = 0;
  while (v == empty) {
    if (++it > limit) {
      atomicOr(err, 2);
      break;
    }
    if ((it & 31) == 0 && __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) break;
    __builtin_amdgcn_s_sleep(1);
    v = pub_ld(p);
  }
  return v;
}

// A wave first waits on one representative word with its lane 0 alone (the
// word its chunk is likely to see published last), so that a waiting wave
// polls one address rather than 64; every lane then checks its own word.
template <typename U>
__device__ __forceinline__ void wait_rep(const U *p, U empty, int32_t *err, int limit) {
  if (wave_lane() == 0) (void)wait_pub(p, empty, err, limit);
}

// Every lane that wants one loads its word; only if some wanted word is not
// yet published does the wave wait: one lane polls the missing word that is
// published last (the highest-numbered one when producers go up the index
// order, the lowest with LOW_LAST), then the missing lanes wait for theirs.
// A wave behind the frontier pays one memory round trip.  Lanes that want
// nothing get `empty`.
template <bool LOW_LAST = false, typename U>
__device__ __forceinline__ U load_or_wait(const U *base, int idx, bool want, U empty, int32_t *err, int limit) {
  U v = want ? pub_ld(base + idx) : empty;
  const bool miss = want && v == empty;
  if (__ballot(miss)) {
    const int rep = LOW_LAST ? -wave_max_int(miss ? -idx : INT32_MIN + 1) : wave_max_int(miss ? idx : -1);
    if (wave_lane() == 0) (void)wait_pub(base + rep, empty, err, limit);
    if (miss) v = wait_pub(base + idx, empty, err, limit);
  }
  return v;
}

struct FlowInit {
  uint64_t *w = nullptr;
  uint32_t *r = nullptr, *cd = nullptr;
  uint64_t *se = nullptr;
  int32_t *err = nullptr;  // cleared at the start of every update
  int km = 0;
  int seed = 1;  // 0: start points are never published (self-test of the bounded waits)
  int reset_blocks = 0;  // trailing workgroups of the net pass that reset the words
};

// Marks of an incremental arrival update (all null for a full one), as
// stamps: an entry equal to the update's epoch is set, any other value is
// not, so nothing is cleared between updates.  A chunk is re-timed when the
// net pass marked it or when a driver of one of its inputs changed in this
// update, which each of its lanes reads for itself (no pushing of marks
// along fanout lists).
struct IncFlags {
  int32_t epoch = 0;
  int32_t *arr = nullptr;               // [n_fw_chunks] the net pass changed an input's delay or the load
  int32_t *lst = nullptr;               // [n_fw_chunks] the chunk's arrivals were re-timed
  int32_t *drv_chg = nullptr;           // [M] the driver's arrival or transition changed
  int32_t *drv_lchg = nullptr;          // [M] its deviation list, hop records or chain depth changed
  const int32_t *snk_chunk = nullptr;   // [A] forward chunk of a combinational input
  const int32_t *nm = nullptr;          // [n_nm_chunks] the net chunk holds a moved cell's pin
};

template <typename T>
__device__ __forceinline__ bool same_bits(T a, T b) {
  if constexpr (sizeof(T) == 4) return __float_as_uint((float)a) == __float_as_uint((float)b);
  else return __double_as_longlong((double)a) == __double_as_longlong((double)b);
}

// v[0, n) = x, 16-byte stores where the alignment allows
__device__ __forceinline__ void fill_u32(uint32_t *p, size_t n, uint32_t x, size_t tid, size_t nth) {
  size_t h = ((16 - ((uintptr_t)p & 15)) & 15) / 4;
  h = h < n ? h : n;
  if (tid < h) p[tid] = x;
  uint4 *q = (uint4 *)(p + h);
  const size_t n4 = (n - h) / 4;
  const uint4 xx = make_uint4(x, x, x, x);
  for (size_t i = tid; i < n4; i += nth) q[i] = xx;
  const size_t t0 = h + n4 * 4;
  if (tid < n - t0) p[t0 + tid] = x;
}

// The words the dataflow sweeps poll return to "not yet published" at the
// start of every update (the start points' words are seeded by the net pass
// itself, so they are left out here): streaming stores in workgroups of their
// own beside the net pass's gathers.
__device__ __forceinline__ void flow_reset(const FlowInit &fl, const Topo &tp, int b) {
  const size_t nth = (size_t)fl.reset_blocks * blockDim.x, tid = (size_t)b * blockDim.x + threadIdx.x;
  const size_t nc = (size_t)(tp.M - tp.n_start);
  if (fl.w) {
    fill_u32((uint32_t *)(fl.w + tp.n_start), 2 * nc, ~0u, tid, nth);
    fill_u32(fl.cd + tp.n_start, nc, 0u, tid, nth);
    if (fl.km) fill_u32((uint32_t *)fl.se, 2 * (size_t)tp.n_comb * fl.km, ~0u, tid, nth);
  }
  if (fl.r) fill_u32(fl.r, (size_t)tp.M, R_EMPTY, tid, nth);
}

template <typename T>
__device__ __forceinline__ void start_point(const Topo &tp, const LutView &L, int v, T ld, T in_slew, T clk_slew,
                                            T *__restrict__ at, T *__restrict__ slew, V2<T> *__restrict__ as,
                                            int32_t *__restrict__ cdep, const FlowInit &fl) {
  T a = 0, s = in_slew;
  if (v >= tp.n_pi && v < tp.n_start) lut_pair<T>(L, tp.ff_type[v - tp.n_pi], clk_slew, ld, a, s);
  if (v < tp.n_start) {
    at[v] = a;
    slew[v] = s;
    as[v] = v2<T>(a, s);
    cdep[v] = 0;
    if (fl.w) {  // seed the start points' words of the dataflow sweeps
      fl.w[v] = fl.seed ? pack2((float)a, (float)s) : W_EMPTY;
      fl.cd[v] = fl.seed ? 1 : 0;
    }
  }
}

// ------------------------------------------------------------- net pass
// one net chunk of the net pass (TREE: the spanning-tree model)
template <typename T, bool TREE>
__device__ __forceinline__ void netpass_chunk(const Topo &tp, const LutView &L, int chunk, const float2 *__restrict__ xy,
                                              const NetModel<T> &nm, T cw, T in_slew, T clk_slew,
                                              T *__restrict__ load, T *__restrict__ dnet, T *__restrict__ dnet_nm,
                                              float2 *__restrict__ cxy_nm, T *__restrict__ at, T *__restrict__ slew,
                                              V2<T> *__restrict__ as, int32_t *__restrict__ cdep, const FlowInit &fl,
                                              const IncFlags &inc) {
  const int lane = wave_lane();
  const int k = chunk * CHUNK + lane;
  const int4 rec = tp.nm_rec[k];
  const int p = rec.x, cell = rec.y;
  const int head = rec.w & 63, tail = (rec.w >> 8) & 63;
  // pin coordinate = cell coordinate + offset; differences are taken as
  // (cell - cell) + (offset - offset), exact to the rounding of the result
  // rather than of a die-scale sum.  A port has no cell and its offset is its
  // position: for the wire lengths it is taken as the base (offset 0), so a
  // port next to a cell far from the origin does not cancel two die-scale
  // numbers
  const float2 q = cell >= 0 ? xy[cell] : make_float2(0.f, 0.f);
  cxy_nm[k] = q;  // kept for the weighted-average wirelength at these positions
  const float fox = tp.nm_ox[k], foy = tp.nm_oy[k];
  const T cx = cell >= 0 ? (T)q.x : (T)fox, cy = cell >= 0 ? (T)q.y : (T)foy;
  const T ox = cell >= 0 ? (T)fox : (T)0, oy = cell >= 0 ? (T)foy : (T)0;
  const T cxd = __shfl(cx, head, 64), cyd = __shfl(cy, head, 64);
  const T oxd = __shfl(ox, head, 64), oyd = __shfl(oy, head, 64);
  const bool sink = p >= 0 && lane != head;
  T len, dn = 0;
  if constexpr (TREE) {
    const ChunkTree<T> tr = tree_chunk_build<T>(cw, lane, head, tail, sink, q.x, q.y, fox, foy, cx, cy, ox, oy,
                                                sink ? (T)tp.type_cap[(rec.w >> 16) & 255] : (T)0);
    len = tr.len;
    dn = tree_chunk_delay<T>(nm, tr);
  } else {
    len = sink ? fabs((cxd - cx) + (oxd - ox)) + fabs((cyd - cy) + (oyd - oy)) : (T)0;
  }
  if (sink) {
    if constexpr (!TREE) dn = nm.delay(len, nm.elmore ? (T)tp.type_cap[(rec.w >> 16) & 255] : (T)0);
    dnet[p - tp.M] = dn;
    dnet_nm[k] = dn;
    // incremental: every sink of a re-timed net gets its chunk re-timed
    if (inc.arr && p - tp.M < tp.A) inc.arr[inc.snk_chunk[p - tp.M]] = inc.epoch;
  }
  const T wl = seg_sum(len, lane, head, tail);
  if (p >= 0 && lane == head) {
    const T ld = (T)tp.net_cpin[p] + cw * wl;
    load[p] = ld;
    start_point<T>(tp, L, p, ld, in_slew, clk_slew, at, slew, as, cdep, fl);
    // incremental: a combinational driver's cell sees its new load
    if (inc.arr && p >= tp.n_start) inc.arr[inc.snk_chunk[tp.comb_inptr[p - tp.n_start]]] = inc.epoch;
  }
}

template <typename T, bool TREE>
__global__ void __launch_bounds__(256) k_netpass(Topo tp, LutView L, const float2 *__restrict__ xy, NetModel<T> nm,
                                                  T cw, T in_slew,
                                                  T clk_slew, T *__restrict__ load, T *__restrict__ dnet,
                                                  T *__restrict__ dnet_nm, float2 *__restrict__ cxy_nm,
                                                  T *__restrict__ at, T *__restrict__ slew,
                                                  V2<T> *__restrict__ as, int32_t *__restrict__ cdep, FlowInit fl) {
  if (blockIdx.x == 0 && threadIdx.x == 0 && fl.err) *fl.err = 0;
  const int main_blocks = (int)gridDim.x - fl.reset_blocks;
  if ((int)blockIdx.x >= main_blocks) {
    flow_reset(fl, tp, (int)blockIdx.x - main_blocks);
    return;
  }
  const int chunk = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (chunk >= tp.n_nm_chunks) return;
  netpass_chunk<T, TREE>(tp, L, chunk, xy, nm, cw, in_slew, clk_slew, load, dnet, dnet_nm, cxy_nm, at, slew, as,
                         cdep, fl, IncFlags{});
}

// the net pass over the marked net chunks of an incremental update (the same
// computation per chunk, so the results are those of a full pass)
template <typename T, bool TREE>
__global__ void __launch_bounds__(256) k_netpass_marked(Topo tp, LutView L, const float2 *__restrict__ xy,
                                                         NetModel<T> nm, T cw, T in_slew, T clk_slew,
                                                         T *__restrict__ load, T *__restrict__ dnet,
                                                         T *__restrict__ dnet_nm, float2 *__restrict__ cxy_nm,
                                                         T *__restrict__ at, T *__restrict__ slew,
                                                         V2<T> *__restrict__ as, int32_t *__restrict__ cdep,
                                                         IncFlags inc) {
  const int chunk = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (chunk >= tp.n_nm_chunks || inc.nm[chunk] != inc.epoch) return;
  netpass_chunk<T, TREE>(tp, L, chunk, xy, nm, cw, in_slew, clk_slew, load, dnet, dnet_nm, cxy_nm, at, slew, as,
                         cdep, FlowInit{}, inc);
}

// nets too wide for one chunk: one thread per net (tree_wl: the spanning-tree
// model, whose delays the tree kernel wrote)
template <typename T>
__global__ void k_netpass_big(Topo tp, LutView L, const float *__restrict__ x, const float *__restrict__ y, NetModel<T> nm,
                              const T *__restrict__ tree_wl, T cw, T in_slew, T clk_slew, T *__restrict__ load,
                              T *__restrict__ dnet,
                              T *__restrict__ at, T *__restrict__ slew, V2<T> *__restrict__ as,
                              int32_t *__restrict__ cdep) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= tp.n_big) return;
  const int v = tp.big_net[i];
  const int dc = tp.drv_cell[v];
  // a port driver: its position as the base (see the chunk form)
  const T cx = dc >= 0 ? (T)x[dc] : (T)tp.drv_ox[v], cy = dc >= 0 ? (T)y[dc] : (T)tp.drv_oy[v];
  const T ox = dc >= 0 ? (T)tp.drv_ox[v] : (T)0, oy = dc >= 0 ? (T)tp.drv_oy[v] : (T)0;
  T wl = tree_wl ? tree_wl[v] : (T)0;
  for (int k = tp.net_ptr[v]; !tree_wl && k < tp.net_ptr[v + 1]; ++k) {
    const int t = tp.net_sink[k];
    const int sc = tp.snk_cell[t];
    const T len = fabs((cx - (T)x[sc]) + (ox - (T)tp.snk_ox[t])) + fabs((cy - (T)y[sc]) + (oy - (T)tp.snk_oy[t]));
    dnet[t] = nm.delay(len, nm.elmore ? (T)tp.snk_cap[t] : (T)0);
    wl += len;
  }
  const T ld = (T)tp.net_cpin[v] + cw * wl;
  load[v] = ld;
  start_point<T>(tp, L, v, ld, in_slew, clk_slew, at, slew, as, cdep, FlowInit{});
}

// insert (c, p) into the ascending list (kc, kp); an entry equal to existing
// ones goes in front of them; the last entry falls off
template <typename T, int KM>
__device__ __forceinline__ void insert_front(T (&kc)[KM], int32_t (&kp)[KM], T c, int32_t p) {
  bool moving = false;
#pragma unroll
  for (int j = 0; j < KM; ++j) {
    const bool go = moving || c <= kc[j];
    const T oc = kc[j];
    const int32_t op = kp[j];
    kc[j] = go ? c : oc;
    kp[j] = go ? p : op;
    c = go ? oc : c;
    p = go ? op : p;
    moving = go;
  }
}

// -------------------------------------------------------------- forward
// One launch per level l does two jobs in separate workgroups: the arrivals
// of level l (the first n_arr workgroups) and, one level behind, the chain
// depths and deviation lists of level l-1, whose critical inputs the previous
// launch settled.  A cell's list extends its critical input's driver's list,
// a dependent load; running it beside the next level's arrivals keeps that
// round trip off the arrival chain.  fw_a keeps each input's arrival through
// its arc (per chunk slot) for the list job.
template <typename T>
__device__ __forceinline__ void fw_arrivals(const Topo &tp, const LutView &L, float *s_lut, int chunk, int ch1,
                                            const T *__restrict__ load, const T *__restrict__ dnet,
                                            T *__restrict__ at, T *__restrict__ slew, V2<T> *__restrict__ as,
                                            T *__restrict__ darc, int32_t *__restrict__ crit, T *__restrict__ fw_a,
                                            const IncFlags &inc) {
  const int lane = wave_lane();
  const int k = chunk * CHUNK + lane;
  // the record and the inputs' loads are issued before the tables are
  // staged, so the latencies overlap (a wave past the level's last chunk
  // reads that chunk's records again and then leaves)
  const int4 rec = tp.fw_rec[(chunk < ch1 ? chunk : ch1 - 1) * CHUNK + lane];
  const int t = rec.x, s = rec.y, c = rec.z;
  const int head = rec.w & 63, tail = (rec.w >> 8) & 63;
  const bool valid = t >= 0 && chunk < ch1;
  T ld = 0, dn = 0;
  V2<T> w = v2<T>(0, 0), old = v2<T>(0, 0);
  if (valid) {
    ld = load[tp.n_start + c];
    w = as[s];
    dn = dnet[t];
  }
  // incremental: whether the net pass marked the chunk or an input's driver
  // changed, and the cell's previous output (issued with the same loads)
  bool mark = false;
  if (inc.arr && valid) {
    mark = inc.drv_chg[s] == inc.epoch || inc.arr[chunk] == inc.epoch;
    if (lane == head) old = as[tp.n_start + c];
  }
  stage_lut(L, s_lut);
  if (chunk >= ch1) return;
  if (inc.arr) {  // only marked chunks, whose cells' lists follow
    if (__ballot(mark) == 0) return;
    if (lane == 0) inc.lst[chunk] = inc.epoch;
  }
  T a = -pos_inf<T>(), o = 0;
  if (valid) {
    const T a_in = w.x + dn;
    T d;
    lut_lds<T>(s_lut, L.nt, L.ns, L.nl, (rec.w >> 16) & 255, sink_slew<T>(L.net_model, w.y, dn), ld, d, o);
    at[tp.M + t] = a_in;
    darc[t] = d;
    a = a_in + d;
  }
  fw_a[k] = a;  // -inf in padding slots
  // the cell's maximum arrival, worst transition and first input attaining
  // the maximum (the head when none does, e.g. NaN)
  T best, so;
  int argl;
  if (((rec.w >> 24) & 127) <= 4) {  // every cell of the chunk has <= 4 inputs
    T ua[4], uo[4];
    seg_fetch<4>(a, head, tail, ua);
    seg_fetch<4>(o, head, tail, uo);
    int aj, oj;
    best = max_first<4>(ua, aj);
    so = max_first<4>(uo, oj);
    argl = head + aj;
  } else {
    best = seg_max(a, lane, head, tail);
    so = seg_max(o, lane, head, tail);
    const int arg0 = seg_min((valid && a == best) ? lane : 64, lane, head, tail);
    argl = arg0 <= tail ? arg0 : head;
  }
  if (valid && lane == head) {  // (the list job records the critical input's hop)
    const int v = tp.n_start + c;
    if (inc.arr && (!same_bits(old.x, best) || !same_bits(old.y, so)))
      inc.drv_chg[v] = inc.epoch;  // a changed output re-times the cells it drives
    at[v] = best;
    slew[v] = so;
    as[v] = v2<T>(best, so);
    crit[c] = argl - head;
  }
}

// hop4 of a cell: its own hop record followed by the first three of its
// critical input's driver's hop4 (terminal records {-1, -1, 0, 0} past a
// start point), so a path walk reads four hops per load
template <typename T, int KM>
__device__ __forceinline__ void fw_lists(const Topo &tp, int chunk, int lc1, const T *__restrict__ fw_a,
                                         int32_t *__restrict__ cdep, T *__restrict__ side_cost,
                                         int32_t *__restrict__ side_pin, int4 *__restrict__ hop4,
                                         const IncFlags &inc) {
  if (chunk >= lc1) return;
  const int lane = wave_lane();
  const int k = chunk * CHUNK + lane;
  const int4 rec = tp.fw_rec[k];
  const int2 ex = tp.fw_ext[k];
  const int t = rec.x, s = rec.y, c = rec.z;
  const int head = rec.w & 63, tail = (rec.w >> 8) & 63;
  const bool valid = t >= 0;
  const T a = fw_a[k];
  if (inc.lst) {  // incremental: the chunk was re-timed or an input's driver's list changed
    const bool mark = (valid && inc.drv_lchg[s] == inc.epoch) || inc.lst[chunk] == inc.epoch;
    if (__ballot(mark) == 0) return;
  }
  // the same maximum and critical input as the arrival job found
  const bool narrow = ((rec.w >> 24) & 127) <= 4;  // wave-uniform
  T ua[4];
  int ut[4], aj = 0;
  T best;
  int argl, pred, tc;
  int2 exc;
  if (narrow) {
    seg_fetch<4>(a, head, tail, ua);
    seg_fetch<4>(t, head, tail, ut);
    best = max_first<4>(ua, aj);
    argl = head + aj;
  } else {
    best = seg_max(a, lane, head, tail);
    const int arg0 = seg_min((valid && a == best) ? lane : 64, lane, head, tail);
    argl = arg0 <= tail ? arg0 : head;
  }
  pred = __shfl(s, argl & 63, 64);
  tc = __shfl(t, argl & 63, 64);
  exc = make_int2(__shfl(ex.x, argl & 63, 64), __shfl(ex.y, argl & 63, 64));
  const bool is_head = valid && lane == head;
  // Every load from the critical input's driver (its deviation list, hop
  // records and chain depth) comes before the first store in program order,
  // so the three share one memory latency (loads are not moved above the
  // stores).
  constexpr int KL = KM > 1 ? KM : 1;
  T kc[KL];
  int32_t kp[KL];
#pragma unroll
  for (int j = 0; j < KL; ++j) {
    kc[j] = pos_inf<T>();
    kp[j] = -1;
  }
  if constexpr (KM > 1) {
    if (is_head && pred >= tp.n_start) {
      const size_t pb = (size_t)(pred - tp.n_start) * KM;
      load_list<KM>(side_cost + pb, kc);
      load_list<KM>(side_pin + pb, kp);
    }
  }
  // incremental: whether this cell's list, hop records or chain depth change
  bool changed = false;
  if (is_head) {
    const int4 none = make_int4(-1, -1, 0, 0);
    int4 up0 = none, up1 = none, up2 = none;
    if (pred >= tp.n_start) {
      const int4 *ph = hop4 + (size_t)(pred - tp.n_start) * 4;
      up0 = ph[0];
      up1 = ph[1];
      up2 = ph[2];
    }
    const int32_t cd = cdep[pred];
    int4 *h = hop4 + (size_t)c * 4;
    const int4 h0 = make_int4(tc, pred, exc.x, exc.y);
    if (inc.lst) {
      auto ne = [](int4 a, int4 b) { return a.x != b.x || a.y != b.y || a.z != b.z || a.w != b.w; };
      changed = cdep[tp.n_start + c] != cd + 1 || ne(h[0], h0) || ne(h[1], up0) || ne(h[2], up1) || ne(h[3], up2);
    }
    cdep[tp.n_start + c] = cd + 1;
    h[0] = h0;
    h[1] = up0;
    h[2] = up1;
    h[3] = up2;
  }
  if constexpr (KM > 1) {
    // own deviations, last arc first so that equal costs keep arc order
    if (narrow) {
      if (is_head) {
#pragma unroll
        for (int j = 3; j >= 0; --j) {
          const T dj = best - ua[j];
          if (j <= tail - head && j != aj && dj < pos_inf<T>()) insert_front<T, KM>(kc, kp, dj, ut[j]);
        }
      }
    } else {
      const T dl = (valid && lane != argl) ? best - a : pos_inf<T>();
      const int width = wave_max_int(valid ? tail - head + 1 : 0);
      for (int r = 0; r < width; ++r) {
        const int j = tail - r;
        const T dj = __shfl(dl, j & 63, 64);
        const int tj = __shfl(t, j & 63, 64);
        if (is_head && j >= head && dj < pos_inf<T>()) insert_front<T, KM>(kc, kp, dj, tj);
      }
    }
    if (is_head) {
      const size_t cb = (size_t)c * KM;
      if (inc.lst) {
        T oc[KM];
        int32_t op[KM];
        load_list<KM>(side_cost + cb, oc);
        load_list<KM>(side_pin + cb, op);
#pragma unroll
        for (int j = 0; j < KM; ++j) changed = changed || !same_bits(oc[j], kc[j]) || op[j] != kp[j];
      }
      store_list<KM>(side_cost + cb, kc);
      store_list<KM>(side_pin + cb, kp);
    }
  }
  // the cells this one drives may take it as their critical input
  if (changed) inc.drv_lchg[tp.n_start + c] = inc.epoch;
}

// arrival chunks [ch0, ch1) in workgroups [0, n_arr); list chunks [lc0, lc1)
// in the rest
template <typename T, int KM>
__global__ void __launch_bounds__(256) k_forward(Topo tp, LutView L, int ch0, int ch1, int n_arr, int lc0, int lc1,
                                                  const T *__restrict__ load, const T *__restrict__ dnet,
                                                  T *__restrict__ at, T *__restrict__ slew, V2<T> *__restrict__ as,
                                                  T *__restrict__ darc, int32_t *__restrict__ crit,
                                                  int32_t *__restrict__ cdep,
                                                  T *__restrict__ side_cost, int32_t *__restrict__ side_pin,
                                                  T *__restrict__ fw_a, int4 *__restrict__ hop4, IncFlags inc) {
  extern __shared__ float4 s_lut4[];
  float *s_lut = (float *)s_lut4;
  const int wave = threadIdx.x >> 6;
  if ((int)blockIdx.x < n_arr)
    fw_arrivals<T>(tp, L, s_lut, ch0 + blockIdx.x * 4 + wave, ch1, load, dnet, at, slew, as, darc, crit, fw_a, inc);
  else
    fw_lists<T, KM>(tp, lc0 + (blockIdx.x - n_arr) * 4 + wave, lc1, fw_a, cdep, side_cost, side_pin, hop4, inc);
}

// ------------------------------------------------------------- endpoints
template <typename T>
__global__ void __launch_bounds__(256) k_endpoint(Topo tp, const double *__restrict__ inst_req,
                                                   const T *__restrict__ dnet, T *__restrict__ at,
                                                   T *__restrict__ rat, T *__restrict__ ep_slack) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= tp.E) return;
  const int t = tp.A + f;
  const T req = (T)inst_req[tp.ff_inst[f]];
  const T a = at[tp.snk_drv[t]] + dnet[t];
  const T s = req - a;
  at[tp.M + t] = a;
  rat[tp.M + t] = req;
  ep_slack[f] = s;
}

// per instance i, chunk j of its endpoint range: partial (min, sum of
// negatives, count of negatives)
template <typename T>
__global__ void __launch_bounds__(256) k_ep_partial(const int32_t *__restrict__ ep_base, int chunks,
                                                     const T *__restrict__ ep_slack, double *__restrict__ part) {
  __shared__ double smin[256], ssum[256], scnt[256];
  const int inst = blockIdx.x / chunks, j = blockIdx.x % chunks;
  const int b = ep_base[inst], e = ep_base[inst + 1];
  const int len = e - b;
  const int lo = b + (int)((long long)len * j / chunks), hi = b + (int)((long long)len * (j + 1) / chunks);
  double mn = 0.0, sm = 0.0, ct = 0.0;
  for (int f = lo + threadIdx.x; f < hi; f += blockDim.x) {
    const double s = (double)ep_slack[f];
    if (s < 0) {
      mn = s < mn ? s : mn;
      sm += s;
      ct += 1.0;
    }
  }
  smin[threadIdx.x] = mn;
  ssum[threadIdx.x] = sm;
  scnt[threadIdx.x] = ct;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      smin[threadIdx.x] = fmin(smin[threadIdx.x], smin[threadIdx.x + o]);
      ssum[threadIdx.x] += ssum[threadIdx.x + o];
      scnt[threadIdx.x] += scnt[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[3 * blockIdx.x + 0] = smin[0];
    part[3 * blockIdx.x + 1] = ssum[0];
    part[3 * blockIdx.x + 2] = scnt[0];
  }
}

// one thread per instance folds its chunks in order; summary[4i..] = wns, tns, n_fail
__global__ void k_ep_final(int num_inst, int chunks, const double *__restrict__ part, double *__restrict__ summary,
                           int32_t *__restrict__ inst_nfail) {
  const int inst = blockIdx.x * blockDim.x + threadIdx.x;
  if (inst >= num_inst) return;
  double mn = 0.0, sm = 0.0, ct = 0.0;
  for (int j = 0; j < chunks; ++j) {
    const double *p = part + 3 * (inst * chunks + j);
    mn = fmin(mn, p[0]);
    sm += p[1];
    ct += p[2];
  }
  summary[4 * inst + 0] = mn;
  summary[4 * inst + 1] = sm;
  summary[4 * inst + 2] = ct;
  summary[4 * inst + 3] = 0.0;
  inst_nfail[inst] = (int32_t)ct;
}

// ------------------------------------------------------------- backward
// A net's pass gives each of its sinks its required time (a combinational
// input: its cell output's minus the arc delay; a flip-flop D pin: set at the
// endpoint), then its driver the minimum over the sinks of (sink required
// time - net delay).  Slack is rat - at, formed where it is exported.  The
// net delays are read in chunk-slot order (dnet_nm).
template <typename T>
__device__ __forceinline__ T sink_required(int p, T r_out, T da, T *__restrict__ rat) {
  const T ri = r_out != pos_inf<T>() ? r_out - da : pos_inf<T>();
  rat[p] = ri;
  return ri;
}

template <typename T>
__global__ void __launch_bounds__(256) k_backward(Topo tp, int ch0, int ch1, const T *__restrict__ dnet_nm,
                                                   const T *__restrict__ darc, T *__restrict__ rat) {
  const int lane = wave_lane();
  const int chunk = ch0 + blockIdx.x * 4 + (threadIdx.x >> 6);
  if (chunk >= ch1) return;
  const int k = chunk * CHUNK + lane;
  const int4 rec = tp.nm_rec[k];
  const int p = rec.x, vo = rec.z;
  const int head = rec.w & 63, tail = (rec.w >> 8) & 63;
  T r = pos_inf<T>();
  if (p >= 0 && lane != head) {
    const T dn = dnet_nm[k];
    const T rt = vo >= 0 ? sink_required<T>(p, rat[vo], darc[p - tp.M], rat) : rat[p];
    if (rt != pos_inf<T>()) r = rt - dn;
  }
  r = seg_min(r, lane, head, tail);
  if (p >= 0 && lane == head) rat[p] = r;
}

template <typename T>
__global__ void k_backward_big(Topo tp, int i0, int i1, const T *__restrict__ dnet, const T *__restrict__ darc,
                               T *__restrict__ rat) {
  const int i = i0 + blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= i1) return;
  const int v = tp.big_net[i];
  T r = pos_inf<T>();
  for (int k = tp.net_ptr[v]; k < tp.net_ptr[v + 1]; ++k) {
    const int t = tp.net_sink[k];
    const int p = tp.M + t;
    const T rt = t < tp.A ? sink_required<T>(p, rat[tp.n_start + tp.snk_comb[t]], darc[t], rat) : rat[p];
    if (rt == pos_inf<T>()) continue;
    const T q = rt - dnet[t];
    r = q < r ? q : r;
  }
  rat[v] = r;
}

// ------------------------------------------------------ dataflow sweeps
// One launch per sweep on a resident grid: every workgroup of the launch is
// on the GPU at once (the grid is sized from the occupancy of the kernel, at
// most a few workgroups per compute unit, so a concurrent kernel on another
// stream cannot keep part of it waiting), and wave w of the W waves owns
// chunks w, w + W, w + 2W, ... in dependency order (forward: level order;
// backward: reverse level order).  For each chunk a wave loads its static
// data (the next chunk's record is already in flight), waits until the words
// it reads are published, computes exactly what the per-level kernels
// compute, and publishes its own words.  A chunk waits only on chunks with
// smaller indices, and every wave takes its chunks in increasing order, so
// the smallest unfinished chunk always has its inputs and its owner at it:
// the sweep completes.  The tables are staged in LDS once per workgroup, not
// once per chunk, and no workgroup is dispatched while the sweep runs.
// Every wait is also bounded, so a broken assumption ends in a reported
// error, not a hang.  One lane per wave polls (the word its chunk is likely
// to see published last) before the others load theirs, which keeps the
// polling traffic of the waiting waves off the frontier's way.
//
// Forward.  Arrival phase of a chunk: a lane loads its driver's {arrival,
// transition} word, waiting only if it is not out yet, and the cell's head
// lane publishes the output's word before anything else.  List phase (head
// lanes): the chain depth and the deviation list follow the critical input,
// every entry its own word, loaded at once and waited for only where still
// empty.  A wave runs the list phase of a chunk after the arrival phase of
// its next chunk: the list chain trails the arrival chain, and a list phase
// run at once would hold the wave (and its next arrivals) until the lists
// below it are out.  Deferral keeps the sweep deadlock-free: give the
// arrival phase of chunk c the key c and its list phase the key c + W; a
// phase waits only on phases of smaller keys, and every wave runs its phases
// in increasing key order (the arrival phase of chunk c, then the list phase
// of chunk c - W, whose key is also c), so the phase of smallest key not yet
// done always has its inputs and its wave at it.
struct FwPend {
  int4 rec;   // the chunk's record (rec.x = -1: nothing pending)
  float a;    // arrival through the lane's arc
  float best; // the cell's arrival
  int argl;   // lane of the critical input
  int pred;   // driver of the critical input
};

template <int KM>
__device__ __forceinline__ void fw_flow_lists(const Topo &tp, const FwPend &q, int32_t *__restrict__ cdep,
                                              float *__restrict__ side_cost, int32_t *__restrict__ side_pin,
                                              uint32_t *__restrict__ fcd, uint64_t *__restrict__ fse,
                                              int32_t *__restrict__ err, int limit) {
  const int lane = wave_lane();
  const int t = q.rec.x, c = q.rec.z;
  const int head = q.rec.w & 63, tail = (q.rec.w >> 8) & 63;
  const bool valid = t >= 0;
  const bool is_head = valid && lane == head;
  const int pred = q.pred;
  const int v = tp.n_start + c;
  // chain depth (+1 in the published word) and deviation list of the
  // critical input's driver
  constexpr int KL = KM > 1 ? KM : 1;
  const bool chain = is_head && pred >= tp.n_start;
  const size_t pb = chain ? (size_t)(pred - tp.n_start) * KM : 0;
  uint32_t cdp = is_head ? pub_ld(&fcd[pred]) : 1u;
  uint64_t pe[KL];
  bool miss = cdp == 0u;
#pragma unroll
  for (int j = 0; j < KL; ++j) {
    pe[j] = (KM > 1 && chain) ? pub_ld(&fse[pb + j]) : 0ull;
    miss = miss || pe[j] == W_EMPTY;
  }
  if (__ballot(miss)) {
    const int p_rep = wave_max_int(miss ? pred : -1);
    if (lane == 0) (void)wait_pub(&fcd[p_rep], 0u, err, limit);
    // then every word still missing is loaded again, all at once (one round
    // trip per poll, not one per word)
    int it = 0;
    while (__ballot(miss)) {
      if (miss) {
        if (cdp == 0u) cdp = pub_ld(&fcd[pred]);
#pragma unroll
        for (int j = 0; j < KL; ++j)
          if (pe[j] == W_EMPTY) pe[j] = pub_ld(&fse[pb + j]);
        miss = cdp == 0u;
#pragma unroll
        for (int j = 0; j < KL; ++j) miss = miss || pe[j] == W_EMPTY;
      }
      if (++it > limit) {
        if (lane == 0) atomicOr(err, 2);
        break;
      }
      if ((it & 31) == 0 && __ballot(__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0)) break;
      if (__ballot(miss)) __builtin_amdgcn_s_sleep(1);
    }
  }
  if (is_head) cdep[v] = (int32_t)cdp;
  if constexpr (KM > 1) {
    const float dl = (valid && lane != q.argl) ? q.best - q.a : __builtin_huge_valf();
    const int width = wave_max_int(valid ? tail - head + 1 : 0);
    float kc[KM];
    int32_t kp[KM];
#pragma unroll
    for (int j = 0; j < KM; ++j) {
      kc[j] = chain ? __uint_as_float((uint32_t)pe[j]) : __builtin_huge_valf();
      kp[j] = chain ? (int32_t)(uint32_t)(pe[j] >> 32) : -1;
    }
    // own deviations, last arc first so that equal costs keep arc order
    for (int r = 0; r < width; ++r) {
      const int j = tail - r;
      const float dj = __shfl(dl, j & 63, 64);
      const int tj = __shfl(t, j & 63, 64);
      if (is_head && j >= head && dj < __builtin_huge_valf()) insert_front<float, KM>(kc, kp, dj, tj);
    }
    if (is_head) {
      const size_t cb = (size_t)c * KM;
#pragma unroll
      for (int j = 0; j < KM; ++j) {
        pub_st(&fse[cb + j], (uint64_t)__float_as_uint(kc[j]) | ((uint64_t)(uint32_t)kp[j] << 32));
        side_cost[cb + j] = kc[j];
        side_pin[cb + j] = kp[j];
      }
    }
  }
  if (is_head) pub_st(&fcd[v], cdp + 1);
}

template <int KM>
__global__ void __launch_bounds__(256) k_forward_flow(Topo tp, LutView L, const float *__restrict__ load,
                                                       const float *__restrict__ dnet, float *__restrict__ at,
                                                       float *__restrict__ slew, float *__restrict__ darc,
                                                       int32_t *__restrict__ crit, int4 *__restrict__ hop,
                                                       int32_t *__restrict__ cdep, float *__restrict__ side_cost,
                                                       int32_t *__restrict__ side_pin, uint64_t *__restrict__ fw,
                                                       uint32_t *__restrict__ fcd, uint64_t *__restrict__ fse,
                                                       int32_t *__restrict__ err,
                                                       int limit) {
  extern __shared__ float4 s_lut4[];
  float *s_lut = (float *)s_lut4;
  const int lane = wave_lane();
  const int wpb = blockDim.x >> 6;
  const int W = gridDim.x * wpb;
  const int nch = tp.n_fw_chunks;
  int chunk = blockIdx.x * wpb + (threadIdx.x >> 6);
  int4 nrec = make_int4(-1, 0, 0, 0);
  int2 nex = make_int2(0, 0);
  if (chunk < nch) {
    nrec = tp.fw_rec[chunk * CHUNK + lane];
    nex = tp.fw_ext[chunk * CHUNK + lane];
  }
  stage_lut(L, s_lut);
  FwPend pend;
  bool pending = false;
  for (; chunk < nch; chunk += W) {
    const int4 rec = nrec;
    const int2 ex = nex;
    if (chunk + W < nch) {  // the next chunk's static data, in flight while this one waits
      nrec = tp.fw_rec[(chunk + W) * CHUNK + lane];
      nex = tp.fw_ext[(chunk + W) * CHUNK + lane];
    }
    const int t = rec.x, s = rec.y, c = rec.z, ty = (rec.w >> 16) & 255;
    const int head = rec.w & 63, tail = (rec.w >> 8) & 63;
    const bool valid = t >= 0;
    float a = -__builtin_huge_valf(), o = 0.f;
    float ld = 0.f, dn = 0.f;
    if (valid) {
      ld = load[tp.n_start + c];
      dn = dnet[t];
    }
    const uint64_t w = load_or_wait(fw, valid ? s : 0, valid, W_EMPTY, err, limit);
    if (valid) {
      const float a_in = __uint_as_float((uint32_t)w) + dn;
      float d;
      lut_lds<float>(s_lut, L.nt, L.ns, L.nl, ty, sink_slew<float>(L.net_model, __uint_as_float((uint32_t)(w >> 32)), dn),
                     ld, d, o);
      at[tp.M + t] = a_in;
      darc[t] = d;
      a = a_in + d;
    }
    const float best = seg_max(a, lane, head, tail);
    const float so = seg_max(o, lane, head, tail);
    // first input attaining the maximum (the head when none does, e.g. NaN)
    const int arg0 = seg_min((valid && a == best) ? lane : 64, lane, head, tail);
    const int argl = arg0 <= tail ? arg0 : head;
    const bool is_head = valid && lane == head;
    const int v = tp.n_start + c;
    if (is_head) pub_st(&fw[v], pack2(best, so));
    const int tc = __shfl(t, argl & 63, 64);
    const int pred = __shfl(s, argl & 63, 64);
    const int2 exc = make_int2(__shfl(ex.x, argl & 63, 64), __shfl(ex.y, argl & 63, 64));
    if (is_head) {
      at[v] = best;
      slew[v] = so;
      crit[c] = argl - head;
      hop[c] = make_int4(tc, pred, exc.x, exc.y);
    }
    if (pending) fw_flow_lists<KM>(tp, pend, cdep, side_cost, side_pin, fcd, fse, err, limit);
    pend.rec = rec;
    pend.a = a;
    pend.best = best;
    pend.argl = argl;
    pend.pred = pred;
    pending = true;
  }
  if (pending) fw_flow_lists<KM>(tp, pend, cdep, side_cost, side_pin, fcd, fse, err, limit);
}

// Backward: chunks from the last; a sink lane loads the required time of its
// cell's output (the D pin of a flip-flop needs nothing), waiting only if it
// is not out yet; the driver lane publishes its own.
__global__ void __launch_bounds__(256) k_backward_flow(Topo tp, const float *__restrict__ dnet_nm,
                                                        const float *__restrict__ darc, float *__restrict__ rat,
                                                        uint32_t *__restrict__ fr, int32_t *__restrict__ err,
                                                        int limit) {
  const int lane = wave_lane();
  const float inf = __builtin_huge_valf();
  const int wpb = blockDim.x >> 6;
  const int W = gridDim.x * wpb;
  const int nch = tp.n_nm_chunks;
  int q = blockIdx.x * wpb + (threadIdx.x >> 6);
  int4 nrec = q < nch ? tp.nm_rec[(nch - 1 - q) * CHUNK + lane] : make_int4(-1, -1, -1, 0);
  for (; q < nch; q += W) {
    const int chunk = nch - 1 - q;
    const int k = chunk * CHUNK + lane;
    const int4 rec = nrec;
    if (q + W < nch) nrec = tp.nm_rec[(nch - 1 - q - W) * CHUNK + lane];
    const int p = rec.x, vo = rec.z;
    const int head = rec.w & 63, tail = (rec.w >> 8) & 63;
    const bool sink = p >= 0 && lane != head;
    const int t = p - tp.M;
    const bool comb_in = sink && vo >= 0;
    const float dn = sink ? dnet_nm[k] : 0.f, da = comb_in ? darc[t] : 0.f;
    const float rq = sink && !comb_in ? rat[p] : 0.f;  // a D pin's, set at the endpoint
    // outputs are numbered in production order of the forward sweep, so the
    // backward sweep publishes the lowest one last
    const uint32_t wr = load_or_wait<true>(fr, comb_in ? vo : 0, comb_in, R_EMPTY, err, limit);
    float r = inf;
    if (sink) {
      const float rt = comb_in ? sink_required<float>(p, __uint_as_float(wr), da, rat) : rq;
      if (rt != inf) r = rt - dn;
    }
    r = seg_min(r, lane, head, tail);
    if (p >= 0 && lane == head) {
      pub_st(&fr[p], __float_as_uint(r));
      rat[p] = r;
    }
  }
}

// hop4 from the hop records, for the dataflow forward sweep (the per-level
// one builds it as it goes): three dependent gathers per cell
__global__ void __launch_bounds__(256) k_hop4_fill(Topo tp, const int4 *__restrict__ hop, int4 *__restrict__ hop4) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= tp.n_comb) return;
  int4 cur = hop[c];
  int4 *h = hop4 + (size_t)c * 4;
  h[0] = cur;
  for (int j = 1; j < 4; ++j) {
    if (cur.x >= 0 && cur.y >= tp.n_start) cur = hop[cur.y - tp.n_start];
    else cur = make_int4(-1, -1, 0, 0);
    h[j] = cur;
  }
}

// --------------------------------------------------------------- export
template <typename T>
__global__ void __launch_bounds__(256) k_export(Topo tp, const T *__restrict__ at, const T *__restrict__ rat,
                                                 const T *__restrict__ slew,
                                                 const T *__restrict__ dnet, const T *__restrict__ load,
                                                 const T *__restrict__ darc, double *o_at, double *o_rat,
                                                 double *o_slack, double *o_slew, double *o_dnet,
                                                 double *o_load, double *o_darc, int net_model) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= tp.P) return;
  const int i = tp.ext_pin_int[p];
  const bool sink = i >= tp.M;
  const int t = i - tp.M;
  if (o_at) o_at[p] = (double)at[i];
  if (o_rat) o_rat[p] = (double)rat[i];
  if (o_slack) o_slack[p] = (double)(rat[i] != pos_inf<T>() ? rat[i] - at[i] : pos_inf<T>());
  if (o_slew) o_slew[p] = (double)(sink ? sink_slew<T>(net_model, slew[tp.snk_drv[t]], dnet[t]) : slew[i]);
  if (o_dnet) o_dnet[p] = sink ? (double)dnet[t] : 0.0;
  if (o_load) o_load[p] = sink ? 0.0 : (double)load[i];
  if (o_darc) o_darc[p] = (sink && t < tp.A) ? (double)darc[t] : 0.0;
}

__global__ void k_export_crit(Topo tp, const int32_t *__restrict__ crit, int32_t *__restrict__ out) {
  const int cell = blockIdx.x * blockDim.x + threadIdx.x;
  if (cell >= tp.N) return;
  const int ci = tp.cell_int[cell];
  out[cell] = ci >= 0 ? crit[ci] : -1;
}

// --------------------------------------------------------------- launchers
static inline int nblk(long long n, int b) { return n > 0 ? (int)((n + b - 1) / b) : 1; }

static inline size_t lut_bytes(const LutView &L) { return sizeof(float4) * (size_t)L.n4; }

template <typename T, int KM>
static void launch_forward(tdp_graph g, int ch0, int ch1, int lc0, int lc1, const IncFlags &inc, hipStream_t s) {
  const Topo &tp = g->topo;
  const int n_arr = ch1 > ch0 ? nblk(ch1 - ch0, 4) : 0;
  const int n_lst = lc1 > lc0 ? nblk(lc1 - lc0, 4) : 0;
  if (n_arr + n_lst == 0) return;
  hipLaunchKernelGGL((k_forward<T, KM>), dim3(n_arr + n_lst), dim3(256), n_arr ? lut_bytes(g->lut) : 0, s, tp,
                     g->lut, ch0, ch1, n_arr, lc0, lc1, (const T *)g->load, (const T *)g->dnet, (T *)g->at,
                     (T *)g->slew, (V2<T> *)g->drv_as, (T *)g->darc, g->crit, g->cdep,
                     (T *)g->side_cost, g->side_pin, (T *)g->fw_a, (int4 *)g->hop4, inc);
}

// arrivals of chunks [ch0, ch1) and the lists of [lc0, lc1), the level before
template <typename T>
static void forward_level(tdp_graph g, int ch0, int ch1, int lc0, int lc1, const IncFlags &inc, hipStream_t s) {
  switch (g->side_k) {
    case 1: launch_forward<T, 1>(g, ch0, ch1, lc0, lc1, inc, s); break;
    case 2: launch_forward<T, 2>(g, ch0, ch1, lc0, lc1, inc, s); break;
    case 4: launch_forward<T, 4>(g, ch0, ch1, lc0, lc1, inc, s); break;
    case 8: launch_forward<T, 8>(g, ch0, ch1, lc0, lc1, inc, s); break;
    case 16: launch_forward<T, 16>(g, ch0, ch1, lc0, lc1, inc, s); break;
    default: launch_forward<T, 32>(g, ch0, ch1, lc0, lc1, inc, s); break;
  }
}

// the per-level forward sweep over every level (incremental: with flags)
template <typename T>
static void forward_levels(tdp_graph g, const IncFlags &inc, hipStream_t s) {
  const Topo &tp = g->topo;
  int lc0 = 0, lc1 = 0;  // the previous non-empty level, whose lists are due
  for (int l = 1; l <= tp.D; ++l) {
    const int ch0 = g->lv.fw_lvl[l - 1], ch1 = g->lv.fw_lvl[l];
    if (ch1 <= ch0) continue;
    forward_level<T>(g, ch0, ch1, lc0, lc1, inc, s);
    lc0 = ch0;
    lc1 = ch1;
  }
  forward_level<T>(g, 0, 0, lc0, lc1, inc, s);
}

// workgroups of a resident grid of `waves`-wave workgroups over nch chunks:
// flow_per_cu per compute unit, within the kernel's occupancy (cached per
// wave count), and no more than the chunks need
static int resident_blocks(tdp_graph g, const void *kern, int32_t *occ_cache, int waves, size_t lds, int nch) {
  const int wi = waves == 1 ? 0 : (waves == 2 ? 1 : 2);
  if (occ_cache[wi] < 0) {
    int occ = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, 64 * waves, lds) != hipSuccess || occ < 1) occ = 1;
    occ_cache[wi] = occ;
  }
  const long long per = std::min(occ_cache[wi], g->flow_per_cu);
  const long long need = nblk(nch, waves);
  return (int)std::max(1LL, std::min(per * std::max(1, g->num_cu), need));
}

template <int KM>
static void launch_forward_flow(tdp_graph g, hipStream_t s) {
  const Topo &tp = g->topo;
  const int w = g->flow_waves;
  const int nb = resident_blocks(g, reinterpret_cast<const void *>(&k_forward_flow<KM>), g->occ_fw, w,
                                 lut_bytes(g->lut), tp.n_fw_chunks);
  hipLaunchKernelGGL((k_forward_flow<KM>), dim3(nb), dim3(64 * w), lut_bytes(g->lut), s, tp, g->lut,
                     (const float *)g->load, (const float *)g->dnet, (float *)g->at, (float *)g->slew,
                     (float *)g->darc, g->crit, (int4 *)g->hop, g->cdep, (float *)g->side_cost, g->side_pin,
                     g->flow_w, g->flow_cd, g->flow_se, g->d_err, g->spin_limit);
}

static void forward_flow(tdp_graph g, hipStream_t s) {
  switch (g->side_k) {
    case 1: launch_forward_flow<1>(g, s); break;
    case 2: launch_forward_flow<2>(g, s); break;
    case 4: launch_forward_flow<4>(g, s); break;
    case 8: launch_forward_flow<8>(g, s); break;
    case 16: launch_forward_flow<16>(g, s); break;
    default: launch_forward_flow<32>(g, s); break;
  }
}

// net pass: pin positions, net delays, driver loads, start points (and the
// reset of the dataflow words in trailing workgroups)
template <typename T>
static void netpass_launch(tdp_graph g, const float *x, const float *y, const FlowInit &fl, hipStream_t s) {
  const Topo &tp = g->topo;
  const NetModel<T> nm = net_model<T>(g);
  const bool tree = g->lut.net_model == 2;
  const T *tree_wl = tree ? (const T *)g->tree.wl : nullptr;
  pack_xy(x, y, g->xy, tp.N, s, g->d_err + 1, ++g->pos_gen);
  const auto k_np = tree ? k_netpass<T, true> : k_netpass<T, false>;
  hipLaunchKernelGGL(k_np, dim3(nblk(tp.n_nm_chunks, 4) + fl.reset_blocks),
                     dim3(256), 0, s, tp, g->lut, g->xy, nm,
                     (T)g->c, (T)g->input_slew, (T)g->clock_slew, (T *)g->load, (T *)g->dnet, (T *)g->dnet_nm,
                     g->cxy_nm, (T *)g->at, (T *)g->slew, (V2<T> *)g->drv_as, g->cdep, fl);
  // nets wider than a chunk: their trees one thread per net first
  if (tp.n_big > 0 && tree) tree_net_impl<T>(g, g->tree, x, y, (T *)g->dnet, tp.big_net, tp.n_big, s);
  if (tp.n_big > 0)
    hipLaunchKernelGGL(k_netpass_big<T>, dim3(nblk(tp.n_big, 64)), dim3(64), 0, s, tp, g->lut, x, y, nm, tree_wl,
                       (T)g->c, (T)g->input_slew, (T)g->clock_slew, (T *)g->load, (T *)g->dnet, (T *)g->at,
                       (T *)g->slew, (V2<T> *)g->drv_as, g->cdep);
}

template <typename T>
void ep_reduce_impl(tdp_graph g, hipStream_t s) {
  const Topo &tp = g->topo;
  hipLaunchKernelGGL(k_ep_partial<T>, dim3(tp.num_inst * g->ep_chunks), dim3(256), 0, s, g->d_ep_base,
                     g->ep_chunks, (const T *)g->ep_slack, g->red_ep);
  hipLaunchKernelGGL(k_ep_final, dim3(nblk(tp.num_inst, 64)), dim3(64), 0, s, tp.num_inst, g->ep_chunks, g->red_ep,
                     g->summary, g->inst_nfail);
}

template <typename T>
void netpass_impl(tdp_graph g, const float *x, const float *y, hipStream_t s) {
  FlowInit fl;
  fl.err = g->d_err;
  netpass_launch<T>(g, x, y, fl, s);
}

// arrivals: net pass, forward sweep, endpoint slacks and WNS / TNS
template <typename T>
void sta_arrivals_impl(tdp_graph g, const float *x, const float *y, hipStream_t s) {
  const Topo &tp = g->topo;
  const NetModel<T> nm = net_model<T>(g);
  // sweep_mode 1 and 2: both sweeps as resident dataflow grids; 3: the
  // backward one only
  const bool flow = sizeof(T) == 4 && g->flow_ok && (g->sweep_mode == 1 || g->sweep_mode == 2);
  const bool bflow = sizeof(T) == 4 && g->flow_ok && g->sweep_mode >= 1;
  FlowInit fl;
  fl.err = g->d_err;
  if (flow) {
    fl.w = g->flow_w;
    fl.cd = g->flow_cd;
    fl.se = g->flow_se;
    fl.km = g->side_k > 1 ? g->side_k : 0;
    fl.seed = g->sweep_mode == 2 ? 0 : 1;
  }
  if (bflow) {
    fl.r = g->flow_r;
    fl.reset_blocks = flow ? 1024 : 64;
  }
  prof_begin(g, TDP_STAGE_NETPASS, s);
  netpass_launch<T>(g, x, y, fl, s);
  g->flow_r_clear = bflow;
  prof_end(g, TDP_STAGE_NETPASS, s);
  prof_begin(g, TDP_STAGE_FORWARD, s);
  g->drv_as_stale = flow;  // the dataflow sweep publishes through its own words
  if (flow) {
    forward_flow(g, s);
    if (tp.n_comb > 0)
      hipLaunchKernelGGL(k_hop4_fill, dim3(nblk(tp.n_comb, 256)), dim3(256), 0, s, tp, (const int4 *)g->hop,
                         (int4 *)g->hop4);
  } else {
    forward_levels<T>(g, IncFlags{}, s);
  }
  prof_end(g, TDP_STAGE_FORWARD, s);
  prof_begin(g, TDP_STAGE_ENDPOINT, s);
  if (tp.E > 0)
    hipLaunchKernelGGL(k_endpoint<T>, dim3(nblk(tp.E, 256)), dim3(256), 0, s, tp, g->d_inst_req, (const T *)g->dnet,
                       (T *)g->at, (T *)g->rat, (T *)g->ep_slack);
  ep_reduce_impl<T>(g, s);
  prof_end(g, TDP_STAGE_ENDPOINT, s);
}

// ---------------------------------------------------- incremental update
// forward chunk of every combinational input; net chunk of every driver
__global__ void k_inc_maps(Topo tp, int32_t *__restrict__ snk_chunk, int32_t *__restrict__ drv_nm_chunk) {
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long nf = (long long)tp.n_fw_chunks * CHUNK, nn = (long long)tp.n_nm_chunks * CHUNK;
  if (k < nf) {
    const int t = tp.fw_rec[k].x;
    if (t >= 0) snk_chunk[t] = (int)(k / CHUNK);
  } else if (k < nf + nn) {
    const long long q = k - nf;
    const int4 rec = tp.nm_rec[q];
    if (rec.x >= 0 && (int)(q % CHUNK) == (rec.w & 63)) drv_nm_chunk[rec.x] = (int)(q / CHUNK);
  }
}

// {arrival, transition} pairs of the combinational drivers from the two
// arrays, and each forward slot's arrival through its arc (the same sum the
// arrival job forms), after a forward sweep that kept neither
template <typename T>
__global__ void k_pack_as(Topo tp, const T *__restrict__ at, const T *__restrict__ slew, const T *__restrict__ darc,
                          V2<T> *__restrict__ as, T *__restrict__ fw_a) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int v = tp.n_start + (int)i;
  if (v < tp.M) as[v] = v2<T>(at[v], slew[v]);
  if (i < (long long)tp.n_fw_chunks * CHUNK) {
    const int t = tp.fw_rec[i].x;
    fw_a[i] = t >= 0 ? at[tp.M + t] + darc[t] : -pos_inf<T>();
  }
}

// the net chunks that hold a moved cell's pins: its output's net and the nets
// of its inputs (bit 2 of err: an id outside [0, N))
__global__ void k_inc_mark(Topo tp, const int32_t *__restrict__ cells, int n, const int32_t *__restrict__ drv_nm_chunk,
                           int32_t *__restrict__ nm, int32_t epoch, int32_t *__restrict__ err) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int e = cells[i];
  if (e < 0 || e >= tp.N) {
    atomicOr(err, 4);
    return;
  }
  const int ci = tp.cell_int[e];
  auto mark = [&](int u) { nm[drv_nm_chunk[u]] = epoch; };
  if (ci >= 0) {
    mark(tp.n_start + ci);
    for (int t = tp.comb_inptr[ci]; t < tp.comb_inptr[ci + 1]; ++t) mark(tp.snk_drv[t]);
  } else {
    const int f = -ci - 1;
    mark(tp.n_pi + f);
    mark(tp.snk_drv[tp.A + f]);
  }
}

template <typename T>
void sta_arrivals_incremental_impl(tdp_graph g, const float *x, const float *y, const int32_t *cells, int n,
                                   hipStream_t s) {
  const Topo &tp = g->topo;
  const NetModel<T> nm = net_model<T>(g);
  IncFlags inc;
  inc.epoch = g->inc_epoch;
  inc.arr = g->inc_arr;
  inc.lst = g->inc_lst;
  inc.drv_chg = g->inc_drv_chg;
  inc.drv_lchg = g->inc_drv_lchg;
  inc.snk_chunk = g->inc_snk_chunk;
  inc.nm = g->inc_nm;
  prof_begin(g, TDP_STAGE_NETPASS, s);
  if (g->drv_as_stale && tp.n_comb > 0)
    hipLaunchKernelGGL(k_pack_as<T>, dim3(nblk(std::max<long long>(tp.n_comb, (long long)tp.n_fw_chunks * CHUNK), 256)),
                       dim3(256), 0, s, tp, (const T *)g->at, (const T *)g->slew, (const T *)g->darc,
                       (V2<T> *)g->drv_as, (T *)g->fw_a);
  g->drv_as_stale = false;
  fill_i32(g->d_err, 1, 0, s);
  if (n > 0)
    hipLaunchKernelGGL(k_inc_mark, dim3(nblk(n, 256)), dim3(256), 0, s, tp, cells, n, g->inc_drv_nm_chunk,
                       g->inc_nm, inc.epoch, g->d_err);
  pack_xy(x, y, g->xy, tp.N, s, g->d_err + 1, ++g->pos_gen);
  // (every net fits a chunk here: graphs with wider nets take full updates)
  const auto k_npm = g->lut.net_model == 2 ? k_netpass_marked<T, true> : k_netpass_marked<T, false>;
  if (n > 0)
    hipLaunchKernelGGL(k_npm, dim3(nblk(tp.n_nm_chunks, 4)),
                       dim3(256), 0, s, tp, g->lut, g->xy, nm, (T)g->c,
                       (T)g->input_slew, (T)g->clock_slew, (T *)g->load, (T *)g->dnet, (T *)g->dnet_nm, g->cxy_nm,
                       (T *)g->at, (T *)g->slew, (V2<T> *)g->drv_as, g->cdep, inc);
  prof_end(g, TDP_STAGE_NETPASS, s);
  prof_begin(g, TDP_STAGE_FORWARD, s);
  forward_levels<T>(g, inc, s);
  prof_end(g, TDP_STAGE_FORWARD, s);
  prof_begin(g, TDP_STAGE_ENDPOINT, s);
  if (tp.E > 0)
    hipLaunchKernelGGL(k_endpoint<T>, dim3(nblk(tp.E, 256)), dim3(256), 0, s, tp, g->d_inst_req, (const T *)g->dnet,
                       (T *)g->at, (T *)g->rat, (T *)g->ep_slack);
  ep_reduce_impl<T>(g, s);
  prof_end(g, TDP_STAGE_ENDPOINT, s);
}

void inc_maps(tdp_graph g, hipStream_t s) {
  const Topo &tp = g->topo;
  const long long total = ((long long)tp.n_fw_chunks + tp.n_nm_chunks) * CHUNK;
  hipLaunchKernelGGL(k_inc_maps, dim3(nblk(total, 256)), dim3(256), 0, s, tp, g->inc_snk_chunk, g->inc_drv_nm_chunk);
}

template <typename T>
void sta_required_impl(tdp_graph g, hipStream_t s) {
  const Topo &tp = g->topo;
  const bool flow = sizeof(T) == 4 && g->flow_ok && g->sweep_mode >= 1;  // modes 1-3
  prof_begin(g, TDP_STAGE_BACKWARD, s);
  if (flow) {
    // the words are reset by a full arrival pass that plans this sweep; after
    // any other (incremental, per-level, or none since the last sweep) they
    // are reset here
    if (!g->flow_r_clear) fill_i32(reinterpret_cast<int32_t *>(g->flow_r), tp.M, (int32_t)R_EMPTY, s);
    g->flow_r_clear = false;
    const int w = g->flow_waves;
    const int nb = resident_blocks(g, reinterpret_cast<const void *>(&k_backward_flow), g->occ_bw, w, 0,
                                   tp.n_nm_chunks);
    hipLaunchKernelGGL(k_backward_flow, dim3(nb), dim3(64 * w), 0, s, tp,
                       (const float *)g->dnet_nm, (const float *)g->darc, (float *)g->rat, g->flow_r, g->d_err,
                       g->spin_limit);
    prof_end(g, TDP_STAGE_BACKWARD, s);
    return;
  }
  for (int l = tp.D; l >= 0; --l) {
    const int ch0 = g->lv.nm_lvl[l], ch1 = g->lv.nm_lvl[l + 1];
    if (ch1 > ch0)
      hipLaunchKernelGGL(k_backward<T>, dim3(nblk(ch1 - ch0, 4)), dim3(256), 0, s, tp, ch0, ch1,
                         (const T *)g->dnet_nm, (const T *)g->darc, (T *)g->rat);
    const int b0 = g->lv.big_lvl[l], b1 = g->lv.big_lvl[l + 1];
    if (b1 > b0)
      hipLaunchKernelGGL(k_backward_big<T>, dim3(nblk(b1 - b0, 64)), dim3(64), 0, s, tp, b0, b1, (const T *)g->dnet,
                         (const T *)g->darc, (T *)g->rat);
  }
  prof_end(g, TDP_STAGE_BACKWARD, s);
}

template <typename T>
void sta_export_impl(tdp_graph g, double *at, double *rat, double *slack, double *slew, double *dnet,
                     double *load, double *darc, hipStream_t s) {
  const Topo &tp = g->topo;
  hipLaunchKernelGGL(k_export<T>, dim3(nblk(tp.P, 256)), dim3(256), 0, s, tp, (const T *)g->at,
                     (const T *)g->rat, (const T *)g->slew, (const T *)g->dnet,
                     (const T *)g->load, (const T *)g->darc, at, rat, slack, slew, dnet, load, darc,
                     g->lut.net_model);
}

void sta_export_crit(tdp_graph g, int32_t *out, hipStream_t s) {
  hipLaunchKernelGGL(k_export_crit, dim3(nblk(g->topo.N, 256)), dim3(256), 0, s, g->topo, g->crit, out);
}

template void ep_reduce_impl<float>(tdp_graph, hipStream_t);
template void ep_reduce_impl<double>(tdp_graph, hipStream_t);
template void netpass_impl<float>(tdp_graph, const float *, const float *, hipStream_t);
template void netpass_impl<double>(tdp_graph, const float *, const float *, hipStream_t);
template void sta_arrivals_incremental_impl<float>(tdp_graph, const float *, const float *, const int32_t *, int,
                                                   hipStream_t);
template void sta_arrivals_incremental_impl<double>(tdp_graph, const float *, const float *, const int32_t *, int,
                                                    hipStream_t);
template void sta_arrivals_impl<float>(tdp_graph, const float *, const float *, hipStream_t);
template void sta_arrivals_impl<double>(tdp_graph, const float *, const float *, hipStream_t);
template void sta_required_impl<float>(tdp_graph, hipStream_t);
template void sta_required_impl<double>(tdp_graph, hipStream_t);
template void sta_export_impl<float>(tdp_graph, double *, double *, double *, double *, double *, double *,
                                     double *, hipStream_t);
template void sta_export_impl<double>(tdp_graph, double *, double *, double *, double *, double *, double *,
                                      double *, hipStream_t);

}  // namespace tdp
