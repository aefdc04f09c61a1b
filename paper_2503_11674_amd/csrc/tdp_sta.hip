// Static timing analysis kernels (Sec. II-B, Eqs. 2-4; net delay Eq. 7).
//
// One update is:
//   net pass   every net as a segment of a 64-lane chunk (driver lane, then
//              its sinks): pin positions, the RC delay into each sink
//              (kappa * L^2, L Manhattan), the driver's load (star model,
//              a segmented sum); start points get arrival and transition.
//   forward    one launch per level; one lane per combinational input pin,
//              a cell's inputs adjacent: arrival = segmented max over inputs of
//              (driver arrival + net delay + table delay at the input's
//              transition and the output load), output transition =
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
#include "tdp_wave.h"

namespace tdp {

template <typename T> __device__ __forceinline__ T pos_inf();
template <> __device__ __forceinline__ float pos_inf<float>() { return __builtin_huge_valf(); }
template <> __device__ __forceinline__ double pos_inf<double>() { return __builtin_huge_val(); }

__device__ __forceinline__ void stage_lut(const LutView &L, float *s_lut) {
  const int nsl = L.nt * L.ns, nld = L.nt * L.nl, ntab = L.nt * L.ns * L.nl;
  for (int i = threadIdx.x; i < nsl; i += blockDim.x) s_lut[i] = L.slew_axis[i];
  for (int i = threadIdx.x; i < nld; i += blockDim.x) s_lut[nsl + i] = L.load_axis[i];
  for (int i = threadIdx.x; i < ntab; i += blockDim.x) {
    s_lut[nsl + nld + i] = L.delay[i];
    s_lut[nsl + nld + ntab + i] = L.slew[i];
  }
  __syncthreads();
}

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

// Poll *p until it differs from `empty`.  The wait is bounded: after `limit`
// polls (or once another wave has given up) it sets bit 2 of *err and returns
// `empty`, so every wave always finishes.
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

struct FlowInit {
  uint64_t *w = nullptr;
  uint32_t *r = nullptr, *cd = nullptr;
  uint64_t *se = nullptr;
  int32_t *tickets = nullptr;
  int32_t *err = nullptr;  // cleared at the start of every update
  int km = 0;
  int seed = 1;  // 0: start points are never published (self-test of the bounded waits)
};

template <typename T>
__device__ __forceinline__ void start_point(const Topo &tp, const LutView &L, int v, T ld, T in_slew, T clk_slew,
                                            T *__restrict__ at, T *__restrict__ slew, int32_t *__restrict__ cdep,
                                            const FlowInit &fl) {
  T a = 0, s = in_slew;
  if (v >= tp.n_pi && v < tp.n_start) lut_pair<T>(L, tp.ff_type[v - tp.n_pi], clk_slew, ld, a, s);
  if (v < tp.n_start) {
    at[v] = a;
    slew[v] = s;
    cdep[v] = 0;
  }
  if (fl.w) {  // reset (or seed) the words the dataflow sweeps poll
    fl.r[v] = R_EMPTY;
    if (v < tp.n_start) {
      fl.w[v] = fl.seed ? pack2((float)a, (float)s) : W_EMPTY;
      fl.cd[v] = fl.seed ? 1 : 0;
    } else {
      fl.w[v] = W_EMPTY;
      fl.cd[v] = 0;
      const size_t b = (size_t)(v - tp.n_start) * fl.km;
      for (int j = 0; j < fl.km; ++j) fl.se[b + j] = W_EMPTY;
    }
  }
}

// ------------------------------------------------------------- net pass
template <typename T>
__global__ void __launch_bounds__(256) k_netpass(Topo tp, LutView L, const float *__restrict__ x,
                                                  const float *__restrict__ y, T kappa, T cw, T in_slew,
                                                  T clk_slew, T *__restrict__ load, T *__restrict__ dnet,
                                                  T *__restrict__ at, T *__restrict__ slew,
                                                  int32_t *__restrict__ cdep, FlowInit fl) {
  if (blockIdx.x == 0 && threadIdx.x == 0 && fl.err) *fl.err = 0;
  if (fl.tickets && blockIdx.x == 0 && threadIdx.x < 4) fl.tickets[threadIdx.x] = 0;
  const int lane = wave_lane();
  const int chunk = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (chunk >= tp.n_nm_chunks) return;
  const int k = chunk * CHUNK + lane;
  const int p = tp.nm_pin[k];
  const int sg = tp.nm_seg[k];
  const int head = sg & 63, tail = (sg >> 8) & 63;
  const int cell = tp.nm_cell[k];
  const T X = (cell >= 0 ? (T)x[cell] : (T)0) + (T)tp.nm_ox[k];
  const T Y = (cell >= 0 ? (T)y[cell] : (T)0) + (T)tp.nm_oy[k];
  const T Xd = __shfl(X, head, 64), Yd = __shfl(Y, head, 64);
  const bool sink = p >= 0 && lane != head;
  const T len = sink ? fabs(Xd - X) + fabs(Yd - Y) : (T)0;
  if (sink) dnet[p - tp.M] = kappa * len * len;
  const T wl = seg_sum(len, lane, head, tail);
  if (p >= 0 && lane == head) {
    const T ld = (T)tp.net_cpin[p] + cw * wl;
    load[p] = ld;
    start_point<T>(tp, L, p, ld, in_slew, clk_slew, at, slew, cdep, fl);
  }
}

// nets too wide for one chunk: one thread per net
template <typename T>
__global__ void k_netpass_big(Topo tp, LutView L, const float *__restrict__ x, const float *__restrict__ y, T kappa,
                              T cw, T in_slew, T clk_slew, T *__restrict__ load, T *__restrict__ dnet,
                              T *__restrict__ at, T *__restrict__ slew, int32_t *__restrict__ cdep) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= tp.n_big) return;
  const int v = tp.big_net[i];
  const int dc = tp.drv_cell[v];
  const T xs = (dc >= 0 ? (T)x[dc] : (T)0) + (T)tp.drv_ox[v];
  const T ys = (dc >= 0 ? (T)y[dc] : (T)0) + (T)tp.drv_oy[v];
  T wl = 0;
  for (int k = tp.net_ptr[v]; k < tp.net_ptr[v + 1]; ++k) {
    const int t = tp.net_sink[k];
    const int sc = tp.snk_cell[t];
    const T len = fabs(xs - ((T)x[sc] + (T)tp.snk_ox[t])) + fabs(ys - ((T)y[sc] + (T)tp.snk_oy[t]));
    dnet[t] = kappa * len * len;
    wl += len;
  }
  const T ld = (T)tp.net_cpin[v] + cw * wl;
  load[v] = ld;
  start_point<T>(tp, L, v, ld, in_slew, clk_slew, at, slew, cdep, FlowInit{});
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
template <typename T, int KM>
__global__ void __launch_bounds__(256) k_forward(Topo tp, LutView L, int ch0, int ch1, const T *__restrict__ load,
                                                  const T *__restrict__ dnet, T *__restrict__ at,
                                                  T *__restrict__ slew, T *__restrict__ darc,
                                                  int32_t *__restrict__ crit, int4 *__restrict__ hop,
                                                  int32_t *__restrict__ cdep, T *__restrict__ side_cost,
                                                  int32_t *__restrict__ side_pin) {
  extern __shared__ float s_lut[];
  stage_lut(L, s_lut);
  const int lane = wave_lane();
  const int chunk = ch0 + blockIdx.x * 4 + (threadIdx.x >> 6);
  if (chunk >= ch1) return;
  const int k = chunk * CHUNK + lane;
  const int t = tp.fw_t[k];
  const int sg = tp.fw_seg[k];
  const int head = sg & 63, tail = (sg >> 8) & 63;
  const bool valid = t >= 0;
  int c = 0, s = 0;
  T a = -pos_inf<T>(), o = 0;
  if (valid) {
    c = tp.snk_comb[t];
    s = tp.snk_drv[t];
    const T ld = load[tp.n_start + c];
    const T a_in = at[s] + dnet[t];
    T d;
    lut_lds<T>(s_lut, L.nt, L.ns, L.nl, tp.comb_type[c], slew[s], ld, d, o);
    at[tp.M + t] = a_in;
    darc[t] = d;
    a = a_in + d;
  }
  const T best = seg_max(a, lane, head, tail);
  const T so = seg_max(o, lane, head, tail);
  // first input attaining the maximum (the head when none does, e.g. NaN)
  const int arg0 = seg_min((valid && a == best) ? lane : 64, lane, head, tail);
  const int argl = arg0 <= tail ? arg0 : head;
  const int tc = __shfl(t, argl & 63, 64);
  const int pred = __shfl(s, argl & 63, 64);
  const bool is_head = valid && lane == head;
  if (is_head) {
    const int v = tp.n_start + c;
    at[v] = best;
    slew[v] = so;
    crit[c] = argl - head;
    // critical input, its driver and their external ids: one record per hop
    // of a path walk
    hop[c] = make_int4(tc, pred, tp.snk_ext[tc], tp.drv_ext[pred]);
    cdep[v] = cdep[pred] + 1;
  }
  if constexpr (KM > 1) {
    const T dl = (valid && lane != argl) ? best - a : pos_inf<T>();
    const int width = wave_max_int(valid ? tail - head + 1 : 0);
    T kc[KM];
    int32_t kp[KM];
#pragma unroll
    for (int j = 0; j < KM; ++j) {
      kc[j] = pos_inf<T>();
      kp[j] = -1;
    }
    if (is_head && pred >= tp.n_start) {
      const size_t pb = (size_t)(pred - tp.n_start) * KM;
#pragma unroll
      for (int j = 0; j < KM; ++j) {
        kc[j] = side_cost[pb + j];
        kp[j] = side_pin[pb + j];
      }
    }
    // own deviations, last arc first so that equal costs keep arc order
    for (int r = 0; r < width; ++r) {
      const int j = tail - r;
      const T dj = __shfl(dl, j & 63, 64);
      const int tj = __shfl(t, j & 63, 64);
      if (is_head && j >= head && dj < pos_inf<T>()) insert_front<T, KM>(kc, kp, dj, tj);
    }
    if (is_head) {
      const size_t cb = (size_t)c * KM;
#pragma unroll
      for (int j = 0; j < KM; ++j) {
        side_cost[cb + j] = kc[j];
        side_pin[cb + j] = kp[j];
      }
    }
  }
}

// ------------------------------------------------------------- endpoints
template <typename T>
__global__ void __launch_bounds__(256) k_endpoint(Topo tp, T req, const T *__restrict__ dnet, T *__restrict__ at,
                                                   T *__restrict__ rat, T *__restrict__ slack,
                                                   T *__restrict__ ep_slack) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= tp.E) return;
  const int t = tp.A + f;
  const T a = at[tp.snk_drv[t]] + dnet[t];
  const T s = req - a;
  at[tp.M + t] = a;
  rat[tp.M + t] = req;
  slack[tp.M + t] = s;
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
template <typename T>
__device__ __forceinline__ void give_inputs(const Topo &tp, int v, T r, const T *__restrict__ darc,
                                            const T *__restrict__ at, T *__restrict__ rat, T *__restrict__ slack) {
  const bool fin = r != pos_inf<T>();
  rat[v] = r;
  slack[v] = fin ? r - at[v] : pos_inf<T>();
  if (v < tp.n_start) return;
  const int c = v - tp.n_start;
  const int b = tp.comb_inptr[c], e = tp.comb_inptr[c + 1];
  for (int t = b; t < e; ++t) {
    const T ri = fin ? r - darc[t] : pos_inf<T>();
    rat[tp.M + t] = ri;
    slack[tp.M + t] = fin ? ri - at[tp.M + t] : pos_inf<T>();
  }
}

template <typename T>
__global__ void __launch_bounds__(256) k_backward(Topo tp, int ch0, int ch1, const T *__restrict__ dnet,
                                                   const T *__restrict__ darc, const T *__restrict__ at,
                                                   T *__restrict__ rat, T *__restrict__ slack) {
  const int lane = wave_lane();
  const int chunk = ch0 + blockIdx.x * 4 + (threadIdx.x >> 6);
  if (chunk >= ch1) return;
  const int k = chunk * CHUNK + lane;
  const int p = tp.nm_pin[k];
  const int sg = tp.nm_seg[k];
  const int head = sg & 63, tail = (sg >> 8) & 63;
  T r = pos_inf<T>();
  if (p >= 0 && lane != head) {
    const T rt = rat[p];
    if (rt != pos_inf<T>()) r = rt - dnet[p - tp.M];
  }
  r = seg_min(r, lane, head, tail);
  if (p >= 0 && lane == head) give_inputs<T>(tp, p, r, darc, at, rat, slack);
}

template <typename T>
__global__ void k_backward_big(Topo tp, int i0, int i1, const T *__restrict__ dnet, const T *__restrict__ darc,
                               const T *__restrict__ at, T *__restrict__ rat, T *__restrict__ slack) {
  const int i = i0 + blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= i1) return;
  const int v = tp.big_net[i];
  T r = pos_inf<T>();
  for (int k = tp.net_ptr[v]; k < tp.net_ptr[v + 1]; ++k) {
    const int t = tp.net_sink[k];
    const T rt = rat[tp.M + t];
    if (rt == pos_inf<T>()) continue;
    const T q = rt - dnet[t];
    r = q < r ? q : r;
  }
  give_inputs<T>(tp, v, r, darc, at, rat, slack);
}

// ------------------------------------------------------ dataflow sweeps
// One persistent launch per sweep.  Each wave takes the next 64-lane chunk
// from a ticket counter (forward: level order; backward: reverse level
// order), waits until the words it reads are published, computes exactly
// what the per-level kernels compute, and publishes its own words.  A chunk
// only waits on chunks with a smaller ticket, which running waves have
// already taken, so the sweep always completes; every wait is also bounded.
//
// Forward, phase 1: a lane polls its driver's {arrival, transition} word.
// Phase 2 (head lanes, after the cell's word is out): the chain depth and the
// deviation list follow the critical input, one polled word per entry.
template <int KM>
__global__ void __launch_bounds__(256) k_forward_flow(Topo tp, LutView L, const float *__restrict__ load,
                                                       const float *__restrict__ dnet, float *__restrict__ at,
                                                       float *__restrict__ slew, float *__restrict__ darc,
                                                       int32_t *__restrict__ crit, int4 *__restrict__ hop,
                                                       int32_t *__restrict__ cdep, float *__restrict__ side_cost,
                                                       int32_t *__restrict__ side_pin, uint64_t *__restrict__ fw,
                                                       uint32_t *__restrict__ fcd, uint64_t *__restrict__ fse,
                                                       int32_t *__restrict__ ticket, int32_t *__restrict__ err,
                                                       int limit) {
  extern __shared__ float s_lut[];
  stage_lut(L, s_lut);
  const int lane = wave_lane();
  for (;;) {
    int chunk = 0;
    if (lane == 0) chunk = atomicAdd(ticket, 1);
    chunk = __shfl(chunk, 0, 64);
    if (chunk >= tp.n_fw_chunks) break;
    const int k = chunk * CHUNK + lane;
    const int t = tp.fw_t[k];
    const int sg = tp.fw_seg[k];
    const int head = sg & 63, tail = (sg >> 8) & 63;
    const bool valid = t >= 0;
    int c = 0, s = 0;
    float a = -__builtin_huge_valf(), o = 0.f;
    if (valid) {
      c = tp.snk_comb[t];
      s = tp.snk_drv[t];
      const float ld = load[tp.n_start + c];
      const float dn = dnet[t];
      const int ty = tp.comb_type[c];
      const uint64_t w = wait_pub(&fw[s], W_EMPTY, err, limit);
      const float a_in = __uint_as_float((uint32_t)w) + dn;
      float d;
      lut_lds<float>(s_lut, L.nt, L.ns, L.nl, ty, __uint_as_float((uint32_t)(w >> 32)), ld, d, o);
      at[tp.M + t] = a_in;
      darc[t] = d;
      a = a_in + d;
    }
    const float best = seg_max(a, lane, head, tail);
    const float so = seg_max(o, lane, head, tail);
    // first input attaining the maximum (the head when none does, e.g. NaN)
  const int arg0 = seg_min((valid && a == best) ? lane : 64, lane, head, tail);
  const int argl = arg0 <= tail ? arg0 : head;
    const int tc = __shfl(t, argl & 63, 64);
    const int pred = __shfl(s, argl & 63, 64);
    const bool is_head = valid && lane == head;
    const int v = tp.n_start + c;
    if (is_head) {
      at[v] = best;
      slew[v] = so;
      crit[c] = argl - head;
      hop[c] = make_int4(tc, pred, tp.snk_ext[tc], tp.drv_ext[pred]);
      pub_st(&fw[v], pack2(best, so));
    }
    // phase 2: chain depth (+1 in the published word) and deviation list
    uint32_t cdp = 0;
    if (is_head) {
      cdp = wait_pub(&fcd[pred], 0u, err, limit);
      cdep[v] = (int32_t)cdp;
    }
    if constexpr (KM > 1) {
      const float dl = (valid && lane != argl) ? best - a : __builtin_huge_valf();
      const int width = wave_max_int(valid ? tail - head + 1 : 0);
      float kc[KM];
      int32_t kp[KM];
#pragma unroll
      for (int j = 0; j < KM; ++j) {
        kc[j] = __builtin_huge_valf();
        kp[j] = -1;
      }
      if (is_head && pred >= tp.n_start) {
        const size_t pb = (size_t)(pred - tp.n_start) * KM;
#pragma unroll
        for (int j = 0; j < KM; ++j) {
          const uint64_t e = wait_pub(&fse[pb + j], W_EMPTY, err, limit);
          kc[j] = __uint_as_float((uint32_t)e);
          kp[j] = (int32_t)(uint32_t)(e >> 32);
        }
      }
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
          side_cost[cb + j] = kc[j];
          side_pin[cb + j] = kp[j];
          pub_st(&fse[cb + j], (uint64_t)__float_as_uint(kc[j]) | ((uint64_t)(uint32_t)kp[j] << 32));
        }
      }
    }
    if (is_head) pub_st(&fcd[v], cdp + 1);
  }
}

// Backward: a sink lane polls the required time of its cell's output (the D
// pin of a flip-flop needs nothing); the driver lane publishes its own.
__global__ void __launch_bounds__(256) k_backward_flow(Topo tp, float req, const float *__restrict__ dnet,
                                                        const float *__restrict__ darc, const float *__restrict__ at,
                                                        float *__restrict__ rat, float *__restrict__ slack,
                                                        uint32_t *__restrict__ fr, int32_t *__restrict__ ticket,
                                                        int32_t *__restrict__ err, int limit) {
  const int lane = wave_lane();
  const float inf = __builtin_huge_valf();
  for (;;) {
    int q = 0;
    if (lane == 0) q = atomicAdd(ticket, 1);
    q = __shfl(q, 0, 64);
    if (q >= tp.n_nm_chunks) break;
    const int chunk = tp.n_nm_chunks - 1 - q;
    const int k = chunk * CHUNK + lane;
    const int p = tp.nm_pin[k];
    const int sg = tp.nm_seg[k];
    const int head = sg & 63, tail = (sg >> 8) & 63;
    float r = inf;
    if (p >= 0 && lane != head) {
      const int t = p - tp.M;
      float rt = req;
      if (t < tp.A) {
        const uint32_t ro = wait_pub(&fr[tp.n_start + tp.snk_comb[t]], R_EMPTY, err, limit);
        const float r_out = __uint_as_float(ro);
        rt = r_out != inf ? r_out - darc[t] : inf;
      }
      if (rt != inf) r = rt - dnet[t];
    }
    r = seg_min(r, lane, head, tail);
    if (p >= 0 && lane == head) {
      give_inputs<float>(tp, p, r, darc, at, rat, slack);
      pub_st(&fr[p], __float_as_uint(r));
    }
  }
}

// --------------------------------------------------------------- export
template <typename T>
__global__ void __launch_bounds__(256) k_export(Topo tp, const T *__restrict__ at, const T *__restrict__ rat,
                                                 const T *__restrict__ slack, const T *__restrict__ slew,
                                                 const T *__restrict__ dnet, const T *__restrict__ load,
                                                 const T *__restrict__ darc, double *o_at, double *o_rat,
                                                 double *o_slack, double *o_slew, double *o_dnet,
                                                 double *o_load, double *o_darc) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= tp.P) return;
  const int i = tp.ext_pin_int[p];
  const bool sink = i >= tp.M;
  const int t = i - tp.M;
  if (o_at) o_at[p] = (double)at[i];
  if (o_rat) o_rat[p] = (double)rat[i];
  if (o_slack) o_slack[p] = (double)slack[i];
  if (o_slew) o_slew[p] = (double)(sink ? slew[tp.snk_drv[t]] : slew[i]);
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

static inline size_t lut_bytes(const LutView &L) {
  return sizeof(float) * (size_t)(L.nt * (L.ns + L.nl) + 2 * L.nt * L.ns * L.nl);
}

template <typename T, int KM>
static void launch_forward(tdp_graph g, int ch0, int ch1, hipStream_t s) {
  const Topo &tp = g->topo;
  hipLaunchKernelGGL((k_forward<T, KM>), dim3(nblk(ch1 - ch0, 4)), dim3(256), lut_bytes(g->lut), s, tp, g->lut, ch0,
                     ch1, (const T *)g->load, (const T *)g->dnet, (T *)g->at, (T *)g->slew, (T *)g->darc, g->crit,
                     (int4 *)g->hop, g->cdep, (T *)g->side_cost, g->side_pin);
}

template <typename T>
static void forward_level(tdp_graph g, int ch0, int ch1, hipStream_t s) {
  switch (g->side_k) {
    case 1: launch_forward<T, 1>(g, ch0, ch1, s); break;
    case 2: launch_forward<T, 2>(g, ch0, ch1, s); break;
    case 4: launch_forward<T, 4>(g, ch0, ch1, s); break;
    case 8: launch_forward<T, 8>(g, ch0, ch1, s); break;
    case 16: launch_forward<T, 16>(g, ch0, ch1, s); break;
    default: launch_forward<T, 32>(g, ch0, ch1, s); break;
  }
}

template <int KM>
static void launch_forward_flow(tdp_graph g, hipStream_t s) {
  const Topo &tp = g->topo;
  hipLaunchKernelGGL((k_forward_flow<KM>), dim3(g->flow_blocks), dim3(256), lut_bytes(g->lut), s, tp, g->lut,
                     (const float *)g->load, (const float *)g->dnet, (float *)g->at, (float *)g->slew,
                     (float *)g->darc, g->crit, (int4 *)g->hop, g->cdep, (float *)g->side_cost, g->side_pin,
                     g->flow_w, g->flow_cd, g->flow_se, g->tickets, g->d_err, g->spin_limit);
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

template <typename T>
void sta_update_impl(tdp_graph g, const float *x, const float *y, hipStream_t s) {
  const Topo &tp = g->topo;
  const T kappa = (T)g->scale * (T)g->r * (T)g->c;
  const bool flow = sizeof(T) == 4 && g->flow_ok && g->sweep_mode >= 1;
  FlowInit fl;
  fl.err = g->d_err;
  if (flow) {
    fl.w = g->flow_w;
    fl.r = g->flow_r;
    fl.cd = g->flow_cd;
    fl.se = g->flow_se;
    fl.tickets = g->tickets;
    fl.km = g->side_k > 1 ? g->side_k : 0;
    fl.seed = g->sweep_mode == 2 ? 0 : 1;
  }
  prof_begin(g, TDP_STAGE_NETPASS, s);
  hipLaunchKernelGGL(k_netpass<T>, dim3(nblk(tp.n_nm_chunks, 4)), dim3(256), 0, s, tp, g->lut, x, y, kappa,
                     (T)g->c, (T)g->input_slew, (T)g->clock_slew, (T *)g->load, (T *)g->dnet, (T *)g->at,
                     (T *)g->slew, g->cdep, fl);
  if (tp.n_big > 0)
    hipLaunchKernelGGL(k_netpass_big<T>, dim3(nblk(tp.n_big, 64)), dim3(64), 0, s, tp, g->lut, x, y, kappa,
                       (T)g->c, (T)g->input_slew, (T)g->clock_slew, (T *)g->load, (T *)g->dnet, (T *)g->at,
                       (T *)g->slew, g->cdep);
  prof_end(g, TDP_STAGE_NETPASS, s);
  prof_begin(g, TDP_STAGE_FORWARD, s);
  if (flow) {
    forward_flow(g, s);
  } else {
    for (int l = 1; l <= tp.D; ++l) {
      const int ch0 = g->lv.fw_lvl[l - 1], ch1 = g->lv.fw_lvl[l];
      if (ch1 > ch0) forward_level<T>(g, ch0, ch1, s);
    }
  }
  prof_end(g, TDP_STAGE_FORWARD, s);
  prof_begin(g, TDP_STAGE_ENDPOINT, s);
  const T req = (T)g->clock_period - (T)g->setup;
  if (tp.E > 0)
    hipLaunchKernelGGL(k_endpoint<T>, dim3(nblk(tp.E, 256)), dim3(256), 0, s, tp, req, (const T *)g->dnet,
                       (T *)g->at, (T *)g->rat, (T *)g->slack, (T *)g->ep_slack);
  hipLaunchKernelGGL(k_ep_partial<T>, dim3(tp.num_inst * g->ep_chunks), dim3(256), 0, s, g->d_ep_base,
                     g->ep_chunks, (const T *)g->ep_slack, g->red_ep);
  hipLaunchKernelGGL(k_ep_final, dim3(nblk(tp.num_inst, 64)), dim3(64), 0, s, tp.num_inst, g->ep_chunks, g->red_ep,
                     g->summary, g->inst_nfail);
  prof_end(g, TDP_STAGE_ENDPOINT, s);
  prof_begin(g, TDP_STAGE_BACKWARD, s);
  if (flow) {
    hipLaunchKernelGGL(k_backward_flow, dim3(g->flow_blocks), dim3(256), 0, s, tp, (float)req, (const float *)g->dnet,
                       (const float *)g->darc, (const float *)g->at, (float *)g->rat, (float *)g->slack, g->flow_r,
                       g->tickets + 1, g->d_err, g->spin_limit);
    prof_end(g, TDP_STAGE_BACKWARD, s);
    return;
  }
  for (int l = tp.D; l >= 0; --l) {
    const int ch0 = g->lv.nm_lvl[l], ch1 = g->lv.nm_lvl[l + 1];
    if (ch1 > ch0)
      hipLaunchKernelGGL(k_backward<T>, dim3(nblk(ch1 - ch0, 4)), dim3(256), 0, s, tp, ch0, ch1, (const T *)g->dnet,
                         (const T *)g->darc, (const T *)g->at, (T *)g->rat, (T *)g->slack);
    const int b0 = g->lv.big_lvl[l], b1 = g->lv.big_lvl[l + 1];
    if (b1 > b0)
      hipLaunchKernelGGL(k_backward_big<T>, dim3(nblk(b1 - b0, 64)), dim3(64), 0, s, tp, b0, b1, (const T *)g->dnet,
                         (const T *)g->darc, (const T *)g->at, (T *)g->rat, (T *)g->slack);
  }
  prof_end(g, TDP_STAGE_BACKWARD, s);
}

template <typename T>
void sta_export_impl(tdp_graph g, double *at, double *rat, double *slack, double *slew, double *dnet,
                     double *load, double *darc, hipStream_t s) {
  const Topo &tp = g->topo;
  hipLaunchKernelGGL(k_export<T>, dim3(nblk(tp.P, 256)), dim3(256), 0, s, tp, (const T *)g->at,
                     (const T *)g->rat, (const T *)g->slack, (const T *)g->slew, (const T *)g->dnet,
                     (const T *)g->load, (const T *)g->darc, at, rat, slack, slew, dnet, load, darc);
}

void sta_export_crit(tdp_graph g, int32_t *out, hipStream_t s) {
  hipLaunchKernelGGL(k_export_crit, dim3(nblk(g->topo.N, 256)), dim3(256), 0, s, g->topo, g->crit, out);
}

template void sta_update_impl<float>(tdp_graph, const float *, const float *, hipStream_t);
template void sta_update_impl<double>(tdp_graph, const float *, const float *, hipStream_t);
template void sta_export_impl<float>(tdp_graph, double *, double *, double *, double *, double *, double *,
                                     double *, hipStream_t);
template void sta_export_impl<double>(tdp_graph, double *, double *, double *, double *, double *, double *,
                                      double *, hipStream_t);

}  // namespace tdp
