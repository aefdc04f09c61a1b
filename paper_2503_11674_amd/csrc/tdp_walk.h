// Path materialisation shared by the per-endpoint and the design-wide
// extraction (Sec. III-B): a path is its endpoint plus the deviations it takes
// from the arrival-time tree; walking back from the endpoint, it follows the
// critical input of every cell except where a deviation names another input.
#pragma once

#include "tdp_internal.h"

namespace tdp {

template <typename T> __device__ __forceinline__ T inf_of();
template <> __device__ __forceinline__ float inf_of<float>() { return __builtin_huge_valf(); }
template <> __device__ __forceinline__ double inf_of<double>() { return __builtin_huge_val(); }

// Writes a path from its last position down to its first, two arrays at
// once.  Values are staged in LDS per aligned group of 32 positions (128
// bytes) and a group goes out in one burst when its lowest position is
// written (or the path starts inside it), so the L2 sees whole lines instead
// of scattered words.  `sa` / `sb`: this thread's 33-word LDS rows (the odd
// stride keeps the lanes of a wave on different banks).
struct RevWriter {
  int32_t *a, *b;
  int32_t *sa, *sb;
  int pos, lo, hi;  // next position (descending), path range [lo, hi)
  __device__ void put(int32_t va, int32_t vb) {
    const int j = pos & 31;
    sa[j] = va;
    sb[j] = vb;
    if (j == 0 || pos == lo) flush(pos, j);
    --pos;
  }
  __device__ void flush(int p0, int j0) {
    const int top = min(hi - 1, p0 | 31);
    if (j0 == 0 && top == p0 + 31) {
#pragma unroll
      for (int q = 0; q < 32; q += 4) {
        *(int4 *)(a + p0 + q) = make_int4(sa[q], sa[q + 1], sa[q + 2], sa[q + 3]);
        *(int4 *)(b + p0 + q) = make_int4(sb[q], sb[q + 1], sb[q + 2], sb[q + 3]);
      }
      return;
    }
    for (int p = p0; p <= top; ++p) {
      a[p] = sa[p & 31];
      b[p] = sb[p & 31];
    }
  }
};

// Deviations of a node of the design-wide search, read through its parent
// links: a node's own deviation is its path's upstream-most one and the
// root's ancestors-first order is the walk's order.  Buffered 16 at a time;
// each refill follows the links from the node, so any number of deviations
// works with a fixed amount of private memory.
struct LinkDevs {
  const int32_t *dev, *par;
  int node, nd, used, nb, bi;
  int buf[16];
  __device__ void refill() {
    const int d0 = used + 1, d1 = min(nd, used + 16);
    int a = node;
    for (int d = nd; d > d1 && a >= 0; --d) a = par[a];
    for (int d = d1; d >= d0; --d) {
      buf[d - d0] = a >= 0 ? dev[a] : -1;
      a = a >= 0 ? par[a] : -1;
    }
    nb = d1 - d0 + 1;
    bi = 0;
  }
  __device__ __forceinline__ int next() {
    if (used >= nd) return -1;
    if (bi >= nb) refill();
    ++used;
    return buf[bi++];
  }
};

// Walks the path into endpoint f (flip-flop index) from its end to its start
// point and writes it through w.  next() yields the path's deviations (sink
// pins), the one nearest the endpoint first, then -1.  Returns whether the
// walk filled the path's range exactly and used every deviation.
//
// Group-synchronous: every iteration all lanes load the four-hop record of
// their current cell together (one memory latency for the wave) and advance
// up to four cells along it; a deviation cell leaves the chain and ends the
// lane's group early.
template <class Next>
__device__ __forceinline__ bool walk_path(const Topo &tp, const int4 *__restrict__ hop4, RevWriter &w, int f,
                                          Next &&next) {
  const int lo = w.lo;
  const int et = tp.A + f;
  w.put(tp.snk_ext[et], tp.M + et);
  int v = tp.snk_drv[et];
  w.put(tp.drv_ext[v], v);
  // the next deviation in registers: its sink and cell
  int dt = next();
  int dc = dt >= 0 ? tp.snk_comb[dt] : -1;
  bool done = v < tp.n_start;
  while (!done && w.pos >= lo) {
    const int4 *hp = hop4 + (size_t)(v - tp.n_start) * 4;
    const int4 g0 = hp[0], g1 = hp[1], g2 = hp[2], g3 = hp[3];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int c = v - tp.n_start;
      int t, text, nv, nvext;
      const bool dev = c == dc;
      if (dev) {
        t = dt;
        text = tp.snk_ext[t];
        nv = tp.snk_drv[t];
        nvext = tp.drv_ext[nv];
        dt = next();
        dc = dt >= 0 ? tp.snk_comb[dt] : -1;
      } else {
        const int4 h = i == 0 ? g0 : (i == 1 ? g1 : (i == 2 ? g2 : g3));
        t = h.x;
        nv = h.y;
        text = h.z;
        nvext = h.w;
      }
      if (w.pos < lo) {
        done = true;
        break;
      }
      w.put(text, tp.M + t);
      if (w.pos < lo) {
        done = true;
        break;
      }
      w.put(nvext, nv);
      v = nv;
      if (v < tp.n_start) {
        done = true;
        break;
      }
      if (dev) break;  // off the chain: reload at the new cell
    }
  }
  return w.pos == lo - 1 && v < tp.n_start && dt < 0;
}

}  // namespace tdp
