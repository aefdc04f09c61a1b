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
// once.  Values are staged in LDS by aligned groups of 16 positions (64
// bytes), three groups deep (group index mod 3), and written out by the lane
// itself at flush points that the whole wave shares, every WALK_FLUSH steps
// of the walk.  A wave's vector loads wait for its earlier stores (they
// retire in order), so batching the stores of several steps leaves fewer
// steps whose next record load waits behind stores.  Between two flushes a
// lane puts at most 8 * WALK_FLUSH = 32 positions, so it completes at most
// three groups and never overwrites a completed group before writing it.
// `row`: this thread's LDS row of WALK_ROW words.
constexpr int WALK_FLUSH = 4;
constexpr int WALK_ROW = 97;  // 3 groups x (16 a + 16 b), +1 against bank conflicts

struct RevWriter {
  int32_t *a, *b;
  int32_t *row;
  int pos, lo, hi;  // next position (descending), path range [lo, hi)
  int np = 0;       // completed groups waiting for the next flush, lowest positions
  int p0a = 0, p0b = 0, p0c = 0;
  __device__ void put(int32_t va, int32_t vb) {
    const int j = pos & 15, g = ((unsigned)pos >> 4) % 3u;
    row[g * 32 + j] = va;
    row[g * 32 + 16 + j] = vb;
    if (j == 0 || pos == lo) {
      if (np == 0) p0a = pos;
      else if (np == 1) p0b = pos;
      else p0c = pos;
      ++np;
    }
    --pos;
  }
  __device__ void write_group(int p0) {
    const int top = min(hi - 1, p0 | 15);
    const int32_t *ga = row + (((unsigned)p0 >> 4) % 3u) * 32, *gb = ga + 16;
    if ((p0 & 15) == 0 && top == p0 + 15) {
#pragma unroll
      for (int q = 0; q < 16; q += 4) {
        *(int4 *)(a + p0 + q) = make_int4(ga[q], ga[q + 1], ga[q + 2], ga[q + 3]);
        *(int4 *)(b + p0 + q) = make_int4(gb[q], gb[q + 1], gb[q + 2], gb[q + 3]);
      }
      return;
    }
    for (int p = p0; p <= top; ++p) {
      a[p] = ga[p & 15];
      b[p] = gb[p & 15];
    }
  }
  __device__ void flush() {
    if (np > 0) write_group(p0a);
    if (np > 1) write_group(p0b);
    if (np > 2) write_group(p0c);
    np = 0;
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
// walk filled the path's range exactly and used every deviation.  Every lane
// of the wave calls it (live = false: no path), so that the steps and the
// flush points are the wave's.
//
// Group-synchronous: every step all lanes load the four-hop record of their
// current cell together (one memory latency for the wave) and advance up to
// four cells along it; a deviation cell leaves the chain and ends the lane's
// step early.
template <class Next>
__device__ __forceinline__ bool walk_path(const Topo &tp, const int4 *__restrict__ hop4, RevWriter &w, int f,
                                          bool live, Next &&next) {
  const int lo = w.lo;
  int v = 0, dt = -1, dc = -1;
  bool done = !live;
  if (live) {
    const int et = tp.A + f;
    w.put(tp.snk_ext[et], tp.M + et);
    v = tp.snk_drv[et];
    w.put(tp.drv_ext[v], v);
    // the next deviation in registers: its sink and cell
    dt = next();
    dc = dt >= 0 ? tp.snk_comb[dt] : -1;
    done = v < tp.n_start;
  }
  w.flush();
  for (int step = 1; __ballot(!done && w.pos >= lo); ++step) {
    if (!done && w.pos >= lo) {
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
    if (step % WALK_FLUSH == 0) w.flush();
  }
  w.flush();
  return live && w.pos == lo - 1 && v < tp.n_start && dt < 0;
}

}  // namespace tdp
