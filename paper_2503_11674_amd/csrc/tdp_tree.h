// The spanning-tree net model on a 64-lane net chunk (a lane per pin, each
// net a segment [head, tail] with its driver at the head): the net pass and
// the smoothed TNS build their trees with these.
//
// Prim's algorithm runs on every segment at once, one pin joining each
// unfinished segment per round: the segment's nearest outside pin (ties to
// the lowest lane, which is the net's order), hung from the tree pin that
// reached it first at that distance.  The minima are exact, so the DPP
// reductions pick the same pins wherever a segment sits in the wave.  Then
// each sink's wire from its parent, the capacitance at and below it (reverse
// joining order) and its Elmore delay (joining order): the operations of the
// one-thread-per-net form, in its order.  Every lane of the wave must call
// these functions.  (fx, fy, fox, foy) are a pin's cell coordinates and
// offset as given (a port: no cell, its position as the offset), which
// decide the topology; (cx, cy, ox, oy) the same position in the timing
// precision with a port's position as the base, for the wire lengths.
#pragma once

#include "tdp_wave.h"

namespace tdp {

template <typename T>
struct ChunkTree {
  int par;     // parent lane (the head for the driver itself)
  int st;      // round in which the lane joined (-1: the driver, padding)
  int who;     // for lane head + 1 + j: the lane that joined in round j
  int rounds;  // rounds of the wave (its widest segment's sink count)
  T len;       // wire from the parent (0 off the sinks)
  T cd;        // capacitance at and below the pin
};

template <typename T>
__device__ __forceinline__ ChunkTree<T> tree_chunk_build(T cw, int lane, int head, int tail, bool sink, float fx,
                                                          float fy, float fox, float foy, T cx, T cy, T ox, T oy,
                                                          T cap) {
  const float hx = __shfl(fx, head, 64), hy = __shfl(fy, head, 64);
  const float hox = __shfl(fox, head, 64), hoy = __shfl(foy, head, 64);
  bool out = sink;  // not yet in the tree
  float dist = sink ? tree_fdist(hx, hy, hox, hoy, fx, fy, fox, foy) : 0.f;
  ChunkTree<T> tr;
  tr.par = head;
  tr.st = -1;
  tr.who = lane;
  int rounds = 0;
  while (__ballot(out)) {
    // non-finite distances (non-finite positions) rank last
    const float key = out && dist == dist ? dist : __builtin_huge_valf();
    const float mn = seg_min_dpp(key, lane, head, tail);
    const int pick = seg_min_dpp(out && key == mn ? lane : 64, lane, head, tail);
    const bool got = pick < 64;
    if (got && lane == pick) {
      out = false;
      tr.st = rounds;
    }
    if (got && lane == head + 1 + rounds) tr.who = pick;
    const int src = got ? pick : lane;
    const float px = __shfl(fx, src, 64), py = __shfl(fy, src, 64);
    const float pox = __shfl(fox, src, 64), poy = __shfl(foy, src, 64);
    if (out && got) {
      const float d = tree_fdist(px, py, pox, poy, fx, fy, fox, foy);
      if (d < dist) {
        dist = d;
        tr.par = pick;
      }
    }
    ++rounds;
  }
  tr.rounds = rounds;
  const T pcx = __shfl(cx, tr.par, 64), pcy = __shfl(cy, tr.par, 64);
  const T pox = __shfl(ox, tr.par, 64), poy = __shfl(oy, tr.par, 64);
  tr.len = sink ? fabs((pcx - cx) + (pox - ox)) + fabs((pcy - cy) + (poy - oy)) : (T)0;
  tr.cd = sink ? cap : (T)0;
  for (int j = rounds - 1; j >= 0; --j) {
    const int slot = head + 1 + j;
    const int w = __shfl(tr.who, slot < 64 ? slot : 63, 64);
    const T c = __shfl(cw * tr.len + tr.cd, w, 64);
    const int pw = __shfl(tr.par, w, 64);
    if (slot <= tail && lane == pw && pw != head) tr.cd += c;
  }
  return tr;
}

// the Elmore delay of the lane's pin (0 at the driver)
template <typename T>
__device__ __forceinline__ T tree_chunk_delay(const NetModel<T> &nm, const ChunkTree<T> &tr) {
  T dl = 0;
  for (int j = 0; j < tr.rounds; ++j) {
    const T pd = __shfl(dl, tr.par, 64);
    if (tr.st == j) dl = pd + nm.rs * tr.len * (nm.hc * tr.len + tr.cd);
  }
  return dl;
}

}  // namespace tdp
