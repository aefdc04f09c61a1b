// Net model 2: every net an RC tree on the rectilinear minimum spanning tree
// of its pins (a fuller model of the wires of Eq. 7, Sec. III-C; the paper's
// timer times nets as RC trees).
//
// Topology: Prim's algorithm from the driver.  The pin outside the tree
// nearest to it joins next (ties: the pin first in the net's list), hung from
// the tree pin that reached it first at that distance (a later pin at equal
// distance does not take it over).  Distances are single precision,
// |(cell x - cell x) + (offset x - offset x)| + the same in y, whatever the
// precision of the timing values, so every precision and every layout of the
// same net takes the same decisions.
// Delays: each edge a uniform wire of its Manhattan length L (resistance
// r L, capacitance c L).  With C_below(v) the capacitance at and below v (its
// pin and the wires and pins of its subtree), the Elmore delay to v is the
// sum over the edges e = (parent, u) on its path of r L_e (c L_e / 2 +
// C_below(u)), times scale; the driver's load is the pin capacitances plus c
// times the tree's length.  Children join after their parents, so the
// reverse joining order accumulates C_below and the joining order the delays.
//
// Two forms: on net chunks, a lane per pin (tdp_tree.h), for every net that
// fits one; and one thread per net with its scratch in global memory per
// sink slot, for nets wider than a chunk.  The net pass builds its chunks'
// trees itself; the kernels here serve its wide nets and the smoothed TNS,
// whose net delays and position gradients for the star models (0 and 1)
// are here too, in the same two forms.
#include "tdp_impl.h"
#include "tdp_prims.h"
#include "tdp_tree.h"

namespace tdp {

static inline int nbt(long long n, int b) { return n > 0 ? (int)((n + b - 1) / b) : 1; }

template <typename T>
struct TreeView {
  float *dist;
  int32_t *par, *ord;
  T *len, *cd, *aux, *aux2, *wl;
};

template <typename T>
static TreeView<T> view(const TreeBuf &b) {
  return TreeView<T>{b.dist, b.par, b.ord, (T *)b.len, (T *)b.cd, (T *)b.aux, (T *)b.aux2, (T *)b.wl};
}

// a pin of net v: its cell's coordinates and its offset (slot -1: the
// driver; a port has no cell, and its offset is its position)
struct PinXY {
  float cx, cy, ox, oy;
  bool port;
};

__device__ __forceinline__ PinXY tree_pin(const Topo &tp, const float *__restrict__ x, const float *__restrict__ y,
                                          int v, int k) {
  if (k < 0) {
    const int dc = tp.drv_cell[v];
    return PinXY{dc >= 0 ? x[dc] : 0.f, dc >= 0 ? y[dc] : 0.f, tp.drv_ox[v], tp.drv_oy[v], dc < 0};
  }
  const int t = tp.net_sink[k];
  const int sc = tp.snk_cell[t];
  return PinXY{x[sc], y[sc], tp.snk_ox[t], tp.snk_oy[t], false};
}

__device__ __forceinline__ float tree_fdist(const PinXY &a, const PinXY &b) {
  return tree_fdist(a.cx, a.cy, a.ox, a.oy, b.cx, b.cy, b.ox, b.oy);
}

// (parent - child) per axis in T: (base difference) + (offset difference),
// a port's position taken as its base (no die-scale cancellation)
template <typename T>
__device__ __forceinline__ void tree_diff(const PinXY &p, const PinXY &c, T &dx, T &dy) {
  auto bx = [](const PinXY &a) { return a.port ? (T)a.ox : (T)a.cx; };
  auto by = [](const PinXY &a) { return a.port ? (T)a.oy : (T)a.cy; };
  auto fx = [](const PinXY &a) { return a.port ? (T)0 : (T)a.ox; };
  auto fy = [](const PinXY &a) { return a.port ? (T)0 : (T)a.oy; };
  dx = (bx(p) - bx(c)) + (fx(p) - fx(c));
  dy = (by(p) - by(c)) + (fy(p) - fy(c));
}

// Prim's tree of net v, then each slot's wire length and capacitance below;
// returns the tree's length
template <typename T>
__device__ T tree_build(const Topo &tp, const float *__restrict__ x, const float *__restrict__ y, T cw, int v,
                        const TreeView<T> &tb) {
  const int k0 = tp.net_ptr[v], k1 = tp.net_ptr[v + 1];
  const PinXY drv = tree_pin(tp, x, y, v, -1);
  for (int k = k0; k < k1; ++k) {
    tb.dist[k] = tree_fdist(drv, tree_pin(tp, x, y, v, k));
    tb.par[k] = -1;
  }
  // a slot in the tree holds distance -1 (a non-finite position gives NaN
  // distances, which still count as outside, so every step takes a slot)
  for (int step = 0; step < k1 - k0; ++step) {
    int j = -1;
    float bd = 0.f;
    for (int k = k0; k < k1; ++k) {
      const float d = tb.dist[k];
      if (!(d < 0.f) && (j < 0 || d < bd)) {
        j = k;
        bd = d;
      }
    }
    tb.ord[k0 + step] = j;
    tb.dist[j] = -1.f;
    const PinXY pj = tree_pin(tp, x, y, v, j);
    for (int k = k0; k < k1; ++k) {
      const float dk = tb.dist[k];
      if (dk < 0.f) continue;
      const float d = tree_fdist(pj, tree_pin(tp, x, y, v, k));
      if (d < dk) {
        tb.dist[k] = d;
        tb.par[k] = j;
      }
    }
  }
  T wl = 0;
  for (int k = k0; k < k1; ++k) {
    T dx, dy;
    tree_diff<T>(tree_pin(tp, x, y, v, tb.par[k]), tree_pin(tp, x, y, v, k), dx, dy);
    const T len = fabs(dx) + fabs(dy);
    tb.len[k] = len;
    tb.cd[k] = (T)tp.snk_cap[tp.net_sink[k]];
    wl += len;
  }
  for (int step = k1 - k0 - 1; step >= 0; --step) {
    const int k = tb.ord[k0 + step], p = tb.par[k];
    if (p >= 0) tb.cd[p] += cw * tb.len[k] + tb.cd[k];
  }
  return wl;
}

// net delays of the sinks of every net (or of the n nets listed) and each
// net's tree length
template <typename T>
__global__ void __launch_bounds__(256) k_tree_net(Topo tp, const float *__restrict__ x, const float *__restrict__ y,
                                                   NetModel<T> nm, T cw, TreeView<T> tb, T *__restrict__ dnet,
                                                   const int32_t *__restrict__ list, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int v = list ? list[i] : i;
  tb.wl[v] = tree_build<T>(tp, x, y, cw, v, tb);
  const int k0 = tp.net_ptr[v], k1 = tp.net_ptr[v + 1];
  for (int step = 0; step < k1 - k0; ++step) {
    const int k = tb.ord[k0 + step], p = tb.par[k];
    const T dp = p >= 0 ? dnet[tp.net_sink[p]] : (T)0;
    const T len = tb.len[k];
    dnet[tp.net_sink[k]] = dp + nm.rs * len * (nm.hc * len + tb.cd[k]);
  }
}

// Gradient of the smoothed TNS through the trees, per pin.  The topology is
// piecewise constant in the positions, so the wire lengths carry the whole
// derivative.  With A(u) the adjoint (d value / d net delay) summed over u's
// subtree and B(u) the sum over the edges e on u's path of scale r L_e
// A(child end of e), the derivative by the length of the edge into u is
//   scale r (c L_u + C_below(u)) A(u) + c B(parent(u)):
// the edge's own term and its capacitance in C_below of every edge above.
// gp[pin] (x) and gp[P + pin] (y) collect d value / d position of each pin.
template <typename T>
__global__ void __launch_bounds__(256) k_st_tree_grad(Topo tp, const float *__restrict__ x,
                                                       const float *__restrict__ y, NetModel<T> nm, T cw,
                                                       TreeView<T> tb, const T *__restrict__ adj, T *__restrict__ gp,
                                                       const int32_t *__restrict__ list, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int v = list[i];
  tree_build<T>(tp, x, y, cw, v, tb);
  const int k0 = tp.net_ptr[v], k1 = tp.net_ptr[v + 1];
  T *gpx = gp, *gpy = gp + tp.P;
  gpx[v] = 0;
  gpy[v] = 0;
  for (int k = k0; k < k1; ++k) {
    const int t = tp.net_sink[k];
    tb.aux[k] = adj[tp.M + t];
    gpx[tp.M + t] = 0;
    gpy[tp.M + t] = 0;
  }
  for (int step = k1 - k0 - 1; step >= 0; --step) {
    const int k = tb.ord[k0 + step], p = tb.par[k];
    if (p >= 0) tb.aux[p] += tb.aux[k];
  }
  for (int step = 0; step < k1 - k0; ++step) {
    const int k = tb.ord[k0 + step], p = tb.par[k];
    const T bp = p >= 0 ? tb.aux2[p] : (T)0;
    const T len = tb.len[k], a = tb.aux[k];
    tb.aux2[k] = bp + nm.rs * len * a;
    const T gl = nm.rs * (cw * len + tb.cd[k]) * a + cw * bp;
    T dx, dy;
    tree_diff<T>(tree_pin(tp, x, y, v, p), tree_pin(tp, x, y, v, k), dx, dy);
    const T gx = gl * (T)((dx > (T)0) - (dx < (T)0)), gy = gl * (T)((dy > (T)0) - (dy < (T)0));
    const int pp = p >= 0 ? tp.M + tp.net_sink[p] : v, pk = tp.M + tp.net_sink[k];
    gpx[pp] += gx;
    gpy[pp] += gy;
    gpx[pk] -= gx;
    gpy[pk] -= gy;
  }
}

// the chunk form of the two kernels above, over the net chunks: a net chunk's
// lane data, its trees, and (forward) the sinks' delays
struct ChunkLane {
  int lane, p, head, tail;
  bool sink, port;
  float fx, fy, fox, foy;
  int ty;
};

// a chunk lane's position in T for the wire lengths: a port's position as
// the base (see the net pass)
template <typename T>
__device__ __forceinline__ void lane_base(const ChunkLane &c, T &cx, T &cy, T &ox, T &oy) {
  cx = c.port ? (T)c.fox : (T)c.fx;
  cy = c.port ? (T)c.foy : (T)c.fy;
  ox = c.port ? (T)0 : (T)c.fox;
  oy = c.port ? (T)0 : (T)c.foy;
}

__device__ __forceinline__ ChunkLane chunk_lane(const Topo &tp, const float2 *__restrict__ xy, int chunk) {
  ChunkLane c;
  c.lane = wave_lane();
  const int k = chunk * CHUNK + c.lane;
  const int4 rec = tp.nm_rec[k];
  c.p = rec.x;
  c.head = rec.w & 63;
  c.tail = (rec.w >> 8) & 63;
  c.ty = (rec.w >> 16) & 255;
  c.sink = c.p >= 0 && c.lane != c.head;
  const float2 q = rec.y >= 0 ? xy[rec.y] : make_float2(0.f, 0.f);
  c.port = rec.y < 0;
  c.fx = q.x;
  c.fy = q.y;
  c.fox = tp.nm_ox[k];
  c.foy = tp.nm_oy[k];
  return c;
}

template <typename T>
__device__ __forceinline__ ChunkTree<T> chunk_tree(const Topo &tp, const ChunkLane &c, T cw) {
  T cx, cy, ox, oy;
  lane_base<T>(c, cx, cy, ox, oy);
  return tree_chunk_build<T>(cw, c.lane, c.head, c.tail, c.sink, c.fx, c.fy, c.fox, c.foy, cx, cy, ox, oy,
                             c.sink ? (T)tp.type_cap[c.ty] : (T)0);
}

template <typename T>
__global__ void __launch_bounds__(256) k_st_tree_chunks(Topo tp, const float2 *__restrict__ xy, NetModel<T> nm, T cw,
                                                        T *__restrict__ dnl) {
  const int chunk = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (chunk >= tp.n_nm_chunks) return;
  const ChunkLane c = chunk_lane(tp, xy, chunk);
  const ChunkTree<T> tr = chunk_tree<T>(tp, c, cw);
  const T dn = tree_chunk_delay<T>(nm, tr);
  if (c.sink) dnl[c.p - tp.M] = dn;
}

template <typename T>
__global__ void __launch_bounds__(256) k_st_tree_grad_chunks(Topo tp, const float2 *__restrict__ xy, NetModel<T> nm,
                                                             T cw, const T *__restrict__ adj, T *__restrict__ gp) {
  const int chunk = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (chunk >= tp.n_nm_chunks) return;
  const ChunkLane c = chunk_lane(tp, xy, chunk);
  const ChunkTree<T> tr = chunk_tree<T>(tp, c, cw);
  const int lane = c.lane, head = c.head, tail = c.tail;
  // A: the adjoint summed over the subtree (reverse joining order)
  T a = c.sink ? adj[c.p] : (T)0;
  for (int j = tr.rounds - 1; j >= 0; --j) {
    const int slot = head + 1 + j;
    const int w = __shfl(tr.who, slot < 64 ? slot : 63, 64);
    const T aw = __shfl(a, w, 64);
    const int pw = __shfl(tr.par, w, 64);
    if (slot <= tail && lane == pw && pw != head) a += aw;
  }
  // B along the path and the derivative by the lane's own wire length
  T b = 0, gl = 0;
  for (int j = 0; j < tr.rounds; ++j) {
    const T bp = __shfl(b, tr.par, 64);
    if (tr.st == j) {
      b = bp + nm.rs * tr.len * a;
      gl = nm.rs * (cw * tr.len + tr.cd) * a + cw * bp;
    }
  }
  T cx, cy, ox, oy;
  lane_base<T>(c, cx, cy, ox, oy);
  const T pcx = __shfl(cx, tr.par, 64), pcy = __shfl(cy, tr.par, 64);
  const T pox = __shfl(ox, tr.par, 64), poy = __shfl(oy, tr.par, 64);
  const T dx = (pcx - cx) + (pox - ox), dy = (pcy - cy) + (poy - oy);
  const T ex = c.sink ? gl * (T)((dx > (T)0) - (dx < (T)0)) : (T)0;
  const T ey = c.sink ? gl * (T)((dy > (T)0) - (dy < (T)0)) : (T)0;
  // per pin, in joining order: minus its own wire's term, plus its children's
  T gx = 0, gy = 0;
  for (int j = 0; j < tr.rounds; ++j) {
    const int slot = head + 1 + j;
    const int w = __shfl(tr.who, slot < 64 ? slot : 63, 64);
    const T exw = __shfl(ex, w, 64), eyw = __shfl(ey, w, 64);
    const int pw = __shfl(tr.par, w, 64);
    if (slot <= tail) {
      if (lane == pw) {
        gx += exw;
        gy += eyw;
      }
      if (lane == w) {
        gx -= ex;
        gy -= ey;
      }
    }
  }
  if (c.p >= 0) {
    gp[c.p] = gx;
    gp[tp.P + c.p] = gy;
  }
}

// The star models on net chunks: a sink's wire runs from the driver (the
// head lane); (driver - sink) per axis as (cell difference) + (offset
// difference), its Manhattan length (0 off the sinks) returned
template <typename T>
__device__ __forceinline__ T star_diff(const ChunkLane &c, T &dx, T &dy) {
  T cx, cy, ox, oy;
  lane_base<T>(c, cx, cy, ox, oy);
  const T cxd = __shfl(cx, c.head, 64), cyd = __shfl(cy, c.head, 64);
  const T oxd = __shfl(ox, c.head, 64), oyd = __shfl(oy, c.head, 64);
  dx = (cxd - cx) + (oxd - ox);
  dy = (cyd - cy) + (oyd - oy);
  return c.sink ? fabs(dx) + fabs(dy) : (T)0;
}

template <typename T>
__global__ void __launch_bounds__(256) k_st_star_chunks(Topo tp, const float2 *__restrict__ xy, NetModel<T> nm,
                                                        T *__restrict__ dnl) {
  const int chunk = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (chunk >= tp.n_nm_chunks) return;
  const ChunkLane c = chunk_lane(tp, xy, chunk);
  T dx, dy;
  const T len = star_diff<T>(c, dx, dy);
  if (c.sink) dnl[c.p - tp.M] = nm.delay(len, nm.elmore ? (T)tp.type_cap[c.ty] : (T)0);
}

// per pin: a sink minus its wire's term, the driver the sum of its sinks'
template <typename T>
__global__ void __launch_bounds__(256) k_st_star_grad_chunks(Topo tp, const float2 *__restrict__ xy, NetModel<T> nm,
                                                             const T *__restrict__ adj, T *__restrict__ gp) {
  const int chunk = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (chunk >= tp.n_nm_chunks) return;
  const ChunkLane c = chunk_lane(tp, xy, chunk);
  T dx, dy;
  const T len = star_diff<T>(c, dx, dy);
  const T gl = c.sink ? adj[c.p] * nm.slope(len, nm.elmore ? (T)tp.type_cap[c.ty] : (T)0) : (T)0;
  const T ex = gl * (T)((dx > (T)0) - (dx < (T)0)), ey = gl * (T)((dy > (T)0) - (dy < (T)0));
  const T sx = seg_sum(ex, c.lane, c.head, c.tail), sy = seg_sum(ey, c.lane, c.head, c.tail);
  if (c.p >= 0) {
    gp[c.p] = c.sink ? -ex : sx;
    gp[tp.P + c.p] = c.sink ? -ey : sy;
  }
}

// the star models on the n nets listed (nets wider than a chunk), one thread
// per net: the sinks' delays (adj null) or the pins' gradients
template <typename T>
__global__ void __launch_bounds__(256) k_st_star_big(Topo tp, const float *__restrict__ x,
                                                      const float *__restrict__ y, NetModel<T> nm,
                                                      const T *__restrict__ adj, T *__restrict__ dnl,
                                                      T *__restrict__ gp, const int32_t *__restrict__ list, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int v = list[i];
  const int dc = tp.drv_cell[v];
  // a port driver: its position as the base
  const T cx = dc >= 0 ? (T)x[dc] : (T)tp.drv_ox[v], cy = dc >= 0 ? (T)y[dc] : (T)tp.drv_oy[v];
  const T ox = dc >= 0 ? (T)tp.drv_ox[v] : (T)0, oy = dc >= 0 ? (T)tp.drv_oy[v] : (T)0;
  T sx = 0, sy = 0;
  for (int k = tp.net_ptr[v]; k < tp.net_ptr[v + 1]; ++k) {
    const int t = tp.net_sink[k];
    const int sc = tp.snk_cell[t];
    const T dx = (cx - (T)x[sc]) + (ox - (T)tp.snk_ox[t]), dy = (cy - (T)y[sc]) + (oy - (T)tp.snk_oy[t]);
    const T len = fabs(dx) + fabs(dy), cap = nm.elmore ? (T)tp.snk_cap[t] : (T)0;
    if (!adj) {
      dnl[t] = nm.delay(len, cap);
      continue;
    }
    const T gl = adj[tp.M + t] * nm.slope(len, cap);
    const T ex = gl * (T)((dx > (T)0) - (dx < (T)0)), ey = gl * (T)((dy > (T)0) - (dy < (T)0));
    gp[tp.M + t] = -ex;
    gp[tp.P + tp.M + t] = -ey;
    sx += ex;
    sy += ey;
  }
  if (adj) {
    gp[v] = sx;
    gp[tp.P + v] = sy;
  }
}

template <typename T>
void tree_net_impl(tdp_graph g, const TreeBuf &b, const float *x, const float *y, T *dnet, const int32_t *list,
                   int n, hipStream_t s) {
  const Topo &tp = g->topo;
  if (!list) n = tp.M;
  if (n <= 0) return;
  hipLaunchKernelGGL(k_tree_net<T>, dim3(nbt(n, 256)), dim3(256), 0, s, tp, x, y, net_model<T>(g), (T)g->c,
                     view<T>(b), dnet, list, n);
}

template <typename T>
void st_net_fwd_impl(tdp_graph g, const float *x, const float *y, T *dnl, hipStream_t s) {
  const Topo &tp = g->topo;
  const bool tree = g->lut.net_model == 2;
  // the chunk kernels read the positions packed once per forward call
  pack_xy(x, y, g->xy_st, tp.N, s);
  if (tp.n_nm_chunks > 0) {
    if (tree)
      hipLaunchKernelGGL(k_st_tree_chunks<T>, dim3(nbt(tp.n_nm_chunks, 4)), dim3(256), 0, s, tp, g->xy_st,
                         net_model<T>(g), (T)g->c, dnl);
    else
      hipLaunchKernelGGL(k_st_star_chunks<T>, dim3(nbt(tp.n_nm_chunks, 4)), dim3(256), 0, s, tp, g->xy_st,
                         net_model<T>(g), dnl);
  }
  if (tp.n_big > 0) {
    if (tree)
      tree_net_impl<T>(g, g->st_tree, x, y, dnl, tp.big_net, tp.n_big, s);
    else
      hipLaunchKernelGGL(k_st_star_big<T>, dim3(nbt(tp.n_big, 256)), dim3(256), 0, s, tp, x, y, net_model<T>(g),
                         (const T *)nullptr, dnl, (T *)nullptr, tp.big_net, tp.n_big);
  }
}

template <typename T>
void st_net_grad_impl(tdp_graph g, const float *x, const float *y, const T *adj, hipStream_t s) {
  const Topo &tp = g->topo;
  const bool tree = g->lut.net_model == 2;
  T *gp = (T *)g->st_gp;
  if (tp.n_nm_chunks > 0) {
    if (tree)
      hipLaunchKernelGGL(k_st_tree_grad_chunks<T>, dim3(nbt(tp.n_nm_chunks, 4)), dim3(256), 0, s, tp, g->xy_st,
                         net_model<T>(g), (T)g->c, adj, gp);
    else
      hipLaunchKernelGGL(k_st_star_grad_chunks<T>, dim3(nbt(tp.n_nm_chunks, 4)), dim3(256), 0, s, tp, g->xy_st,
                         net_model<T>(g), adj, gp);
  }
  if (tp.n_big > 0) {
    if (tree)
      hipLaunchKernelGGL(k_st_tree_grad<T>, dim3(nbt(tp.n_big, 256)), dim3(256), 0, s, tp, x, y, net_model<T>(g),
                         (T)g->c, view<T>(g->st_tree), adj, gp, tp.big_net, tp.n_big);
    else
      hipLaunchKernelGGL(k_st_star_big<T>, dim3(nbt(tp.n_big, 256)), dim3(256), 0, s, tp, x, y, net_model<T>(g),
                         adj, (T *)nullptr, gp, tp.big_net, tp.n_big);
  }
}

template void tree_net_impl<float>(tdp_graph, const TreeBuf &, const float *, const float *, float *,
                                   const int32_t *, int, hipStream_t);
template void tree_net_impl<double>(tdp_graph, const TreeBuf &, const float *, const float *, double *,
                                    const int32_t *, int, hipStream_t);
template void st_net_fwd_impl<float>(tdp_graph, const float *, const float *, float *, hipStream_t);
template void st_net_fwd_impl<double>(tdp_graph, const float *, const float *, double *, hipStream_t);
template void st_net_grad_impl<float>(tdp_graph, const float *, const float *, const float *, hipStream_t);
template void st_net_grad_impl<double>(tdp_graph, const float *, const float *, const double *, hipStream_t);

}  // namespace tdp
