// Internal definitions of the HIP timing library (not part of the ABI).
//
// Device numbering (chosen at build, see tdp_build.cpp):
//   drivers  v in [0, M):  [primary-input ports][flip-flop Q pins][combinational
//            outputs in (level, external cell id) order]; driver v drives net v.
//            Combinational cell c (level-major index) owns driver n_start + c.
//   sinks    t in [0, S):  [combinational input pins, cell-major, arc order]
//            [flip-flop D pins in ascending external pin id];  A = number of
//            combinational inputs, so the D pin of flip-flop f is sink A + f.
//   pins     per-pin arrays use [drivers | sinks]: pin M + t is sink t.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/tdp.h"

#define TDP_MAX_K 32

namespace tdp {

// ---------------------------------------------------------------- library
struct LutView {
  int nt, ns, nl;
  const float *slew_axis;   // [nt][ns]
  const float *load_axis;   // [nt][nl]
  const float *delay;       // [nt][ns][nl]
  const float *slew;        // [nt][ns][nl]
  // the four arrays above are consecutive in one buffer, padded to whole
  // float4s: the image a kernel stages in LDS
  const float4 *flat4;
  int n4;
  int net_model;  // 0: lumped wires; 1: Elmore star nets with degraded sink transitions
};

// Net delay into a sink at Manhattan distance len (Eq. 7: wire R and C both
// linear in length).  Lumped: the wire's R times its C, kappa * len^2 with
// kappa = scale * r * c.  Elmore: each sink on a branch of its own from the
// driver, a uniform RC line loaded by the sink's pin capacitance; the first
// moment of its response is scale * r * len * (c * len / 2 + cap).  The
// spanning-tree model (elmore == 2) takes its delays from each net's tree
// instead (the tree kernels); delay() and slope() serve models 0 and 1.
template <typename T>
struct NetModel {
  int elmore;
  T kappa;  // scale * r * c
  T rs;     // scale * r
  T hc;     // c / 2
  __device__ __forceinline__ T delay(T len, T cap) const {
    return elmore ? rs * len * (hc * len + cap) : kappa * len * len;
  }
  // d delay / d len
  __device__ __forceinline__ T slope(T len, T cap) const {
    return elmore ? rs * ((T)2 * hc * len + cap) : (T)2 * kappa * len;
  }
};

// Scratch of the spanning-tree net model (element type T of the timing values
// for len, cd, aux, aux2 and wl)
struct TreeBuf {
  float *dist;
  int32_t *par, *ord;
  void *len, *cd, *aux, *aux2, *wl;
};

// The spanning-tree model's topology metric: the single-precision Manhattan
// distance of two pins, each given as cell coordinates and offset, each axis
// taken as (cell difference) + (offset difference)
__device__ __forceinline__ float tree_fdist(float ax, float ay, float aox, float aoy, float bx, float by, float box,
                                            float boy) {
  return fabsf((ax - bx) + (aox - box)) + fabsf((ay - by) + (aoy - boy));
}

// Transition at a sink: the driver's, or under the Elmore model that one
// degraded by the wire (PERI: root sum of squares of the input transition and
// the wire's step-response transition, ln 9 times its Elmore delay, the 10-90%
// time of a single pole).
// The fused multiply-add is written out: left to the compiler, the sum of
// squares may be contracted one way in one kernel and another way in the
// next, and the sweeps that compute the same arrivals would then differ in
// the last bit.
template <typename T>
__device__ __forceinline__ T sink_slew(int net_model, T s, T dn) {
  if (!net_model) return s;
  const T w = (T)2.1972245773362196 * dn;  // ln 9
  return sqrt(fma(s, s, w * w));
}

// Bilinear lookup with clamping: the breakpoint interval is the last one whose
// left end is <= the value (the top interval for values at or past the end).
template <typename T>
__device__ __forceinline__ void lut_pair(const LutView &L, int type, T s, T l, T &d_out, T &s_out) {
  const float *sa = L.slew_axis + type * L.ns;
  const float *la = L.load_axis + type * L.nl;
  T s0 = (T)sa[0], s1 = (T)sa[L.ns - 1];
  T l0 = (T)la[0], l1 = (T)la[L.nl - 1];
  s = s < s0 ? s0 : (s > s1 ? s1 : s);
  l = l < l0 ? l0 : (l > l1 ? l1 : l);
  int i = 0;
  while (i + 1 < L.ns - 1 && (T)sa[i + 1] <= s) ++i;
  int j = 0;
  while (j + 1 < L.nl - 1 && (T)la[j + 1] <= l) ++j;
  T tau = (s - (T)sa[i]) / ((T)sa[i + 1] - (T)sa[i]);
  T ups = (l - (T)la[j]) / ((T)la[j + 1] - (T)la[j]);
  int base = (type * L.ns + i) * L.nl + j;
  T w00 = (1 - tau) * (1 - ups), w10 = tau * (1 - ups), w01 = (1 - tau) * ups, w11 = tau * ups;
  d_out = w00 * (T)L.delay[base] + w10 * (T)L.delay[base + L.nl] + w01 * (T)L.delay[base + 1] +
          w11 * (T)L.delay[base + L.nl + 1];
  s_out = w00 * (T)L.slew[base] + w10 * (T)L.slew[base + L.nl] + w01 * (T)L.slew[base + 1] +
          w11 * (T)L.slew[base + L.nl + 1];
}

// bin grid of the density term: bin (i, j) covers [x0 + i bw, x0 + (i+1) bw)
// x [y0 + j bh, y0 + (j+1) bh), stored at j * gx + i; window radius R bins
struct DensityGrid {
  float x0, y0, bw, bh, target;
  int gx, gy, R;
};

// ---------------------------------------------------------------- topology
// Device topology; plain data so kernels take it by value.
struct Topo {
  int32_t N = 0, P = 0, M = 0, S = 0, A = 0, E = 0;
  int32_t n_pi = 0, n_ff = 0, n_start = 0, n_comb = 0, D = 0;
  int32_t num_inst = 1;
  // drivers [M]
  int32_t *drv_cell = nullptr;  // external cell, -1 for a port
  float *drv_ox = nullptr, *drv_oy = nullptr;
  int32_t *drv_ext = nullptr;   // external pin id
  int32_t *net_ptr = nullptr;   // [M+1] into net_sink
  int32_t *net_sink = nullptr;  // [S] sinks of each net
  double *net_cpin = nullptr;   // [M] sum of sink pin capacitances
  float *snk_cap = nullptr;     // [S] input-pin capacitance of each sink
  float *type_cap = nullptr;    // [num_types] input-pin capacitance of each cell type
  // sinks [S]
  int32_t *snk_cell = nullptr;
  float *snk_ox = nullptr, *snk_oy = nullptr;
  int32_t *snk_drv = nullptr;   // driver of the sink's net
  int32_t *snk_ext = nullptr;
  int32_t *snk_comb = nullptr;  // [A] combinational cell of an input pin
  // combinational cells [n_comb]
  uint8_t *comb_type = nullptr;
  int32_t *comb_inptr = nullptr;  // [n_comb+1] into sinks [0, A)
  int32_t *comb_ext = nullptr;
  // flip-flops [n_ff]
  int32_t *ff_ext = nullptr;
  uint8_t *ff_type = nullptr;
  int32_t *ff_inst = nullptr;    // instance of each flip-flop (batched graphs)
  // maps
  int32_t *ext_pin_int = nullptr;  // [P] external pin -> internal pin
  int32_t *cell_int = nullptr;     // [N] external cell -> comb index, or -(ff index)-1
  uint8_t *cell_fixed = nullptr;   // [N]
  // 64-lane chunks of combinational inputs: a cell's inputs never straddle a
  // chunk; chunks are level-pure.  One record per lane: {sink t (-1 =
  // padding), its driver, its combinational cell, head lane | tail lane << 8 |
  // cell type << 16 | widest cell of the chunk << 24}, so a lane finds
  // everything static in one load.
  int32_t n_fw_chunks = 0;
  int4 *fw_rec = nullptr;
  int2 *fw_ext = nullptr;  // per lane: external ids of its sink and of that sink's driver
  // 64-lane chunks of nets (driver lane first, then its sinks); a net never
  // straddles a chunk; chunks are level-pure by driver level.  Nets with more
  // than 63 sinks are "big" and handled one thread per net.
  // One record per lane: {internal pin (driver v or M + t; -1 = padding),
  // external cell (-1 for a port or padding), for a combinational-input sink
  // the output driver of its cell (else -1), head lane | tail lane << 8 |
  // for a sink, its cell's type << 16}.
  int32_t n_nm_chunks = 0, n_big = 0;
  int4 *nm_rec = nullptr;
  float *nm_ox = nullptr, *nm_oy = nullptr;
  int32_t *big_net = nullptr;    // [n_big] drivers of big nets, level-major
};

constexpr int CHUNK = 64;

struct HostLevels {
  std::vector<int32_t> fw_lvl;    // [D+1]: level l input chunks are [fw_lvl[l-1], fw_lvl[l])
  std::vector<int32_t> nm_lvl;    // [D+2]: level l net chunks are [nm_lvl[l], nm_lvl[l+1]) (0 = start points)
  std::vector<int32_t> big_lvl;   // [D+2]: level l big nets are [big_lvl[l], big_lvl[l+1])
  std::vector<int32_t> lvl;       // [D+1]: level l cells are [lvl[l-1], lvl[l])
  std::vector<int32_t> ep_base;   // [num_inst+1] endpoint range per instance
  std::vector<int32_t> pin_base;  // [num_inst+1]
  std::vector<int32_t> cell_base; // [num_inst+1]
};

// host-side image of the device topology, produced by the build
struct HostTopo {
  Topo dims;  // sizes only
  HostLevels lv;
  std::vector<int32_t> drv_cell, drv_ext, net_ptr, net_sink, snk_cell, snk_drv, snk_ext, snk_comb,
      comb_inptr, comb_ext, ff_ext, ff_inst, ext_pin_int, cell_int;
  std::vector<float> drv_ox, drv_oy, snk_ox, snk_oy, snk_cap, type_cap;
  std::vector<double> net_cpin;
  std::vector<int4> fw_rec, nm_rec;
  std::vector<int2> fw_ext;
  std::vector<int32_t> big_net;
  std::vector<float> nm_ox, nm_oy;
  std::vector<uint8_t> comb_type, ff_type, cell_fixed;
};

tdp_status build_host_topology(const tdp_netlist *const *nls, int32_t count, const tdp_library *lib,
                               HostTopo &out, std::string &err);

// ---------------------------------------------------------------- graph
struct Profiler {
  bool on = false;
  int32_t mask = 0;                       // stages being timed
  hipEvent_t open[TDP_NUM_STAGES] = {};
  struct Mark { int stage; hipEvent_t a, b; };
  std::vector<Mark> marks;
  std::vector<hipEvent_t> pool;           // events reused between reads
  double ms[TDP_NUM_STAGES] = {0};
  int calls[TDP_NUM_STAGES] = {0};
  hipEvent_t take() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    return hipEventCreate(&e) == hipSuccess ? e : nullptr;
  }
};

}  // namespace tdp

struct tdp_graph_s {
  int device = 0;
  tdp_precision prec = TDP_F32;
  int esz = 4;  // bytes per timing value
  tdp::Topo topo;
  tdp::HostLevels lv;
  tdp::LutView lut{};
  float r = 0, c = 0, scale = 0;
  float input_slew = 0, clock_slew = 0;
  // required time at the D pins of each instance (period - setup, rounded as
  // the graph's precision rounds it); device copy in d_inst_req
  std::vector<double> h_inst_req;
  double *d_inst_req = nullptr;
  int32_t max_paths = 0, max_k = 1, side_k = 1, max_out = 0, max_out_inst = 0, slot_cap = 0, pin_cap = 0;
  int32_t key_bits32 = 40, ep_chunks = 1;
  int32_t tune_block = 256, tune_chunk = 1, sweep_mode = 0;
  std::string last_error;
  bool updated = false, extracted = false, pairs_built = false, stns_ready = false;
  std::vector<void *> allocs;  // every device allocation, freed at destroy
  std::vector<int32_t> h_snk_ext;  // host copy: external pin of each sink
  int32_t *d_err = nullptr;    // device flag for internal consistency errors
  double *consts = nullptr;    // [4] device constants: {1, 0, 0, 0}

  // timing state (element type per precision)
  // slack is not stored: export derives it as rat - at.  dnet_nm holds the
  // net delays again in net-chunk slot order (the backward passes read them
  // there); drv_as packs {arrival, transition} of each driver for the
  // forward passes' gathers.
  void *load = nullptr, *dnet = nullptr, *at = nullptr, *slew = nullptr, *rat = nullptr, *darc = nullptr,
       *dnet_nm = nullptr, *drv_as = nullptr, *fw_a = nullptr;
  int32_t *crit = nullptr;       // [n_comb] arc index of the critical input
  int32_t *hop = nullptr;        // [n_comb][4] {critical sink, its driver, their external ids}
  int32_t *hop4 = nullptr;       // [n_comb][4][4] the hop records of a cell and of the next three up its chain
  int32_t *cdep = nullptr;       // [M] combinational cells on the critical chain
  void *side_cost = nullptr;     // [n_comb][side_k] cheapest deviations along the chain
  int32_t *side_pin = nullptr;   // [n_comb][side_k]
  void *ep_slack = nullptr;      // [E]
  // dataflow sweeps (single precision): published words polled by consumers
  uint64_t *flow_w = nullptr;    // [M] {arrival, transition} of a driver; all ones = not yet
  uint32_t *flow_r = nullptr;    // [M] required time of a driver; all ones = not yet
  uint32_t *flow_cd = nullptr;   // [M] chain depth + 1 of a driver; 0 = not yet
  uint64_t *flow_se = nullptr;   // [n_comb][side_k] deviation entries {cost, sink}; all ones = not yet
  int32_t flow_waves = 4, spin_limit = 1 << 20;
  int32_t flow_per_cu = 1;       // workgroups per compute unit of the resident dataflow grids
  int32_t num_cu = 0;            // compute units of the device
  int32_t occ_fw[3] = {-1, -1, -1}, occ_bw[3] = {-1, -1, -1};  // occupancy per 1 / 2 / 4 waves, -1 = not yet
  bool flow_ok = false;          // the graph can use the dataflow sweeps
  int32_t pos_gen = 0;           // arrival passes so far; d_err[1] == pos_gen: a position was not finite
  bool flow_r_clear = false;     // flow_r holds no published word (the last net pass reset it)
  bool drv_as_stale = false;     // drv_as (combinational drivers) and fw_a predate the last forward sweep
  double *red_ep = nullptr, *red_loss = nullptr, *red_wa = nullptr;
  double *summary = nullptr;     // [4 * num_inst]: wns, tns, n_fail, 0
  int32_t *inst_nfail = nullptr, *d_ep_base = nullptr;

  // extraction
  int32_t *sel_flag = nullptr, *sel_pos = nullptr, *sel_list = nullptr, *d_nsel = nullptr;
  int32_t *inst_nsel = nullptr, *inst_nvalid = nullptr, *inst_seg = nullptr, *inst_outb = nullptr,
          *inst_kept = nullptr, *inst_selb = nullptr, *sel_npop = nullptr;
  void *slot_key = nullptr;      // path slack per slot
  int32_t *slot_dev = nullptr, *slot_par = nullptr, *slot_len = nullptr, *slot_cells = nullptr,
          *d_nslots = nullptr;
  uint64_t *sort_k0 = nullptr, *sort_k1 = nullptr;
  uint32_t *sort_v0 = nullptr, *sort_v1 = nullptr;
  int32_t *sort_hist = nullptr, *scan_tmp = nullptr;
  int32_t *out_slot = nullptr, *out_len = nullptr;
  int32_t *slot_out = nullptr;  // [slot_cap] output index of a slot's path, -1 when cut
  int32_t *path_ptr = nullptr, *path_pins = nullptr, *path_int = nullptr, *path_ep = nullptr,
          *path_epi = nullptr, *path_rank = nullptr, *d_num_paths = nullptr;
  void *path_slack = nullptr;
  int32_t last_k = 1;

  // design-wide extraction, report_timing(K): a store of gcap search nodes
  // and its sort / scan buffers, allocated by the first such call
  int32_t gcap = 0;
  void *gt_cost = nullptr, *gt_key = nullptr, *gt_theta = nullptr;
  int32_t *gt_dev = nullptr, *gt_par = nullptr, *gt_ep = nullptr, *gt_cells = nullptr, *gt_nd = nullptr;
  int32_t *gt_cnt = nullptr, *gt_off = nullptr, *gt_start = nullptr, *gt_end = nullptr;
  int32_t *gt_misc = nullptr;  // [4] device counters read back per round
  uint64_t *gt_k0 = nullptr, *gt_k1 = nullptr;
  uint32_t *gt_v0 = nullptr, *gt_v1 = nullptr;
  int32_t *gt_hist = nullptr, *gt_scan = nullptr;

  // pairs
  float *pw = nullptr;                 // [S] weight per sink pin
  uint8_t *pin_p = nullptr;            // [S] membership in P
  unsigned long long *pacc = nullptr;  // [S] fixed-point accumulator
  int32_t *pfirst = nullptr;           // [S] first occurrence (path index)
  int32_t *pflag = nullptr;            // [S] compaction positions
  int32_t *d_npairs = nullptr;
  int32_t *pair_sink = nullptr, *pair_cs = nullptr, *pair_ct = nullptr;
  float *pair_dox = nullptr, *pair_doy = nullptr, *pair_w = nullptr;
  int32_t *cell_cnt = nullptr, *cell_ptr = nullptr, *cell_cur = nullptr, *cell_flag = nullptr,
          *touched = nullptr, *d_ntouched = nullptr;
  int32_t *inc_other = nullptr, *inc_key = nullptr;
  float *inc_dx = nullptr, *inc_dy = nullptr, *inc_w = nullptr;

  // smoothed TNS (st_gp: the gradient per pin and axis [2P])
  void *st_at = nullptr, *st_adj = nullptr, *st_dnet = nullptr, *st_gp = nullptr;
  float st_gamma = 0;
  const float *st_x = nullptr, *st_y = nullptr;

  // early (hold) analysis, allocated by its first call: packed {arrival,
  // transition} per driver, arrival per sink, arc delay per comb input
  void *ea_as = nullptr, *ea_at = nullptr, *ea_darc = nullptr;
  double *ea_part = nullptr, *ea_summary = nullptr;
  float ea_hold = 0;
  bool ea_ready = false;

  // incremental arrival update, allocated by its first call: marks as epoch
  // stamps per forward chunk (arrivals, lists), per driver (arrival or
  // transition changed, list changed) and per net chunk; the forward chunk of
  // each combinational input and the net chunk of each driver
  bool inc_ready = false;
  int32_t inc_epoch = 0;
  int32_t *inc_arr = nullptr, *inc_lst = nullptr, *inc_drv_chg = nullptr, *inc_drv_lchg = nullptr,
          *inc_nm = nullptr, *inc_snk_chunk = nullptr, *inc_drv_nm_chunk = nullptr;

  // rise / fall timing (tdp_rf_setup): per-pin arrays [2 * pin + transition]
  // in device pin order, arc delays [4 * input + 2 * x + y], critical (input,
  // transition) per cell and output transition, the fall tables, unateness
  bool rf_ready = false, rf_updated = false;
  void *rf_at = nullptr, *rf_slew = nullptr, *rf_rat = nullptr, *rf_darc4 = nullptr;
  int32_t *rf_crit = nullptr, *rf_unate = nullptr;
  float *rf_delay_fall = nullptr, *rf_slew_fall = nullptr;  // inside rf_flat
  float4 *rf_flat = nullptr;  // the fall tables' image: [slew axes | load axes | delay | slew], as lut.flat4
  uint8_t *rf_path_tran = nullptr;  // [pin_cap] transition of each path pin

  // density term and Nesterov steps (tdp_density_setup)
  bool dn_ready = false;
  tdp::DensityGrid dn{};
  int dn_key_bits = 8, dn_alloc_bins = 0, dn_alloc_R = -1;
  double dn_total_area = 0;
  float *dn_area = nullptr;                    // [N]
  uint64_t *dn_k0 = nullptr, *dn_k1 = nullptr;  // [N] bin keys (sort ping-pong)
  uint32_t *dn_v0 = nullptr, *dn_v1 = nullptr;  // [N] cell ids
  int32_t *dn_hist = nullptr, *dn_scan = nullptr, *dn_start = nullptr;  // start [bins + 1]
  int32_t *dn_heavy = nullptr, *dn_nheavy = nullptr;  // crowded bins [bins] and their count
  float *dn_w = nullptr;                       // [2 (2R+1)][N] window weights of the sorted cells
  float *dn_map = nullptr;                     // [bins]
  double *dn_part = nullptr, *nest_part = nullptr, *nest_alpha = nullptr;

  // net model 2 (spanning-tree RC nets), allocated at build when the library
  // selects it: the net pass's scratch and the smoothed TNS's, per sink slot
  // of net_sink (Prim's distance, parent slot or -1 for the driver, joining
  // order, wire length, capacitance below, two adjoint sums) and per net (the
  // tree's length)
  tdp::TreeBuf tree{}, st_tree{};

  // weighted-average wirelength: per-pin gradient [2P]
  float *wa_gpin = nullptr;
  float2 *xy = nullptr;        // [N] positions packed by the last timing update
  float2 *xy_wa = nullptr;     // [N] positions packed by a WA call
  float2 *xy_st = nullptr;     // [N] positions packed by the last smoothed-TNS forward call
  float2 *cxy_nm = nullptr;    // [net-chunk slots] cell coordinates the last update gathered

  tdp::Profiler prof;
};

namespace tdp {
// the graph's net model in the precision T of its timing values
template <typename T>
inline NetModel<T> net_model(const tdp_graph_s *g) {
  return NetModel<T>{g->lut.net_model, (T)g->scale * (T)g->r * (T)g->c, (T)g->scale * (T)g->r, (T)0.5 * (T)g->c};
}
}  // namespace tdp
