// Host-side graph construction: validation, levelisation and the device
// numbering described in tdp_internal.h.
//
// The timing graph (Sec. II-B) has net arcs (driver -> sink) and cell arcs
// (combinational input -> output).  Start points are primary-input ports and
// flip-flop Q pins (level 0); a combinational cell sits one level above the
// highest level among the drivers of its inputs.  Kahn's algorithm over cells
// both assigns the levels and rejects combinational loops.
#include <algorithm>
#include <cmath>
#include <numeric>

#include "tdp_internal.h"

namespace tdp {

namespace {
enum Role : int8_t { R_NONE = 0, R_PORT, R_CIN, R_COUT, R_FFD, R_FFQ };

bool fail(std::string &err, const std::string &m) {
  err = m;
  return false;
}

bool check_library(const tdp_library *lib, std::string &err) {
  if (!lib) return fail(err, "library is NULL");
  if (lib->num_types < 1 || lib->n_slew < 2 || lib->n_load < 2 || lib->n_slew > 16 || lib->n_load > 16)
    return fail(err, "library: need >= 1 type and 2..16 breakpoints per axis");
  // cell types travel in 8-bit fields of the lane records
  if (lib->num_types > 256) return fail(err, "library: at most 256 cell types");
  if (!lib->slew_axis || !lib->load_axis || !lib->delay_lut || !lib->slew_lut || !lib->pin_cap)
    return fail(err, "library: NULL array");
  for (int t = 0; t < lib->num_types; ++t) {
    for (int i = 0; i + 1 < lib->n_slew; ++i)
      if (!(lib->slew_axis[t * lib->n_slew + i] < lib->slew_axis[t * lib->n_slew + i + 1]))
        return fail(err, "library: slew axis not strictly increasing");
    for (int i = 0; i + 1 < lib->n_load; ++i)
      if (!(lib->load_axis[t * lib->n_load + i] < lib->load_axis[t * lib->n_load + i + 1]))
        return fail(err, "library: load axis not strictly increasing");
    if (!std::isfinite(lib->pin_cap[t])) return fail(err, "library: pin capacitance not finite");
  }
  size_t n = (size_t)lib->num_types * lib->n_slew * lib->n_load;
  for (size_t q = 0; q < n; ++q)
    if (!std::isfinite(lib->delay_lut[q]) || !std::isfinite(lib->slew_lut[q]))
      return fail(err, "library: table entry not finite");
  if (!std::isfinite(lib->r_per_um) || !std::isfinite(lib->c_per_um) || !std::isfinite(lib->delay_scale))
    return fail(err, "library: wire parameters not finite");
  if (lib->net_model < 0 || lib->net_model > 2) return fail(err, "library: net_model must be 0, 1 or 2");
  return true;
}

// Validate one netlist; fills role / driver / level arrays in its own ids.
struct Checked {
  std::vector<int8_t> role;
  std::vector<int32_t> net_of_driver;  // [P] net driven by a driver pin
  std::vector<int32_t> driver_of;      // [P] driver pin of a sink pin
  std::vector<int32_t> level;          // [N] level of a combinational cell
  int32_t depth = 0;
};

bool check_netlist(const tdp_netlist *nl, const tdp_library *lib, Checked &ck, std::string &err,
                   bool &cycle) {
  cycle = false;
  if (!nl) return fail(err, "netlist is NULL");
  const int N = nl->num_cells, P = nl->num_pins, M = nl->num_nets;
  if (N < 1 || P < 1 || M < 1) return fail(err, "netlist: empty");
  if (!nl->pin_cell || !nl->pin_off_x || !nl->pin_off_y || !nl->net_ptr || !nl->net_pins ||
      !nl->cell_type || !nl->cell_in_ptr || !nl->cell_in_pins || !nl->cell_out_pin || !nl->cell_is_ff)
    return fail(err, "netlist: NULL array");
  ck.role.assign(P, R_NONE);
  for (int p = 0; p < P; ++p) {
    if (nl->pin_cell[p] < -1 || nl->pin_cell[p] >= N) return fail(err, "netlist: pin_cell out of range");
    if (!std::isfinite(nl->pin_off_x[p]) || !std::isfinite(nl->pin_off_y[p]))
      return fail(err, "netlist: pin offset not finite");
    if (nl->pin_cell[p] == -1) ck.role[p] = R_PORT;
  }
  if (nl->cell_in_ptr[0] != 0) return fail(err, "netlist: cell_in_ptr[0] != 0");
  for (int c = 0; c < N; ++c) {
    if (nl->cell_type[c] < 0 || nl->cell_type[c] >= lib->num_types)
      return fail(err, "netlist: cell_type out of range");
    int b = nl->cell_in_ptr[c], e = nl->cell_in_ptr[c + 1];
    if (e < b) return fail(err, "netlist: cell_in_ptr not monotone");
    bool ff = nl->cell_is_ff[c] != 0;
    if (ff && e - b != 1) return fail(err, "netlist: a flip-flop must have exactly one input (D)");
    if (!ff && e - b < 1) return fail(err, "netlist: a combinational cell needs at least one input");
    for (int k = b; k < e; ++k) {
      int p = nl->cell_in_pins[k];
      if (p < 0 || p >= P) return fail(err, "netlist: cell_in_pins out of range");
      if (nl->pin_cell[p] != c) return fail(err, "netlist: input pin not owned by its cell");
      if (ck.role[p] != R_NONE) return fail(err, "netlist: pin listed twice");
      ck.role[p] = ff ? R_FFD : R_CIN;
    }
    int o = nl->cell_out_pin[c];
    if (o < 0 || o >= P) return fail(err, "netlist: cell_out_pin out of range");
    if (nl->pin_cell[o] != c) return fail(err, "netlist: output pin not owned by its cell");
    if (ck.role[o] != R_NONE) return fail(err, "netlist: pin listed twice");
    ck.role[o] = ff ? R_FFQ : R_COUT;
  }
  for (int p = 0; p < P; ++p)
    if (ck.role[p] == R_NONE) return fail(err, "netlist: pin is neither a port nor a cell pin");
  if (nl->net_ptr[0] != 0) return fail(err, "netlist: net_ptr[0] != 0");
  ck.net_of_driver.assign(P, -1);
  ck.driver_of.assign(P, -1);
  for (int n = 0; n < M; ++n) {
    int b = nl->net_ptr[n], e = nl->net_ptr[n + 1];
    if (e <= b) return fail(err, "netlist: a net needs a driver");
    for (int k = b; k < e; ++k)
      if (nl->net_pins[k] < 0 || nl->net_pins[k] >= P) return fail(err, "netlist: net_pins out of range");
    int d = nl->net_pins[b];
    int8_t r = ck.role[d];
    if (r != R_PORT && r != R_COUT && r != R_FFQ) return fail(err, "netlist: net driver is not an output pin or port");
    if (ck.net_of_driver[d] >= 0) return fail(err, "netlist: pin drives two nets");
    ck.net_of_driver[d] = n;
    for (int k = b + 1; k < e; ++k) {
      int t = nl->net_pins[k];
      if (ck.role[t] != R_CIN && ck.role[t] != R_FFD) return fail(err, "netlist: net sink is not an input pin");
      if (ck.driver_of[t] >= 0) return fail(err, "netlist: input pin in two nets");
      ck.driver_of[t] = d;
    }
  }
  for (int p = 0; p < P; ++p) {
    int8_t r = ck.role[p];
    if ((r == R_PORT || r == R_COUT || r == R_FFQ) && ck.net_of_driver[p] < 0)
      return fail(err, "netlist: an output pin or port drives no net");
    if ((r == R_CIN || r == R_FFD) && ck.driver_of[p] < 0) return fail(err, "netlist: an input pin is in no net");
  }
  // Kahn over combinational cells
  std::vector<int32_t> indeg(N, 0);
  std::vector<std::vector<int32_t>> fanout_cells;  // built lazily via CSR below
  std::vector<int32_t> fo_cnt(N + 1, 0);
  for (int c = 0; c < N; ++c) {
    if (nl->cell_is_ff[c]) continue;
    for (int k = nl->cell_in_ptr[c]; k < nl->cell_in_ptr[c + 1]; ++k) {
      int d = ck.driver_of[nl->cell_in_pins[k]];
      if (ck.role[d] == R_COUT) {
        indeg[c]++;
        fo_cnt[nl->pin_cell[d] + 1]++;
      }
    }
  }
  std::partial_sum(fo_cnt.begin(), fo_cnt.end(), fo_cnt.begin());
  std::vector<int32_t> fo(fo_cnt[N]);
  std::vector<int32_t> cur(fo_cnt.begin(), fo_cnt.end() - 1);
  for (int c = 0; c < N; ++c) {
    if (nl->cell_is_ff[c]) continue;
    for (int k = nl->cell_in_ptr[c]; k < nl->cell_in_ptr[c + 1]; ++k) {
      int d = ck.driver_of[nl->cell_in_pins[k]];
      if (ck.role[d] == R_COUT) fo[cur[nl->pin_cell[d]]++] = c;
    }
  }
  ck.level.assign(N, 0);
  std::vector<int32_t> queue;
  queue.reserve(N);
  int n_comb = 0;
  for (int c = 0; c < N; ++c)
    if (!nl->cell_is_ff[c]) {
      n_comb++;
      if (indeg[c] == 0) { ck.level[c] = 1; queue.push_back(c); }
    }
  size_t head = 0;
  while (head < queue.size()) {
    int c = queue[head++];
    for (int k = fo_cnt[c]; k < fo_cnt[c + 1]; ++k) {
      int s = fo[k];
      ck.level[s] = std::max(ck.level[s], ck.level[c] + 1);
      if (--indeg[s] == 0) queue.push_back(s);
    }
  }
  if ((int)queue.size() != n_comb) {
    cycle = true;
    return fail(err, "netlist: combinational loop");
  }
  ck.depth = 0;
  for (int c = 0; c < N; ++c) if (!nl->cell_is_ff[c]) ck.depth = std::max(ck.depth, ck.level[c]);
  return true;
}
}  // namespace

tdp_status build_host_topology(const tdp_netlist *const *nls, int32_t count, const tdp_library *lib,
                               HostTopo &H, std::string &err) {
  if (count < 1 || !nls) { err = "no netlist"; return TDP_E_INVALID; }
  if (!check_library(lib, err)) return TDP_E_INVALID;
  std::vector<Checked> cks(count);
  int64_t tot_cells = 0, tot_pins = 0, tot_nets = 0;
  for (int i = 0; i < count; ++i) {
    bool cycle = false;
    if (!check_netlist(nls[i], lib, cks[i], err, cycle)) {
      if (count > 1) err = "instance " + std::to_string(i) + ": " + err;
      return cycle ? TDP_E_CYCLE : TDP_E_INVALID;
    }
    tot_cells += nls[i]->num_cells;
    tot_pins += nls[i]->num_pins;
    tot_nets += nls[i]->num_nets;
  }
  if (tot_pins >= (int64_t)1 << 30 || tot_cells >= (int64_t)1 << 30) { err = "graph too large"; return TDP_E_INVALID; }
  Topo &T = H.dims;
  T.num_inst = count;
  T.N = (int32_t)tot_cells;
  T.P = (int32_t)tot_pins;
  T.M = (int32_t)tot_nets;
  H.lv.pin_base.assign(count + 1, 0);
  H.lv.cell_base.assign(count + 1, 0);
  for (int i = 0; i < count; ++i) {
    H.lv.pin_base[i + 1] = H.lv.pin_base[i] + nls[i]->num_pins;
    H.lv.cell_base[i + 1] = H.lv.cell_base[i] + nls[i]->num_cells;
  }
  // union-wide lists in external (offset) ids
  struct CombRec { int32_t level, cell; };
  std::vector<CombRec> combs;
  std::vector<int32_t> ports, ffs;  // external pin id of port / external cell of FF
  T.D = 0;
  for (int i = 0; i < count; ++i) {
    const tdp_netlist *nl = nls[i];
    int pb = H.lv.pin_base[i], cb = H.lv.cell_base[i];
    T.D = std::max(T.D, cks[i].depth);
    for (int p = 0; p < nl->num_pins; ++p) if (cks[i].role[p] == R_PORT) ports.push_back(pb + p);
    for (int c = 0; c < nl->num_cells; ++c) {
      if (nl->cell_is_ff[c]) ffs.push_back(cb + c);
      else combs.push_back({cks[i].level[c], cb + c});
    }
  }
  auto inst_of_cell = [&](int32_t cell) {
    return (int)(std::upper_bound(H.lv.cell_base.begin(), H.lv.cell_base.end(), cell) - H.lv.cell_base.begin()) - 1;
  };
  auto d_pin_of_ff = [&](int32_t cell) {
    int i = inst_of_cell(cell);
    const tdp_netlist *nl = nls[i];
    int c = cell - H.lv.cell_base[i];
    return H.lv.pin_base[i] + nl->cell_in_pins[nl->cell_in_ptr[c]];
  };
  std::sort(ports.begin(), ports.end());
  std::sort(ffs.begin(), ffs.end(), [&](int32_t a, int32_t b) { return d_pin_of_ff(a) < d_pin_of_ff(b); });
  std::sort(combs.begin(), combs.end(), [](const CombRec &a, const CombRec &b) {
    return a.level != b.level ? a.level < b.level : a.cell < b.cell;
  });
  T.n_pi = (int32_t)ports.size();
  T.n_ff = (int32_t)ffs.size();
  T.n_start = T.n_pi + T.n_ff;
  T.n_comb = (int32_t)combs.size();
  T.E = T.n_ff;
  if (T.n_start + T.n_comb != T.M) { err = "internal: driver count mismatch"; return TDP_E_INVALID; }
  H.lv.lvl.assign(T.D + 1, 0);
  for (int l = 1; l <= T.D; ++l) {
    auto it = std::lower_bound(combs.begin(), combs.end(), l + 1,
                               [](const CombRec &r, int v) { return r.level < v; });
    H.lv.lvl[l] = (int32_t)(it - combs.begin());
  }
  // endpoint ranges per instance (flip-flops are ordered by D pin, which is
  // instance-major because external ids are offset per instance)
  H.lv.ep_base.assign(count + 1, 0);
  for (int32_t f : ffs) H.lv.ep_base[inst_of_cell(f) + 1]++;
  for (int i = 0; i < count; ++i) H.lv.ep_base[i + 1] += H.lv.ep_base[i];

  // ---------------------------------------------------------- numbering
  H.ext_pin_int.assign(T.P, -1);
  H.cell_int.assign(T.N, 0);
  H.drv_cell.assign(T.M, -1);
  H.drv_ext.assign(T.M, -1);
  H.drv_ox.assign(T.M, 0.f);
  H.drv_oy.assign(T.M, 0.f);
  // drivers
  auto get_nl = [&](int32_t extpin, int &inst, int &local) {
    inst = (int)(std::upper_bound(H.lv.pin_base.begin(), H.lv.pin_base.end(), extpin) - H.lv.pin_base.begin()) - 1;
    local = extpin - H.lv.pin_base[inst];
    return nls[inst];
  };
  std::vector<int32_t> drv_pin(T.M);
  for (int q = 0; q < T.n_pi; ++q) drv_pin[q] = ports[q];
  for (int f = 0; f < T.n_ff; ++f) {
    int32_t cell = ffs[f];
    int i = inst_of_cell(cell);
    drv_pin[T.n_pi + f] = H.lv.pin_base[i] + nls[i]->cell_out_pin[cell - H.lv.cell_base[i]];
    H.cell_int[cell] = -(f + 1);
  }
  for (int c = 0; c < T.n_comb; ++c) {
    int32_t cell = combs[c].cell;
    int i = inst_of_cell(cell);
    drv_pin[T.n_start + c] = H.lv.pin_base[i] + nls[i]->cell_out_pin[cell - H.lv.cell_base[i]];
    H.cell_int[cell] = c;
  }
  for (int v = 0; v < T.M; ++v) {
    int inst, local;
    const tdp_netlist *nl = get_nl(drv_pin[v], inst, local);
    H.drv_ext[v] = drv_pin[v];
    int pc = nl->pin_cell[local];
    H.drv_cell[v] = pc < 0 ? -1 : pc + H.lv.cell_base[inst];
    H.drv_ox[v] = nl->pin_off_x[local];
    H.drv_oy[v] = nl->pin_off_y[local];
    H.ext_pin_int[drv_pin[v]] = v;
  }
  // sinks: comb inputs cell-major, then D pins
  H.comb_inptr.assign(T.n_comb + 1, 0);
  H.comb_type.assign(T.n_comb, 0);
  H.comb_ext.assign(T.n_comb, 0);
  std::vector<int32_t> snk_pin;
  snk_pin.reserve(T.P);
  for (int c = 0; c < T.n_comb; ++c) {
    int32_t cell = combs[c].cell;
    int i = inst_of_cell(cell);
    const tdp_netlist *nl = nls[i];
    int lc = cell - H.lv.cell_base[i];
    H.comb_type[c] = (uint8_t)nl->cell_type[lc];
    H.comb_ext[c] = cell;
    for (int k = nl->cell_in_ptr[lc]; k < nl->cell_in_ptr[lc + 1]; ++k) snk_pin.push_back(H.lv.pin_base[i] + nl->cell_in_pins[k]);
    H.comb_inptr[c + 1] = (int32_t)snk_pin.size();
  }
  T.A = (int32_t)snk_pin.size();
  H.ff_ext.assign(T.n_ff, 0);
  H.ff_type.assign(T.n_ff, 0);
  H.ff_inst.assign(T.n_ff, 0);
  for (int f = 0; f < T.n_ff; ++f) {
    int32_t cell = ffs[f];
    int i = inst_of_cell(cell);
    H.ff_ext[f] = cell;
    H.ff_type[f] = (uint8_t)nls[i]->cell_type[cell - H.lv.cell_base[i]];
    H.ff_inst[f] = i;
    snk_pin.push_back(d_pin_of_ff(cell));
  }
  T.S = (int32_t)snk_pin.size();
  if (T.M + T.S != T.P) { err = "internal: pin count mismatch"; return TDP_E_INVALID; }
  H.snk_cell.assign(T.S, 0);
  H.snk_ext.assign(T.S, 0);
  H.snk_drv.assign(T.S, 0);
  H.snk_ox.assign(T.S, 0.f);
  H.snk_oy.assign(T.S, 0.f);
  H.snk_comb.assign(T.A, 0);
  for (int c = 0; c < T.n_comb; ++c)
    for (int t = H.comb_inptr[c]; t < H.comb_inptr[c + 1]; ++t) H.snk_comb[t] = c;
  for (int t = 0; t < T.S; ++t) {
    int inst, local;
    const tdp_netlist *nl = get_nl(snk_pin[t], inst, local);
    H.snk_ext[t] = snk_pin[t];
    H.snk_cell[t] = nl->pin_cell[local] + H.lv.cell_base[inst];
    H.snk_ox[t] = nl->pin_off_x[local];
    H.snk_oy[t] = nl->pin_off_y[local];
    H.ext_pin_int[snk_pin[t]] = T.M + t;
    int dl = cks[inst].driver_of[local];
    H.snk_drv[t] = H.ext_pin_int[H.lv.pin_base[inst] + dl];
  }
  // nets, in driver order, sinks in the netlist's own order
  H.net_ptr.assign(T.M + 1, 0);
  H.net_sink.clear();
  H.net_sink.reserve(T.S);
  H.net_cpin.assign(T.M, 0.0);
  H.snk_cap.assign(T.S, 0.f);
  H.type_cap.assign(lib->pin_cap, lib->pin_cap + lib->num_types);
  for (int v = 0; v < T.M; ++v) {
    int inst, local;
    const tdp_netlist *nl = get_nl(drv_pin[v], inst, local);
    int n = cks[inst].net_of_driver[local];
    double cp = 0.0;
    for (int k = nl->net_ptr[n] + 1; k < nl->net_ptr[n + 1]; ++k) {
      int tl = nl->net_pins[k];
      int t = H.ext_pin_int[H.lv.pin_base[inst] + tl] - T.M;
      H.net_sink.push_back(t);
      H.snk_cap[t] = lib->pin_cap[nl->cell_type[nl->pin_cell[tl]]];
      cp += lib->pin_cap[nl->cell_type[nl->pin_cell[tl]]];
    }
    H.net_cpin[v] = cp;
    H.net_ptr[v + 1] = (int32_t)H.net_sink.size();
  }
  H.cell_fixed.assign(T.N, 0);
  for (int i = 0; i < count; ++i)
    if (nls[i]->cell_fixed)
      for (int c = 0; c < nls[i]->num_cells; ++c) H.cell_fixed[H.lv.cell_base[i] + c] = nls[i]->cell_fixed[c] ? 1 : 0;

  // ---------------------------------------------------------- 64-lane chunks
  auto seg = [](int head, int tail) { return head | (tail << 8); };
  // combinational inputs, cell by cell, one level after another
  {
    int64_t lane = 0;
    auto pad = [&]() {
      while (lane % CHUNK) {
        const int l = (int)(lane % CHUNK);
        H.fw_rec.push_back(make_int4(-1, 0, 0, seg(l, l)));
        H.fw_ext.push_back(make_int2(0, 0));
        ++lane;
      }
    };
    H.lv.fw_lvl.assign(T.D + 1, 0);
    for (int l = 1; l <= T.D; ++l) {
      for (int c = H.lv.lvl[l - 1]; c < H.lv.lvl[l]; ++c) {
        const int n = H.comb_inptr[c + 1] - H.comb_inptr[c];
        if (n > CHUNK) { err = "cells with more than 64 inputs are not supported"; return TDP_E_UNSUPPORTED; }
        if (lane % CHUNK + n > CHUNK) pad();
        const int head = (int)(lane % CHUNK);
        for (int t = H.comb_inptr[c]; t < H.comb_inptr[c + 1]; ++t) {
          H.fw_rec.push_back(make_int4(t, H.snk_drv[t], c, seg(head, head + n - 1) | (int)H.comb_type[c] << 16));
          H.fw_ext.push_back(make_int2(H.snk_ext[t], H.drv_ext[H.snk_drv[t]]));
          ++lane;
        }
      }
      pad();
      H.lv.fw_lvl[l] = (int32_t)(lane / CHUNK);
    }
    T.n_fw_chunks = (int32_t)(lane / CHUNK);
    // the widest cell of each chunk, in bits 24-30 of every lane's record:
    // a wave-uniform bound for the segmented reductions
    for (int64_t k0 = 0; k0 < lane; k0 += CHUNK) {
      int w = 1;
      for (int64_t k = k0; k < k0 + CHUNK; ++k)
        if (H.fw_rec[k].x >= 0) w = std::max(w, ((H.fw_rec[k].w >> 8) & 63) - (H.fw_rec[k].w & 63) + 1);
      for (int64_t k = k0; k < k0 + CHUNK; ++k) H.fw_rec[k].w |= w << 24;
    }
  }
  // nets: driver lane then sinks, drivers level by level (start points first)
  {
    int64_t lane = 0;
    auto pad = [&]() {
      while (lane % CHUNK) {
        const int l = (int)(lane % CHUNK);
        H.nm_rec.push_back(make_int4(-1, -1, -1, seg(l, l)));
        H.nm_ox.push_back(0.f);
        H.nm_oy.push_back(0.f);
        ++lane;
      }
    };
    H.lv.nm_lvl.assign(T.D + 2, 0);
    H.lv.big_lvl.assign(T.D + 2, 0);
    for (int l = 0; l <= T.D; ++l) {
      const int v0 = l == 0 ? 0 : T.n_start + H.lv.lvl[l - 1];
      const int v1 = l == 0 ? T.n_start : T.n_start + H.lv.lvl[l];
      for (int v = v0; v < v1; ++v) {
        const int n = 1 + H.net_ptr[v + 1] - H.net_ptr[v];
        if (n > CHUNK) {
          H.big_net.push_back(v);
          continue;
        }
        if (lane % CHUNK + n > CHUNK) pad();
        const int head = (int)(lane % CHUNK);
        H.nm_rec.push_back(make_int4(v, H.drv_cell[v], -1, seg(head, head + n - 1)));
        H.nm_ox.push_back(H.drv_ox[v]);
        H.nm_oy.push_back(H.drv_oy[v]);
        ++lane;
        for (int k = H.net_ptr[v]; k < H.net_ptr[v + 1]; ++k) {
          const int t = H.net_sink[k];
          const int vo = t < T.A ? T.n_start + H.snk_comb[t] : -1;
          const int ty = t < T.A ? H.comb_type[H.snk_comb[t]] : H.ff_type[t - T.A];
          H.nm_rec.push_back(make_int4(T.M + t, H.snk_cell[t], vo, seg(head, head + n - 1) | ty << 16));
          H.nm_ox.push_back(H.snk_ox[t]);
          H.nm_oy.push_back(H.snk_oy[t]);
          ++lane;
        }
      }
      pad();
      H.lv.nm_lvl[l + 1] = (int32_t)(lane / CHUNK);
      H.lv.big_lvl[l + 1] = (int32_t)H.big_net.size();
    }
    T.n_nm_chunks = (int32_t)(lane / CHUNK);
    T.n_big = (int32_t)H.big_net.size();
  }
  return TDP_OK;
}

}  // namespace tdp
