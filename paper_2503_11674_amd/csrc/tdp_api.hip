// C ABI entry points (include/tdp.h): argument checks, device allocation,
// precision dispatch.  Every failure returns a status and leaves the graph
// unchanged; nothing throws across the ABI.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>
#include <map>
#include <vector>
#include <mutex>
#include <new>
#include <string>

#include "tdp_impl.h"
#include "tdp_prims.h"

using namespace tdp;

// The no-allocation variant of report_timing keeps its node store in this
// fixed array, one copy per device, held until the process ends.  Host code
// never uses the array's name as an address: the device address comes from
// hipGetSymbolAddress, once per device with that device current.
static constexpr size_t kNoallocBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kNoallocBytes];

namespace {

thread_local std::string g_loose_error;  // errors before a graph exists

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) hipSetDevice(dev);
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) hipSetDevice(prev);
  }
};

tdp_status fail(tdp_graph g, tdp_status st, const std::string &msg) {
  if (g) g->last_error = msg;
  else g_loose_error = msg;
  return st;
}

tdp_status check_launch(tdp_graph g, const char *what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(g, TDP_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
  return TDP_OK;
}

template <typename P>
bool dalloc(tdp_graph g, P *&ptr, size_t count, size_t elem = sizeof(P), int fill = 0) {
  void *p = nullptr;
  size_t bytes = std::max<size_t>(count * elem, 16);
  if (hipMalloc(&p, bytes) != hipSuccess) return false;
  if (hipMemset(p, fill, bytes) != hipSuccess) {
    hipFree(p);
    return false;
  }
  g->allocs.push_back(p);
  ptr = (P *)p;
  return true;
}

template <typename P>
bool upload(tdp_graph g, P *&ptr, const std::vector<P> &h) {
  if (!dalloc(g, ptr, h.size())) return false;
  if (h.empty()) return true;
  return hipMemcpy(ptr, h.data(), sizeof(P) * h.size(), hipMemcpyHostToDevice) == hipSuccess;
}

void free_all(tdp_graph g) {
  for (void *p : g->allocs) hipFree(p);
  g->allocs.clear();
  for (auto &m : g->prof.marks) {
    hipEventDestroy(m.a);
    hipEventDestroy(m.b);
  }
  g->prof.marks.clear();
  for (auto &e : g->prof.open)
    if (e) { hipEventDestroy(e); e = nullptr; }
  for (hipEvent_t e : g->prof.pool) hipEventDestroy(e);
  g->prof.pool.clear();
}

// required time at the D pins: period - setup as the graph's precision
// computes it (so a batch of one equals the single-netlist graph bitwise)
static double required_time(tdp_precision prec, float period, float setup) {
  return prec == TDP_F32 ? (double)(period - setup) : (double)period - (double)setup;
}

// host-side copies kept for export / import
struct HostSide {
  std::vector<int32_t> snk_ext;
};

tdp_status build_common(const tdp_netlist *const *nls, int32_t count, const tdp_library *lib, tdp_precision prec,
                        int32_t max_paths, int32_t per_inst_paths, int32_t max_k, int device, tdp_graph *out) {
  if (!out) return fail(nullptr, TDP_E_INVALID, "out is NULL");
  *out = nullptr;
  if (prec != TDP_F32 && prec != TDP_F64) return fail(nullptr, TDP_E_INVALID, "unknown precision");
  if (max_k < 1 || max_k > TDP_MAX_K) return fail(nullptr, TDP_E_INVALID, "max_k must be in 1..32");
  if (max_paths < 1) return fail(nullptr, TDP_E_INVALID, "max_paths must be >= 1");
  if (prec == TDP_F64 && count > 1)
    return fail(nullptr, TDP_E_UNSUPPORTED, "batched graphs are single precision only");
  // host-side validation first: it needs no device
  HostTopo H;
  std::string err;
  tdp_status st = build_host_topology(nls, count, lib, H, err);
  if (st != TDP_OK) return fail(nullptr, st, err);
  // path storage is indexed with 32-bit offsets: up to 2 D + 2 pins per path
  // and max_k path slots per endpoint
  if ((int64_t)max_paths * (2 * (int64_t)H.dims.D + 2) > INT32_MAX)
    return fail(nullptr, TDP_E_INVALID, "max_paths * (2 depth + 2) exceeds 2^31 - 1 path pins");
  if ((int64_t)H.dims.E * max_k > INT32_MAX)
    return fail(nullptr, TDP_E_INVALID, "endpoints * max_k exceeds 2^31 - 1 path slots");
  // the tables are staged in LDS by the forward sweep
  if ((size_t)lib->num_types * (lib->n_slew + lib->n_load + 2 * lib->n_slew * lib->n_load) > 8192)
    return fail(nullptr, TDP_E_UNSUPPORTED, "library tables exceed 32 KB");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
    return fail(nullptr, TDP_E_DEVICE, "no such HIP device");

  tdp_graph g = new (std::nothrow) tdp_graph_s();
  if (!g) return fail(nullptr, TDP_E_NOMEM, "host allocation failed");
  DeviceGuard dg(device);
  g->device = device;
  if (hipDeviceGetAttribute(&g->num_cu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess ||
      g->num_cu < 1)
    g->num_cu = 1;
  g->prec = prec;
  g->esz = prec == TDP_F64 ? 8 : 4;
  g->lv = H.lv;
  Topo &T = g->topo;
  T = H.dims;
  g->r = lib->r_per_um;
  g->c = lib->c_per_um;
  g->scale = lib->delay_scale;
  g->input_slew = nls[0]->input_slew_ps;
  g->clock_slew = nls[0]->clock_slew_ps;
  g->h_inst_req.resize(count);
  for (int i = 0; i < count; ++i) g->h_inst_req[i] = required_time(prec, nls[i]->clock_period_ps, nls[i]->setup_ps);
  g->max_paths = max_paths;
  g->max_k = max_k;
  g->side_k = 1;
  while (g->side_k < max_k) g->side_k <<= 1;
  if (max_k == 1) g->side_k = 1;
  g->max_out = max_paths;
  g->max_out_inst = per_inst_paths;
  g->slot_cap = std::max(1, T.E * max_k);
  g->pin_cap = (int32_t)((int64_t)max_paths * (2 * T.D + 2));
  g->key_bits32 = T.num_inst <= 1 ? 32 : (T.num_inst <= 256 ? 40 : 48);
  int max_inst_e = 1;
  for (int i = 0; i < T.num_inst; ++i) max_inst_e = std::max(max_inst_e, H.lv.ep_base[i + 1] - H.lv.ep_base[i]);
  g->ep_chunks = std::min(64, std::max(1, (max_inst_e + 4095) / 4096));

  bool ok = true;
  // library
  const int nt = lib->num_types, ns = lib->n_slew, nl = lib->n_load;
  // one buffer [slew axes | load axes | delay tables | slew tables], padded
  // to whole float4s (the layout kernels stage in LDS)
  const size_t n_sa = (size_t)nt * ns, n_la = (size_t)nt * nl, n_tab = (size_t)nt * ns * nl;
  const size_t n_all = n_sa + n_la + 2 * n_tab, n4 = (n_all + 3) / 4;
  float4 *flat = nullptr;
  ok = ok && dalloc(g, flat, n4);
  float *sa = (float *)flat, *la = sa + n_sa, *dl = la + n_la, *sl = dl + n_tab;
  if (ok) {
    std::vector<float> img(4 * n4, 0.f);
    std::copy(lib->slew_axis, lib->slew_axis + n_sa, img.begin());
    std::copy(lib->load_axis, lib->load_axis + n_la, img.begin() + n_sa);
    std::copy(lib->delay_lut, lib->delay_lut + n_tab, img.begin() + n_sa + n_la);
    std::copy(lib->slew_lut, lib->slew_lut + n_tab, img.begin() + n_sa + n_la + n_tab);
    ok = hipMemcpy(flat, img.data(), sizeof(float) * img.size(), hipMemcpyHostToDevice) == hipSuccess;
  }
  g->lut = LutView{nt, ns, nl, sa, la, dl, sl, flat, (int)n4, lib->net_model};
  // topology
  ok = ok && upload(g, T.drv_cell, H.drv_cell) && upload(g, T.drv_ox, H.drv_ox) && upload(g, T.drv_oy, H.drv_oy) &&
       upload(g, T.drv_ext, H.drv_ext) && upload(g, T.net_ptr, H.net_ptr) && upload(g, T.net_sink, H.net_sink) &&
       upload(g, T.net_cpin, H.net_cpin) && upload(g, T.snk_cap, H.snk_cap) && upload(g, T.type_cap, H.type_cap) &&
       upload(g, T.snk_cell, H.snk_cell) && upload(g, T.snk_ox, H.snk_ox) && upload(g, T.snk_oy, H.snk_oy) &&
       upload(g, T.snk_drv, H.snk_drv) && upload(g, T.snk_ext, H.snk_ext) && upload(g, T.snk_comb, H.snk_comb) &&
       upload(g, T.comb_type, H.comb_type) &&
       upload(g, T.comb_inptr, H.comb_inptr) && upload(g, T.comb_ext, H.comb_ext) && upload(g, T.ff_ext, H.ff_ext) &&
       upload(g, T.ff_type, H.ff_type) && upload(g, T.ff_inst, H.ff_inst) &&
       upload(g, T.ext_pin_int, H.ext_pin_int) && upload(g, T.cell_int, H.cell_int) &&
       upload(g, T.cell_fixed, H.cell_fixed) && upload(g, g->d_ep_base, H.lv.ep_base) &&
       upload(g, T.fw_rec, H.fw_rec) && upload(g, T.fw_ext, H.fw_ext) && upload(g, T.nm_rec, H.nm_rec) &&
       upload(g, T.nm_ox, H.nm_ox) && upload(g, T.nm_oy, H.nm_oy) && upload(g, T.big_net, H.big_net);
  g->h_snk_ext = H.snk_ext;
  // timing state
  const size_t es = g->esz;
  ok = ok && dalloc(g, g->load, T.M, es) && dalloc(g, g->dnet, T.S, es) && dalloc(g, g->at, T.P, es) &&
       dalloc(g, g->slew, T.M, es) && dalloc(g, g->rat, T.P, es) &&
       dalloc(g, g->dnet_nm, (size_t)T.n_nm_chunks * CHUNK, es) && dalloc(g, g->drv_as, (size_t)2 * T.M, es) &&
       dalloc(g, g->fw_a, (size_t)T.n_fw_chunks * CHUNK, es) &&
       dalloc(g, g->darc, T.A, es) && dalloc(g, g->crit, T.n_comb) && dalloc(g, g->hop, (size_t)T.n_comb * 4) &&
       dalloc(g, g->hop4, (size_t)T.n_comb * 16) &&
       dalloc(g, g->cdep, T.M) && dalloc(g, g->ep_slack, T.E, es) &&
       dalloc(g, g->red_ep, (size_t)3 * T.num_inst * g->ep_chunks) && dalloc(g, g->red_loss, 4096) &&
       dalloc(g, g->red_wa, 4096) && dalloc(g, g->summary, (size_t)4 * T.num_inst) &&
       dalloc(g, g->inst_nfail, T.num_inst) && dalloc(g, g->d_err, 4) && dalloc(g, g->consts, 4) &&
       upload(g, g->d_inst_req, g->h_inst_req);
  if (ok && g->side_k > 1)
    ok = dalloc(g, g->side_cost, (size_t)T.n_comb * g->side_k, es) &&
         dalloc(g, g->side_pin, (size_t)T.n_comb * g->side_k);
  // dataflow sweeps: single precision, every net fits one 64-lane chunk
  g->flow_ok = prec == TDP_F32 && T.n_big == 0;
  g->sweep_mode = g->flow_ok ? 3 : 0;
  if (ok && g->flow_ok) {
    ok = dalloc(g, g->flow_w, T.M) && dalloc(g, g->flow_r, T.M) && dalloc(g, g->flow_cd, T.M) &&
         dalloc(g, g->flow_se, (size_t)T.n_comb * g->side_k);
  }
  if (ok) {
    const double one[4] = {1.0, 0.0, 0.0, 0.0};
    ok = hipMemcpy(g->consts, one, sizeof one, hipMemcpyHostToDevice) == hipSuccess;
  }
  // extraction
  const int sc = g->slot_cap, mo = g->max_out, ni = T.num_inst;
  const int scan_cap = std::max({T.S, T.N, T.E, mo, sc, sort_hist_size(sc)});
  ok = ok && dalloc(g, g->sel_flag, T.E) && dalloc(g, g->sel_pos, T.E) && dalloc(g, g->sel_list, T.E) &&
       dalloc(g, g->d_nsel, 1) && dalloc(g, g->inst_nsel, ni) && dalloc(g, g->inst_nvalid, ni) &&
       dalloc(g, g->inst_seg, ni) && dalloc(g, g->inst_outb, ni) && dalloc(g, g->inst_kept, ni) &&
       dalloc(g, g->inst_selb, ni) && dalloc(g, g->sel_npop, T.E) &&
       dalloc(g, g->slot_key, sc, es) && dalloc(g, g->slot_dev, sc) && dalloc(g, g->slot_par, sc) &&
       dalloc(g, g->slot_len, sc) && dalloc(g, g->slot_out, std::max(sc, mo)) && dalloc(g, g->slot_cells, sc) && dalloc(g, g->d_nslots, 1) &&
       dalloc(g, g->sort_k0, sc) && dalloc(g, g->sort_k1, sc) && dalloc(g, g->sort_v0, sc) &&
       dalloc(g, g->sort_v1, sc) && dalloc(g, g->sort_hist, sort_hist_size(sc)) &&
       dalloc(g, g->scan_tmp, scan_tmp_size(scan_cap)) && dalloc(g, g->out_slot, mo) &&
       dalloc(g, g->out_len, mo) && dalloc(g, g->path_ptr, (size_t)mo + 1) && dalloc(g, g->path_pins, g->pin_cap) &&
       dalloc(g, g->path_int, g->pin_cap) && dalloc(g, g->path_ep, mo) && dalloc(g, g->path_epi, mo) &&
       dalloc(g, g->path_rank, mo) && dalloc(g, g->d_num_paths, 1) && dalloc(g, g->path_slack, mo, es);
  // pairs
  ok = ok && dalloc(g, g->pw, T.S) && dalloc(g, g->pin_p, T.S) && dalloc(g, g->pacc, T.S) &&
       dalloc(g, g->pfirst, T.S, sizeof(int32_t), 0x7F) && dalloc(g, g->pflag, T.S) && dalloc(g, g->d_npairs, 1) &&
       dalloc(g, g->pair_sink, T.S) && dalloc(g, g->pair_cs, T.S) && dalloc(g, g->pair_ct, T.S) &&
       dalloc(g, g->pair_dox, T.S) && dalloc(g, g->pair_doy, T.S) && dalloc(g, g->pair_w, T.S) &&
       dalloc(g, g->cell_cnt, T.N) && dalloc(g, g->cell_ptr, (size_t)T.N + 1) && dalloc(g, g->cell_cur, T.N) &&
       dalloc(g, g->cell_flag, T.N) && dalloc(g, g->touched, T.N) && dalloc(g, g->d_ntouched, 1) &&
       dalloc(g, g->inc_other, (size_t)2 * T.S) && dalloc(g, g->inc_key, (size_t)2 * T.S) &&
       dalloc(g, g->inc_dx, (size_t)2 * T.S) && dalloc(g, g->inc_dy, (size_t)2 * T.S) &&
       dalloc(g, g->inc_w, (size_t)2 * T.S);
  // smoothed TNS, WA
  ok = ok && dalloc(g, g->st_at, T.P, es) && dalloc(g, g->st_adj, T.P, es) && dalloc(g, g->st_dnet, T.S, es) &&
       dalloc(g, g->st_gp, (size_t)2 * T.P, es) &&
       dalloc(g, g->wa_gpin, (size_t)2 * T.P) && dalloc(g, g->xy, T.N) &&
       dalloc(g, g->xy_wa, T.N) && dalloc(g, g->xy_st, T.N) && dalloc(g, g->cxy_nm, (size_t)T.n_nm_chunks * CHUNK);
  // spanning-tree net model: scratch of the net pass and of the smoothed TNS
  if (lib->net_model == 2) {
    auto tree_alloc = [&](TreeBuf &b) {
      return dalloc(g, b.dist, T.S) && dalloc(g, b.par, T.S) && dalloc(g, b.ord, T.S) && dalloc(g, b.len, T.S, es) &&
             dalloc(g, b.cd, T.S, es) && dalloc(g, b.aux, T.S, es) && dalloc(g, b.aux2, T.S, es) &&
             dalloc(g, b.wl, T.M, es);
    };
    ok = ok && tree_alloc(g->tree) && tree_alloc(g->st_tree);
  }
  if (!ok || hipDeviceSynchronize() != hipSuccess) {
    free_all(g);
    delete g;
    return fail(nullptr, TDP_E_NOMEM, "device allocation or upload failed");
  }
  *out = g;
  return TDP_OK;
}

#define GUARD(g)                                                     \
  if (!(g)) return fail(nullptr, TDP_E_INVALID, "graph is NULL"); \
  DeviceGuard _dg((g)->device)

template <typename F>
tdp_status dispatch(tdp_graph g, F &&f) {
  if (g->prec == TDP_F64) f((double)0);
  else f((float)0);
  return TDP_OK;
}

}  // namespace

extern "C" {

tdp_status tdp_sta_build(const tdp_netlist *netlist, const tdp_library *lib, tdp_precision prec, int32_t max_paths,
                         int32_t max_k, int device, tdp_graph *out) {
  const tdp_netlist *one[1] = {netlist};
  return build_common(one, 1, lib, prec, max_paths, max_paths, max_k, device, out);
}

tdp_status tdp_batch_build(const tdp_netlist *const *netlists, int32_t count, const tdp_library *lib,
                           tdp_precision prec, int32_t max_paths_each, int32_t max_k, int device, tdp_graph *out) {
  if (!netlists || count < 1) return fail(nullptr, TDP_E_INVALID, "no netlists");
  for (int i = 1; i < count; ++i)
    if (!netlists[i] || !netlists[0] || netlists[i]->input_slew_ps != netlists[0]->input_slew_ps ||
        netlists[i]->clock_slew_ps != netlists[0]->clock_slew_ps)
      return fail(nullptr, TDP_E_INVALID, "batched netlists must share input and clock slews");
  int64_t cap = (int64_t)max_paths_each * count;
  if (max_paths_each < 1 || cap > (1 << 30)) return fail(nullptr, TDP_E_INVALID, "bad max_paths_each");
  return build_common(netlists, count, lib, prec, (int32_t)cap, max_paths_each, max_k, device, out);
}

tdp_status tdp_batch_offsets(tdp_graph g, int32_t *pin_base, int32_t *cell_base) {
  if (!g) return fail(nullptr, TDP_E_INVALID, "graph is NULL");
  for (int i = 0; i <= g->topo.num_inst; ++i) {
    if (pin_base) pin_base[i] = g->lv.pin_base[i];
    if (cell_base) cell_base[i] = g->lv.cell_base[i];
  }
  return TDP_OK;
}

void tdp_destroy(tdp_graph g) {
  if (!g) return;
  DeviceGuard dg(g->device);
  hipDeviceSynchronize();
  free_all(g);
  delete g;
}

tdp_status tdp_sta_set_clock(tdp_graph g, float period, float setup) {
  GUARD(g);
  if (!std::isfinite(period) || !std::isfinite(setup)) return fail(g, TDP_E_INVALID, "clock not finite");
  for (double &r : g->h_inst_req) r = required_time(g->prec, period, setup);
  if (hipMemcpy(g->d_inst_req, g->h_inst_req.data(), sizeof(double) * g->h_inst_req.size(),
                hipMemcpyHostToDevice) != hipSuccess)
    return fail(g, TDP_E_DEVICE, "clock upload failed");
  return TDP_OK;
}

tdp_status tdp_sta_update(tdp_graph g, const float *x, const float *y, hipStream_t s) {
  GUARD(g);
  if (!x || !y) return fail(g, TDP_E_INVALID, "positions are NULL");
  g->ea_ready = false;  // the hold results belong to the previous placement
  g->rf_updated = false;
  dispatch(g, [&](auto z) {
    sta_arrivals_impl<decltype(z)>(g, x, y, s);
    sta_required_impl<decltype(z)>(g, s);
  });
  tdp_status st = check_launch(g, "sta_update");
  if (st == TDP_OK) g->updated = true;
  return st;
}

tdp_status tdp_sta_update_arrivals_incremental(tdp_graph g, const float *x, const float *y, const int32_t *cells,
                                               int32_t n_cells, hipStream_t s) {
  GUARD(g);
  if (!x || !y) return fail(g, TDP_E_INVALID, "positions are NULL");
  if (n_cells < 0 || (n_cells > 0 && !cells)) return fail(g, TDP_E_INVALID, "bad moved-cell list");
  if (!g->updated) return fail(g, TDP_E_STATE, "an incremental update needs a full one first");
  if (g->topo.n_big > 0) return fail(g, TDP_E_UNSUPPORTED, "incremental updates need every net within one chunk");
  const Topo &T = g->topo;
  if (!g->inc_ready) {
    const bool ok = dalloc(g, g->inc_arr, T.n_fw_chunks) && dalloc(g, g->inc_lst, T.n_fw_chunks) &&
                    dalloc(g, g->inc_drv_chg, T.M) && dalloc(g, g->inc_drv_lchg, T.M) &&
                    dalloc(g, g->inc_nm, T.n_nm_chunks) && dalloc(g, g->inc_snk_chunk, T.A) &&
                    dalloc(g, g->inc_drv_nm_chunk, T.M);
    if (!ok) return fail(g, TDP_E_NOMEM, "incremental update: device allocation failed");
    inc_maps(g, s);
    g->inc_ready = true;
    g->inc_epoch = 0;
  }
  if (g->inc_epoch == INT32_MAX) {  // the stamps start over
    fill_i32(g->inc_arr, T.n_fw_chunks, 0, s);
    fill_i32(g->inc_lst, T.n_fw_chunks, 0, s);
    fill_i32(g->inc_drv_chg, T.M, 0, s);
    fill_i32(g->inc_drv_lchg, T.M, 0, s);
    fill_i32(g->inc_nm, T.n_nm_chunks, 0, s);
    g->inc_epoch = 0;
  }
  ++g->inc_epoch;
  g->ea_ready = false;
  g->rf_updated = false;
  dispatch(g, [&](auto z) { sta_arrivals_incremental_impl<decltype(z)>(g, x, y, cells, n_cells, s); });
  return check_launch(g, "sta_update_arrivals_incremental");
}

tdp_status tdp_sta_update_arrivals(tdp_graph g, const float *x, const float *y, hipStream_t s) {
  GUARD(g);
  if (!x || !y) return fail(g, TDP_E_INVALID, "positions are NULL");
  g->ea_ready = false;
  g->rf_updated = false;
  dispatch(g, [&](auto z) { sta_arrivals_impl<decltype(z)>(g, x, y, s); });
  tdp_status st = check_launch(g, "sta_update_arrivals");
  if (st == TDP_OK) g->updated = true;
  return st;
}

tdp_status tdp_sta_update_required(tdp_graph g, hipStream_t s) {
  GUARD(g);
  if (!g->updated) return fail(g, TDP_E_STATE, "no arrival pass yet");
  dispatch(g, [&](auto z) { sta_required_impl<decltype(z)>(g, s); });
  return check_launch(g, "sta_update_required");
}

tdp_status tdp_sta_summary(tdp_graph g, double *wns, double *tns, int32_t *n_fail, hipStream_t s) {
  GUARD(g);
  if (!g->updated) return fail(g, TDP_E_STATE, "no timing update yet");
  const int ni = g->topo.num_inst;
  std::vector<double> h(4 * ni);
  int32_t errs[2] = {0, 0};
  if (hipStreamSynchronize(s) != hipSuccess ||
      hipMemcpy(h.data(), g->summary, sizeof(double) * 4 * ni, hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(errs, g->d_err, 8, hipMemcpyDeviceToHost) != hipSuccess)
    return fail(g, TDP_E_DEVICE, "summary copy failed");
  const int32_t err = errs[0];
  if (errs[1] == g->pos_gen) return fail(g, TDP_E_INVALID, "a cell position of the last update is NaN or infinite");
  if (err & 2) return fail(g, TDP_E_DEVICE, "a dataflow sweep gave up waiting (results are invalid)");
  if (err & 4) return fail(g, TDP_E_DEVICE, "an incremental update was given a cell id outside [0, num_cells)");
  double w = 0, t = 0, n = 0;
  for (int i = 0; i < ni; ++i) {
    w = std::min(w, h[4 * i]);
    t += h[4 * i + 1];
    n += h[4 * i + 2];
  }
  if (wns) *wns = w;
  if (tns) *tns = t;
  if (n_fail) *n_fail = (int32_t)n;
  return TDP_OK;
}

tdp_status tdp_batch_summary(tdp_graph g, double *wns, double *tns, int32_t *n_fail, hipStream_t s) {
  GUARD(g);
  if (!g->updated) return fail(g, TDP_E_STATE, "no timing update yet");
  const int ni = g->topo.num_inst;
  std::vector<double> h(4 * ni);
  if (hipStreamSynchronize(s) != hipSuccess ||
      hipMemcpy(h.data(), g->summary, sizeof(double) * 4 * ni, hipMemcpyDeviceToHost) != hipSuccess)
    return fail(g, TDP_E_DEVICE, "summary copy failed");
  for (int i = 0; i < ni; ++i) {
    if (wns) wns[i] = h[4 * i];
    if (tns) tns[i] = h[4 * i + 1];
    if (n_fail) n_fail[i] = (int32_t)h[4 * i + 2];
  }
  return TDP_OK;
}

tdp_status tdp_sta_export(tdp_graph g, double *at, double *rat, double *slack, double *slew, double *dnet,
                          double *load, double *darc, hipStream_t s) {
  GUARD(g);
  if (!g->updated) return fail(g, TDP_E_STATE, "no timing update yet");
  dispatch(g, [&](auto z) { sta_export_impl<decltype(z)>(g, at, rat, slack, slew, dnet, load, darc, s); });
  return check_launch(g, "sta_export");
}

tdp_status tdp_rf_setup(tdp_graph g, const tdp_rf_tables *rt) {
  GUARD(g);
  if (!rt || !rt->delay_fall || !rt->slew_fall || !rt->unate) return fail(g, TDP_E_INVALID, "NULL rise/fall table");
  if (g->topo.num_inst > 1) return fail(g, TDP_E_UNSUPPORTED, "rise / fall timing on a batched graph");
  const Topo &T = g->topo;
  const int nt = g->lut.nt, ntab = nt * g->lut.ns * g->lut.nl;
  for (int t = 0; t < nt; ++t)
    if (rt->unate[t] < 0 || rt->unate[t] > 2) return fail(g, TDP_E_INVALID, "unate must be 0, 1 or 2");
  for (int i = 0; i < ntab; ++i)
    if (!std::isfinite(rt->delay_fall[i]) || !std::isfinite(rt->slew_fall[i]))
      return fail(g, TDP_E_INVALID, "rise/fall tables must be finite");
  if (!g->rf_ready) {
    const size_t es = g->esz;
    const bool ok = dalloc(g, g->rf_at, (size_t)2 * T.P, es) && dalloc(g, g->rf_slew, (size_t)2 * T.P, es) &&
                    dalloc(g, g->rf_rat, (size_t)2 * T.P, es) && dalloc(g, g->rf_darc4, (size_t)4 * T.A, es) &&
                    dalloc(g, g->rf_crit, (size_t)2 * T.n_comb) && dalloc(g, g->rf_unate, nt) &&
                    dalloc(g, g->rf_flat, (size_t)g->lut.n4) && dalloc(g, g->rf_path_tran, g->pin_cap);
    if (!ok) return fail(g, TDP_E_NOMEM, "rise/fall: device allocation failed");
    // the same axes as the rise tables, then the fall tables
    const size_t n_ax = (size_t)nt * (g->lut.ns + g->lut.nl);
    g->rf_delay_fall = (float *)g->rf_flat + n_ax;
    g->rf_slew_fall = g->rf_delay_fall + ntab;
    if (hipMemcpy(g->rf_flat, g->lut.flat4, sizeof(float) * n_ax, hipMemcpyDeviceToDevice) != hipSuccess)
      return fail(g, TDP_E_DEVICE, "rise/fall: table upload failed");
  }
  if (hipMemcpy(g->rf_unate, rt->unate, sizeof(int32_t) * nt, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(g->rf_delay_fall, rt->delay_fall, sizeof(float) * ntab, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(g->rf_slew_fall, rt->slew_fall, sizeof(float) * ntab, hipMemcpyHostToDevice) != hipSuccess)
    return fail(g, TDP_E_DEVICE, "rise/fall: table upload failed");
  g->rf_ready = true;
  g->rf_updated = false;
  return TDP_OK;
}

tdp_status tdp_sta_update_rf(tdp_graph g, const float *x, const float *y, hipStream_t s) {
  GUARD(g);
  if (!g->rf_ready) return fail(g, TDP_E_STATE, "rise/fall tables not set (tdp_rf_setup)");
  if (!x || !y) return fail(g, TDP_E_INVALID, "positions are NULL");
  // the single-transition results (and everything derived from them) are
  // replaced: the endpoint slacks and WNS / TNS now hold the rise/fall ones
  g->updated = false;
  g->extracted = false;
  g->ea_ready = false;
  g->stns_ready = false;
  dispatch(g, [&](auto z) { rf_update_impl<decltype(z)>(g, x, y, s); });
  tdp_status st = check_launch(g, "sta_update_rf");
  if (st == TDP_OK) g->rf_updated = true;
  return st;
}

tdp_status tdp_sta_rf_summary(tdp_graph g, double *wns, double *tns, int32_t *n_fail, hipStream_t s) {
  GUARD(g);
  if (!g->rf_updated) return fail(g, TDP_E_STATE, "no rise/fall update yet");
  double h[4] = {0, 0, 0, 0};
  if (hipStreamSynchronize(s) != hipSuccess ||
      hipMemcpy(h, g->summary, sizeof h, hipMemcpyDeviceToHost) != hipSuccess)
    return fail(g, TDP_E_DEVICE, "summary copy failed");
  if (wns) *wns = std::min(0.0, h[0]);
  if (tns) *tns = h[1];
  if (n_fail) *n_fail = (int32_t)h[2];
  return TDP_OK;
}

tdp_status tdp_sta_rf_export(tdp_graph g, double *at, double *rat, double *slack, double *slew, hipStream_t s) {
  GUARD(g);
  if (!g->rf_updated) return fail(g, TDP_E_STATE, "no rise/fall update yet");
  dispatch(g, [&](auto z) { rf_export_impl<decltype(z)>(g, at, rat, slack, slew, s); });
  return check_launch(g, "sta_rf_export");
}

tdp_status tdp_extract_paths_rf(tdp_graph g, int32_t n, int32_t K, hipStream_t s, tdp_paths *out,
                                const uint8_t **d_path_tran) {
  GUARD(g);
  if (!g->rf_updated) return fail(g, TDP_E_STATE, "no rise/fall update yet");
  if (K < 0) return fail(g, TDP_E_INVALID, "K < 0");
  if (n > g->max_paths) return fail(g, TDP_E_CAPACITY, "n > max_paths");
  dispatch(g, [&](auto z) { rf_extract_impl<decltype(z)>(g, n, K, s); });
  tdp_status st = check_launch(g, "extract_paths_rf");
  if (st != TDP_OK) return st;
  g->extracted = true;
  g->last_k = 1;
  if (out) {
    out->max_paths = g->max_out;
    out->d_num_paths = g->d_num_paths;
    out->path_ptr = g->path_ptr;
    out->path_pins = g->path_pins;
    out->path_ep = g->path_ep;
    out->path_rank = g->path_rank;
    out->path_slack = g->path_slack;
  }
  if (d_path_tran) *d_path_tran = g->rf_path_tran;
  return TDP_OK;
}

tdp_status tdp_sta_export_crit(tdp_graph g, int32_t *crit, hipStream_t s) {
  GUARD(g);
  if (!g->updated) return fail(g, TDP_E_STATE, "no timing update yet");
  if (!crit) return fail(g, TDP_E_INVALID, "crit is NULL");
  sta_export_crit(g, crit, s);
  return check_launch(g, "sta_export_crit");
}

tdp_status tdp_sta_views(tdp_graph g, const void **at, const void **rat, const int32_t **pin_index) {
  GUARD(g);
  if (!g->updated) return fail(g, TDP_E_STATE, "no timing update yet");
  if (at) *at = g->at;
  if (rat) *rat = g->rat;
  if (pin_index) *pin_index = g->topo.ext_pin_int;
  return TDP_OK;
}

tdp_status tdp_extract_paths(tdp_graph g, int32_t n, int32_t k, int32_t K, float slack_limit, hipStream_t s,
                             tdp_paths *out) {
  GUARD(g);
  if (!g->updated) return fail(g, TDP_E_STATE, "no timing update yet");
  if (k < 1 || k > g->max_k) return fail(g, TDP_E_CAPACITY, "k outside 1..max_k");
  if (K < 0) return fail(g, TDP_E_INVALID, "K < 0");
  if (std::isnan(slack_limit)) return fail(g, TDP_E_INVALID, "slack_limit is NaN");
  const int Keff = std::min(K, g->max_out_inst);
  dispatch(g, [&](auto z) { extract_impl<decltype(z)>(g, n, k, Keff, slack_limit, s); });
  tdp_status st = check_launch(g, "extract_paths");
  if (st != TDP_OK) return st;
  g->extracted = true;
  g->last_k = k;
  if (out) {
    out->max_paths = g->max_out;
    out->d_num_paths = g->d_num_paths;
    out->path_ptr = g->path_ptr;
    out->path_pins = g->path_pins;
    out->path_ep = g->path_ep;
    out->path_rank = g->path_rank;
    out->path_slack = g->path_slack;
  }
  return TDP_OK;
}

// the node store of report_timing(K), made on its first call
}  // extern "C" (reopened below)

namespace tdp {
int report_node_cap(const tdp_graph_s *g) {
  const int64_t want = std::max<int64_t>({(int64_t)8 * g->max_out, (int64_t)g->slot_cap, 4096});
  return (int)std::min<int64_t>(want, (int64_t)1 << 27);
}
}  // namespace tdp

namespace {

// the graph's node store, allocated by the first report_timing call
tdp_status ensure_global(tdp_graph g) {
  if (g->gcap > 0) return TDP_OK;
  const Topo &T = g->topo;
  const int cap = report_node_cap(g);
  const size_t es = g->esz;
  const int scan_cap = std::max(cap, sort_hist_size(cap));
  const bool ok = dalloc(g, g->gt_cost, cap, es) && dalloc(g, g->gt_key, cap, es) &&
                  dalloc(g, g->gt_theta, T.num_inst, es) && dalloc(g, g->gt_dev, cap) && dalloc(g, g->gt_par, cap) &&
                  dalloc(g, g->gt_ep, cap) && dalloc(g, g->gt_cells, cap) && dalloc(g, g->gt_nd, cap) &&
                  dalloc(g, g->gt_cnt, cap) && dalloc(g, g->gt_off, cap) && dalloc(g, g->gt_start, T.num_inst) &&
                  dalloc(g, g->gt_end, T.num_inst) && dalloc(g, g->gt_misc, 4) && dalloc(g, g->gt_k0, cap) &&
                  dalloc(g, g->gt_k1, cap) && dalloc(g, g->gt_v0, cap) && dalloc(g, g->gt_v1, cap) &&
                  dalloc(g, g->gt_hist, sort_hist_size(cap)) && dalloc(g, g->gt_scan, scan_tmp_size(scan_cap));
  if (!ok) return fail(g, TDP_E_NOMEM, "report_timing: device allocation failed");
  g->gcap = cap;
  return TDP_OK;
}

GtStore graph_store(tdp_graph g) {
  GtStore st;
  st.cap = g->gcap;
  st.gt_cost = g->gt_cost;
  st.gt_key = g->gt_key;
  st.gt_theta = g->gt_theta;
  st.gt_dev = g->gt_dev;
  st.gt_par = g->gt_par;
  st.gt_ep = g->gt_ep;
  st.gt_cells = g->gt_cells;
  st.gt_nd = g->gt_nd;
  st.gt_cnt = g->gt_cnt;
  st.gt_off = g->gt_off;
  st.gt_start = g->gt_start;
  st.gt_end = g->gt_end;
  st.gt_misc = g->gt_misc;
  st.gt_k0 = g->gt_k0;
  st.gt_k1 = g->gt_k1;
  st.gt_v0 = g->gt_v0;
  st.gt_v1 = g->gt_v1;
  st.gt_hist = g->gt_hist;
  st.gt_scan = g->gt_scan;
  return st;
}

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char *g_scratch_ptr[kMaxDevices] = {};

tdp_status scratch_address(tdp_graph g, unsigned char **out) {
  if (g->device < 0 || g->device >= kMaxDevices) return fail(g, TDP_E_UNSUPPORTED, "device index beyond 63");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[g->device]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(g, TDP_E_DEVICE, std::string("no-allocation scratch: hipGetSymbolAddress failed: ") +
                                       hipGetErrorString(e));
    g_scratch_ptr[g->device] = (unsigned char *)p;
  }
  *out = g_scratch_ptr[g->device];
  return TDP_OK;
}

// carve the node store for `cap` nodes out of [base, base + limit); returns
// the bytes it needs (more than limit: nothing carved)
size_t carve_store(const tdp_graph_s *g, int cap, unsigned char *base, size_t limit, GtStore &st) {
  const size_t es = g->esz, ni = (size_t)g->topo.num_inst;
  const int scan_cap = std::max(cap, sort_hist_size(cap));
  size_t off = 0;
  auto take = [&](size_t bytes) -> void * {
    void *p = base + off;
    off += (std::max<size_t>(bytes, 16) + 255) & ~(size_t)255;
    return p;
  };
  const size_t c = (size_t)cap;
  st.cap = cap;
  st.gt_cost = take(c * es);
  st.gt_key = take(c * es);
  st.gt_theta = take(ni * es);
  st.gt_dev = (int32_t *)take(c * 4);
  st.gt_par = (int32_t *)take(c * 4);
  st.gt_ep = (int32_t *)take(c * 4);
  st.gt_cells = (int32_t *)take(c * 4);
  st.gt_nd = (int32_t *)take(c * 4);
  st.gt_cnt = (int32_t *)take(c * 4);
  st.gt_off = (int32_t *)take(c * 4);
  st.gt_start = (int32_t *)take(ni * 4);
  st.gt_end = (int32_t *)take(ni * 4);
  st.gt_misc = (int32_t *)take(16);
  st.gt_k0 = (uint64_t *)take(c * 8);
  st.gt_k1 = (uint64_t *)take(c * 8);
  st.gt_v0 = (uint32_t *)take(c * 4);
  st.gt_v1 = (uint32_t *)take(c * 4);
  st.gt_hist = (int32_t *)take((size_t)sort_hist_size(cap) * 4);
  st.gt_scan = (int32_t *)take((size_t)scan_tmp_size(scan_cap) * 4);
  if (off > limit) st = GtStore{};
  return off;
}

tdp_status report_common(tdp_graph g, const GtStore &st, int32_t K, float slack_limit, hipStream_t s,
                         tdp_paths *out) {
  const int Keff = std::min(K, g->max_out_inst);
  tdp_status rs = TDP_OK;
  dispatch(g, [&](auto z) { rs = report_impl<decltype(z)>(g, st, Keff, slack_limit, s); });
  if (rs != TDP_OK) return rs;
  rs = check_launch(g, "report_timing");
  if (rs != TDP_OK) return rs;
  g->extracted = true;
  g->last_k = 1;
  if (out) {
    out->max_paths = g->max_out;
    out->d_num_paths = g->d_num_paths;
    out->path_ptr = g->path_ptr;
    out->path_pins = g->path_pins;
    out->path_ep = g->path_ep;
    out->path_rank = g->path_rank;
    out->path_slack = g->path_slack;
  }
  return TDP_OK;
}

}  // namespace

extern "C" {

tdp_status tdp_report_timing(tdp_graph g, int32_t K, float slack_limit, hipStream_t s, tdp_paths *out) {
  GUARD(g);
  if (!g->updated) return fail(g, TDP_E_STATE, "no timing update yet");
  if (K < 0) return fail(g, TDP_E_INVALID, "K < 0");
  if (std::isnan(slack_limit)) return fail(g, TDP_E_INVALID, "slack_limit is NaN");
  tdp_status st = ensure_global(g);
  if (st != TDP_OK) return st;
  return report_common(g, graph_store(g), K, slack_limit, s, out);
}

tdp_status tdp_report_timing_noalloc(tdp_graph g, int32_t K, float slack_limit, hipStream_t s, tdp_paths *out) {
  GUARD(g);
  if (!g->updated) return fail(g, TDP_E_STATE, "no timing update yet");
  if (K < 0) return fail(g, TDP_E_INVALID, "K < 0");
  if (std::isnan(slack_limit)) return fail(g, TDP_E_INVALID, "slack_limit is NaN");
  unsigned char *base = nullptr;
  tdp_status st = scratch_address(g, &base);
  if (st != TDP_OK) return st;
  GtStore gs;
  const size_t need = carve_store(g, report_node_cap(g), base, kNoallocBytes, gs);
  if (need > kNoallocBytes)
    return fail(g, TDP_E_CAPACITY,
                "report_timing_noalloc: this graph's node store needs " + std::to_string(need) +
                    " bytes, more than the fixed " + std::to_string(kNoallocBytes) +
                    " (max_paths and max_k set its size; use tdp_report_timing)");
  return report_common(g, gs, K, slack_limit, s, out);
}

tdp_status tdp_paths_count(tdp_graph g, int32_t *num_paths, int32_t *num_pins, hipStream_t s) {
  GUARD(g);
  if (!g->extracted) return fail(g, TDP_E_STATE, "no extraction yet");
  int32_t n = 0, pins = 0, err = 0;
  if (hipStreamSynchronize(s) != hipSuccess ||
      hipMemcpy(&n, g->d_num_paths, 4, hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(&pins, g->path_ptr + n, 4, hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(&err, g->d_err, 4, hipMemcpyDeviceToHost) != hipSuccess)
    return fail(g, TDP_E_DEVICE, "count copy failed");
  if (err & 1) return fail(g, TDP_E_DEVICE, "internal: a path walk did not match its length");
  if (err & 2) return fail(g, TDP_E_DEVICE, "a dataflow sweep gave up waiting (results are invalid)");
  if (num_paths) *num_paths = n;
  if (num_pins) *num_pins = pins;
  return TDP_OK;
}

tdp_status tdp_pairs_update(tdp_graph g, int32_t rule, float w0, float w1, hipStream_t s) {
  GUARD(g);
  if (!g->extracted) return fail(g, TDP_E_STATE, "no extraction yet");
  if (rule != 0 && rule != 1) return fail(g, TDP_E_INVALID, "rule must be 0 or 1");
  if (!std::isfinite(w0) || !std::isfinite(w1)) return fail(g, TDP_E_INVALID, "weights not finite");
  dispatch(g, [&](auto z) { pairs_update_impl<decltype(z)>(g, rule, w0, w1, s); });
  return check_launch(g, "pairs_update");
}

static __global__ void k_zero_pairs(int S, float *w, uint8_t *in_p) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < S) {
    w[t] = 0.f;
    in_p[t] = 0;
  }
}

tdp_status tdp_pairs_reset(tdp_graph g, hipStream_t s) {
  GUARD(g);
  const int S = g->topo.S;
  hipLaunchKernelGGL(k_zero_pairs, dim3((S + 255) / 256), dim3(256), 0, s, S, g->pw, g->pin_p);
  pairs_rebuild(g, s);
  return check_launch(g, "pairs_reset");
}

tdp_status tdp_pairs_export(tdp_graph g, float *h_w, uint8_t *h_in_p, hipStream_t s) {
  GUARD(g);
  const int S = g->topo.S, P = g->topo.P;
  std::vector<float> w(S);
  std::vector<uint8_t> m(S);
  if (hipStreamSynchronize(s) != hipSuccess ||
      hipMemcpy(w.data(), g->pw, sizeof(float) * S, hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(m.data(), g->pin_p, S, hipMemcpyDeviceToHost) != hipSuccess)
    return fail(g, TDP_E_DEVICE, "pair copy failed");
  if (h_w) std::fill(h_w, h_w + P, 0.f);
  if (h_in_p) std::fill(h_in_p, h_in_p + P, (uint8_t)0);
  for (int t = 0; t < S; ++t) {
    const int p = g->h_snk_ext[t];
    if (h_w) h_w[p] = w[t];
    if (h_in_p) h_in_p[p] = m[t];
  }
  return TDP_OK;
}

tdp_status tdp_pairs_import(tdp_graph g, const float *h_w, const uint8_t *h_in_p, hipStream_t s) {
  GUARD(g);
  if (!h_w || !h_in_p) return fail(g, TDP_E_INVALID, "NULL arrays");
  const int S = g->topo.S;
  std::vector<float> w(S);
  std::vector<uint8_t> m(S);
  for (int t = 0; t < S; ++t) {
    const int p = g->h_snk_ext[t];
    if (!std::isfinite(h_w[p])) return fail(g, TDP_E_INVALID, "weight not finite");
    w[t] = h_in_p[p] ? h_w[p] : 0.f;
    m[t] = h_in_p[p] ? 1 : 0;
  }
  if (hipStreamSynchronize(s) != hipSuccess ||
      hipMemcpy(g->pw, w.data(), sizeof(float) * S, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(g->pin_p, m.data(), S, hipMemcpyHostToDevice) != hipSuccess)
    return fail(g, TDP_E_DEVICE, "pair upload failed");
  pairs_rebuild(g, s);
  return check_launch(g, "pairs_import");
}

tdp_status tdp_pairs_count(tdp_graph g, int32_t *num_pairs, hipStream_t s) {
  GUARD(g);
  int32_t n = 0;
  if (hipStreamSynchronize(s) != hipSuccess || hipMemcpy(&n, g->d_npairs, 4, hipMemcpyDeviceToHost) != hipSuccess)
    return fail(g, TDP_E_DEVICE, "count copy failed");
  if (num_pairs) *num_pairs = n;
  return TDP_OK;
}

tdp_status tdp_p2p_loss_fwd(tdp_graph g, const float *x, const float *y, double *loss, hipStream_t s) {
  GUARD(g);
  if (!x || !y || !loss) return fail(g, TDP_E_INVALID, "NULL argument");
  dispatch(g, [&](auto z) { p2p_fwd_impl<decltype(z)>(g, 0, x, y, loss, s); });
  return check_launch(g, "p2p_loss_fwd");
}

tdp_status tdp_pair_loss_fwd(tdp_graph g, int32_t kind, const float *x, const float *y, double *loss,
                             hipStream_t s) {
  GUARD(g);
  if (kind < 0 || kind > 2) return fail(g, TDP_E_INVALID, "kind must be 0, 1 or 2");
  if (!x || !y || !loss) return fail(g, TDP_E_INVALID, "NULL argument");
  dispatch(g, [&](auto z) { p2p_fwd_impl<decltype(z)>(g, kind, x, y, loss, s); });
  return check_launch(g, "pair_loss_fwd");
}

tdp_status tdp_p2p_loss_bwd(tdp_graph g, const float *x, const float *y, const double *gout, float *gx, float *gy,
                            hipStream_t s) {
  GUARD(g);
  if (!x || !y || !gx || !gy) return fail(g, TDP_E_INVALID, "NULL argument");
  dispatch(g, [&](auto z) { p2p_bwd_impl<decltype(z)>(g, 0, x, y, gout ? gout : g->consts, gx, gy, s); });
  return check_launch(g, "p2p_loss_bwd");
}

tdp_status tdp_pair_loss_bwd(tdp_graph g, int32_t kind, const float *x, const float *y, const double *gout,
                             float *gx, float *gy, hipStream_t s) {
  GUARD(g);
  if (kind < 0 || kind > 2) return fail(g, TDP_E_INVALID, "kind must be 0, 1 or 2");
  if (!x || !y || !gx || !gy) return fail(g, TDP_E_INVALID, "NULL argument");
  dispatch(g, [&](auto z) { p2p_bwd_impl<decltype(z)>(g, kind, x, y, gout ? gout : g->consts, gx, gy, s); });
  return check_launch(g, "pair_loss_bwd");
}

tdp_status tdp_stns_fwd(tdp_graph g, const float *x, const float *y, float gamma, double *val, hipStream_t s) {
  GUARD(g);
  if (!g->updated) return fail(g, TDP_E_STATE, "no timing update yet");
  if (!x || !y || !val) return fail(g, TDP_E_INVALID, "NULL argument");
  if (!(gamma > 0) || !std::isfinite(gamma)) return fail(g, TDP_E_INVALID, "gamma must be > 0");
  dispatch(g, [&](auto z) { stns_fwd_impl<decltype(z)>(g, x, y, gamma, val, s); });
  tdp_status st = check_launch(g, "stns_fwd");
  if (st == TDP_OK) g->stns_ready = true;
  return st;
}

tdp_status tdp_stns_bwd(tdp_graph g, const double *gout, float *gx, float *gy, hipStream_t s) {
  GUARD(g);
  if (!g->stns_ready) return fail(g, TDP_E_STATE, "no smoothed-TNS forward yet");
  if (!gx || !gy) return fail(g, TDP_E_INVALID, "NULL argument");
  dispatch(g, [&](auto z) { stns_bwd_impl<decltype(z)>(g, gout ? gout : g->consts, gx, gy, s); });
  return check_launch(g, "stns_bwd");
}

tdp_status tdp_wa_fwd_bwd(tdp_graph g, const float *x, const float *y, float gamma, double *wl, float *gx, float *gy,
                          hipStream_t s) {
  GUARD(g);
  if (!x || !y || !wl || !gx || !gy) return fail(g, TDP_E_INVALID, "NULL argument");
  if (!(gamma > 0) || !std::isfinite(gamma)) return fail(g, TDP_E_INVALID, "gamma must be > 0");
  wa_impl(g, x, y, gamma, wl, gx, gy, s);
  return check_launch(g, "wa_fwd_bwd");
}

tdp_status tdp_wa_fwd_bwd_at_update(tdp_graph g, float gamma, double *wl, float *gx, float *gy, hipStream_t s) {
  GUARD(g);
  if (!g->updated) return fail(g, TDP_E_STATE, "no timing update yet");
  if (!wl || !gx || !gy) return fail(g, TDP_E_INVALID, "NULL argument");
  if (!(gamma > 0) || !std::isfinite(gamma)) return fail(g, TDP_E_INVALID, "gamma must be > 0");
  wa_impl(g, nullptr, nullptr, gamma, wl, gx, gy, s);
  return check_launch(g, "wa_fwd_bwd_at_update");
}

tdp_status tdp_sta_update_early(tdp_graph g, float hold_ps, hipStream_t s) {
  GUARD(g);
  if (!g->updated) return fail(g, TDP_E_STATE, "no timing update yet");
  if (!std::isfinite(hold_ps)) return fail(g, TDP_E_INVALID, "hold time not finite");
  if (!g->ea_as) {
    const Topo &T = g->topo;
    const size_t es = g->esz;
    const bool ok = dalloc(g, g->ea_as, std::max(T.M, 1), 2 * es) && dalloc(g, g->ea_at, std::max(T.S, 1), es) &&
                    dalloc(g, g->ea_darc, std::max(T.A, 1), es) && dalloc(g, g->ea_part, 3 * early_parts()) &&
                    dalloc(g, g->ea_summary, 3);
    if (!ok) return fail(g, TDP_E_NOMEM, "early analysis: device allocation failed");
  }
  g->ea_hold = hold_ps;
  dispatch(g, [&](auto z) { early_impl<decltype(z)>(g, hold_ps, s); });
  g->ea_ready = true;
  return check_launch(g, "sta_update_early");
}

tdp_status tdp_sta_early_summary(tdp_graph g, double *whs, double *ths, int32_t *n_fail, hipStream_t s) {
  GUARD(g);
  if (!g->ea_ready) return fail(g, TDP_E_STATE, "no early update yet");
  double h[3];
  if (hipStreamSynchronize(s) != hipSuccess ||
      hipMemcpy(h, g->ea_summary, sizeof(h), hipMemcpyDeviceToHost) != hipSuccess)
    return fail(g, TDP_E_DEVICE, "early summary copy failed");
  if (whs) *whs = h[0];
  if (ths) *ths = h[1];
  if (n_fail) *n_fail = (int32_t)h[2];
  return TDP_OK;
}

tdp_status tdp_sta_early_export(tdp_graph g, double *d_at, double *d_slew, double *d_darc, double *d_hold_slack,
                                hipStream_t s) {
  GUARD(g);
  if (!g->ea_ready) return fail(g, TDP_E_STATE, "no early update yet");
  dispatch(g, [&](auto z) { early_export_impl<decltype(z)>(g, d_at, d_slew, d_darc, d_hold_slack, s); });
  return check_launch(g, "sta_early_export");
}

tdp_status tdp_density_setup(tdp_graph g, const tdp_density_grid *grid, const float *h_area) {
  GUARD(g);
  if (!grid || !h_area) return fail(g, TDP_E_INVALID, "NULL argument");
  const tdp_density_grid &q = *grid;
  if (q.bins_x < 1 || q.bins_y < 1 || q.bins_x > 4096 || q.bins_y > 4096)
    return fail(g, TDP_E_INVALID, "density grid: bins_x and bins_y must be in 1..4096");
  if (q.radius < 0 || q.radius > 8) return fail(g, TDP_E_INVALID, "density grid: radius must be in 0..8");
  if (!(q.bin_w > 0) || !(q.bin_h > 0) || !std::isfinite(q.bin_w) || !std::isfinite(q.bin_h) ||
      !std::isfinite(q.x0) || !std::isfinite(q.y0))
    return fail(g, TDP_E_INVALID, "density grid: origin and bin sizes must be finite, sizes > 0");
  if (!(q.target > 0) || !std::isfinite(q.target)) return fail(g, TDP_E_INVALID, "density grid: target must be > 0");
  const int N = g->topo.N;
  double total = 0.0;
  for (int c = 0; c < N; ++c) {
    if (!std::isfinite(h_area[c]) || h_area[c] < 0) return fail(g, TDP_E_INVALID, "cell areas must be finite, >= 0");
    total += h_area[c];
  }
  const int bins = q.bins_x * q.bins_y, K = 2 * q.radius + 1;
  bool ok = true;
  if (!g->dn_area) {
    const int scan_cap = std::max(std::max(N, 1), sort_hist_size(std::max(N, 1)));
    ok = dalloc(g, g->dn_area, N) && dalloc(g, g->dn_k0, N) && dalloc(g, g->dn_k1, N) && dalloc(g, g->dn_v0, N) &&
         dalloc(g, g->dn_v1, N) && dalloc(g, g->dn_hist, sort_hist_size(std::max(N, 1))) &&
         dalloc(g, g->dn_scan, scan_tmp_size(scan_cap)) && dalloc(g, g->dn_part, 2 * density_parts()) &&
         dalloc(g, g->nest_part, 2 * density_parts()) && dalloc(g, g->nest_alpha, 1) && dalloc(g, g->dn_nheavy, 1);
  }
  if (ok && bins > g->dn_alloc_bins) {  // a smaller grid reuses the buffers
    ok = dalloc(g, g->dn_start, (size_t)bins + 1) && dalloc(g, g->dn_map, bins) && dalloc(g, g->dn_heavy, bins);
    if (ok) g->dn_alloc_bins = bins;
  }
  if (ok && q.radius > g->dn_alloc_R) {
    ok = dalloc(g, g->dn_w, (size_t)2 * K * std::max(N, 1));
    if (ok) g->dn_alloc_R = q.radius;
  }
  if (!ok) return fail(g, TDP_E_NOMEM, "density: device allocation failed");
  if (N > 0 && hipMemcpy(g->dn_area, h_area, sizeof(float) * N, hipMemcpyHostToDevice) != hipSuccess)
    return fail(g, TDP_E_DEVICE, "density: area upload failed");
  int bits = 0;
  while (bits < 62 && ((int64_t)1 << bits) < (int64_t)bins) ++bits;
  g->dn_key_bits = std::max(8, (bits + 7) / 8 * 8);
  g->dn = DensityGrid{q.x0, q.y0, q.bin_w, q.bin_h, q.target, q.bins_x, q.bins_y, q.radius};
  g->dn_total_area = total;
  g->dn_ready = true;
  return TDP_OK;
}

tdp_status tdp_density_fwd_bwd(tdp_graph g, const float *x, const float *y, float scale, double *d_value,
                               double *d_overflow, float *d_gx, float *d_gy, float *d_map, hipStream_t s) {
  GUARD(g);
  if (!g->dn_ready) return fail(g, TDP_E_STATE, "density: no tdp_density_setup yet");
  if (!x || !y) return fail(g, TDP_E_INVALID, "NULL positions");
  if ((d_gx == nullptr) != (d_gy == nullptr)) return fail(g, TDP_E_INVALID, "d_gx and d_gy: both or neither");
  if (!std::isfinite(scale)) return fail(g, TDP_E_INVALID, "scale not finite");
  density_impl(g, x, y, scale, d_value, d_overflow, d_gx, d_gy, d_map, s);
  return check_launch(g, "density_fwd_bwd");
}

tdp_status tdp_nesterov_step(tdp_graph g, const float *d_gx, const float *d_gy, const float *d_pdiv, float *d_vx,
                             float *d_vy, float *d_ux, float *d_uy, float *d_vpx, float *d_vpy, float *d_gpx,
                             float *d_gpy, double coef, double alpha0, int32_t first, float xlo, float xhi, float ylo,
                             float yhi, double *d_alpha, hipStream_t s) {
  GUARD(g);
  if (!g->dn_ready) return fail(g, TDP_E_STATE, "nesterov: no tdp_density_setup yet");
  if (!d_gx || !d_gy || !d_pdiv || !d_vx || !d_vy || !d_ux || !d_uy || !d_vpx || !d_vpy || !d_gpx || !d_gpy)
    return fail(g, TDP_E_INVALID, "NULL argument");
  if (!std::isfinite(coef) || !(alpha0 > 0) || !std::isfinite(alpha0))
    return fail(g, TDP_E_INVALID, "coef must be finite and alpha0 > 0");
  if (!(xlo <= xhi) || !(ylo <= yhi) || !std::isfinite(xlo) || !std::isfinite(xhi) || !std::isfinite(ylo) ||
      !std::isfinite(yhi))
    return fail(g, TDP_E_INVALID, "bounds must be finite with lo <= hi");
  nesterov_impl(g, d_gx, d_gy, d_pdiv, d_vx, d_vy, d_ux, d_uy, d_vpx, d_vpy, d_gpx, d_gpy, coef, alpha0, first ? 1 : 0,
                xlo, xhi, ylo, yhi, d_alpha, s);
  return check_launch(g, "nesterov_step");
}

tdp_status tdp_abs_sum(tdp_graph g, const float *d_a, const float *d_b, double *d_out, hipStream_t s) {
  GUARD(g);
  if (!g->dn_ready) return fail(g, TDP_E_STATE, "abs_sum: no tdp_density_setup yet");
  if (!d_a || !d_b || !d_out) return fail(g, TDP_E_INVALID, "NULL argument");
  abs_sum_impl(g, d_a, d_b, d_out, s);
  return check_launch(g, "abs_sum");
}

tdp_status tdp_profile_enable(tdp_graph g, int32_t stage_mask) {
  GUARD(g);
  g->prof.mask = stage_mask;
  g->prof.on = stage_mask != 0;
  return TDP_OK;
}

tdp_status tdp_profile_read(tdp_graph g, double *ms, int32_t *calls) {
  GUARD(g);
  for (auto &m : g->prof.marks) {
    float e = 0.f;
    if (hipEventSynchronize(m.b) == hipSuccess && hipEventElapsedTime(&e, m.a, m.b) == hipSuccess) {
      g->prof.ms[m.stage] += e;
      g->prof.calls[m.stage] += 1;
    }
    g->prof.pool.push_back(m.a);
    g->prof.pool.push_back(m.b);
  }
  g->prof.marks.clear();
  for (int i = 0; i < TDP_NUM_STAGES; ++i) {
    if (ms) ms[i] = g->prof.ms[i];
    if (calls) calls[i] = g->prof.calls[i];
    g->prof.ms[i] = 0;
    g->prof.calls[i] = 0;
  }
  return TDP_OK;
}

tdp_status tdp_set_tuning(tdp_graph g, int32_t flow_waves, int32_t flow_per_cu, int32_t spin_log2,
                          int32_t sweep_mode) {
  GUARD(g);
  if (flow_waves != 0 && flow_waves != 1 && flow_waves != 2 && flow_waves != 4)
    return fail(g, TDP_E_INVALID, "flow_waves must be 0, 1, 2 or 4");
  if (flow_per_cu < 0 || flow_per_cu > 4) return fail(g, TDP_E_INVALID, "flow_per_cu must be 0..4");
  if (spin_log2 != 0 && (spin_log2 < 1 || spin_log2 > 30)) return fail(g, TDP_E_INVALID, "spin_log2 out of range");
  if (sweep_mode < 0 || sweep_mode > 3) return fail(g, TDP_E_INVALID, "sweep_mode must be 0..3");
  if (sweep_mode >= 1 && !g->flow_ok)
    return fail(g, TDP_E_UNSUPPORTED, "dataflow sweeps need single precision and nets of at most 63 sinks");
  if (flow_waves) g->flow_waves = flow_waves;
  if (flow_per_cu) g->flow_per_cu = flow_per_cu;
  if (spin_log2) g->spin_limit = 1 << spin_log2;
  g->sweep_mode = sweep_mode;
  return TDP_OK;
}

// autotuner choices of this process, by graph signature: device, precision,
// sizes, depth, instances, deviation-list width and the extraction asked for
struct TuneChoice {
  int mode, waves, per_cu, us;
};
static std::mutex g_tune_mu;
static std::map<std::vector<int64_t>, TuneChoice> g_tune_cache;

tdp_status tdp_autotune(tdp_graph g, const float *x, const float *y, int32_t n, int32_t k, int32_t K, int32_t reps,
                        int32_t *choice, hipStream_t s) {
  GUARD(g);
  if (!x || !y) return fail(g, TDP_E_INVALID, "positions are NULL");
  if (reps < 1 || reps > 1000) return fail(g, TDP_E_INVALID, "reps must be 1..1000");
  if (k < 0 || k > g->max_k) return fail(g, TDP_E_CAPACITY, "k outside 0..max_k");
  const Topo &T = g->topo;
  const std::vector<int64_t> sig = {g->device, (int64_t)g->prec, T.N, T.P, T.M, T.S, T.A, T.E, T.D, T.n_comb,
                                    T.num_inst, g->side_k, g->flow_ok ? 1 : 0, g->num_cu, n, k, K};
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune_cache.find(sig);
    if (it != g_tune_cache.end()) {  // tuned before: no trials
      g->sweep_mode = it->second.mode;
      g->flow_waves = it->second.waves;
      g->flow_per_cu = it->second.per_cu;
      if (choice) {
        choice[0] = it->second.mode;
        choice[1] = it->second.waves;
        choice[2] = it->second.per_cu;
        choice[3] = it->second.us;
      }
      tdp_status r = tdp_sta_update(g, x, y, s);
      if (r == TDP_OK && k > 0) r = tdp_extract_paths(g, n, k, K, std::numeric_limits<float>::infinity(), s, nullptr);
      return r;
    }
  }
  struct Cand {
    int mode, waves, per_cu;
  };
  std::vector<Cand> cands = {{0, g->flow_waves, g->flow_per_cu}};
  if (g->flow_ok)
    for (int w : {1, 2, 4})
      for (int pc : {1, 2, 4})
        for (int m : {1, 3}) cands.push_back({m, w, pc});
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) hipEventDestroy(e0);
    return fail(g, TDP_E_DEVICE, "event creation failed");
  }
  const bool prof = g->prof.on;
  g->prof.on = false;
  const float no_limit = std::numeric_limits<float>::infinity();
  Cand best_c = {g->sweep_mode, g->flow_waves, g->flow_per_cu};
  float best = std::numeric_limits<float>::infinity();
  tdp_status st = TDP_OK;
  auto run = [&]() {
    tdp_status r = tdp_sta_update(g, x, y, s);
    if (r == TDP_OK && k > 0) r = tdp_extract_paths(g, n, k, K, no_limit, s, nullptr);
    return r;
  };
  for (const Cand &c : cands) {
    g->sweep_mode = c.mode;
    g->flow_waves = c.waves;
    g->flow_per_cu = c.per_cu;
    st = run();  // warm-up
    if (st == TDP_OK && hipEventRecord(e0, s) != hipSuccess) st = fail(g, TDP_E_DEVICE, "event record failed");
    for (int r = 0; r < reps && st == TDP_OK; ++r) st = run();
    if (st == TDP_OK && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess))
      st = fail(g, TDP_E_DEVICE, "event wait failed");
    if (st != TDP_OK) break;
    int32_t err = 0;
    if (hipMemcpy(&err, g->d_err, 4, hipMemcpyDeviceToHost) != hipSuccess) {
      st = fail(g, TDP_E_DEVICE, "status copy failed");
      break;
    }
    float ms = 0.f;
    hipEventElapsedTime(&ms, e0, e1);
    ms /= (float)reps;
    if (err == 0 && ms < best) {  // a sweep whose waits gave up does not qualify
      best = ms;
      best_c = c;
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  g->sweep_mode = best_c.mode;
  g->flow_waves = best_c.waves;
  g->flow_per_cu = best_c.per_cu;
  g->prof.on = prof;
  if (st != TDP_OK) return st;
  // leave the results of the chosen configuration behind
  st = run();
  if (st != TDP_OK) return st;
  const int us = std::isfinite(best) ? (int32_t)std::lround(best * 1000.0f) : -1;
  if (choice) {
    choice[0] = best_c.mode;
    choice[1] = best_c.waves;
    choice[2] = best_c.per_cu;
    choice[3] = us;
  }
  if (std::isfinite(best)) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache[sig] = TuneChoice{best_c.mode, best_c.waves, best_c.per_cu, us};
  }
  return TDP_OK;
}

tdp_status tdp_graph_info(tdp_graph g, int32_t *info8) {
  GUARD(g);
  if (!info8) return fail(g, TDP_E_INVALID, "NULL argument");
  const Topo &T = g->topo;
  const int32_t v[8] = {T.N, T.P, T.M, T.D, T.E, T.n_start, T.n_comb, T.S};
  std::memcpy(info8, v, sizeof v);
  return TDP_OK;
}

const char *tdp_status_str(tdp_status st) {
  switch (st) {
    case TDP_OK: return "ok";
    case TDP_E_INVALID: return "invalid argument";
    case TDP_E_CYCLE: return "combinational cycle";
    case TDP_E_NOMEM: return "out of memory";
    case TDP_E_DEVICE: return "device error";
    case TDP_E_CAPACITY: return "capacity exceeded";
    case TDP_E_STATE: return "call out of order";
    case TDP_E_UNSUPPORTED: return "unsupported";
  }
  return "unknown status";
}

const char *tdp_last_error(tdp_graph g) { return g ? g->last_error.c_str() : g_loose_error.c_str(); }

}  // extern "C"
