"""Parity at the full workload sizes, in the launch configuration the
benchmark times (single precision, the sweep form its autotuner picks, the
benchmark's step: timing update, extraction, pair update, WA and p2p
forward/backward on three streams).

* 2M cells (depth 100, 12 % flip-flops, K = 100k paths): every pin's timing,
  every path, the pair set and its weights, both losses and their gradients,
  against the FP64 oracle on the same input (the oracle runs the whole size
  in seconds); every other sweep form (per level, both sweeps on resident
  grids, required times only on a resident grid) bitwise against that; then
  report_timing(K) on the same graph against the oracle's.
* 1M cells (depth 80, K = 50k, exponential pair weights): the two
  differentiable objectives through torch.autograd against the oracle's
  gradients and against central finite differences (h = 1e-3 um) of the
  double-precision graph on 1,000 random cells.
"""
import time

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import ref  # noqa: E402
from paper_2503_11674_amd import netgen  # noqa: E402
from tests.comparator import arc_tables, compare_global, compare_paths_fast, pair_sinks, timing_close  # noqa: E402
from tests.conftest import with_clock  # noqa: E402

pytestmark = pytest.mark.gpu


def _tdp():
    from paper_2503_11674_amd import tdp
    return tdp


def _dev():
    return torch.device("cuda", 0)


def _log(msg):
    print(f"[{time.strftime('%H:%M:%S')}] {msg}", flush=True)


def _xy(nl):
    return (torch.tensor(np.asarray(nl["x"], np.float32), device=_dev()),
            torch.tensor(np.asarray(nl["y"], np.float32), device=_dev()))


def _timing_checks(nl, st, o):
    inf_ok, bad, worst = timing_close(o["at"], st["at"])
    assert inf_ok and bad == 0, ("at", bad, worst)
    scale = np.maximum(np.abs(np.where(np.isfinite(st["at"]), st["at"], 0)),
                       np.abs(np.where(np.isfinite(st["rat"]), st["rat"], 0)))
    scale = np.maximum(scale, abs(float(nl["clock_period"])))
    for key in ("rat", "slack"):
        inf_ok, bad, worst = timing_close(o[key], st[key], scale=scale)
        _log(f"{key}: worst relative error {worst:.3g}")
        assert inf_ok and bad == 0, (key, bad, worst)
    for key in ("dnet", "load", "darc", "slew"):
        inf_ok, bad, worst = timing_close(o[key], st[key], rtol=2e-5)
        assert inf_ok and bad == 0, (key, bad, worst)


def _pinned_pair_checks(nl, gp, rp, pinned_ref, w_gpu, in_gpu, w_ref, in_ref, rtol=1e-4):
    """Pairs on pinned violating paths are in both sets; weights agree for
    pairs that occur on pinned paths only."""
    viol = rp["path_slack"] < 0
    pinned_sinks = np.unique(pair_sinks(rp, pinned_ref & viol))
    assert pinned_sinks.shape[0] > 0
    assert in_gpu[pinned_sinks].all() and in_ref[pinned_sinks].all()
    # occurrences on unpinned paths (either side) make a weight order-dependent
    # in single precision: leave those pairs out
    key_r = set(zip(rp["path_ep"][pinned_ref].tolist(), rp["path_rank"][pinned_ref].tolist()))
    g_pinned = np.array([(int(e), int(r)) in key_r for e, r in zip(gp["path_ep"], gp["path_rank"])], bool)
    loose = np.union1d(pair_sinks(rp, ~pinned_ref), pair_sinks(gp, ~g_pinned))
    cmp = np.setdiff1d(pinned_sinks, loose)
    assert cmp.shape[0] > 0.5 * pinned_sinks.shape[0]
    np.testing.assert_allclose(w_gpu[cmp], w_ref[cmp], rtol=rtol)
    return cmp


def _p2p_abs_scale(nl, sinks, w):
    """Per cell: sum of |dPP/dx| terms that reach it (vectorised)."""
    driver_of = arc_tables(nl)[0]
    pc = np.asarray(nl["pin_cell"])
    px = np.where(pc >= 0, nl["x"][np.maximum(pc, 0)], 0) + nl["pin_off_x"]
    py = np.where(pc >= 0, nl["y"][np.maximum(pc, 0)], 0) + nl["pin_off_y"]
    s = driver_of[sinks]
    m = 2 * np.asarray(w, np.float64) * (np.abs(px[s] - px[sinks]) + np.abs(py[s] - py[sinks]))
    scale = np.zeros(int(nl["num_cells"]))
    for q in (s, sinks):
        ok = pc[q] >= 0
        np.add.at(scale, pc[q][ok], m[ok])
    return scale


def test_full_size_step_2m_cells(library):
    tdp = _tdp()
    cfg = netgen.CONFIGS["C5"]
    _log("generating the 2M-cell workload")
    nl = with_clock(netgen.make_netlist(cfg), library)
    st = ref.sta(nl, library)
    K = cfg.top_k_paths
    k = max(1, K // st["n_fail"])
    _log(f"oracle timing done: n_fail={st['n_fail']} k={k}")
    g = tdp.TimingGraph(nl, library, max_paths=K, max_k=k)
    x, y = _xy(nl)
    gx = torch.zeros_like(x)
    gy = torch.zeros_like(y)
    wl = torch.zeros((), dtype=torch.float64, device=_dev())
    pp = torch.zeros((), dtype=torch.float64, device=_dev())
    one = torch.ones((), dtype=torch.float64, device=_dev())

    # the benchmark's step, with its side streams (beta = 1 here), in the
    # sweep form the benchmark's autotuner picks
    import bench
    step = bench.build_step(g, x, y, k, K, gx, gy, wl, pp, one, overlap=True)
    tune = g.autotune(x, y, n=-1, k=k, K=K, reps=2)
    _log(f"autotuner: {tune}")

    def run():
        g.pairs_reset()
        step()
        torch.cuda.synchronize()
        o = {kk: v.cpu().numpy() for kk, v in g.export().items()}
        w, inp = g.pairs_export()
        return o, g.paths(), (w, inp), gx.cpu().numpy(), gy.cpu().numpy(), float(wl), float(pp), g.summary()

    step()
    res0 = run()
    _log("GPU step done")
    # every sweep form computes the same step bitwise
    for mode in (0, 1, 3):
        if mode == tune["sweep_mode"]:
            continue
        g.set_tuning(sweep_mode=mode)
        r = run()
        for key in res0[0]:
            assert np.array_equal(res0[0][key], r[0][key]), (mode, key)
        for key in ("path_ptr", "path_pins", "path_ep", "path_rank", "path_slack"):
            assert np.array_equal(res0[1][key], r[1][key]), (mode, key)
        assert np.array_equal(res0[2][0], r[2][0]) and np.array_equal(res0[2][1], r[2][1]), mode
        assert np.array_equal(res0[3], r[3]) and np.array_equal(res0[4], r[4]), mode
        assert res0[5:] == r[5:], mode
        _log(f"sweep mode {mode}: bitwise equal to mode {tune['sweep_mode']}")
    g.set_tuning(sweep_mode=tune["sweep_mode"])
    o = res0[0]
    _timing_checks(nl, st, o)
    wns, tns, nf = g.summary()
    assert nf == st["n_fail"]
    assert abs(wns - st["wns"]) <= 1e-4 * abs(st["wns"]) and abs(tns - st["tns"]) <= 1e-4 * abs(st["tns"])
    # paths
    gp = g.paths()
    rp = ref.extract(nl, library, st, n=-1, k=k, K=K)
    _log(f"oracle extraction done: {rp['num_paths']} paths")
    assert gp["num_paths"] == rp["num_paths"] and rp["num_paths"] > 0.9 * min(K, st["n_fail"] * k)
    c, pinned = compare_paths_fast(gp, rp, st, arc_tables(nl), k)
    _log(f"paths: {c}")
    assert c["missing"] == 0 and c["extra"] == 0 and c["gpu_valid"] == gp["num_paths"]
    assert c["pinned_ok"] == c["pinned"] and c["unpinned_ok"] == c["unpinned"]
    assert c["pinned"] > 0.9 * rp["num_paths"]
    # at any size: the sorted path slacks agree element by element
    tol = 1e-4 * max(abs(float(nl["clock_period"])), abs(st["wns"]))
    assert np.all(np.abs(np.sort(gp["path_slack"]) - np.sort(rp["path_slack"])) <= tol)
    # pairs (one Eq. 9 round)
    w_gpu, in_gpu = res0[2]
    ps = ref.PairState(nl["num_pins"])
    ref.pairs_update(ps, rp, st["wns"], rule=0)
    _pinned_pair_checks(nl, gp, rp, pinned, w_gpu, in_gpu.astype(bool), ps.w, ps.in_p.astype(bool))
    # losses on the GPU's own pair set
    sinks = np.nonzero(in_gpu)[0]
    l_ref, px_ref, py_ref = ref.p2p(nl, sinks, w_gpu[sinks].astype(np.float64))
    assert abs(res0[6] - l_ref) <= 1e-4 * abs(l_ref)
    v_wa, wx_ref, wy_ref, ax, ay = ref.wa(nl, 5.0, with_abs=True)
    assert abs(res0[5] - v_wa) <= 1e-4 * abs(v_wa)
    scale = _p2p_abs_scale(nl, sinks, w_gpu[sinks])
    ex = np.abs(res0[3] - (wx_ref + px_ref))
    ey = np.abs(res0[4] - (wy_ref + py_ref))
    _log(f"gradient: worst scaled error {(ex / np.maximum(ax + scale, 1e-12)).max():.3g}")
    assert np.all(ex <= 1e-4 * (ax + scale) + 1e-6)
    assert np.all(ey <= 1e-4 * (ay + scale) + 1e-6)

    # report_timing(K) on the same graph: the K worst paths of the design
    g.report_timing(K)
    gk = g.paths()
    _log(f"GPU report_timing({K}): {gk['num_paths']} paths")
    rk = ref.report_timing(nl, library, st, K)
    _log(f"oracle report_timing done: {rk['num_paths']} paths on {len(set(rk['path_ep'].tolist()))} endpoints")
    res = compare_global(gk, rk, st, arc_tables(nl))
    _log(f"report_timing: {res}")
    assert res["count_ok"] and res["num"] == K
    assert res["valid"] == K and res["slack_ok"] == K and res["distinct"] and res["sorted"] and res["ranks_ok"]
    assert res["order_stat_ok"] and res["pinned_found"] == res["pinned"] and res["pinned"] > 0


# ------------------------------------------------------------------ 1M cells
_U64 = 2.0 ** -53
# smoothed TNS, single precision against the oracle: per cell, relative to
# the summed magnitudes of its net-arc gradient terms.  Each term carries an
# adjoint made of softmax weights exp((a - A) / gamma); with arrivals below
# 2^17 ps held to about two ulps (2^-7 ps) each, the argument is off by up to
# 4 * 2^-7 / 10 = 3.1e-3, which is what one weight's relative error can be
STNS_RTOL = 4e-3


def _central_fd(fwd, x, y, cells, axis, h=1e-3):
    """Central differences of a scalar GPU objective at the given cells: the
    perturbed coordinates are the single-precision values nearest to x +- h,
    and the step is their exact difference."""
    base = (x if axis == 0 else y)
    v0 = base[cells].double().cpu().numpy()
    plus = torch.tensor((v0 + h).astype(np.float32), device=_dev())
    minus = torch.tensor((v0 - h).astype(np.float32), device=_dev())
    out = torch.zeros((len(cells), 2), dtype=torch.float64, device=_dev())
    work = base.clone()
    xs = (work, y) if axis == 0 else (x, work)
    for i, c in enumerate(cells.tolist()):
        work[c] = plus[i]
        fwd(*xs, out[i, 0])
        work[c] = minus[i]
        fwd(*xs, out[i, 1])
        work[c] = base[c]
    step = (plus.double() - minus.double()).cpu().numpy()
    vals = out.cpu().numpy()
    return (vals[:, 0] - vals[:, 1]) / step, np.abs(vals).max(), step


def test_objectives_1m_cells_against_oracle_and_finite_differences(library):
    tdp = _tdp()
    cfg = netgen.CONFIGS["C3"]
    _log("generating the 1M-cell workload")
    nl = with_clock(netgen.make_netlist(cfg), library)
    st = ref.sta(nl, library)
    K = cfg.top_k_paths
    k = max(1, K // st["n_fail"])
    g = tdp.TimingGraph(nl, library, max_paths=K, max_k=k)
    x, y = _xy(nl)
    g.sta_update(x, y)
    g.extract_paths(n=-1, k=k, K=K)
    g.pairs_update(rule=1)
    w_gpu, in_gpu = g.pairs_export()
    in_gpu = in_gpu.astype(bool)
    _log(f"GPU: {g.pairs_count()} pairs")
    # exponential weights against the oracle on pinned paths
    gp = g.paths()
    rp = ref.extract(nl, library, st, n=-1, k=k, K=K)
    c, pinned = compare_paths_fast(gp, rp, st, arc_tables(nl), k)
    _log(f"paths: {c}")
    assert c["missing"] == 0 and c["extra"] == 0
    assert c["pinned_ok"] == c["pinned"] and c["unpinned_ok"] == c["unpinned"]
    ps = ref.PairState(nl["num_pins"])
    ref.pairs_update(ps, rp, st["wns"], rule=1)
    _pinned_pair_checks(nl, gp, rp, pinned, w_gpu, in_gpu, ps.w, ps.in_p.astype(bool))
    # autograd, single precision
    xr = x.clone().requires_grad_(True)
    yr = y.clone().requires_grad_(True)
    pp = tdp.P2PLoss.apply(xr, yr, g)
    stns = tdp.SmoothTNS.apply(xr, yr, g, 10.0)
    (pp + stns).backward()
    gx32 = xr.grad.cpu().numpy().astype(np.float64)
    gy32 = yr.grad.cpu().numpy().astype(np.float64)
    # oracle values and gradients (p2p on the GPU's own pair set)
    sinks = np.nonzero(in_gpu)[0]
    l_ref, px_ref, py_ref = ref.p2p(nl, sinks, w_gpu[sinks].astype(np.float64))
    v_ref, sx_ref, sy_ref, sax, say = ref.stns(nl, library, st, gamma=10.0, with_abs=True)
    assert abs(float(pp) - l_ref) <= 1e-4 * abs(l_ref)
    assert abs(float(stns) - v_ref) <= 1e-4 * abs(v_ref)
    # single-precision gradient of the sum against the oracle, per cell: p2p
    # at 1e-4 of the magnitudes of its terms as at 2M cells; the smoothed TNS
    # at STNS_RTOL of the magnitudes of its net-arc terms (each term carries
    # an adjoint built from log-sum-exp weights exp((a - A) / gamma) of
    # single-precision arrival times)
    p_scale = _p2p_abs_scale(nl, sinks, w_gpu[sinks])
    ex = np.abs(gx32 - (px_ref + sx_ref))
    ey = np.abs(gy32 - (py_ref + sy_ref))
    # single precision cannot carry an adjoint below its resolution of the
    # largest entry (a far-from-critical endpoint's sigmoid underflows): an
    # absolute floor of 2^-23 of the largest smoothed-TNS entry
    s_floor = 2.0 ** -23 * max(np.abs(sx_ref).max(), np.abs(sy_ref).max())
    big_x, big_y = sax > 64 * s_floor, say > 64 * s_floor
    rx = (ex - 1e-4 * p_scale)[big_x] / sax[big_x]
    ry = (ey - 1e-4 * p_scale)[big_y] / say[big_y]
    _log(f"autograd vs oracle: {int(big_x.sum())} / {int(big_y.sum())} cells above the floor, worst smoothed-TNS "
         f"excess per cell scale {max(rx.max(), ry.max()):.3g} (p99 {np.percentile(np.r_[rx, ry], 99):.3g})")
    assert np.all(ex <= 1e-4 * p_scale + STNS_RTOL * sax + s_floor)
    assert np.all(ey <= 1e-4 * p_scale + STNS_RTOL * say + s_floor)
    # central differences of the double-precision graph (same pair set and
    # weights) on 1,000 random movable cells
    g64 = tdp.TimingGraph(nl, library, precision="f64", max_paths=K, max_k=k)
    g64.sta_update(x, y)
    g64.pairs_import(w_gpu, in_gpu.astype(np.uint8))
    rng = np.random.default_rng(2503)
    movable = np.nonzero(np.asarray(nl["cell_fixed"]) == 0)[0]
    cells = torch.tensor(np.sort(rng.choice(movable, 1000, replace=False)), device=_dev())
    cn = cells.cpu().numpy()
    for axis, gref, g32 in ((0, (px_ref, sx_ref), gx32), (1, (py_ref, sy_ref), gy32)):
        fd_p, vmax_p, _ = _central_fd(lambda a, b, o: g64.p2p_loss_fwd(a, b, out=o), x, y, cells, axis)
        fd_s, vmax_s, _ = _central_fd(lambda a, b, o: g64.stns_fwd(a, b, 10.0, out=o), x, y, cells, axis)
        # rounding of two double-precision sums over the whole design,
        # divided by the step (the objectives are smooth at this scale:
        # cells with a pin within 2h of alignment with a net neighbour sit on
        # an |dx| kink and are left out)
        atol_p = 64 * _U64 * vmax_p / 1e-3
        atol_s = 64 * _U64 * vmax_s / 1e-3
        keep = ~_near_kink(nl, cn, axis, 2e-3)
        _log(f"axis {axis}: {int(keep.sum())} cells; p2p fd atol {atol_p:.3g}, stns fd atol {atol_s:.3g}")
        e_p = np.abs(fd_p - gref[0][cn])[keep]
        e_s = np.abs(fd_s - gref[1][cn])[keep]
        _log(f"fd vs oracle: p2p worst {e_p.max():.3g}, stns worst {e_s.max():.3g}")
        assert np.all(e_p <= atol_p + 1e-6 * np.abs(gref[0][cn])[keep])
        assert np.all(e_s <= atol_s + 1e-6 * np.abs(gref[1][cn])[keep])
        # and the single-precision autograd gradient against the differences
        s_abs = (sax if axis == 0 else say)[cn][keep]
        e32 = np.abs(g32[cn] - (fd_p + fd_s))[keep]
        assert np.all(e32 <= 1e-4 * p_scale[cn][keep] + STNS_RTOL * s_abs + s_floor + atol_p + atol_s)
        assert np.count_nonzero(np.abs(fd_p[keep]) > 0) > 10 and np.count_nonzero(np.abs(fd_s[keep]) > 0) > 10


def _near_kink(nl, cells, axis, eps):
    """Cells with a pin whose coordinate on the axis is within eps of the
    other end of one of its net arcs."""
    driver_of = arc_tables(nl)[0]
    pc = np.asarray(nl["pin_cell"])
    coord = np.asarray(nl["x"] if axis == 0 else nl["y"], np.float64)
    off = np.asarray(nl["pin_off_x"] if axis == 0 else nl["pin_off_y"], np.float64)
    pos = np.where(pc >= 0, coord[np.maximum(pc, 0)], 0) + off
    sinks = np.nonzero(driver_of >= 0)[0]
    close = np.abs(pos[sinks] - pos[driver_of[sinks]]) < eps
    bad = np.zeros(int(nl["num_cells"]), bool)
    for q in (sinks[close], driver_of[sinks[close]]):
        ok = pc[q] >= 0
        bad[pc[q][ok]] = True
    return bad[cells]


# ------------------------------------------------------------- batched form
def test_batched_workload_matches_instances_and_oracle(library):
    """The 40-instance batch (32 uneven netlists, 8 jittered snapshots) as one
    union graph: every instance's timing and paths equal its own graph's
    bitwise, and two instances (the largest netlist and one snapshot) match
    the oracle."""
    tdp = _tdp()
    _log("generating the batched workload")
    nls = netgen.batch_workload()
    k, K = 10, 5000
    singles = []
    for nl in nls:
        x, y = _xy(nl)
        g = tdp.TimingGraph(nl, library, max_paths=K, max_k=k)
        # a snapshot keeps the clock period of the unperturbed placement
        g.sta_update(*_xy({"x": nl.get("x_base", nl["x"]), "y": nl.get("y_base", nl["y"])}))
        at = g.export()["at"].cpu().numpy()
        T = netgen.clock_period_for_fail_fraction(at[ref.endpoint_pins(nl)], 0.05)
        g.set_clock(T)
        nl["clock_period"] = np.float32(T)
        g.sta_update(x, y)
        g.extract_paths(n=-1, k=k, K=K)
        singles.append((g, x, y))
    gb = tdp.TimingGraph(nls, library, max_paths=K, max_k=k)
    pb, _ = gb.batch_offsets()
    xb, yb = torch.cat([s[1] for s in singles]), torch.cat([s[2] for s in singles])
    # the union in the configuration the benchmark's autotuner picks for it
    _log(f"union autotuner: {gb.autotune(xb, yb, n=-1, k=k, K=K, reps=2)}")
    gb.sta_update(xb, yb)
    gb.extract_paths(n=-1, k=k, K=K)
    ob = gb.export()
    P = gb.paths()
    wb, tb, nb = gb.batch_summary()
    _log(f"union: {gb.num_cells} cells, {P['num_paths']} paths")
    for i, (g, _, _) in enumerate(singles):
        o = g.export()
        for key in ("at", "rat", "slack"):
            assert torch.equal(o[key], ob[key][pb[i]:pb[i + 1]]), (i, key)
        w, t, n = g.summary()
        assert (w, n) == (wb[i], nb[i])
        p = g.paths()
        idx = np.nonzero((P["path_ep"] >= pb[i]) & (P["path_ep"] < pb[i + 1]))[0]
        assert len(idx) == p["num_paths"] and 0 < p["num_paths"] <= min(K, n * k), i
        assert np.array_equal(P["path_slack"][idx], p["path_slack"])
        mine = np.concatenate([P["path_pins"][P["path_ptr"][j]:P["path_ptr"][j + 1]] for j in idx]) - pb[i]
        assert np.array_equal(mine, p["path_pins"]), i
    largest = int(np.argmax([nl["num_cells"] for nl in nls[:32]]))
    for i in (largest, 32):
        nl = nls[i]
        st = ref.sta(nl, library)
        o = {kk: v.cpu().numpy() for kk, v in singles[i][0].export().items()}
        _timing_checks(nl, st, o)
        rp = ref.extract(nl, library, st, n=-1, k=k, K=K)
        c, _ = compare_paths_fast(singles[i][0].paths(), rp, st, arc_tables(nl), k)
        _log(f"instance {i}: {c}")
        assert c["missing"] == 0 and c["extra"] == 0
        assert c["pinned_ok"] == c["pinned"] and c["unpinned_ok"] == c["unpinned"]
    for g, _, _ in singles:
        g.close()
