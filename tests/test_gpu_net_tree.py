"""Parity of the HIP path with the FP64 oracle under the spanning-tree net
model (net_model 2: Elmore delays on each net's rectilinear minimum spanning
tree, PERI-degraded sink transitions): timing, paths and report_timing(K),
the smoothed TNS and its gradient, FP64, every sweep form bitwise, nets wider
than a 64-lane chunk, and incremental updates bitwise equal to full ones
(rise / fall and early timing under this model are in their own test files).
Both sides decide the trees' topologies in single precision; a different
topology would show as net delays far outside the tolerance."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import ref  # noqa: E402
from paper_2503_11674_amd import netgen  # noqa: E402
from tests.bruteforce import Graph  # noqa: E402
from tests.comparator import arc_tables, compare_global, compare_paths, timing_close  # noqa: E402
from tests.conftest import with_clock  # noqa: E402
from tests.test_gpu_net_model import _check_sta, _fanout_design, _xy  # noqa: E402

pytestmark = pytest.mark.gpu


def _tdp():
    from paper_2503_11674_amd import tdp
    return tdp


def _tree(library):
    return dict(library, net_model=2)


_CASES = {}


def _case(name, library):
    if name in _CASES:
        return _CASES[name]
    print(f"[tree case] building {name}", flush=True)
    lib = _tree(library)
    nl = with_clock(netgen.make_netlist(netgen.CONFIGS[name]), lib)
    st = ref.sta(nl, lib)
    E = len(ref.endpoint_pins(nl))
    K = netgen.CONFIGS[name].top_k_paths
    k = max(1, K // max(1, st["n_fail"]))
    g = _tdp().TimingGraph(nl, lib, max_paths=max(K, E), max_k=max(k, 4))
    x, y = _xy(nl)
    g.sta_update(x, y)
    out = {kk: v.cpu().numpy() for kk, v in g.export().items()}
    _CASES[name] = dict(nl=nl, lib=lib, st=st, g=g, x=x, y=y, gpu=out, K=K, k=k)
    return _CASES[name]


@pytest.mark.parametrize("name", ["C1", "C2"])
def test_tree_sta_parity(name, library):
    c = _case(name, library)
    nl, st, o = c["nl"], c["st"], c["gpu"]
    _check_sta(o, st, nl)
    wns, tns, nf = c["g"].summary()
    assert nf == st["n_fail"] == len(ref.endpoint_pins(nl)) // 20
    assert abs(wns - st["wns"]) <= 1e-4 * abs(st["wns"])
    assert abs(tns - st["tns"]) <= 1e-4 * abs(st["tns"])
    # the model is in effect: the trees are not stars, and the loads are the
    # trees' (not longer than the stars')
    par = ref.rc_tree(nl)
    g = Graph(nl)
    sinks = np.nonzero(par >= 0)[0]
    assert np.mean(par[sinks] != np.array([g.driver[t] for t in sinks])) > 0.1
    st1 = ref.sta(nl, dict(library, net_model=1))
    drv = np.asarray(sorted({g.driver[t] for t in sinks}))
    assert np.all(o["load"][drv] <= st1["load"][drv] * (1 + 1e-5))


@pytest.mark.parametrize("name", ["C1", "C2"])
def test_tree_paths_and_report_timing(name, library):
    c = _case(name, library)
    nl, lib, st, g, k, K = c["nl"], c["lib"], c["st"], c["g"], c["k"], c["K"]
    print(f"[tree] {name} extract n_fail k={k} K={K}", flush=True)
    g.extract_paths(n=-1, k=k, K=K)
    gp = g.paths()
    rp = ref.extract(nl, lib, st, n=-1, k=k, K=K)
    assert gp["num_paths"] == rp["num_paths"]
    res = compare_paths(gp, rp, st, Graph(nl), k)
    assert res["missing"] == 0 and res["extra"] == 0
    assert res["pinned_ok"] == res["pinned"] and res["unpinned_ok"] == res["unpinned"]
    print(f"[tree] {name} report_timing K={K}", flush=True)
    g.report_timing(K)
    gp = g.paths()
    rp = ref.report_timing(nl, lib, st, K)
    r = compare_global(gp, rp, st, arc_tables(nl), fp32=True)
    assert r["count_ok"] and r["valid"] == r["num"] and r["slack_ok"] == r["num"]
    assert r["distinct"] and r["sorted"] and r["ranks_ok"] and r["order_stat_ok"]
    assert r["pinned_found"] == r["pinned"]


@pytest.mark.parametrize("precision", ["f32", "f64"])
def test_tree_smoothed_tns_parity(precision, library):
    tdp = _tdp()
    c = _case("C1", library)
    nl, lib, st = c["nl"], c["lib"], c["st"]
    g = tdp.TimingGraph(nl, lib, precision=precision, max_paths=200, max_k=4)
    g.sta_update(c["x"], c["y"])
    v_ref, gx_ref, gy_ref, ax, ay = ref.stns(nl, lib, st, gamma=10.0, with_abs=True)
    xr = c["x"].clone().requires_grad_(True)
    yr = c["y"].clone().requires_grad_(True)
    v = tdp.SmoothTNS.apply(xr, yr, g, 10.0)
    v.backward()
    tol = 1e-4 if precision == "f32" else 1e-10
    assert abs(float(v) - v_ref) <= tol * abs(v_ref)
    # per cell, against the magnitudes of the terms summed into it
    for got, want, mag in ((xr.grad, gx_ref, ax), (yr.grad, gy_ref, ay)):
        got = got.cpu().numpy().astype(np.float64)
        lim = (1e-4 if precision == "f32" else 1e-6) * np.maximum(mag, 1e-3 * np.abs(want).max())
        assert np.all(np.abs(got - want) <= lim), np.max(np.abs(got - want) / lim)
    assert np.abs(gx_ref).max() > 0
    g.close()


def test_tree_f64_and_sweeps_agree(library):
    """FP64 graphs meet the oracle to 1e-12; the dataflow sweeps compute
    bitwise what the per-level sweeps compute under this model too."""
    tdp = _tdp()
    c = _case("C2", library)
    nl, lib, st = c["nl"], c["lib"], c["st"]
    g = tdp.TimingGraph(nl, lib, precision="f64", max_paths=200, max_k=4)
    g.sta_update(c["x"], c["y"])
    o = {kk: v.cpu().numpy() for kk, v in g.export().items()}
    for key in ("at", "rat", "slew", "dnet", "load"):
        inf_ok, bad, worst = timing_close(o[key], st[key], rtol=1e-12)
        assert inf_ok and bad == 0, (key, bad, worst)
    g.close()
    outs = []
    for mode in (0, 1, 3):
        g = tdp.TimingGraph(nl, lib, max_paths=c["K"], max_k=c["k"])
        g.set_tuning(sweep_mode=mode)
        g.sta_update(c["x"], c["y"])
        outs.append({kk: v.cpu().numpy() for kk, v in g.export().items()})
        g.close()
    for o in outs[1:]:
        for key in outs[0]:
            assert np.array_equal(outs[0][key], o[key]), key


def test_tree_nets_wider_than_a_chunk(library):
    tdp = _tdp()
    lib = _tree(library)
    nl = _fanout_design()
    fo = np.diff(nl["net_ptr"]) - 1
    assert (fo > 63).sum() == 2
    nl = with_clock(nl, lib, 0.3)
    st = ref.sta(nl, lib)
    E = len(ref.endpoint_pins(nl))
    g = tdp.TimingGraph(nl, lib, max_paths=4 * E, max_k=4)
    g.sta_update(*_xy(nl))
    o = {kk: v.cpu().numpy() for kk, v in g.export().items()}
    _check_sta(o, st, nl)
    g.extract_paths(n=-1, k=4)
    gp = g.paths()
    rp = ref.extract(nl, lib, st, n=-1, k=4)
    assert gp["num_paths"] == rp["num_paths"]
    res = compare_paths(gp, rp, st, Graph(nl), 4)
    assert res["missing"] == 0 and res["extra"] == 0
    # the smoothed TNS through the wide nets' trees (one thread per net) and
    # the others' (a lane per pin)
    v_ref, gx_ref, gy_ref, ax, ay = ref.stns(nl, lib, st, gamma=10.0, with_abs=True)
    x, y = _xy(nl)
    xr, yr = x.clone().requires_grad_(True), y.clone().requires_grad_(True)
    v = tdp.SmoothTNS.apply(xr, yr, g, 10.0)
    v.backward()
    assert abs(float(v) - v_ref) <= 1e-4 * abs(v_ref)
    for got, want, mag in ((xr.grad, gx_ref, ax), (yr.grad, gy_ref, ay)):
        got = got.cpu().numpy().astype(np.float64)
        lim = 1e-4 * np.maximum(mag, 1e-3 * np.abs(want).max())
        assert np.all(np.abs(got - want) <= lim), np.max(np.abs(got - want) / lim)
    assert np.abs(gx_ref[:160]).max() > 0  # the wide nets' cells carry gradient
    g.close()


def test_tree_incremental_equals_full(library):
    from tests.test_gpu_incremental import _same, _state
    tdp = _tdp()
    lib = _tree(library)
    cfg = netgen.CONFIGS["C2"]
    nl = with_clock(netgen.make_netlist(cfg), lib)
    E = int(np.count_nonzero(nl["cell_is_ff"]))
    k = 4
    K = min(cfg.top_k_paths, E * k)
    dev = torch.device("cuda", 0)
    x = torch.tensor(nl["x"], device=dev)
    y = torch.tensor(nl["y"], device=dev)
    gi = tdp.TimingGraph(nl, lib, max_paths=K, max_k=k)
    gf = tdp.TimingGraph(nl, lib, max_paths=K, max_k=k)
    gi.sta_update(x, y)
    rng = np.random.default_rng(11)
    movable = np.nonzero(np.asarray(nl["cell_fixed"]) == 0)[0]
    for m in (1, 200, 5000):
        cells = rng.choice(movable, m, replace=False).astype(np.int32)
        xn, yn = x.clone(), y.clone()
        ct = torch.tensor(cells, device=dev, dtype=torch.long)
        xn[ct] += torch.tensor(rng.normal(0, 20.0, m).astype(np.float32), device=dev)
        yn[ct] += torch.tensor(rng.normal(0, 20.0, m).astype(np.float32), device=dev)
        gi.sta_update_arrivals_incremental(xn, yn, torch.tensor(cells, device=dev, dtype=torch.int32))
        gf.sta_update(xn, yn)
        _same(_state(gi, k, K), _state(gf, k, K))
        print(f"[tree] incremental, {m} cells moved: equal to a full update", flush=True)
        x, y = xn, yn
    # and both still meet the oracle at the final positions
    st = ref.sta(nl, lib, x.cpu().numpy(), y.cpu().numpy())
    o = {kk: v.cpu().numpy() for kk, v in gi.export().items()}
    for key in ("dnet", "load"):
        inf_ok, bad, worst = timing_close(o[key], st[key], rtol=2e-5)
        assert inf_ok and bad == 0, (key, bad, worst)
    gi.close()
    gf.close()


@pytest.mark.parametrize("wide", [False, True])
@pytest.mark.parametrize("precision", ["f32", "f64"])
def test_tree_hand_net_is_exact(wide, precision):
    """Dyadic positions and library: every wire length, capacitance and
    Elmore delay is a short binary fraction, so both sides compute them
    exactly.  A port drives sinks at (8, 0), (16, 0), (16, 8), (24, 0): the
    tree is port -> (8, 0) -> (16, 0) -> {(16, 8), (24, 0)}, the last two tied
    at distance 8 (the first listed joins first).  C_below = 14, 10, 2, 2 fF,
    delays 7.5, 13, 14.5, 14.5 ps, load 16 fF.  The wide form adds 64 sinks
    on the line y = 0 (one thread per net instead of a chunk's lanes)."""
    from tests import handnets
    tdp = _tdp()
    lib = dict(handnets.dyadic_library(), net_model=2)
    sx = [8.0, 16.0, 16.0, 24.0] + ([32.0 + 8 * i for i in range(64)] if wide else [])
    sy = [0.0, 0.0, 8.0, 0.0] + ([0.0] * 64 if wide else [])
    n = len(sx)
    cells = [(0, 1)] * n + [(netgen.FF_TYPE, 1)] * n
    port = 4 * n
    nets = [(port, [2 * i for i in range(n)])] + [(2 * i + 1, [2 * n + 2 * i]) for i in range(n)] + \
        [(2 * n + 2 * i + 1, []) for i in range(n)]
    x = sx + [v + 4.0 for v in sx]
    y = sy + sy
    nl, _ = handnets.build(cells, 1, nets, x, y, port_xy=[(0.0, 0.0)], clock_period=400.0)
    st = ref.sta(nl, lib)
    par = ref.rc_tree(nl)
    assert [int(par[2 * i]) for i in range(4)] == [port, 0, 2, 2]
    if not wide:
        assert st["dnet"][[0, 2, 4, 6]].tolist() == [7.5, 13.0, 14.5, 14.5]
        assert st["load"][port] == 16.0
    g = tdp.TimingGraph(nl, lib, precision=precision, max_paths=4 * n, max_k=2)
    g.sta_update(*_xy(nl))
    o = {kk: v.cpu().numpy() for kk, v in g.export().items()}
    assert np.array_equal(o["dnet"], st["dnet"]) and np.array_equal(o["load"], st["load"])
    inf_ok, bad, worst = timing_close(o["at"], st["at"], rtol=1e-6 if precision == "f32" else 1e-12)
    assert inf_ok and bad == 0, (bad, worst)
    g.close()


def test_tree_full_size_2m_cells(library):
    """The 2M-cell workload under the spanning-tree model: every pin's timing
    against the oracle in the library's default sweep form and in the
    per-level one, the summary, and the extraction's path count."""
    from tests.test_gpu_fullsize import _timing_checks
    tdp = _tdp()
    lib = _tree(library)
    cfg = netgen.CONFIGS["C5"]
    print("[tree] generating the 2M-cell workload", flush=True)
    nl = with_clock(netgen.make_netlist(cfg), lib)
    st = ref.sta(nl, lib)
    K = cfg.top_k_paths
    k = max(1, K // st["n_fail"])
    print(f"[tree] oracle timing done: n_fail={st['n_fail']} k={k}", flush=True)
    g = tdp.TimingGraph(nl, lib, max_paths=K, max_k=k)
    x, y = _xy(nl)
    for mode in (None, 0):
        if mode is not None:
            g.set_tuning(sweep_mode=mode)
        g.sta_update(x, y)
        o = {kk: v.cpu().numpy() for kk, v in g.export().items()}
        _timing_checks(nl, st, o)
        wns, tns, nf = g.summary()
        assert nf == st["n_fail"]
        assert abs(wns - st["wns"]) <= 1e-4 * abs(st["wns"]) and abs(tns - st["tns"]) <= 1e-4 * abs(st["tns"])
        g.extract_paths(n=-1, k=k, K=K)
        assert g.paths_count()[0] == min(K, st["n_fail"] * k)
        print(f"[tree] sweep form {mode}: timing and summary match the oracle", flush=True)
    g.close()
