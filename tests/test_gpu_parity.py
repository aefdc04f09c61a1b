"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Sizes: hand chains (exact binary fractions, bit-equal in FP32), small random
DAGs, C1 (2,000 cells) and C2 (200,000 cells, several hundred tiles per
level and ragged tails).  Tolerances: see tests/comparator.py.
"""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import ref  # noqa: E402
from paper_2503_11674_amd import netgen  # noqa: E402
from tests import handnets  # noqa: E402
from tests.bruteforce import Graph  # noqa: E402
from tests.comparator import arc_tables, compare_global, compare_paths, pairs_of, timing_close  # noqa: E402
from tests.conftest import with_clock  # noqa: E402

pytestmark = pytest.mark.gpu


def _tdp():
    from paper_2503_11674_amd import tdp
    return tdp


def _dev():
    return torch.device("cuda", 0)


def _xy(nl, x=None, y=None):
    x = nl["x"] if x is None else x
    y = nl["y"] if y is None else y
    return (torch.tensor(np.asarray(x, np.float32), device=_dev()),
            torch.tensor(np.asarray(y, np.float32), device=_dev()))


_CASES = {}


def case(name, library):
    """netlist + oracle STA + GPU graph after one update (cached per name)."""
    if name in _CASES:
        return _CASES[name]
    print(f"[case] building {name}", flush=True)
    if name in netgen.CONFIGS:
        nl = with_clock(netgen.make_netlist(netgen.CONFIGS[name]), library)
    else:
        raise KeyError(name)
    st = ref.sta(nl, library)
    E = len(ref.endpoint_pins(nl))
    K = netgen.CONFIGS[name].top_k_paths
    k = max(1, K // max(1, st["n_fail"]))
    g = _tdp().TimingGraph(nl, library, max_paths=max(K, E), max_k=max(k, 4))
    x, y = _xy(nl)
    g.sta_update(x, y)
    out = {k2: v.cpu().numpy() for k2, v in g.export().items()}
    _CASES[name] = dict(nl=nl, st=st, g=g, x=x, y=y, gpu=out, K=K, k=k)
    return _CASES[name]


# ---------------------------------------------------------------- exact
def test_hand_chain_bit_exact():
    tdp = _tdp()
    nl, _ = handnets.chain_netlist()
    lib = handnets.dyadic_library()
    g = tdp.TimingGraph(nl, lib, max_paths=8, max_k=3)
    x, y = _xy(nl)
    g.sta_update(x, y)
    o = {k: v.cpu().numpy() for k, v in g.export().items()}
    exp_at = {6: 0.0, 0: 9.0, 1: 15.625, 2: 24.625, 3: 31.25, 4: 40.25, 5: 25.0625}
    exp_rat = {4: 32.0, 3: 23.0, 2: 16.375, 1: 7.375, 0: 0.75, 6: -8.25, 5: math.inf}
    for p, v in exp_at.items():
        assert o["at"][p] == v, p
    for p, v in exp_rat.items():
        assert o["rat"][p] == v, p
    assert g.summary() == (-8.25, -8.25, 1)
    g.extract_paths(n=-1, k=3)
    p = g.paths()
    assert p["num_paths"] == 1 and p["path_pins"].tolist() == [6, 0, 1, 2, 3, 4]
    assert p["path_slack"][0] == -8.25


def test_hand_diamond_paths_exact():
    tdp = _tdp()
    nl, _ = handnets.diamond_netlist()
    lib = handnets.dyadic_library()
    st = ref.sta(nl, lib)
    g = tdp.TimingGraph(nl, lib, max_paths=8, max_k=2)
    x, y = _xy(nl)
    g.sta_update(x, y)
    o = {k: v.cpu().numpy() for k, v in g.export().items()}
    for key in ("at", "rat", "slack", "dnet", "load", "darc"):
        assert np.array_equal(o[key], st[key]), key
    assert o["crit"].tolist() == st["crit"].tolist()
    g.extract_paths(n=-1, k=2)
    p = g.paths()
    assert p["path_pins"].tolist() == [7, 3, 4, 5, 7, 0, 1, 2, 4, 5]
    assert p["path_ptr"].tolist() == [0, 4, 10]
    assert p["path_slack"].tolist() == [-3.625, 7.75]
    assert p["path_rank"].tolist() == [0, 1]


def test_tie_takes_lowest_arc():
    tdp = _tdp()
    cells = [(1, 2), (7, 1)]
    nets = [(5, [0]), (6, [1]), (2, [3]), (4, [])]
    nl, _ = handnets.build(cells, 2, nets, [24.0, 48.0], [0.0, 0.0], port_xy=[(0.0, 0.0), (48.0, 0.0)],
                           clock_period=10.0)
    g = tdp.TimingGraph(nl, handnets.dyadic_library(), max_paths=8, max_k=2)
    g.sta_update(*_xy(nl))
    assert g.export()["crit"].cpu().tolist() == [0, -1]
    g.extract_paths(n=-1, k=2)
    p = g.paths()
    assert p["path_pins"].tolist() == [5, 0, 2, 3, 6, 1, 2, 3]


# ------------------------------------------------------------ timing parity
@pytest.mark.parametrize("name", ["C1", "C2"])
def test_sta_parity(name, library):
    c = case(name, library)
    st, o = c["st"], c["gpu"]
    inf_ok, bad, worst = timing_close(o["at"], st["at"])
    assert inf_ok and bad == 0, ("at", bad, worst)
    # required time and slack are the clock period minus a downstream delay:
    # their scale is the largest of |AT|, |RAT| and the period at the pin
    scale = np.maximum(np.abs(np.where(np.isfinite(st["at"]), st["at"], 0)),
                       np.abs(np.where(np.isfinite(st["rat"]), st["rat"], 0)))
    scale = np.maximum(scale, abs(float(c["nl"]["clock_period"])))
    for key in ("rat", "slack"):
        inf_ok, bad, worst = timing_close(o[key], st[key], scale=scale)
        print(key, "worst relative error", worst)
        assert inf_ok and bad == 0, (key, bad, worst)
    for key in ("dnet", "load", "darc", "slew"):
        inf_ok, bad, worst = timing_close(o[key], st[key], rtol=2e-5)
        assert inf_ok and bad == 0, (key, bad, worst)
    wns, tns, nf = c["g"].summary()
    assert nf == st["n_fail"] == len(ref.endpoint_pins(c["nl"])) // 20
    assert abs(wns - st["wns"]) <= 1e-4 * abs(st["wns"])
    assert abs(tns - st["tns"]) <= 1e-4 * abs(st["tns"])
    # critical inputs agree wherever the best two arcs are apart by more than rounding
    nl = c["nl"]
    comb = np.nonzero(nl["cell_is_ff"] == 0)[0]
    ptr, pins = nl["cell_in_ptr"], nl["cell_in_pins"]
    mism = 0
    for cell in comb:
        ins = pins[ptr[cell]:ptr[cell + 1]]
        a = st["at"][ins] + st["darc"][ins]
        if len(ins) > 1:
            srt = np.sort(a)
            if srt[-1] - srt[-2] <= 1e-4 * max(1.0, abs(srt[-1])):
                continue
        mism += int(o["crit"][cell] != st["crit"][cell])
    assert mism == 0


@pytest.mark.parametrize("name", ["C1", "C2"])
def test_paths_parity(name, library):
    c = case(name, library)
    nl, st, g, k, K = c["nl"], c["st"], c["g"], c["k"], c["K"]
    g.extract_paths(n=-1, k=k, K=K)
    gp = g.paths()
    rp = ref.extract(nl, library, st, n=-1, k=k, K=K)
    assert gp["num_paths"] == rp["num_paths"]
    assert np.all(np.diff(gp["path_slack"]) >= 0)
    res = compare_paths(gp, rp, st, Graph(nl), k)
    print({kk: v for kk, v in res.items() if kk != "pinned_keys"})
    assert res["missing"] == 0 and res["extra"] == 0
    assert res["pinned_ok"] == res["pinned"] and res["pinned"] > 0.9 * rp["num_paths"]
    assert res["unpinned_ok"] == res["unpinned"]
    # (n, 1) covers n distinct endpoints
    g.extract_paths(n=-1, k=1)
    p1 = g.paths()
    assert p1["num_paths"] == st["n_fail"] and len(set(p1["path_ep"].tolist())) == st["n_fail"]
    # explicit n with a slack limit
    g.extract_paths(n=7, k=3, slack_limit=0.0)
    p2 = g.paths()
    r2 = ref.extract(nl, library, st, n=7, k=3, slack_limit=0.0)
    assert p2["num_paths"] == r2["num_paths"]
    assert np.all(p2["path_slack"] < 0)


def test_paths_on_small_random_dags(library):
    tdp = _tdp()
    for seed in range(6):
        cfg = netgen.NetlistConfig("tiny", 60, ff_frac=0.25, depth=6, fanin_lo=1, fanin_hi=4, fanout_cap=8,
                                   die=300.0, seed=100 + seed)
        nl = with_clock(netgen.make_netlist(cfg), library, 0.3)
        st = ref.sta(nl, library)
        E = len(ref.endpoint_pins(nl))
        g = tdp.TimingGraph(nl, library, max_paths=E * 8, max_k=8)
        g.sta_update(*_xy(nl))
        g.extract_paths(n=E, k=8)
        gp = g.paths()
        rp = ref.extract(nl, library, st, n=E, k=8)
        res = compare_paths(gp, rp, st, Graph(nl), 8)
        assert gp["num_paths"] == rp["num_paths"], seed
        assert res["missing"] == 0 and res["extra"] == 0, seed
        assert res["pinned_ok"] == res["pinned"] and res["unpinned_ok"] == res["unpinned"], (seed, res)


# ------------------------------------------------------ report_timing(K)
def _check_global(gp, rp, st, nl, fp32=True):
    res = compare_global(gp, rp, st, arc_tables(nl), fp32=fp32)
    print(res, flush=True)
    assert res["count_ok"], (gp["num_paths"], rp["num_paths"])
    assert res["valid"] == res["num"] and res["slack_ok"] == res["num"]
    assert res["distinct"] and res["sorted"] and res["ranks_ok"]
    assert res["order_stat_ok"]
    assert res["pinned_found"] == res["pinned"]
    return res


@pytest.mark.parametrize("name", ["C1", "C2"])
def test_report_timing_parity(name, library):
    c = case(name, library)
    nl, st, g, K = c["nl"], c["st"], c["g"], c["K"]
    for KK in (1, 37, K):
        print(f"[report_timing] {name} K={KK}", flush=True)
        g.report_timing(KK)
        gp = g.paths()
        rp = ref.report_timing(nl, library, st, KK)
        res = _check_global(gp, rp, st, nl)
        assert res["pinned"] > 0
    # fewer distinct endpoints than report_timing_endpoint(n_fail, 1) covers
    # whenever the worst endpoints hold several of the K worst paths
    g.report_timing(K)
    n_ep = len(set(g.paths()["path_ep"].tolist()))
    assert n_ep <= K
    # a slack limit keeps only the violating part
    g.report_timing(K, slack_limit=0.0)
    gp = g.paths()
    rp = ref.report_timing(nl, library, st, K, slack_limit=0.0)
    _check_global(gp, rp, st, nl)
    assert np.all(gp["path_slack"] < 0)


@pytest.mark.parametrize("max_k", [1, 2])
def test_report_timing_short_lists_and_refinement(library, max_k):
    """max_k = 1 keeps no deviation lists (every expansion walks the chain)
    and gives a loose first bound, so the node store overflows and the bound
    is refined; max_k = 2 cuts the lists short almost everywhere."""
    tdp = _tdp()
    nl = with_clock(netgen.make_netlist(netgen.CONFIGS["C1"]), library)
    st = ref.sta(nl, library)
    E = len(ref.endpoint_pins(nl))
    g = tdp.TimingGraph(nl, library, max_paths=E, max_k=max_k)
    g.sta_update(*_xy(nl))
    for KK in (E // 2, E):
        print(f"[report_timing] max_k={max_k} K={KK}", flush=True)
        g.report_timing(KK)
        gp = g.paths()
        rp = ref.report_timing(nl, library, st, KK)
        _check_global(gp, rp, st, nl)


def test_report_timing_small_random_dags(library):
    tdp = _tdp()
    for seed in range(6):
        cfg = netgen.NetlistConfig("tiny", 60, ff_frac=0.25, depth=6, fanin_lo=1, fanin_hi=4, fanout_cap=8,
                                   die=300.0, seed=100 + seed)
        nl = with_clock(netgen.make_netlist(cfg), library, 0.3)
        st = ref.sta(nl, library)
        E = len(ref.endpoint_pins(nl))
        g = tdp.TimingGraph(nl, library, max_paths=E * 8, max_k=4)
        g.sta_update(*_xy(nl))
        for KK in (5, E * 8):
            g.report_timing(KK)
            gp = g.paths()
            rp = ref.report_timing(nl, library, st, KK)
            _check_global(gp, rp, st, nl)
        g.close()


def test_report_timing_f64_and_determinism(library):
    tdp = _tdp()
    nl = with_clock(netgen.make_netlist(netgen.CONFIGS["C1"]), library)
    st = ref.sta(nl, library)
    g = tdp.TimingGraph(nl, library, precision="f64", max_paths=200, max_k=10)
    g.sta_update(*_xy(nl))
    g.report_timing(100)
    gp = g.paths()
    rp = ref.report_timing(nl, library, st, 100)
    _check_global(gp, rp, st, nl, fp32=False)
    assert np.allclose(gp["path_slack"], rp["path_slack"], rtol=0, atol=1e-9)
    g.close()
    outs = []
    for _ in range(2):
        g = tdp.TimingGraph(nl, library, max_paths=200, max_k=10)
        g.sta_update(*_xy(nl))
        g.report_timing(200)
        p = g.paths()
        outs.append((p["path_pins"], p["path_slack"], p["path_rank"]))
        g.close()
    for a, b in zip(*outs):
        assert np.array_equal(a, b)


def test_report_timing_batch_matches_single_instances(library):
    tdp = _tdp()
    nls = []
    for i, n in enumerate((3000, 800, 5000)):
        cfg = netgen.NetlistConfig(f"b{i}", n, depth=10 + 5 * i, fanout_cap=16, die=600.0, seed=40 + i)
        nls.append(with_clock(netgen.make_netlist(cfg), library))
    gb = tdp.TimingGraph(nls, library, max_paths=2000, max_k=4)
    pb, cb = gb.batch_offsets()
    xb = torch.tensor(np.concatenate([nl["x"] for nl in nls]), device=_dev())
    yb = torch.tensor(np.concatenate([nl["y"] for nl in nls]), device=_dev())
    gb.sta_update(xb, yb)
    gb.report_timing(300)
    P = gb.paths()
    for i, nl in enumerate(nls):
        g = tdp.TimingGraph(nl, library, max_paths=2000, max_k=4)
        g.sta_update(*_xy(nl))
        g.report_timing(300)
        p = g.paths()
        sel = (P["path_ep"] >= pb[i]) & (P["path_ep"] < pb[i + 1])
        idx = np.nonzero(sel)[0]
        assert len(idx) == p["num_paths"] == 300
        assert np.array_equal(P["path_slack"][idx], p["path_slack"])
        assert np.array_equal(P["path_rank"][idx], p["path_rank"])
        mine = np.concatenate([P["path_pins"][P["path_ptr"][j]:P["path_ptr"][j + 1]] for j in idx]) - pb[i]
        assert np.array_equal(mine, p["path_pins"])
        g.close()


def test_pairs_from_report_timing(library):
    """Eq. 9 weights over the paths of report_timing(K) match the oracle's
    rule applied to the same paths."""
    c = case("C1", library)
    nl, st, g, K = c["nl"], c["st"], c["g"], c["K"]
    g.pairs_reset()
    g.report_timing(K)
    gp = g.paths()
    g.pairs_update(rule=0, w0=10.0, w1=0.2)
    w_gpu, in_gpu = g.pairs_export()
    ps = ref.PairState(nl["num_pins"])
    ref.pairs_update(ps, gp, st["wns"], rule=0)
    assert np.array_equal(in_gpu.astype(bool), ps.in_p.astype(bool))
    sel = np.nonzero(ps.in_p)[0]
    assert sel.shape[0] > 0
    assert np.allclose(w_gpu[sel], ps.w[sel], rtol=1e-4)
    g.pairs_reset()


# ------------------------------------------------------------- pairs, loss
@pytest.mark.parametrize("name", ["C1", "C2"])
def test_pairs_and_p2p(name, library):
    tdp = _tdp()
    c = case(name, library)
    nl, st, g, k, K = c["nl"], c["st"], c["g"], c["k"], c["K"]
    g.pairs_reset()
    g.extract_paths(n=-1, k=k, K=K)
    gp = g.paths()
    rp = ref.extract(nl, library, st, n=-1, k=k, K=K)
    res = compare_paths(gp, rp, st, Graph(nl), k)
    g.pairs_update(rule=0, w0=10.0, w1=0.2)
    w_gpu, in_gpu = g.pairs_export()
    ps = ref.PairState(nl["num_pins"])
    ref.pairs_update(ps, rp, st["wns"], rule=0)
    # pairs of pinned violating paths are identical as a set (Eq. 9 counts
    # violating paths only)
    viol = {(int(rp["path_ep"][i]), int(rp["path_rank"][i])) for i in range(rp["num_paths"])
            if rp["path_slack"][i] < 0}
    pinned_viol = res["pinned_keys"] & viol
    pinned_pairs = pairs_of(rp, pinned_viol)
    assert pinned_pairs <= set(np.nonzero(in_gpu)[0].tolist())
    assert set(np.nonzero(ps.in_p)[0].tolist()) >= pinned_pairs
    # weights: pairs whose every occurrence is on a pinned path
    all_unpinned = (pairs_of(rp) - pairs_of(rp, res["pinned_keys"])) | (pairs_of(gp) - pairs_of(gp, res["pinned_keys"]))
    cmp = [t for t in pinned_pairs if t not in all_unpinned]
    assert len(cmp) > 0
    assert np.allclose(w_gpu[cmp], ps.w[cmp], rtol=1e-4)
    # loss and gradient against the oracle on the GPU's own pair set
    sinks = np.nonzero(in_gpu)[0]
    l_ref, gx_ref, gy_ref = ref.p2p(nl, sinks, w_gpu[sinks].astype(np.float64))
    xr = c["x"].clone().requires_grad_(True)
    yr = c["y"].clone().requires_grad_(True)
    loss = tdp.P2PLoss.apply(xr, yr, g)
    loss.backward()
    assert abs(float(loss) - l_ref) <= 1e-4 * abs(l_ref)
    # per-cell scale: sum of |contributions| to that cell
    scale = _p2p_abs_scale(nl, sinks, w_gpu[sinks])
    gx = xr.grad.cpu().numpy()
    gy = yr.grad.cpu().numpy()
    assert np.all(np.abs(gx - gx_ref) <= 1e-4 * scale + 1e-6)
    assert np.all(np.abs(gy - gy_ref) <= 1e-4 * scale + 1e-6)
    # a second round adds to existing pairs (Eq. 9 state persists)
    g.pairs_update(rule=0, w0=10.0, w1=0.2)
    w2, in2 = g.pairs_export()
    ref.pairs_update(ps, rp, st["wns"], rule=0)
    assert np.array_equal(in2, in_gpu)
    assert np.allclose(w2[cmp], ps.w[cmp], rtol=1e-4)
    # exponential rule
    g.pairs_update(rule=1)
    w3, in3 = g.pairs_export()
    ps3 = ref.PairState(nl["num_pins"])
    ref.pairs_update(ps3, rp, st["wns"], rule=1)
    assert np.allclose(w3[cmp], ps3.w[cmp], rtol=1e-4)
    # checkpoint: export / reset / import restores the loss
    l1 = float(g.p2p_loss_fwd(c["x"], c["y"]))
    g.pairs_reset()
    assert g.pairs_count() == 0 and float(g.p2p_loss_fwd(c["x"], c["y"])) == 0.0
    g.pairs_import(w3, in3)
    assert float(g.p2p_loss_fwd(c["x"], c["y"])) == l1


def test_whole_chain_against_the_oracle_chain(library):
    """On the 2k-cell design every extracted path is pinned (separated from
    its neighbours by more than the comparison threshold), so the pair set
    is determined: the GPU's chain (timing, extraction, two Eq. 9 rounds,
    loss) against the oracle's own chain, with no GPU value fed to the
    oracle."""
    tdp = _tdp()
    c = case("C1", library)
    nl, st, g, k, K = c["nl"], c["st"], c["g"], c["k"], c["K"]
    g.pairs_reset()
    g.sta_update(c["x"], c["y"])
    g.extract_paths(n=-1, k=k, K=K)
    gp = g.paths()
    rp = ref.extract(nl, library, st, n=-1, k=k, K=K)
    res = compare_paths(gp, rp, st, Graph(nl), k)
    assert res["pinned"] == rp["num_paths"] == gp["num_paths"] and res["pinned_ok"] == res["pinned"]
    ps = ref.PairState(nl["num_pins"])
    for _ in range(2):
        g.pairs_update(rule=0, w0=10.0, w1=0.2)
        ref.pairs_update(ps, rp, st["wns"], rule=0)
    w_gpu, in_gpu = g.pairs_export()
    assert np.array_equal(in_gpu.astype(bool), ps.in_p.astype(bool))
    sinks, w_ref = ps.pairs()
    np.testing.assert_allclose(w_gpu[sinks], w_ref, rtol=1e-4)
    l_ref, gx_ref, gy_ref = ref.p2p(nl, sinks, w_ref)
    xr = c["x"].clone().requires_grad_(True)
    yr = c["y"].clone().requires_grad_(True)
    loss = tdp.P2PLoss.apply(xr, yr, g)
    loss.backward()
    assert abs(float(loss.detach()) - l_ref) <= 1e-4 * abs(l_ref)
    scale = _p2p_abs_scale(nl, sinks, w_ref)
    assert np.all(np.abs(xr.grad.cpu().numpy() - gx_ref) <= 1e-4 * scale + 1e-6)
    assert np.all(np.abs(yr.grad.cpu().numpy() - gy_ref) <= 1e-4 * scale + 1e-6)
    g.pairs_reset()


@pytest.mark.parametrize("precision", ["f32", "f64"])
def test_zero_copy_timing_views(precision, library):
    """tdp_sta_views: the graph's own arrival / required arrays in device pin
    order, read through the external-to-device pin map, equal the export;
    the same tensors show the next update's values."""
    tdp = _tdp()
    c = case("C1", library)
    nl = c["nl"]
    g = tdp.TimingGraph(nl, library, precision=precision, max_paths=200, max_k=4)
    g.sta_update(c["x"], c["y"])
    v = g.views()
    assert v["at"].dtype == (torch.float64 if precision == "f64" else torch.float32)
    idx = v["pin_index"].long()
    o = g.export()
    assert torch.equal(v["at"][idx].double(), o["at"]) and torch.equal(v["rat"][idx].double(), o["rat"])
    g.sta_update(c["x"] + 7.0, c["y"])
    o2 = g.export()
    assert not torch.equal(o2["at"], o["at"])
    assert torch.equal(v["at"][idx].double(), o2["at"]) and torch.equal(v["rat"][idx].double(), o2["rat"])
    del v
    g.close()


@pytest.mark.parametrize("bad", [float("nan"), float("inf"), -float("inf")])
def test_non_finite_positions_are_reported(bad, library):
    """A NaN or infinite cell coordinate makes the summary of that update an
    invalid-argument error; the next update at finite positions is clean,
    and so is its incremental form."""
    tdp = _tdp()
    c = case("C1", library)
    nl = c["nl"]
    g = tdp.TimingGraph(nl, library, max_paths=200, max_k=2)
    g.sta_update(c["x"], c["y"])
    ref_summary = g.summary()
    for axis in (0, 1):
        x, y = c["x"].clone(), c["y"].clone()
        (x if axis == 0 else y)[17] = bad
        g.sta_update(x, y)
        with pytest.raises(tdp.TdpError) as e:
            g.summary()
        assert e.value.status == 1
        g.sta_update(c["x"], c["y"])
        assert g.summary() == ref_summary
    x = c["x"].clone()
    x[17] = bad
    cells = torch.tensor([17], dtype=torch.int32, device=x.device)
    g.sta_update_arrivals_incremental(x, c["y"], cells)
    g.sta_update_required()
    with pytest.raises(tdp.TdpError) as e:
        g.summary()
    assert e.value.status == 1
    g.sta_update_arrivals_incremental(c["x"], c["y"], cells)
    g.sta_update_required()
    assert g.summary() == ref_summary
    g.close()


def test_autograd_on_column_views_of_a_position_matrix(library):
    # placers keep positions as one [N, 2] tensor; its columns are strided
    # views, which the autograd Functions must hand to the kernels as
    # contiguous arrays in both directions
    tdp = _tdp()
    c = case("C1", library)
    nl, st, g, k, K = c["nl"], c["st"], c["g"], c["k"], c["K"]
    g.pairs_reset()
    g.extract_paths(n=-1, k=k, K=K)
    g.pairs_update(rule=0, w0=10.0, w1=0.2)
    w_gpu, in_gpu = g.pairs_export()
    sinks = np.nonzero(in_gpu)[0]
    l_ref, gx_ref, gy_ref = ref.p2p(nl, sinks, w_gpu[sinks].astype(np.float64))
    scale = _p2p_abs_scale(nl, sinks, w_gpu[sinks])
    pos = torch.stack([c["x"], c["y"]], dim=1).clone().requires_grad_(True)
    assert not pos[:, 0].is_contiguous()
    for fn in (lambda a, b: tdp.P2PLoss.apply(a, b, g), lambda a, b: tdp.PairLoss.apply(a, b, g, 0)):
        pos.grad = None
        loss = fn(pos[:, 0], pos[:, 1])
        loss.backward()
        assert abs(float(loss) - l_ref) <= 1e-4 * abs(l_ref)
        gr = pos.grad.cpu().numpy()
        assert np.all(np.abs(gr[:, 0] - gx_ref) <= 1e-4 * scale + 1e-6)
        assert np.all(np.abs(gr[:, 1] - gy_ref) <= 1e-4 * scale + 1e-6)
    # the smoothed TNS through the same views
    v_ref, sx_ref, sy_ref = ref.stns(nl, library, st, gamma=10.0)
    pos.grad = None
    v = tdp.SmoothTNS.apply(pos[:, 0], pos[:, 1], g, 10.0)
    v.backward()
    gr = pos.grad.cpu().numpy()
    sc = np.abs(sx_ref).max()
    assert np.allclose(gr[:, 0], sx_ref, atol=1e-4 * sc, rtol=1e-3)
    assert np.allclose(gr[:, 1], sy_ref, atol=1e-4 * sc, rtol=1e-3)


def test_per_cell_tensors_are_checked(library):
    tdp = _tdp()
    c = case("C1", library)
    g = c["g"]
    short = c["x"][:-1].clone()
    with pytest.raises(ValueError):
        g.sta_update(short, c["y"])
    with pytest.raises(ValueError):
        g.p2p_loss_fwd(c["x"], c["y"].double())
    gx = torch.zeros_like(c["x"])
    with pytest.raises(ValueError):
        g.p2p_loss_bwd(c["x"], c["y"], torch.ones((), dtype=torch.float64, device=_dev()), gx, gx[:-1])
    with pytest.raises(ValueError):
        g.wa_fwd_bwd(c["x"], c["y"], 5.0, gx, torch.zeros(2 * g.num_cells, device=_dev())[::2])


def _p2p_abs_scale(nl, sinks, w):
    gr = Graph(nl)
    scale = np.zeros(nl["num_cells"])
    pc = nl["pin_cell"]
    px = np.where(pc >= 0, nl["x"][np.maximum(pc, 0)], 0) + nl["pin_off_x"]
    py = np.where(pc >= 0, nl["y"][np.maximum(pc, 0)], 0) + nl["pin_off_y"]
    for t, wt in zip(sinks, w):
        s = gr.driver[t]
        m = 2 * wt * (abs(px[s] - px[t]) + abs(py[s] - py[t]))
        for q in (s, t):
            if pc[q] >= 0:
                scale[pc[q]] += m
    return scale


# --------------------------------------------------- smoothed TNS and WA
def test_smoothed_tns_parity(library):
    tdp = _tdp()
    c = case("C1", library)
    nl, st, g = c["nl"], c["st"], c["g"]
    v_ref, gx_ref, gy_ref = ref.stns(nl, library, st, gamma=10.0)
    xr = c["x"].clone().requires_grad_(True)
    yr = c["y"].clone().requires_grad_(True)
    v = tdp.SmoothTNS.apply(xr, yr, g, 10.0)
    v.backward()
    assert abs(float(v) - v_ref) <= 1e-4 * abs(v_ref)
    sc = np.abs(gx_ref).max()
    assert np.allclose(xr.grad.cpu().numpy(), gx_ref, atol=1e-4 * sc, rtol=1e-3)
    assert np.allclose(yr.grad.cpu().numpy(), gy_ref, atol=1e-4 * sc, rtol=1e-3)


@pytest.mark.parametrize("name", ["C1", "C2"])
def test_wa_parity(name, library):
    c = case(name, library)
    nl, g = c["nl"], c["g"]
    v_ref, gx_ref, gy_ref, ax, ay = ref.wa(nl, 5.0, with_abs=True)
    gx = torch.zeros_like(c["x"])
    gy = torch.zeros_like(c["y"])
    v = g.wa_fwd_bwd(c["x"], c["y"], 5.0, gx, gy)
    assert abs(float(v) - v_ref) <= 1e-4 * abs(v_ref)
    # per cell: 1e-4 of the summed magnitudes of the summands of its pins' derivatives
    ex = np.abs(gx.cpu().numpy() - gx_ref)
    ey = np.abs(gy.cpu().numpy() - gy_ref)
    print("WA worst scaled error", (ex / np.maximum(ax, 1e-12)).max(), (ey / np.maximum(ay, 1e-12)).max())
    assert np.all(ex <= 1e-4 * ax + 1e-7)
    assert np.all(ey <= 1e-4 * ay + 1e-7)
    # at the last update's positions (the case's update used these): bitwise
    gx2 = torch.zeros_like(c["x"])
    gy2 = torch.zeros_like(c["y"])
    g.sta_update(c["x"], c["y"])
    v2 = g.wa_fwd_bwd_at_update(5.0, gx2, gy2)
    assert float(v2) == float(v) and torch.equal(gx2, gx) and torch.equal(gy2, gy)


# ------------------------------------------------------------ FP64 mode
def test_f64_mode_literal_threshold(library):
    tdp = _tdp()
    nl = with_clock(netgen.make_netlist(netgen.CONFIGS["C1"]), library)
    st = ref.sta(nl, library)
    g = tdp.TimingGraph(nl, library, precision="f64", max_paths=200, max_k=10)
    g.sta_update(*_xy(nl))
    o = {k: v.cpu().numpy() for k, v in g.export().items()}
    for key in ("at", "rat"):
        inf_ok, bad, worst = timing_close(o[key], st[key], rtol=1e-12)
        assert inf_ok and bad == 0, key
    g.extract_paths(n=-1, k=10, K=100)
    gp = g.paths()
    rp = ref.extract(nl, library, st, n=-1, k=10, K=100)
    res = compare_paths(gp, rp, st, Graph(nl), 10, fp32=False)
    assert res["pinned_ok"] == res["pinned"] and res["unpinned_ok"] == res["unpinned"]
    assert res["missing"] == 0 and res["extra"] == 0


# --------------------------------------------------------- determinism
def test_bitwise_determinism(library):
    tdp = _tdp()
    nl = with_clock(netgen.make_netlist(netgen.CONFIGS["C1"]), library)
    outs = []
    for _ in range(2):
        g = tdp.TimingGraph(nl, library, max_paths=200, max_k=10)
        x, y = _xy(nl)
        g.sta_update(x, y)
        g.extract_paths(n=-1, k=10, K=100)
        g.pairs_update()
        gx = torch.zeros_like(x)
        gy = torch.zeros_like(y)
        loss = g.p2p_loss_fwd(x, y)
        g.p2p_loss_bwd(x, y, torch.ones((), dtype=torch.float64, device=x.device), gx, gy)
        p = g.paths()
        outs.append((g.export()["slack"].cpu().numpy(), p["path_pins"], p["path_slack"], g.pairs_export()[0],
                     float(loss), gx.cpu().numpy(), gy.cpu().numpy()))
        g.close()
    for a, b in zip(*outs):
        assert np.array_equal(np.asarray(a), np.asarray(b))


# -------------------------------------------------------------- batching
@pytest.mark.parametrize("net_model", [0, 2])
def test_batch_matches_single_instances(net_model, library):
    # the spanning-tree model builds its trees per chunk segment: an instance's
    # nets give the same bits wherever they sit in the union's chunks
    tdp = _tdp()
    library = dict(library, net_model=net_model)
    nls = []
    for i, n in enumerate((3000, 800, 5000)):
        cfg = netgen.NetlistConfig(f"b{i}", n, depth=10 + 5 * i, fanout_cap=16, die=600.0, seed=40 + i)
        nls.append(netgen.make_netlist(cfg))
    # a shared clock period, tight enough that every instance has violations
    T = math.inf
    for nl in nls:
        st0 = ref.sta(nl, library, clock_period=0.0)
        T = min(T, netgen.clock_period_for_fail_fraction(st0["at"][ref.endpoint_pins(nl)], 0.05))
    for nl in nls:
        nl["clock_period"] = np.float32(T)
    gb = tdp.TimingGraph(nls, library, max_paths=2000, max_k=4)
    pb, cb = gb.batch_offsets()
    xb = torch.tensor(np.concatenate([nl["x"] for nl in nls]), device=_dev())
    yb = torch.tensor(np.concatenate([nl["y"] for nl in nls]), device=_dev())
    gb.sta_update(xb, yb)
    wb, tb, nb = gb.batch_summary()
    gb.extract_paths(n=-1, k=4, K=300)
    P = gb.paths()
    ob = gb.export()
    for i, nl in enumerate(nls):
        g = tdp.TimingGraph(nl, library, max_paths=2000, max_k=4)
        g.sta_update(*_xy(nl))
        w, t, n = g.summary()
        assert (w, n) == (wb[i], nb[i]) and abs(t - tb[i]) <= 1e-9 * max(1.0, abs(t))
        o = g.export()
        for key in ("slack", "dnet", "load", "slew"):
            assert torch.equal(o[key], ob[key][pb[i]:pb[i + 1]]), key
        g.extract_paths(n=-1, k=4, K=300)
        p = g.paths()
        sel = (P["path_ep"] >= pb[i]) & (P["path_ep"] < pb[i + 1])
        idx = np.nonzero(sel)[0]
        assert len(idx) == p["num_paths"] > 0
        assert np.array_equal(P["path_slack"][idx], p["path_slack"])
        mine = np.concatenate([P["path_pins"][P["path_ptr"][j]:P["path_ptr"][j + 1]] for j in idx]) - pb[i]
        assert np.array_equal(mine, p["path_pins"])
        g.close()


# ------------------------------------------------------------ sweep modes
def test_level_and_dataflow_sweeps_agree_bitwise(library):
    """The resident dataflow sweeps (both, or the required times only) compute
    exactly what the one-launch-per-level sweeps compute (same operations in
    the same order per value)."""
    tdp = _tdp()
    c = case("C2", library)
    nl = c["nl"]
    outs = []
    for mode in (0, 1, 3):
        g = tdp.TimingGraph(nl, library, max_paths=c["K"], max_k=c["k"])
        g.set_tuning(sweep_mode=mode)
        g.sta_update(c["x"], c["y"])
        o = {k: v.cpu().numpy() for k, v in g.export().items()}
        g.extract_paths(n=-1, k=c["k"], K=c["K"])
        p = g.paths()
        outs.append((o, p, g.summary()))
        g.close()
    o0, p0, s0 = outs[0]
    for o1, p1, s1 in outs[1:]:
        for key in o0:
            assert np.array_equal(o0[key], o1[key]), key
        for key in ("path_ptr", "path_pins", "path_ep", "path_rank", "path_slack"):
            assert np.array_equal(p0[key], p1[key]), key
        assert s0 == s1


def test_wide_cells_match_oracle_and_dataflow(library):
    """Fan-in up to 8: chunks whose cells all have <= 4 inputs take the
    gathered reductions, wider ones the shuffle scan; both against the
    oracle and bitwise against the dataflow sweep (scan only)."""
    tdp = _tdp()
    cfg = netgen.NetlistConfig("wide", 20000, ff_frac=0.1, depth=30, fanin_lo=1, fanin_hi=8, fanout_cap=16,
                               die=2000.0, seed=7)
    nl = with_clock(netgen.make_netlist(cfg), library)
    st = ref.sta(nl, library)
    widths = np.diff(nl["cell_in_ptr"])[np.asarray(nl["cell_is_ff"]) == 0]
    assert widths.max() > 4 and (widths <= 4).mean() > 0.3
    k, K = 4, 2000
    outs = []
    for mode in (0, 1, 3):
        g = tdp.TimingGraph(nl, library, max_paths=K, max_k=k)
        g.set_tuning(sweep_mode=mode)
        g.sta_update(*_xy(nl))
        o = {kk: v.cpu().numpy() for kk, v in g.export().items()}
        g.extract_paths(n=-1, k=k, K=K)
        outs.append((o, g.paths()))
        g.close()
    o0, p0 = outs[0]
    for o1, p1 in outs[1:]:
        for key in o0:
            assert np.array_equal(o0[key], o1[key]), key
        for key in ("path_ptr", "path_pins", "path_slack"):
            assert np.array_equal(p0[key], p1[key]), key
    for key in ("at", "rat"):
        inf_ok, bad, worst = timing_close(o0[key], st[key],
                                          scale=np.maximum(np.abs(np.nan_to_num(st["at"], posinf=0, neginf=0)),
                                                           abs(float(nl["clock_period"]))))
        assert inf_ok and bad == 0, (key, bad, worst)
    rp = ref.extract(nl, library, st, n=-1, k=k, K=K)
    res = compare_paths(p0, rp, st, Graph(nl), k)
    assert p0["num_paths"] == rp["num_paths"]
    assert res["missing"] == 0 and res["extra"] == 0
    assert res["pinned_ok"] == res["pinned"] and res["unpinned_ok"] == res["unpinned"]


def test_dataflow_wait_gives_up_cleanly(library):
    """Self-test of the bounded waits: with the start points withheld every
    wait runs out of polls, the kernels still finish and the summary reports
    a device error; the next normal update is correct again."""
    tdp = _tdp()
    nl = with_clock(netgen.make_netlist(netgen.CONFIGS["C1"]), library)
    st = ref.sta(nl, library)
    g = tdp.TimingGraph(nl, library, max_paths=200, max_k=10)
    x, y = _xy(nl)
    g.set_tuning(spin_log2=4, sweep_mode=2)
    g.sta_update(x, y)
    with pytest.raises(tdp.TdpError) as e:
        g.summary()
    assert e.value.status == 4
    g.set_tuning(spin_log2=20, sweep_mode=1)
    g.sta_update(x, y)
    wns, tns, nf = g.summary()
    assert nf == st["n_fail"] and abs(wns - st["wns"]) <= 1e-4 * abs(st["wns"])


# ------------------------------------------------------------------ errors
def test_error_paths(library):
    tdp = _tdp()
    nl, _ = handnets.chain_netlist()
    g = tdp.TimingGraph(nl, handnets.dyadic_library(), max_paths=4, max_k=2)
    with pytest.raises(tdp.TdpError) as e:
        g.extract_paths(n=-1, k=1)
    assert e.value.status == 6
    g.sta_update(*_xy(nl))
    with pytest.raises(tdp.TdpError) as e:
        g.extract_paths(n=-1, k=3)
    assert e.value.status == 5
    # no violation: no paths, pair update keeps P empty, loss 0
    g.set_clock(1000.0)
    g.sta_update(*_xy(nl))
    assert g.summary() == (0.0, 0.0, 0)
    g.extract_paths(n=-1, k=2)
    assert g.paths()["num_paths"] == 0
    g.pairs_update()
    assert g.pairs_count() == 0
    x, y = _xy(nl)
    assert float(g.p2p_loss_fwd(x, y)) == 0.0


def test_empty_requests_and_a_design_without_logic(library):
    """K = 0, n = 0 and a slack limit below WNS give no paths from either
    extraction; a design of flip-flops and ports only (no combinational
    cell, depth 0) times, extracts and scores exactly."""
    tdp = _tdp()
    c = case("C1", library)
    st, g = c["st"], c["g"]
    lim = float(st["wns"]) - 1.0
    for call in (lambda: g.extract_paths(n=-1, k=2, K=0), lambda: g.extract_paths(n=0, k=2),
                 lambda: g.report_timing(0), lambda: g.report_timing(50, slack_limit=lim),
                 lambda: g.extract_paths(n=-1, k=2, slack_limit=lim)):
        call()
        p = g.paths()
        assert p["num_paths"] == 0 and p["path_ptr"].tolist() == [0]
    # ports 6, 7 and flip-flops 0, 1, 2 (D pins 0, 2, 4; Q pins 1, 3, 5); Q 3
    # and Q 5 drive nothing.  Distances 10, 130 and 120 um give the exact
    # arrivals 1.5625, 264.0625 and 26 + 225 = 251 under the dyadic library.
    nl0, _ = handnets.build([(netgen.FF_TYPE, 1)] * 3, 2, [(6, [0]), (7, [2]), (1, [4]), (3, []), (5, [])],
                            x=[10.0, 50.0, 90.0], y=[0.0, 20.0, 40.0], port_xy=[(0.0, 0.0), (100.0, 100.0)],
                            clock_period=200.0)
    lib = handnets.dyadic_library()
    st0 = ref.sta(nl0, lib)
    assert st0["at"][[0, 2, 4]].tolist() == [1.5625, 264.0625, 251.0]
    g0 = tdp.TimingGraph(nl0, lib, max_paths=8, max_k=2)
    x0, y0 = _xy(nl0)
    g0.sta_update(x0, y0)
    o = {k: v.cpu().numpy() for k, v in g0.export().items()}
    fin = np.isfinite(st0["rat"])
    assert np.array_equal(o["at"], st0["at"]) and np.array_equal(o["rat"][fin], st0["rat"][fin])
    assert g0.summary() == (-64.0625, -115.0625, 2)
    g0.extract_paths(n=-1, k=2)
    gp = g0.paths()
    rp = ref.extract(nl0, lib, st0, n=-1, k=2)
    assert gp["num_paths"] == rp["num_paths"] == 2
    assert np.array_equal(gp["path_pins"], rp["path_pins"]) and np.array_equal(gp["path_slack"], rp["path_slack"])
    g0.report_timing(5)
    gk = g0.paths()
    rk = ref.report_timing(nl0, lib, st0, 5)
    assert gk["num_paths"] == rk["num_paths"] == 3
    assert np.array_equal(gk["path_pins"], rk["path_pins"]) and np.array_equal(gk["path_slack"], rk["path_slack"])
    g0.pairs_reset()
    g0.extract_paths(n=-1, k=2)
    g0.pairs_update()
    w, inp = g0.pairs_export()
    assert sorted(np.nonzero(inp)[0].tolist()) == [2, 4]
    gx = torch.zeros_like(x0)
    gy = torch.zeros_like(y0)
    wl = g0.wa_fwd_bwd(x0, y0, 5.0, gx, gy)
    v_wa, wx, wy = ref.wa(nl0, 5.0)
    assert abs(float(wl) - v_wa) <= 1e-5 * max(1.0, abs(v_wa))
    assert np.allclose(gx.cpu().numpy(), wx, rtol=1e-4, atol=1e-6)
    g0.close()


# -------------------------------------------------------------- autotuner
def test_autotune_keeps_results(library):
    """The autotuner picks a supported configuration and the results after it
    are bitwise those of the default configuration."""
    tdp = _tdp()
    c = case("C2", library)
    g = tdp.TimingGraph(c["nl"], library, max_paths=c["K"], max_k=c["k"])
    ch = g.autotune(c["x"], c["y"], n=-1, k=c["k"], K=c["K"], reps=2)
    print("autotune choice", ch)
    assert ch["sweep_mode"] in (0, 1, 3) and ch["flow_waves"] in (1, 2, 4) and ch["flow_per_cu"] in (1, 2, 4)
    assert ch["us_per_run"] > 0
    o = {k: v.cpu().numpy() for k, v in g.export().items()}
    for key in o:
        assert np.array_equal(o[key], c["gpu"][key]), key
    g.extract_paths(n=-1, k=c["k"], K=c["K"])
    p = g.paths()
    c["g"].extract_paths(n=-1, k=c["k"], K=c["K"])
    p0 = c["g"].paths()
    for key in ("path_ptr", "path_pins", "path_slack"):
        assert np.array_equal(p[key], p0[key]), key
    with pytest.raises(tdp.TdpError):
        g.autotune(c["x"], c["y"], reps=0)
    # a second graph of the same signature takes the kept choice (the time
    # reported is the one measured when the choice was made) and its results
    g2 = tdp.TimingGraph(c["nl"], library, max_paths=c["K"], max_k=c["k"])
    ch2 = g2.autotune(c["x"], c["y"], n=-1, k=c["k"], K=c["K"], reps=2)
    assert ch2 == ch
    o2 = {k: v.cpu().numpy() for k, v in g2.export().items()}
    for key in o:
        assert np.array_equal(o2[key], o[key]), key
    g2.close()
    g.close()


# ------------------------------------------------------ pair-loss variants
@pytest.mark.parametrize("kind", [0, 1, 2])
def test_pair_loss_variants(library, kind):
    """The three pair distances of Sec. III-C over the GPU's pair set, value
    and gradient against the oracle (per cell: 1e-4 of the summed magnitudes
    of the terms that reach it)."""
    tdp = _tdp()
    c = case("C2", library)
    nl, g = c["nl"], c["g"]
    g.pairs_reset()
    g.extract_paths(n=-1, k=c["k"], K=c["K"])
    g.pairs_update(rule=1)
    w, in_p = g.pairs_export()
    sinks = np.nonzero(in_p)[0]
    ws = w[sinks].astype(np.float64)
    if kind == 0:
        v_ref, gx_ref, gy_ref = ref.p2p(nl, sinks, ws)
        scale = _p2p_abs_scale(nl, sinks, w[sinks])
    else:
        v_ref, gx_ref, gy_ref = ref.pair_loss(nl, kind, sinks, ws)
        # every term's gradient has magnitude at most w per axis
        gr = Graph(nl)
        pc = nl["pin_cell"]
        scale = np.zeros(nl["num_cells"])
        for t, wt in zip(sinks, ws):
            for q in (gr.driver[t], t):
                if pc[q] >= 0:
                    scale[pc[q]] += wt
    xr = c["x"].clone().requires_grad_(True)
    yr = c["y"].clone().requires_grad_(True)
    v = tdp.PairLoss.apply(xr, yr, g, kind)
    v.backward()
    assert abs(float(v) - v_ref) <= 1e-4 * abs(v_ref)
    ex = np.abs(xr.grad.cpu().numpy() - gx_ref)
    ey = np.abs(yr.grad.cpu().numpy() - gy_ref)
    print("kind", kind, "worst scaled error", (ex / np.maximum(scale, 1e-12)).max())
    assert np.all(ex <= 1e-4 * scale + 1e-6) and np.all(ey <= 1e-4 * scale + 1e-6)
    if kind == 0:  # the variant entry equals the p2p entry bitwise
        assert float(g.pair_loss_fwd(0, c["x"], c["y"])) == float(g.p2p_loss_fwd(c["x"], c["y"]))
    with pytest.raises(tdp.TdpError):
        g.pair_loss_fwd(3, c["x"], c["y"])


def test_quadratic_pair_loss_spaces_a_chain_on_the_gpu(library):
    """Sec. III-C / Fig. 3 on the GPU path: gradient descent on the pair loss
    of a chain of movable buffers between a fixed port and a fixed flip-flop.
    The quadratic loss moves the buffers to equal spacing; the Manhattan and
    linear Euclidean losses give every interior buffer a zero gradient, so a
    skewed chain stays where it is."""
    from tests.test_pair_losses import _chain
    tdp = _tdp()
    skew = [0.0, 0.5, 1.0, 1.5, 2.0, 9.0, 10.0]
    nl, sinks = _chain(skew)
    n = len(skew) - 2
    for kind in (0, 1, 2):
        g = tdp.TimingGraph(nl, library, max_paths=4, max_k=1)
        x, y = _xy(nl)
        g.sta_update(x, y)
        w = np.zeros(nl["num_pins"], np.float32)
        inp = np.zeros(nl["num_pins"], np.uint8)
        w[sinks], inp[sinks] = 1.0, 1
        g.pairs_import(w, inp)
        x = x.clone()
        for _ in range(400):
            xr = x.clone().requires_grad_(True)
            tdp.PairLoss.apply(xr, y, g, kind).backward()
            if kind != 0:
                # the interior buffers feel no pull at all
                assert torch.count_nonzero(xr.grad[:n]) == 0
                break
            x = x - 0.1 * xr.grad
        if kind == 0:
            pos = [0.0] + x.cpu().numpy()[:n].tolist() + [10.0]
            assert np.allclose(np.diff(pos), 10.0 / (n + 1), atol=1e-3), pos
        g.close()


def test_two_pass_update_on_two_streams(library):
    """The arrival pass and the required-time pass, the second on another
    stream ordered by events, give bitwise what the one-call update gives."""
    tdp = _tdp()
    c = case("C2", library)
    g = tdp.TimingGraph(c["nl"], library, max_paths=c["K"], max_k=c["k"])
    side = torch.cuda.Stream()
    main = torch.cuda.current_stream()
    ev = torch.cuda.Event()
    g.sta_update_arrivals(c["x"], c["y"])
    ev.record(main)
    side.wait_event(ev)
    g.sta_update_required(stream=side)
    ev2 = torch.cuda.Event()
    ev2.record(side)
    main.wait_event(ev2)
    o = {k: v.cpu().numpy() for k, v in g.export().items()}
    for key in o:
        assert np.array_equal(o[key], c["gpu"][key]), key
    g2 = tdp.TimingGraph(c["nl"], library, max_paths=8, max_k=1)
    with pytest.raises(tdp.TdpError) as e:
        g2.sta_update_required()
    assert e.value.status == 6
    g.close()
    g2.close()


# ------------------------------------------------------------- HIP graphs
def test_step_replays_from_a_captured_graph(library):
    """The benchmark's step (three streams) captured in a HIP graph: every
    replay, with eager work and synchronisations between replays, gives
    bitwise the eager step's paths, pair weights, losses and gradients."""
    import bench
    tdp = _tdp()
    c = case("C2", library)
    g = tdp.TimingGraph(c["nl"], library, max_paths=c["K"], max_k=c["k"])
    x, y = c["x"], c["y"]
    gx = torch.zeros_like(x)
    gy = torch.zeros_like(y)
    wl = torch.zeros((), dtype=torch.float64, device=_dev())
    pp = torch.zeros((), dtype=torch.float64, device=_dev())
    beta = torch.full((), 2.5e-5, dtype=torch.float64, device=_dev())
    step = bench.build_step(g, x, y, c["k"], c["K"], gx, gy, wl, pp, beta, overlap=True)

    def snapshot():
        torch.cuda.synchronize()
        p = g.paths()
        w, _ = g.pairs_export()
        return (p["path_pins"].copy(), p["path_slack"].copy(), w.copy(), float(wl), float(pp),
                gx.cpu().numpy().copy(), gy.cpu().numpy().copy(), g.export()["slack"].cpu().numpy())

    # eager reference: reset P, one step
    g.pairs_reset()
    step()
    ref_out = snapshot()
    # capture (the pair set then holds one round; reset before every replay)
    step()
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        step()
    torch.cuda.synchronize()
    for rep in range(3):
        g.pairs_reset()
        torch.cuda.synchronize()
        graph.replay()
        out = snapshot()
        for a, b in zip(out, ref_out):
            assert np.array_equal(np.asarray(a), np.asarray(b)), rep
        # eager work between replays
        g.sta_update(x, y)
        g.extract_paths(n=-1, k=1)
        torch.cuda.synchronize()
    g.close()
