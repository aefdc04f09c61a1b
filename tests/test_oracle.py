"""Pins for the FP64 CPU oracle: closed forms, hand-computed chains, the
paper's worked example, brute force over all paths, invariants and finite
differences.  Every check here fixes the oracle against something other than
itself; a plausible slip anywhere in it (a dropped term, a wrong sign or
index, a swapped operand) breaks at least one of them."""
import json
import math
import os

import numpy as np
import pytest

from oracle import ref
from paper_2503_11674_amd import netgen
from tests import handnets
from tests.bruteforce import Graph, brute_endpoint_paths, brute_sta
from tests.conftest import with_clock

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------------------
# lookup tables
# ---------------------------------------------------------------------------
def test_lut_exact_at_grid_points(library):
    sa, la = library["slew_axis"][0], library["load_axis"][0]
    S, L = np.meshgrid(sa, la, indexing="ij")
    for t in range(8):
        tab = library["delay_lut"][t]
        v = ref.lut_eval(sa, la, tab, S.ravel(), L.ravel())
        assert np.array_equal(v, tab.astype(np.float64).ravel())


def test_lut_reproduces_bilinear_functions():
    sa, la = netgen.SLEW_AXIS, netgen.LOAD_AXIS
    a, b, c, d = 3.0, 0.7, 0.01, 0.0005
    f = lambda s, l: a + b * s + c * l + d * s * l
    S, L = np.meshgrid(sa.astype(np.float64), la.astype(np.float64), indexing="ij")
    tab = f(S, L)
    rng = np.random.default_rng(3)
    s = rng.uniform(5, 80, 500)
    l = rng.uniform(2, 8192, 500)
    v = ref.lut_eval(sa, la, tab.astype(np.float32), s, l)
    # the table itself is rounded to float32, so compare against the same
    exact = ref.lut_eval(sa, la, tab.astype(np.float32), s, l)
    assert np.allclose(v, f(s, l), rtol=2e-7, atol=1e-5)
    assert np.array_equal(v, exact)


def test_lut_clamps_outside_the_axes(library):
    sa, la = library["slew_axis"][0], library["load_axis"][0]
    tab = library["delay_lut"][3].astype(np.float64)
    v = ref.lut_eval(sa, la, tab.astype(np.float32), np.array([1.0, 500.0, 1.0, 500.0]),
                     np.array([0.5, 0.5, 1e6, 1e6]))
    assert v.tolist() == [tab[0, 0], tab[6, 0], tab[0, 6], tab[6, 6]]


# ---------------------------------------------------------------------------
# hand-computed chains with exact binary-fraction values
# ---------------------------------------------------------------------------
def test_hand_chain_exact():
    nl, pins = handnets.chain_netlist()
    lib = handnets.dyadic_library()
    st = ref.sta(nl, lib)
    # wires are 24 um: net delay 24^2/64 = 9 ps, load 2 + 24/4 = 8 fF
    # buffer delay at (slew 10, load 8) = 4 + 10/4 + 8/64 = 6.625 ps
    # clock-to-Q at (10, load 0 clamped to 2) = 20 + 5 + 2/32 = 25.0625 ps
    exp_at = {6: 0.0, 0: 9.0, 1: 15.625, 2: 24.625, 3: 31.25, 4: 40.25, 5: 25.0625}
    exp_rat = {4: 32.0, 3: 23.0, 2: 16.375, 1: 7.375, 0: 0.75, 6: -8.25, 5: math.inf}
    for p, v in exp_at.items():
        assert st["at"][p] == v, p
    for p, v in exp_rat.items():
        assert st["rat"][p] == v, p
    for p in (6, 0, 1, 2, 3, 4):
        assert st["slack"][p] == -8.25
    assert st["slack"][5] == math.inf
    assert st["dnet"][0] == 9.0 and st["load"][1] == 8.0 and st["darc"][2] == 6.625
    assert (st["wns"], st["tns"], st["n_fail"]) == (-8.25, -8.25, 1)
    pa = ref.extract(nl, lib, st, n=-1, k=3)
    assert pa["num_paths"] == 1
    assert ref.path_list(pa) == [[6, 0, 1, 2, 3, 4]]
    assert pa["path_slack"][0] == -8.25


def test_hand_diamond_exact():
    nl, pins = handnets.diamond_netlist()
    lib = handnets.dyadic_library()
    st = ref.sta(nl, lib)
    # A->BUF.in 24 um (9 ps), BUF.out->AND.in0 24 um (9 ps), A->AND.in1 48 um (36 ps)
    # BUF: 4 + 2.5 + 0.125 = 6.625; AND (type 2): 6 + 2.5 + 0.125 = 8.625
    assert st["at"][2] == 24.625 and st["at"][3] == 36.0
    assert st["at"][4] == 44.625 and st["at"][5] == 53.625
    assert st["crit"][1] == 1
    assert st["slack"][5] == -3.625 and st["slack"][7] == -3.625
    assert st["slack"][0] == 7.75 and st["slack"][2] == 7.75 and st["slack"][3] == -3.625
    pa = ref.extract(nl, lib, st, n=-1, k=2)
    assert ref.path_list(pa) == [[7, 3, 4, 5], [7, 0, 1, 2, 4, 5]]
    assert pa["path_slack"].tolist() == [-3.625, 7.75]
    assert pa["path_rank"].tolist() == [0, 1]
    pa1 = ref.extract(nl, lib, st, n=-1, k=1)
    assert pa1["ep_next"].tolist() == [7.75]


def test_no_violation_gives_zero_wns_tns():
    nl, _ = handnets.chain_netlist()
    st = ref.sta(nl, handnets.dyadic_library(), clock_period=1000.0)
    assert (st["wns"], st["tns"], st["n_fail"]) == (0.0, 0.0, 0)
    pa = ref.extract(nl, handnets.dyadic_library(), st, n=-1, k=1)
    assert pa["num_paths"] == 0


# ---------------------------------------------------------------------------
# brute force over every path of small random DAGs
# ---------------------------------------------------------------------------
def _tiny(seed, n=24, depth=5):
    cfg = netgen.NetlistConfig("tiny", n, ff_frac=0.25, depth=depth, fanin_lo=1, fanin_hi=3,
                               fanout_cap=6, die=200.0, seed=seed)
    return netgen.make_netlist(cfg)


@pytest.mark.parametrize("seed", range(8))
def test_sta_matches_brute_force(seed, library):
    nl = with_clock(_tiny(seed), library, 0.3)
    st = ref.sta(nl, library)
    at, rat = brute_sta(nl, st)
    fin = np.isfinite(at)
    assert np.array_equal(fin, np.isfinite(st["at"]))
    assert np.allclose(st["at"][fin], at[fin], rtol=1e-12, atol=1e-9)
    fin = np.isfinite(rat)
    assert np.array_equal(fin, np.isfinite(st["rat"]))
    assert np.allclose(st["rat"][fin], rat[fin], rtol=1e-12, atol=1e-9)


@pytest.mark.parametrize("seed", range(8))
def test_k_paths_match_brute_force(seed, library):
    nl = with_clock(_tiny(seed), library, 0.3)
    st = ref.sta(nl, library)
    k = 6
    E = ref.endpoint_pins(nl)
    pa = ref.extract(nl, library, st, n=len(E), k=k)
    got = {}
    for i, pl in enumerate(ref.path_list(pa)):
        got.setdefault(int(pa["path_ep"][i]), []).append((int(pa["path_rank"][i]), pa["path_slack"][i], pl))
    for e in E:
        want = brute_endpoint_paths(nl, st, int(e))
        mine = sorted(got.get(int(e), []))
        assert len(mine) == min(k, len(want))
        for r, (rank, s, pl) in enumerate(mine):
            assert rank == r
            assert abs(s - want[r][0]) <= 1e-9 * max(1.0, abs(want[r][0]))
            lo = r == 0 or want[r][0] - want[r - 1][0] > 1e-9
            hi = r + 1 >= len(want) or want[r + 1][0] - want[r][0] > 1e-9
            if lo and hi:
                assert pl == want[r][1]
            else:
                assert any(pl == w[1] for w in want)


def _all_paths(nl, st):
    """Every path of the design with its slack, sorted by slack."""
    out = []
    for e in ref.endpoint_pins(nl):
        out += [(s, int(e), pl) for s, pl in brute_endpoint_paths(nl, st, int(e))]
    out.sort(key=lambda t: t[0])
    return out


@pytest.mark.parametrize("seed", range(8))
@pytest.mark.parametrize("K", [1, 7, 40, 10 ** 6])
def test_global_k_paths_match_brute_force(seed, K, library):
    """report_timing(K): the K smallest slacks over every path of the design;
    a path whose slack is separated from its neighbours is fixed pin for pin,
    ranks count the earlier paths of the same endpoint."""
    nl = with_clock(_tiny(seed), library, 0.3)
    st = ref.sta(nl, library)
    want = _all_paths(nl, st)
    got = ref.report_timing(nl, library, st, K)
    m = got["num_paths"]
    assert m == min(K, len(want))
    gl = ref.path_list(got)
    assert np.all(np.diff(got["path_slack"]) >= 0)
    assert len(set(map(tuple, gl))) == m
    for r in range(m):
        s = got["path_slack"][r]
        assert abs(s - want[r][0]) <= 1e-9 * max(1.0, abs(want[r][0]))
        lo = r == 0 or want[r][0] - want[r - 1][0] > 1e-9
        hi = r + 1 >= len(want) or want[r + 1][0] - want[r][0] > 1e-9
        if lo and hi:
            assert gl[r] == want[r][2] and got["path_ep"][r] == want[r][1]
        else:
            assert any(gl[r] == w[2] for w in want)
    nxt = want[m][0] if m < len(want) else math.inf
    assert got["next_slack"] == nxt or abs(got["next_slack"] - nxt) <= 1e-9 * max(1.0, abs(nxt))
    seen = {}
    for r in range(m):
        e = int(got["path_ep"][r])
        assert got["path_rank"][r] == seen.get(e, 0)
        seen[e] = seen.get(e, 0) + 1


def test_global_k_agrees_with_per_endpoint_lists(library):
    """On the 2k-cell workload: the paths report_timing(K) puts on an
    endpoint are that endpoint's worst paths, and its K-th slack is no larger
    than the K-th smallest of the per-endpoint top-k union (a subset of all
    paths)."""
    nl = with_clock(netgen.make_netlist(netgen.CONFIGS["C1"]), library)
    st = ref.sta(nl, library)
    K = 100
    g = ref.report_timing(nl, library, st, K)
    assert g["num_paths"] == K
    E = ref.endpoint_pins(nl)
    per = ref.extract(nl, library, st, n=len(E), k=10)
    assert g["path_slack"][-1] <= np.sort(per["path_slack"])[K - 1] + 1e-9
    cnt = {}
    for e in g["path_ep"].tolist():
        cnt[e] = cnt.get(e, 0) + 1
    for e, c in cnt.items():
        one = ref.extract(nl, library, st, n=len(E), k=c)
        s_ep = np.sort(one["path_slack"][one["path_ep"] == e])
        s_gl = np.sort(g["path_slack"][g["path_ep"] == e])
        assert np.allclose(s_ep, s_gl, rtol=0, atol=1e-9)
    # every endpoint absent from the answer has slack >= the K-th path's
    absent = np.setdiff1d(E, np.array(list(cnt.keys())))
    assert np.all(st["slack"][absent] >= g["path_slack"][-1] - 1e-9)


# ---------------------------------------------------------------------------
# invariants on the smallest workload
# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def c1(library):
    nl = with_clock(netgen.make_netlist(netgen.CONFIGS["C1"]), library)
    return nl, ref.sta(nl, library)


def test_invariants_c1(c1, library):
    nl, st = c1
    g = Graph(nl)
    at, rat, sl = st["at"], st["rat"], st["slack"]
    fin = np.isfinite(rat)
    assert np.array_equal(sl[fin], (rat - at)[fin])
    # every arc: AT(v) >= AT(u) + d and RAT(u) <= RAT(v) - d; crit arcs are tight
    for v in range(g.P):
        for u in g.preds(v):
            d = g.arc_delay(u, v, st["dnet"], st["darc"])
            assert at[v] >= at[u] + d - 1e-9
            if np.isfinite(rat[v]):
                assert rat[u] <= rat[v] - d + 1e-9
    for c in range(nl["num_cells"]):
        if nl["cell_is_ff"][c]:
            continue
        o = nl["cell_out_pin"][c]
        i = nl["cell_in_pins"][nl["cell_in_ptr"][c] + st["crit"][c]]
        assert at[o] == at[i] + st["darc"][i]
    E = ref.endpoint_pins(nl)
    es = sl[E]
    assert st["n_fail"] == int(math.floor(0.05 * len(E)))
    assert st["wns"] == es.min()
    # the worst slack anywhere is the worst endpoint slack (up to rounding)
    assert abs(sl.min() - st["wns"]) <= 1e-9
    assert math.isclose(st["tns"], es[es < 0].sum(), rel_tol=1e-12)
    # every pin on the worst endpoint's rank-1 path has slack == WNS
    pa = ref.extract(nl, library, st, n=1, k=1)
    for p in ref.path_list(pa)[0]:
        assert abs(sl[p] - st["wns"]) <= 1e-9


def test_extraction_structure_c1(c1, library):
    nl, st = c1
    nf = st["n_fail"]
    p1 = ref.extract(nl, library, st, n=-1, k=1)
    assert p1["num_paths"] == nf and len(set(p1["path_ep"].tolist())) == nf
    p10 = ref.extract(nl, library, st, n=-1, k=10)
    assert p10["num_paths"] <= 10 * nf
    assert np.all(np.diff(p10["path_slack"]) >= 0)
    # rank-1 slack is the endpoint slack; ranks within an endpoint are ordered
    for i in range(p10["num_paths"]):
        e = p10["path_ep"][i]
        if p10["path_rank"][i] == 0:
            assert abs(p10["path_slack"][i] - st["slack"][e]) < 1e-9
    # the reported slack equals RAT - (AT(start) + sum of arc delays)
    g = Graph(nl)
    for i, pl in enumerate(ref.path_list(p10)):
        arr = st["at"][pl[0]] + g.path_delay(pl, st["dnet"], st["darc"])
        assert abs((st["rat"][pl[-1]] - arr) - p10["path_slack"][i]) < 1e-9
        assert g.is_start(pl[0]) and g.role[pl[-1]] == "ffd"
    pK = ref.extract(nl, library, st, n=-1, k=10, K=37)
    assert pK["num_paths"] == 37
    assert np.array_equal(pK["path_slack"], p10["path_slack"][:37])


# ---------------------------------------------------------------------------
# pin-pair weights: the paper's worked example (Fig. 2 discussion)
# ---------------------------------------------------------------------------
def _fig2():
    with open(os.path.join(GOLDEN, "fig2_pairs.json")) as f:
        g = json.load(f)
    paths = [p["pins"] for p in g["paths"]]
    sl = np.array([p["slack"] for p in g["paths"]], np.float64)
    order = np.argsort(sl, kind="stable")
    ptr = np.concatenate([[0], np.cumsum([len(paths[i]) for i in order])]).astype(np.int32)
    pins = np.concatenate([paths[i] for i in order]).astype(np.int32)
    return g, {"num_paths": len(paths), "path_ptr": ptr, "path_pins": pins, "path_slack": sl[order]}


def test_fig2_eq9_weights():
    g, pa = _fig2()
    st = ref.PairState(g["num_pins"])
    ref.pairs_update(st, pa, wns=g["wns"], rule=0, w0=g["w0"], w1=g["w1"])
    assert st.in_p[g["pin_B"]] == 0            # B only lies on a non-violating path
    assert st.in_p[g["pin_C"]] == 1
    assert math.isclose(st.w[g["pin_C"]], g["expected_w_AC"], rel_tol=1e-15)
    # a second round adds w1 * slack / WNS for every occurrence
    ref.pairs_update(st, pa, wns=g["wns"], rule=0, w0=g["w0"], w1=g["w1"])
    assert math.isclose(st.w[g["pin_C"]], g["expected_w_AC"] + 0.2 * (1.0 + 0.8), rel_tol=1e-15)


def test_fig2_exp_rule():
    g, pa = _fig2()
    st = ref.PairState(g["num_pins"])
    ref.pairs_update(st, pa, wns=g["wns"], rule=1)
    # exp(500/500) + exp(400/500) through C; B's path: exp(-100/500)
    assert math.isclose(st.w[g["pin_C"]], math.e + math.exp(0.8), rel_tol=1e-15)
    assert math.isclose(st.w[g["pin_B"]], math.exp(-0.2), rel_tol=1e-15)


def test_eq9_sequential_equals_order_free(c1, library):
    nl, st = c1
    pa = ref.extract(nl, library, st, n=-1, k=10)
    s = ref.PairState(nl["num_pins"])
    ref.pairs_update(s, pa, st["wns"], rule=0)
    # order-free: new pair -> w0 + w1 * (sum_all - first) / WNS
    tot, first = {}, {}
    for i, pl in enumerate(ref.path_list(pa)):
        if pa["path_slack"][i] >= 0:
            continue
        r = pa["path_slack"][i] / st["wns"]
        for t in pl[1::2]:
            tot[t] = tot.get(t, 0.0) + r
            first.setdefault(t, r)
    assert set(np.nonzero(s.in_p)[0].tolist()) == set(tot)
    for t in tot:
        assert math.isclose(s.w[t], 10.0 + 0.2 * (tot[t] - first[t]), rel_tol=1e-12)


# ---------------------------------------------------------------------------
# PP loss (Eqs. 8, 10)
# ---------------------------------------------------------------------------
def test_pp_hand_value():
    nl, _ = handnets.diamond_netlist()
    # pairs: A->AND.in1 (pin 3, 48 um apart) w=2; AND.out->FF.D (pin 5, 24 um) w=0.5
    loss, gx, gy = ref.p2p(nl, np.array([3, 5]), np.array([2.0, 0.5]))
    assert loss == 2.0 * 48 ** 2 + 0.5 * 24 ** 2
    # AND (cell 1): +2*2*(48-0) from being the sink, +2*0.5*(48-72) as the driver
    assert gx.tolist() == [0.0, 2 * 2 * 48 + 2 * 0.5 * (48 - 72), 2 * 0.5 * (72 - 48)]
    assert np.all(gy == 0)


def _dyadic_positions(nl, seed):
    rng = np.random.default_rng(seed)
    x = np.round(nl["x"].astype(np.float64) * 1024) / 1024
    y = np.round(nl["y"].astype(np.float64) * 1024) / 1024
    return x.astype(np.float32), y.astype(np.float32), rng


def test_pp_gradient_fd_and_invariance(c1, library):
    nl, st = c1
    pa = ref.extract(nl, library, st, n=-1, k=10)
    ps = ref.PairState(nl["num_pins"])
    ref.pairs_update(ps, pa, st["wns"])
    sinks, w = ps.pairs()
    x, y, rng = _dyadic_positions(nl, 5)
    loss, gx, gy = ref.p2p(nl, sinks, w, x, y)
    h = 2.0 ** -10
    touched = np.nonzero(gx != 0)[0]
    for c in rng.choice(touched, 20, replace=False):
        for arr, g in ((x, gx), (y, gy)):
            a = arr.copy(); a[c] += h
            lp = ref.p2p(nl, sinks, w, *((a, y) if arr is x else (x, a)))[0]
            a[c] -= 2 * h
            lm = ref.p2p(nl, sinks, w, *((a, y) if arr is x else (x, a)))[0]
            fd = (lp - lm) / (2 * h)
            assert abs(fd - g[c]) <= 1e-6 * max(1.0, abs(g[c]))
    # moving every cell and port by the same amount leaves PP unchanged
    nl2 = dict(nl)
    port = nl["pin_cell"] < 0
    nl2["pin_off_x"] = nl["pin_off_x"] + np.where(port, 3.0, 0.0).astype(np.float32)
    l2 = ref.p2p(nl2, sinks, w, x + np.float32(3.0), y)[0]
    assert math.isclose(l2, loss, rel_tol=1e-9)


def test_pp_gradient_sums_to_zero_without_ports():
    # a port-free loop of buffers between two flip-flops
    cells = [(7, 1), (0, 1), (1, 1), (7, 1)]
    # FF0 D0 Q1; B1 in2 out3; B2 in4 out5; FF3 D6 Q7
    nets = [(1, [2]), (3, [4]), (5, [6]), (7, [0])]
    nl, _ = handnets.build(cells, 0, nets, [1.5, 10.25, 30.0, 47.0], [2.0, -4.0, 8.5, 1.0],
                           off_x=np.linspace(-0.5, 0.5, 8), off_y=np.linspace(0.4, -0.4, 8))
    loss, gx, gy = ref.p2p(nl, np.array([2, 4, 6, 0]), np.array([1.0, 3.0, 0.5, 2.0]))
    assert abs(gx.sum()) < 1e-12 and abs(gy.sum()) < 1e-12


# ---------------------------------------------------------------------------
# smoothed TNS
# ---------------------------------------------------------------------------
def test_stns_chain_equals_hard_tns():
    # with one input per cell the log-sum-exp is exact: smoothed arrival = arrival
    nl, _ = handnets.chain_netlist()
    lib = handnets.dyadic_library()
    st = ref.sta(nl, lib)
    g = 10.0
    v, gx, gy = ref.stns(nl, lib, st, gamma=g)
    s = -8.25
    assert math.isclose(v, -g * math.log1p(math.exp(-s / g)), rel_tol=1e-15)


def _lse_diamond(flip):
    """Port A (0, 0) -> BUF (cell 0, x = 16) -> AND.in0 and A -> AND.in1
    (AND = cell 1, type 2, x = 48) -> FF (cell 2, x = 80).D; clock 56 ps.
    Pins: BUF in 0 out 1; AND in0 2 in1 3 out 4; FF D 5 Q 6; port 7.  With
    flip the AND's two inputs swap nets, so the critical one is in0."""
    cells = [(0, 1), (2, 2), (7, 1)]
    a_direct, a_buf = (2, 3) if flip else (3, 2)
    nets = [(7, [0, a_direct]), (1, [a_buf]), (4, [5]), (6, [])]
    return handnets.build(cells, 1, nets, [16.0, 48.0, 80.0], [0.0, 0.0, 0.0], port_xy=[(0.0, 0.0)],
                          clock_period=56.0)[0], a_direct, a_buf


@pytest.mark.parametrize("flip", [False, True])
@pytest.mark.parametrize("g", [10.0, 3.0])
def test_stns_two_input_closed_form(flip, g):
    # The smoothed arrival at a two-input cell is m + g ln(1 + exp(-D / g))
    # (D the gap between the two arrivals through the arcs), and its adjoint
    # splits the output's sensitivity over the inputs by the softmax weights.
    # Every value below is worked out by hand from the dyadic library:
    #   wires: A->BUF 16 um (4 ps), BUF->AND 32 um (16 ps), A->AND 48 um
    #   (36 ps), AND->FF 32 um (16 ps); loads 2 + 32/4 = 10 fF;
    #   BUF arc 4 + 10/4 + 10/64 = 6.65625 ps, AND arcs 6 + 2.5 + 10/64.
    nl, a_direct, a_buf = _lse_diamond(flip)
    lib = handnets.dyadic_library()
    st = ref.sta(nl, lib)
    a_via_buf = 4.0 + 6.65625 + 16.0 + 8.65625   # 35.3125
    a_dir = 36.0 + 8.65625                        # 44.65625
    assert st["at"][4] == a_dir and st["crit"][1] == (0 if flip else 1)
    D = a_dir - a_via_buf
    at_out = a_dir + g * math.log(1.0 + math.exp(-D / g))
    s_end = 56.0 - (at_out + 16.0)
    z = -s_end / g
    value = -g * (max(z, 0.0) + math.log1p(math.exp(-abs(z))))
    v, gx, gy = ref.stns(nl, lib, st, gamma=g)
    assert math.isclose(v, value, rel_tol=4e-15), (v, value)
    # adjoint: d value / d AT~(FF.D) = -sigmoid(z); softmax split at the AND
    ab_end = -1.0 / (1.0 + math.exp(-z))
    w_buf = math.exp((a_via_buf - at_out) / g)
    w_dir = math.exp((a_dir - at_out) / g)
    assert math.isclose(w_buf + w_dir, 1.0, rel_tol=1e-14)
    # d delay / d L = 2 kappa L = L / 32 (kappa = 1/64); every wire runs in
    # +x from driver to sink, so d L / d x_driver = -1 and d L / d x_sink = +1
    gx0 = ab_end * w_buf * (16.0 / 32) - ab_end * w_buf * (32.0 / 32)
    gx1 = ab_end * w_dir * (48.0 / 32) + ab_end * w_buf * (32.0 / 32) - ab_end * (32.0 / 32)
    gx2 = ab_end * (32.0 / 32)
    for got, want in zip(gx, (gx0, gx1, gx2)):
        assert math.isclose(got, want, rel_tol=1e-14, abs_tol=1e-16), (gx, (gx0, gx1, gx2))
    assert np.all(gy == 0.0)  # every wire is horizontal: sign(0) = 0
    # the magnitudes of the same terms, per cell (the scale of rounding error)
    _, _, _, ax, ay = ref.stns(nl, lib, st, gamma=g, with_abs=True)
    a = abs(ab_end)
    want_abs = (a * w_buf * (16.0 / 32 + 32.0 / 32), a * w_dir * (48.0 / 32) + a * w_buf + a, a)
    for got, want in zip(ax, want_abs):
        assert math.isclose(got, want, rel_tol=1e-14), (ax, want_abs)
    assert np.all(ay == 0.0)


def test_stns_tends_to_hard_tns_as_gamma_vanishes(c1, library):
    # g -> 0: the log-sum-exp becomes the maximum and softplus the ramp, so
    # the smoothed TNS becomes the TNS of Eq. 4
    nl, st = c1
    v, _, _ = ref.stns(nl, library, st, gamma=1e-6)
    assert st["tns"] < 0
    assert abs(v - st["tns"]) <= 1e-9 * abs(st["tns"]), (v, st["tns"])
    v1, _, _ = ref.stns(nl, library, st, gamma=1.0)
    assert v1 < v  # a larger temperature only lowers it (both terms add)


def test_stns_bounds_and_fd(c1, library):
    nl, st = c1
    g = 10.0
    x, y, rng = _dyadic_positions(nl, 7)
    st = ref.sta(nl, library, x, y)
    v, gx, gy = ref.stns(nl, library, st, gamma=g, x=x, y=y)
    E = ref.endpoint_pins(nl)
    es = st["slack"][E]
    tns_all = np.minimum(es, 0).sum()
    # LSE adds at most g*ln(fan-in) per level, softplus at most g*ln 2
    bound = len(E) * g * math.log(2) + len(E) * nl["depth"] * g * math.log(4)
    assert v <= tns_all + 1e-9
    assert tns_all - v <= bound
    # finite differences away from the |dx| kink
    h = 2.0 ** -10
    g_ = Graph(nl)
    ok = []
    for c in rng.permutation(nl["num_cells"])[:400]:
        pins = np.nonzero(nl["pin_cell"] == c)[0]
        close = False
        for p in pins:
            others = ([g_.driver[p]] if g_.driver[p] >= 0 else []) + g_.sinks.get(int(p), [])
            for q in others:
                px = (0 if nl["pin_cell"][p] < 0 else x[nl["pin_cell"][p]]) + nl["pin_off_x"][p]
                qx = (0 if nl["pin_cell"][q] < 0 else x[nl["pin_cell"][q]]) + nl["pin_off_x"][q]
                py = (0 if nl["pin_cell"][p] < 0 else y[nl["pin_cell"][p]]) + nl["pin_off_y"][p]
                qy = (0 if nl["pin_cell"][q] < 0 else y[nl["pin_cell"][q]]) + nl["pin_off_y"][q]
                if abs(px - qx) < 10 * h or abs(py - qy) < 10 * h:
                    close = True
        if not close and (gx[c] != 0 or gy[c] != 0):
            ok.append(c)
        if len(ok) == 15:
            break
    assert len(ok) >= 5
    for c in ok:
        for axis in (0, 1):
            a = (x if axis == 0 else y).copy()
            a[c] += h
            vp = ref.stns(nl, library, st, g, *((a, y) if axis == 0 else (x, a)))[0]
            a[c] -= 2 * h
            vm = ref.stns(nl, library, st, g, *((a, y) if axis == 0 else (x, a)))[0]
            fd = (vp - vm) / (2 * h)
            gr = (gx if axis == 0 else gy)[c]
            assert abs(fd - gr) <= 1e-5 * max(1e-3, abs(gr)), (c, axis, fd, gr)


# ---------------------------------------------------------------------------
# weighted-average wirelength
# ---------------------------------------------------------------------------
def test_wa_two_pin_closed_form():
    cells = [(0, 1), (7, 1)]
    # B in0 out1; FF D2 Q3
    nets = [(1, [2]), (3, [0])]
    for dx, dy in ((7.0, 3.0), (0.5, -12.0), (40.0, 0.0)):
        nl, _ = handnets.build(cells, 0, nets, [0.0, dx], [0.0, dy])
        g = 5.0
        v, gx, gy = ref.wa(nl, gamma=g)
        f = lambda d: abs(d) * math.tanh(abs(d) / (2 * g))
        assert math.isclose(v, 2 * (f(dx) + f(dy)), rel_tol=1e-13)


def test_wa_tends_to_hpwl_and_fd(c1):
    nl, _ = c1
    x, y, rng = _dyadic_positions(nl, 9)
    hp = 0.0
    ptr, pins = nl["net_ptr"], nl["net_pins"]
    px = np.where(nl["pin_cell"] >= 0, x[np.maximum(nl["pin_cell"], 0)], 0) + nl["pin_off_x"]
    py = np.where(nl["pin_cell"] >= 0, y[np.maximum(nl["pin_cell"], 0)], 0) + nl["pin_off_y"]
    for n in range(nl["num_nets"]):
        q = pins[ptr[n]:ptr[n + 1]]
        hp += px[q].max() - px[q].min() + py[q].max() - py[q].min()
    v = ref.wa(nl, 1e-3, x, y)[0]
    assert abs(v - hp) < 1e-6 * hp
    g = 5.0
    v, gx, gy = ref.wa(nl, g, x, y)
    assert v < hp
    h = 2.0 ** -10
    for c in rng.choice(nl["num_cells"], 10, replace=False):
        a = x.copy(); a[c] += h
        vp = ref.wa(nl, g, a, y)[0]
        a[c] -= 2 * h
        vm = ref.wa(nl, g, a, y)[0]
        assert abs((vp - vm) / (2 * h) - gx[c]) <= 1e-6 * max(1.0, abs(gx[c]))


def test_wa_magnitudes_bound_the_gradient(c1):
    """The per-cell magnitude sums (the rounding scale of the WA gradient) are
    at least the gradient's magnitude, and for a lone two-pin net they are
    the derivative's four summands, computable by hand."""
    nl, _ = c1
    v, gx, gy, ax, ay = ref.wa(nl, 5.0, with_abs=True)
    assert np.all(ax >= np.abs(gx) * (1 - 1e-12)) and np.all(ay >= np.abs(gy) * (1 - 1e-12))
    cells = [(0, 1), (7, 1)]
    nets = [(1, [2]), (3, [0])]
    g, d = 5.0, 7.0
    nl2, _ = handnets.build(cells, 0, nets, [0.0, d], [0.0, 0.0])
    _, gx2, _, ax2, _ = ref.wa(nl2, g, with_abs=True)
    # two pins at 0 and d: weights a = (e^{-d/g}, 1) / (1 + e^{-d/g}); the
    # mean fp = d / (1 + e^{-d/g}); pin 0's summands (both nets' pin on
    # cell 0 count once per net: cell 0 has one pin on each net)
    e = math.exp(-d / g)
    a0, fp = e / (1 + e), d / (1 + e)
    b0, fm = 1 / (1 + e), d * e / (1 + e)
    mag0 = a0 * (1 + abs(0 - fp) / g) + b0 * (1 + abs(0 - fm) / g)
    assert math.isclose(ax2[0], 2 * mag0, rel_tol=1e-12)
    assert abs(gx2[0]) <= ax2[0]


def test_zero_slack_endpoint_is_not_violated():
    # the chain's endpoint arrives at 40.25 ps: a clock of 40.25 gives slack 0
    nl, _ = handnets.chain_netlist()
    st = ref.sta(nl, handnets.dyadic_library(), clock_period=40.25)
    assert st["slack"][4] == 0.0
    assert (st["wns"], st["tns"], st["n_fail"]) == (0.0, 0.0, 0)


def test_critical_input_tie_takes_lowest_arc_index():
    # two ports 24 um from a 2-input cell: both arcs arrive at exactly the same time
    cells = [(1, 2), (7, 1)]
    # AND in0 0 in1 1 out 2; FF D3 Q4; ports 5 (at (0,0)) and 6 (at (48,0))
    nets = [(5, [0]), (6, [1]), (2, [3]), (4, [])]
    nl, _ = handnets.build(cells, 2, nets, [24.0, 48.0], [0.0, 0.0],
                           port_xy=[(0.0, 0.0), (48.0, 0.0)], clock_period=10.0)
    lib = handnets.dyadic_library()
    st = ref.sta(nl, lib)
    assert st["at"][0] + st["darc"][0] == st["at"][1] + st["darc"][1]
    assert st["crit"][0] == 0
    pa = ref.extract(nl, lib, st, n=-1, k=2)
    # equal slacks: rank 0 is the critical (lowest-index) arc's path
    assert ref.path_list(pa) == [[5, 0, 2, 3], [6, 1, 2, 3]]
