"""Pins for the oracle's rise / fall timing (both transitions of every pin,
cell arcs by unateness) and its report_timing_endpoint(n, 1):

* with the fall tables equal to the rise tables and every arc positive
  unate, both transitions reduce to the single-transition timer (itself
  pinned by hand chains and brute force), bitwise, paths included;
* a hand chain of two inverting cells in exact binary fractions (arrivals,
  required times, slacks, WNS / TNS and the path with its transitions);
* brute force over every (path, transition) sequence of small random DAGs
  that the arcs' unateness allows: arrival = the longest such path into a
  (pin, transition), required time = the shortest one out of it, using the
  graph-based transitions for the arc delays;
* on a generated design: every extracted path's delay, summed along its
  pins and transitions, is its endpoint's arrival, and its slack the
  endpoint's slack."""
import math

import numpy as np
import pytest

from oracle import ref
from paper_2503_11674_amd import netgen
from tests import handnets
from tests.bruteforce import Graph
from tests.conftest import with_clock


def _tiny(seed, n=24, depth=5):
    cfg = netgen.NetlistConfig("tiny", n, ff_frac=0.25, depth=depth, fanin_lo=1, fanin_hi=3,
                               fanout_cap=6, die=200.0, seed=seed)
    return netgen.make_netlist(cfg)


def _same_tables(lib):
    out = dict(lib)
    out["delay_fall"] = lib["delay_lut"].copy()
    out["slew_fall"] = lib["slew_lut"].copy()
    out["unate"] = np.zeros(int(lib["num_types"]), np.int32)
    return out


@pytest.mark.parametrize("net_model", [0, 1, 2])
def test_equal_tables_and_positive_arcs_reduce_to_one_transition(net_model, library):
    lib = dict(library, net_model=net_model)
    nl = with_clock(netgen.make_netlist(netgen.CONFIGS["C1"]), lib)
    st = ref.sta(nl, lib)
    rf = ref.sta_rf(nl, _same_tables(lib))
    for key in ("at", "slew", "rat", "slack"):
        assert np.array_equal(rf[key][:, 0], st[key]) and np.array_equal(rf[key][:, 1], st[key]), key
    comb = np.asarray(nl["cell_is_ff"]) == 0
    assert np.array_equal(rf["crit"][comb, 0], 2 * st["crit"][comb])
    assert np.array_equal(rf["crit"][comb, 1], 2 * st["crit"][comb] + 1)
    assert (rf["wns"], rf["tns"], rf["n_fail"]) == (st["wns"], st["tns"], st["n_fail"])
    ep = ref.endpoint_pins(nl)
    assert np.array_equal(rf["ep_slack"][ep], st["slack"][ep])
    p1 = ref.extract(nl, lib, st, n=-1, k=1, K=1000)
    p2 = ref.extract_rf(nl, rf, n=-1, K=1000)
    assert p1["num_paths"] == p2["num_paths"] == st["n_fail"]
    for key in ("path_ptr", "path_pins", "path_slack", "path_ep"):
        assert np.array_equal(p1[key], p2[key]), key
    assert np.all(p2["path_tran"] == 0)  # equal slacks: rise


def _rf_dyadic_library():
    """handnets.dyadic_library as the rise tables; falls in exact binary
    fractions too: comb type t falls by (2 + 2t) + s/8 + l/32 with a 12 ps
    output transition, the flip-flop's Q by 24 + s/4 + l/16.  Types 3 and 4
    invert (negative unate)."""
    lib = handnets.dyadic_library()
    sa = netgen.SLEW_AXIS.astype(np.float64)
    la = netgen.LOAD_AXIS.astype(np.float64)
    fall = np.zeros((8, 7, 7))
    for t in range(7):
        fall[t] = (2 + 2 * t) + sa[:, None] / 8 + la[None, :] / 32
    fall[7] = 24 + sa[:, None] / 4 + la[None, :] / 16
    lib["delay_fall"] = fall.astype(np.float32)
    lib["slew_fall"] = np.full((8, 7, 7), 12.0, np.float32)
    unate = np.zeros(8, np.int32)
    unate[3:6] = 1
    unate[6] = 2
    lib["unate"] = unate
    return lib


def test_hand_inverter_chain():
    # port -> INV1 (type 3) -> INV2 (type 4) -> FF.D, 24 um wires: net delay
    # 24^2 / 64 = 9 ps, every load 2 + 24/4 = 8 fF, clock period 48 ps.
    cells = [(3, 1), (4, 1), (7, 1)]
    # pins: INV1 in 0 out 1; INV2 in 2 out 3; FF D 4 Q 5; port 6
    nets = [(6, [0]), (1, [2]), (3, [4]), (5, [])]
    nl, _ = handnets.build(cells, 1, nets, [24.0, 48.0, 72.0], [0.0, 0.0, 0.0], port_xy=[(0.0, 0.0)],
                           clock_period=48.0)
    rf = ref.sta_rf(nl, _rf_dyadic_library())
    at, rat, slack = rf["at"], rf["rat"], rf["slack"]
    # INV1: rise from the input's fall, 9 + (7 + 10/4 + 8/64); fall from its
    # rise, 9 + (8 + 10/8 + 8/32); transitions 10 (rise) and 12 (fall)
    assert tuple(at[1]) == (18.625, 18.5) and tuple(rf["slew"][1]) == (10.0, 12.0)
    assert tuple(at[2]) == (27.625, 27.5)
    # INV2: rise from the fall (slew 12): 27.5 + (8 + 12/4 + 8/64);
    # fall from the rise (slew 10): 27.625 + (10 + 10/8 + 8/32)
    assert tuple(at[3]) == (38.625, 39.125)
    assert tuple(at[4]) == (47.625, 48.125)
    assert tuple(slack[4]) == (0.375, -0.125) and rf["ep_slack"][4] == -0.125
    assert (rf["wns"], rf["tns"], rf["n_fail"]) == (-0.125, -0.125, 1)
    # required: 48 at D, 39 at INV2's output; INV2's input rise must not be
    # later than 39 - 11.5, its fall 39 - 11.125
    assert tuple(rat[3]) == (39.0, 39.0) and tuple(rat[2]) == (27.5, 27.875)
    assert tuple(slack[2]) == (-0.125, 0.375)
    assert tuple(rf["crit"][1]) == (1, 0) and tuple(rf["crit"][0]) == (1, 0)  # input 0, the other transition
    p = ref.extract_rf(nl, rf, n=-1)
    assert p["num_paths"] == 1 and p["path_slack"][0] == -0.125 and p["path_ep"][0] == 4
    assert list(p["path_pins"]) == [6, 0, 1, 2, 3, 4]
    assert list(p["path_tran"]) == [1, 1, 0, 0, 1, 1]


def test_ties_take_the_first_input_and_the_rise():
    # one port drives both inputs of a non-unate cell (type 6) over equal
    # wires: all four (input, transition) candidates of either output
    # transition tie, and the first input's rise sets it
    cells = [(6, 2), (7, 1)]
    # pins: X in0 0 in1 1 out 2; FF D 3 Q 4; port 5
    nets = [(5, [0, 1]), (2, [3]), (4, [])]
    # wires 16 um (4 ps) and 24 um (9 ps), load 8 fF: the output rises at
    # 4 + 12.625 = 16.625 and falls at 4 + 15.5 = 19.5; D falls at 28.5
    nl, _ = handnets.build(cells, 1, nets, [16.0, 40.0], [0.0, 0.0], port_xy=[(0.0, 0.0)], clock_period=28.0)
    rf = ref.sta_rf(nl, _rf_dyadic_library())
    assert rf["at"][0, 0] == rf["at"][1, 0] == rf["at"][0, 1] == rf["at"][1, 1] == 4.0
    assert tuple(rf["at"][2]) == (16.625, 19.5)
    assert tuple(rf["crit"][0]) == (0, 0)
    p = ref.extract_rf(nl, rf, n=-1)
    assert p["num_paths"] == 1 and p["path_slack"][0] == -0.5
    assert list(p["path_pins"]) == [5, 0, 2, 3] and list(p["path_tran"]) == [0, 0, 1, 1]


def _arc_delay(lib, tables, type_, slew, load):
    return float(ref.lut_eval(lib["slew_axis"][type_], lib["load_axis"][type_], tables[type_],
                              np.array([slew]), np.array([load]))[0])


def _rf_arcs(nl, lib, rf, st):
    """Every (pin, transition) -> (pin, transition) arc with its delay, from
    the netlist and the library alone (arc delays at the oracle's graph-based
    transitions and loads)."""
    g = Graph(nl)
    dt = (lib["delay_lut"], lib["delay_fall"])
    arcs = {}
    for v in range(g.P):
        r = g.role[v]
        if r in ("port", "cout", "ffq"):
            for t in g.sinks.get(v, []):
                for y in (0, 1):
                    arcs.setdefault((v, y), []).append(((t, y), st["dnet"][t]))
        elif r == "cin":
            o = g.cell_out_of(v)
            ty = int(nl["cell_type"][nl["pin_cell"][v]])
            u = int(lib["unate"][ty])
            for y in (0, 1):
                for x in (0, 1):
                    if u == 2 or (u == 0 and x == y) or (u == 1 and x != y):
                        arcs.setdefault((v, y), []).append(
                            ((o, x), _arc_delay(lib, dt[x], ty, rf["slew"][v, y], st["load"][o])))
    return g, arcs


@pytest.mark.parametrize("seed", range(6))
def test_brute_force_over_transition_paths(seed, library):
    lib = netgen.make_rf_library(library)
    nl = _tiny(seed)
    nl["clock_period"] = np.float32(150.0)
    st = ref.sta(nl, lib)
    rf = ref.sta_rf(nl, lib)
    g, arcs = _rf_arcs(nl, lib, rf, st)
    # start arrivals: 0 at ports; clock-to-Q by transition at the clock slew
    start = {}
    for v in range(g.P):
        if g.role[v] == "port":
            start[(v, 0)] = start[(v, 1)] = 0.0
        elif g.role[v] == "ffq":
            ty = int(nl["cell_type"][nl["pin_cell"][v]])
            for y, tab in ((0, lib["delay_lut"]), (1, lib["delay_fall"])):
                start[(v, y)] = _arc_delay(lib, tab, ty, float(nl["clock_slew"]), st["load"][v])
    best = {}

    def walk(node, acc):
        if acc <= best.get(node, -math.inf):
            pass
        best[node] = max(best.get(node, -math.inf), acc)
        for nxt, d in arcs.get(node, []):
            walk(nxt, acc + d)

    for node, a0 in start.items():
        walk(node, a0)
    checked = 0
    for v in range(g.P):
        for y in (0, 1):
            want = best.get((v, y), -math.inf)
            got = rf["at"][v, y]
            if want == -math.inf:
                assert got == -math.inf
                continue
            assert math.isclose(got, want, rel_tol=1e-12, abs_tol=1e-9), (v, y, got, want)
            checked += 1
    assert checked > 40
    # required times: the shortest (T - setup - delays) over paths to any D pin
    req = float(nl["clock_period"]) - float(nl["setup"])
    memo = {}

    def rq(node):
        if node in memo:
            return memo[node]
        v, _ = node
        r = req if g.role[v] == "ffd" else math.inf
        for nxt, d in arcs.get(node, []):
            r = min(r, rq(nxt) - d)
        memo[node] = r
        return r

    for v in range(g.P):
        for y in (0, 1):
            want = rq((v, y))
            got = rf["rat"][v, y]
            if want == math.inf:
                assert got == math.inf
            else:
                assert math.isclose(got, want, rel_tol=1e-12, abs_tol=1e-9), (v, y, got, want)


def test_paths_sum_to_their_endpoint_arrival(library):
    lib = netgen.make_rf_library(library)
    nl = netgen.make_netlist(netgen.CONFIGS["C1"])
    nl["clock_period"] = np.float32(0.0)
    rf0 = ref.sta_rf(nl, lib)
    ep = ref.endpoint_pins(nl)
    worst = np.max(rf0["at"][ep], axis=1)
    nl["clock_period"] = np.float32(netgen.clock_period_for_fail_fraction(worst, 0.05))
    st = ref.sta(nl, lib)
    rf = ref.sta_rf(nl, lib)
    assert rf["n_fail"] == len(ep) // 20
    g, arcs = _rf_arcs(nl, lib, rf, st)
    p = ref.extract_rf(nl, rf, n=-1)
    assert p["num_paths"] == rf["n_fail"]
    assert np.all(np.diff(p["path_slack"]) >= 0)
    for i in range(p["num_paths"]):
        pins = p["path_pins"][p["path_ptr"][i]:p["path_ptr"][i + 1]]
        tr = p["path_tran"][p["path_ptr"][i]:p["path_ptr"][i + 1]]
        s0, e = (int(pins[0]), int(tr[0])), (int(pins[-1]), int(tr[-1]))
        total = rf["at"][s0[0], s0[1]]
        for a, b in zip(zip(pins[:-1], tr[:-1]), zip(pins[1:], tr[1:])):
            d = [dd for nxt, dd in arcs[(int(a[0]), int(a[1]))] if nxt == (int(b[0]), int(b[1]))]
            assert len(d) == 1
            total += d[0]
        assert math.isclose(total, rf["at"][e[0], e[1]], rel_tol=1e-12)
        assert math.isclose(p["path_slack"][i], rf["ep_slack"][e[0]], rel_tol=0, abs_tol=0)
        assert rf["slack"][e[0], e[1]] == rf["ep_slack"][e[0]]
