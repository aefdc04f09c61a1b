"""Pins for the oracle's early (hold) analysis: brute force over every path of
small random DAGs (earliest arrival = minimum over start-to-pin paths), a hand
diamond in exact binary fractions, the single-fan-in chain (early = late),
and early <= late at every pin of a generated design (the tables grow with
the transition)."""
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


@pytest.mark.parametrize("seed", range(8))
@pytest.mark.parametrize("net_model", [0, 1, 2])
def test_early_arrivals_are_the_shortest_paths(seed, net_model, library):
    lib = dict(library, net_model=net_model)
    nl = _tiny(seed)
    late = ref.sta(nl, lib, clock_period=0.0)
    early = ref.sta_early(nl, lib)
    g = Graph(nl)
    checked = 0
    for v in range(g.P):
        ps = g.paths_to(v)
        if not ps:  # unreachable from any start point
            assert early["at"][v] == math.inf
            continue
        want = min(early["at"][p[0]] + g.path_delay(p, late["dnet"], early["darc"]) for p in ps)
        assert math.isclose(early["at"][v], want, rel_tol=1e-12, abs_tol=1e-9), (v, early["at"][v], want)
        checked += 1
    assert checked > 20


def test_hand_diamond_takes_the_short_branch():
    # port -> BUF -> AND.in0 (9 + 6.625 + 9 = 24.625) and port -> AND.in1
    # (36): early 24.625 + 8.625 = 33.25 at the AND, 42.25 at the D pin
    # (late: 36 + 8.625 + 9 = 53.625)
    nl, _ = handnets.diamond_netlist()
    lib = handnets.dyadic_library()
    e = ref.sta_early(nl, lib, hold=50.0)
    late = ref.sta(nl, lib)
    assert e["at"][4] == 33.25 and late["at"][4] == 44.625
    assert e["at"][5] == 42.25 and late["at"][5] == 53.625
    assert e["hold_slack"][5] == 42.25 - 50.0
    assert (e["whs"], e["ths"], e["n_hold_fail"]) == (-7.75, -7.75, 1)
    assert e["darc"][2] == 8.625 and e["darc"][3] == 8.625
    ok = ref.sta_early(nl, lib, hold=42.25)
    assert (ok["whs"], ok["ths"], ok["n_hold_fail"]) == (0.0, 0.0, 0)  # slack exactly 0 is met


@pytest.mark.parametrize("net_model", [0, 1, 2])
def test_single_fan_in_chain_has_equal_early_and_late(net_model):
    nl, _ = handnets.chain_netlist()
    lib = dict(handnets.dyadic_library(), net_model=net_model)
    e = ref.sta_early(nl, lib)
    late = ref.sta(nl, lib)
    assert np.array_equal(e["at"], late["at"]) and np.array_equal(e["slew"], late["slew"])


@pytest.mark.parametrize("net_model", [0, 1, 2])
def test_early_bounds_late_on_a_generated_design(net_model, library):
    lib = dict(library, net_model=net_model)
    nl = with_clock(netgen.make_netlist(netgen.CONFIGS["C1"]), lib)
    late = ref.sta(nl, lib)
    e = ref.sta_early(nl, lib)
    fin = np.isfinite(late["at"])
    assert np.array_equal(fin, np.isfinite(e["at"]))
    assert np.all(e["at"][fin] <= late["at"][fin] + 1e-9)
    assert np.all(e["slew"][fin] <= late["slew"][fin] + 1e-9)
    assert np.sum(e["at"][fin] < late["at"][fin] - 1e-6) > 100  # multi-input cells differ
    # hold: with the hold time at the 5 % quantile of the early D arrivals,
    # the count and sums follow from the D pins' slacks
    D = ref.endpoint_pins(nl)
    hold = float(np.quantile(e["at"][D], 0.05))
    h = ref.sta_early(nl, lib, hold=hold)
    hs = h["hold_slack"][D]
    assert np.allclose(hs, e["at"][D] - hold, rtol=0, atol=1e-9)
    assert h["n_hold_fail"] == int(np.sum(hs < 0)) > 0
    assert math.isclose(h["ths"], float(hs[hs < 0].sum()), rel_tol=1e-12)
    assert h["whs"] == hs.min()
    off = np.ones(nl["num_pins"], bool)
    off[D] = False
    assert np.all(np.isinf(h["hold_slack"][off]))


def test_best_case_transition_at_a_two_input_cell():
    # output transition table s/2 + 5: the port's 40 ps reaches AND.in1
    # directly, the BUF turns it into 25 ps for AND.in0; the AND's output
    # transition is 17.5 early (from in0) and 25 late (from in1), and the
    # arc delays follow the input transitions: 6 + 25/4 + 8/64 = 12.375 and
    # 6 + 40/4 + 8/64 = 16.125
    nl, _ = handnets.diamond_netlist()
    nl["input_slew"] = np.float32(40.0)
    lib = handnets.dyadic_library()
    sa = netgen.SLEW_AXIS.astype(np.float64)
    lib["slew_lut"] = np.broadcast_to((sa[:, None] / 2 + 5)[None], (8, 7, 7)).astype(np.float32).copy()
    e = ref.sta_early(nl, lib)
    late = ref.sta(nl, lib)
    assert e["slew"][1] == 25.0 and e["slew"][2] == 25.0 and e["slew"][3] == 40.0
    assert e["slew"][4] == 17.5 and late["slew"][4] == 25.0
    assert e["slew"][5] == 17.5 and late["slew"][5] == 25.0  # the D pin sees its driver's
    assert e["darc"][2] == 12.375 and e["darc"][3] == 16.125
    # BUF: 4 + 40/4 + 8/64 = 14.125, so in0 arrives at 9 + 14.125 + 9
    assert e["darc"][0] == 14.125
    assert e["at"][4] == min(9 + 14.125 + 9 + 12.375, 36 + 16.125) == 44.5
