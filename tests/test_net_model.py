"""Pins for the oracle's second net model: the Elmore delay of a star RC net
with PERI slew degradation at the sinks (a fuller model of the RC wires of
Eq. 7, as an RC-tree timer computes them).

Each check fixes the model against something computed another way: the first
moment of the discretised RC network solved as a linear system, the 10-90%
time of a numerically integrated single-pole step response, the lumped model
in the limit of pins without capacitance, and the zero-length wire."""
import math

import numpy as np
import pytest
from scipy.integrate import solve_ivp

from oracle import ref
from paper_2503_11674_amd import netgen
from tests import handnets
from tests.bruteforce import Graph
from tests.conftest import with_clock


def _lib(library, **kw):
    lib = dict(library)
    lib["net_model"] = 1
    lib.update(kw)
    return lib


def _star(port_xy=(0.0, 0.0), input_slew=10.0):
    """A port drives the inputs of three single-input cells of types 0, 3 and
    5 (distinct pin capacitances); each drives a flip-flop just to its right.
    Pins: cell c in 2c, out 2c+1 (c < 3); FF D 6/8/10, Q 7/9/11; port 12."""
    cells = [(0, 1), (3, 1), (5, 1), (7, 1), (7, 1), (7, 1)]
    cx = [10.0, 20.0, -30.0]
    cy = [0.0, 17.5, 50.0]
    x = cx + [v + 5.0 for v in cx]
    y = cy + cy
    nets = [(12, [0, 2, 4]), (1, [6]), (3, [8]), (5, [10]), (7, []), (9, []), (11, [])]
    nl, ids = handnets.build(cells, 1, nets, x, y, port_xy=[port_xy], clock_period=100.0,
                             input_slew=input_slew)
    return nl, [0, 2, 4], 12


def _pin_xy(nl, p):
    c = nl["pin_cell"][p]
    bx = 0.0 if c < 0 else float(nl["x"][c])
    by = 0.0 if c < 0 else float(nl["y"][c])
    return bx + float(nl["pin_off_x"][p]), by + float(nl["pin_off_y"][p])


def _first_moment_of_star(lengths, caps, r, c, m):
    """Elmore delays of the sinks of a star net, by the first moment of the
    impulse response of the discretised network: each branch is m equal
    RC segments, each segment's capacitance split between its two ends, the
    sink's pin capacitance at the far end; the driver is an ideal source.
    With G the conductance matrix of the non-source nodes and C their
    capacitances, the first moments solve G m1 = C 1."""
    nb = len(lengths)
    n = nb * m
    G = np.zeros((n, n))
    C = np.zeros(n)
    for b, (L, cp) in enumerate(zip(lengths, caps)):
        g = m / (r * L)
        for j in range(m):
            i = b * m + j
            # segment j joins node j-1 (the source for j = 0) to node j
            G[i, i] += g
            if j > 0:
                G[i - 1, i - 1] += g
                G[i, i - 1] -= g
                G[i - 1, i] -= g
            C[i] += 0.5 * c * L / m
            if j > 0:
                C[i - 1] += 0.5 * c * L / m
        C[b * m + m - 1] += cp
    m1 = np.linalg.solve(G, C)
    return np.array([m1[b * m + m - 1] for b in range(nb)])


@pytest.mark.parametrize("m", [1, 3, 8])
def test_elmore_delay_is_the_first_moment_of_the_rc_network(library, m):
    nl, sinks, port = _star()
    lib = _lib(library)
    st = ref.sta(nl, lib)
    px, py = _pin_xy(nl, port)
    lengths = []
    for t in sinks:
        tx, ty = _pin_xy(nl, t)
        lengths.append(abs(px - tx) + abs(py - ty))
    caps = [float(lib["pin_cap"][nl["cell_type"][nl["pin_cell"][t]]]) for t in sinks]
    assert len(set(caps)) == 3  # the three sinks see different pin capacitances
    r, c, scale = (float(np.float32(lib[k])) for k in ("r_per_um", "c_per_um", "delay_scale"))
    want = scale * _first_moment_of_star(lengths, caps, r, c, m)
    got = st["dnet"][sinks]
    assert np.allclose(got, want, rtol=1e-11, atol=0), (got, want)
    # the driver's load is the net's total capacitance in either model
    assert math.isclose(st["load"][port], sum(caps) + c * sum(lengths), rel_tol=1e-12)
    st0 = ref.sta(nl, library)
    assert st0["load"][port] == st["load"][port]


def test_single_pole_wire_transition_is_its_10_90_percent_time(library):
    # without wire capacitance every branch is one resistor charging the sink
    # pin: a single pole whose time constant is the Elmore delay.  A step at
    # the driver (input transition 0) leaves the sink with exactly the 10-90%
    # rise time of that pole.
    nl, sinks, port = _star(input_slew=0.0)
    lib = _lib(library, c_per_um=np.float32(0.0), r_per_um=np.float32(100.0))
    st = ref.sta(nl, lib)
    for t in sinks:
        tau = st["dnet"][t]
        assert tau > 1.0

        def hit(level):
            ev = lambda _t, v: v[0] - level
            ev.terminal = False
            return ev

        sol = solve_ivp(lambda _t, v: [(1.0 - v[0]) / tau], (0.0, 10.0 * tau), [0.0],
                        events=[hit(0.1), hit(0.9)], rtol=1e-12, atol=1e-14)
        t10, t90 = sol.t_events[0][0], sol.t_events[1][0]
        assert math.isclose(st["slew"][t], t90 - t10, rel_tol=1e-7), (st["slew"][t], t90 - t10)
        assert st["slew"][port] == 0.0


def test_ramp_through_a_single_pole_wire_is_near_peri(library):
    # a ramp into a single-pole wire: the exact 10-90% time at the sink, by
    # integrating the response, is within the published accuracy of PERI's
    # root sum of squares (a few percent) across input/wire ratios, far from
    # what a plain sum or the larger of the two would give
    s_in = 20.0
    nl, sinks, port = _star(input_slew=s_in)
    lib = _lib(library, c_per_um=np.float32(0.0), r_per_um=np.float32(100.0))
    st = ref.sta(nl, lib)
    ramp = s_in / 0.8  # 0-100% duration of a ramp whose 10-90% time is s_in
    ratios = []
    for t in sinks:
        tau = st["dnet"][t]

        def hit(level):
            return lambda _t, v: v[0] - level

        sol = solve_ivp(lambda tt, v: [(min(tt / ramp, 1.0) - v[0]) / tau], (0.0, ramp + 40.0 * tau), [0.0],
                        events=[hit(0.1), hit(0.9)], rtol=1e-11, atol=1e-13, max_step=ramp / 200)
        exact = sol.t_events[1][0] - sol.t_events[0][0]
        w = math.log(9.0) * tau
        assert abs(st["slew"][t] / exact - 1) < 0.03, (t, st["slew"][t], exact)
        assert abs((s_in + w) / exact - 1) > 0.1 or abs(max(s_in, w) / exact - 1) > 0.1
        ratios.append(s_in / w)
    assert min(ratios) < 1.0 < max(ratios)  # both regimes are covered


def test_zero_length_wire_passes_the_transition_through(library):
    # the first cell's input sits on the port: no wire, no delay, no degradation
    nl, sinks, port = _star(input_slew=23.0)
    nl["x"][0], nl["y"][0] = 0.0, 0.0
    st = ref.sta(nl, _lib(library))
    assert st["dnet"][sinks[0]] == 0.0
    assert st["slew"][sinks[0]] == 23.0
    assert st["at"][sinks[0]] == 0.0
    # the other sinks are degraded, and the degradation grows with the wire
    d = st["dnet"][sinks[1:]]
    s = st["slew"][sinks[1:]]
    assert np.all(s > 23.0)
    assert (d[0] < d[1]) == (s[0] < s[1])


def test_models_differ_by_the_distributed_half_without_pin_capacitance(library):
    # a uniform line charges through half its own resistance on average: with
    # no pin capacitance the Elmore delay is half of the lumped r*c*L^2
    nl = with_clock(netgen.make_netlist(netgen.CONFIGS["C1"]), library)
    lib0 = dict(library, pin_cap=np.zeros_like(library["pin_cap"]))
    st0 = ref.sta(nl, lib0)
    st1 = ref.sta(nl, _lib(lib0))
    sink = np.nonzero(st0["dnet"] > 0)[0]
    assert sink.size > 1000
    assert np.allclose(st1["dnet"][sink], 0.5 * st0["dnet"][sink], rtol=1e-14, atol=0)
    assert np.array_equal(st1["load"], st0["load"])


def test_degraded_transitions_feed_the_cell_arcs(library):
    # on a generated design: every sink's transition lies between its
    # driver's and driver's + ln 9 * delay (a root sum of squares of the two),
    # and every cell arc is looked up at the sink's own (degraded) transition
    nl = with_clock(netgen.make_netlist(netgen.CONFIGS["C1"]), library)
    lib = _lib(library)
    st = ref.sta(nl, lib)
    g = Graph(nl)
    sl, dn = st["slew"], st["dnet"]
    w = math.log(9.0) * dn
    checked = 0
    for t in range(g.P):
        u = g.driver[t]
        if u < 0:
            continue
        lo = max(sl[u], w[t])
        assert lo - 1e-12 <= sl[t] <= sl[u] + w[t] + 1e-12
        if w[t] > 0:
            assert sl[t] > sl[u]
        checked += 1
    assert checked > 1000
    n_deg = 0
    for c in range(nl["num_cells"]):
        if nl["cell_is_ff"][c]:
            continue
        o = nl["cell_out_pin"][c]
        ty = int(nl["cell_type"][c])
        ins = nl["cell_in_pins"][nl["cell_in_ptr"][c]:nl["cell_in_ptr"][c + 1]]
        dl = ref.lut_eval(lib["slew_axis"][ty], lib["load_axis"][ty], lib["delay_lut"][ty], sl[ins],
                          np.full(len(ins), st["load"][o]))
        so = ref.lut_eval(lib["slew_axis"][ty], lib["load_axis"][ty], lib["slew_lut"][ty], sl[ins],
                          np.full(len(ins), st["load"][o]))
        assert np.allclose(st["darc"][ins], dl, rtol=1e-13, atol=1e-12)
        assert math.isclose(sl[o], so.max(), rel_tol=1e-13)
        n_deg += int(np.any(sl[ins] != sl[[g.driver[i] for i in ins]]))
    assert n_deg > 100
    # the model changes the timing: the degraded transitions are slower
    st0 = ref.sta(nl, library)
    assert not np.allclose(st["at"], st0["at"])


def test_stns_gradient_under_the_elmore_model_matches_finite_differences(library):
    nl = with_clock(netgen.make_netlist(netgen.CONFIGS["C1"]), library)
    lib = _lib(library)
    st = ref.sta(nl, lib)
    g = 10.0
    v, gx, gy = ref.stns(nl, lib, st, gamma=g)
    E = ref.endpoint_pins(nl)
    es = st["slack"][E]
    assert v <= np.minimum(es, 0).sum() + 1e-9
    h = 2.0 ** -10
    x = np.asarray(nl["x"], np.float64)
    y = np.asarray(nl["y"], np.float64)
    gr_ = Graph(nl)

    def near_kink(c):
        # a pin of c level with a pin it connects to, in x or y: |dx| kink
        for p in np.nonzero(nl["pin_cell"] == c)[0]:
            others = ([gr_.driver[p]] if gr_.driver[p] >= 0 else []) + gr_.sinks.get(int(p), [])
            px, py = _pin_xy(nl, p)
            for q in others:
                qx, qy = _pin_xy(nl, q)
                if abs(px - qx) < 10 * h or abs(py - qy) < 10 * h:
                    return True
        return False

    # the cells with the largest gradients, where a wrong term cannot hide
    order = np.argsort(-(np.abs(gx) + np.abs(gy)))
    cells = [int(c) for c in order[:40] if not near_kink(c)][:10]
    assert len(cells) == 10 and abs(gx[cells[-1]]) + abs(gy[cells[-1]]) > 1e-3
    for c in cells:
        for axis, a0 in ((0, x), (1, y)):
            a = a0.copy()
            a[c] += h
            vp = ref.stns(nl, lib, st, g, *((a, y) if axis == 0 else (x, a)))[0]
            a[c] -= 2 * h
            vm = ref.stns(nl, lib, st, g, *((a, y) if axis == 0 else (x, a)))[0]
            fd = (vp - vm) / (2 * h)
            gr = (gx if axis == 0 else gy)[c]
            assert abs(fd - gr) <= 1e-5 * max(1e-3, abs(gr)), (c, axis, fd, gr)
