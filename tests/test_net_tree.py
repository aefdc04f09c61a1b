"""Pins for the oracle's third net model: the Elmore delay of an RC tree whose
topology is the net's rectilinear minimum spanning tree (grown from the
driver by Prim's algorithm), with the sink transitions degraded as in the
star model.

Each check fixes the model against something computed another way: the
spanning tree against scipy's minimum spanning tree and against every
spanning tree of small nets (Cayley's enumeration by Pruefer sequences), the
delays against the first moment of the discretised RC network solved as a
linear system, the two-pin nets against the star model, the loads against
the star's (a spanning tree is never longer than the star, itself one), and
the smoothed-TNS gradient against central differences."""
import itertools
import math

import numpy as np
import pytest
from scipy.sparse.csgraph import minimum_spanning_tree

from oracle import ref
from paper_2503_11674_amd import netgen
from tests.conftest import with_clock


def _lib(library, model=2, **kw):
    lib = dict(library)
    lib["net_model"] = model
    lib.update(kw)
    return lib


@pytest.fixture(scope="module")
def c1(library):
    return with_clock(netgen.make_netlist(netgen.CONFIGS["C1"]), library)


def _pins_xy32(nl, pins):
    """(cell, offset) coordinates of pins in single precision."""
    pins = np.asarray(pins)
    c = np.asarray(nl["pin_cell"])[pins]
    x = np.asarray(nl["x"], np.float32)
    y = np.asarray(nl["y"], np.float32)
    bx = np.where(c >= 0, x[np.maximum(c, 0)], np.float32(0))
    by = np.where(c >= 0, y[np.maximum(c, 0)], np.float32(0))
    return bx, by, np.asarray(nl["pin_off_x"], np.float32)[pins], np.asarray(nl["pin_off_y"], np.float32)[pins]


def _fdist_matrix(nl, pins):
    """Pairwise single-precision Manhattan distances, each axis taken as
    (cell difference) + (offset difference)."""
    bx, by, ox, oy = _pins_xy32(nl, pins)
    dx = (bx[:, None] - bx[None, :]) + (ox[:, None] - ox[None, :])
    dy = (by[:, None] - by[None, :]) + (oy[:, None] - oy[None, :])
    return np.abs(dx) + np.abs(dy)


def _pin_xy(nl, p):
    c = nl["pin_cell"][p]
    bx = 0.0 if c < 0 else float(nl["x"][c])
    by = 0.0 if c < 0 else float(nl["y"][c])
    return bx + float(nl["pin_off_x"][p]), by + float(nl["pin_off_y"][p])


def _nets(nl):
    ptr, pins = nl["net_ptr"], nl["net_pins"]
    for n in range(int(nl["num_nets"])):
        yield [int(p) for p in pins[ptr[n]:ptr[n + 1]]]


def _tree_weight(D, parent_of):
    return sum(float(D[i, parent_of[i]]) for i in range(1, D.shape[0]))


def test_tree_is_a_minimum_spanning_tree(c1):
    par = ref.rc_tree(c1)
    checked = brute = 0
    for pins in _nets(c1):
        if len(pins) < 2:
            continue
        idx = {p: i for i, p in enumerate(pins)}
        assert par[pins[0]] == -1
        parent_of = {}
        for i, p in enumerate(pins[1:], 1):
            assert par[p] in idx and par[p] != p
            parent_of[i] = idx[int(par[p])]
        for i in parent_of:  # every sink reaches the driver: a spanning tree
            seen, u = set(), i
            while u != 0:
                assert u not in seen
                seen.add(u)
                u = parent_of[u]
        D = _fdist_matrix(c1, pins).astype(np.float64)
        w = _tree_weight(D, parent_of)
        # scipy drops zero entries as missing edges: coincident pins get a
        # negligible positive weight instead
        ref_w = float(minimum_spanning_tree(np.where(D > 0, D, 1e-300)).sum())
        assert math.isclose(w, ref_w, rel_tol=1e-12, abs_tol=1e-9), (pins, w, ref_w)
        checked += 1
        n = len(pins)
        if 3 <= n <= 6:
            # every labelled tree on n nodes, from its Pruefer sequence
            best = math.inf
            for seq in itertools.product(range(n), repeat=n - 2):
                deg = [1] * n
                for s in seq:
                    deg[s] += 1
                tot = 0.0
                for s in seq:
                    leaf = min(i for i in range(n) if deg[i] == 1)
                    tot += D[leaf, s]
                    deg[leaf] -= 1
                    deg[s] -= 1
                u, v = [i for i in range(n) if deg[i] == 1]
                best = min(best, tot + D[u, v])
            assert math.isclose(w, best, rel_tol=1e-12, abs_tol=1e-9)
            brute += 1
    assert checked > 1000 and brute > 200


def test_ties_go_to_the_first_pin_and_the_first_parent(library):
    # a port at the origin and three sinks listed as (10, 10), (10, 0),
    # (0, 10).  (10, 0) and (0, 10) tie at distance 10 from the port: the one
    # listed first joins first, so (10, 10) hangs from (10, 0) (had (0, 10)
    # joined first, from it).  (0, 10) then lies 10 from the port and 10 from
    # (10, 10): it keeps the parent that reached it first, the port.
    from tests import handnets
    cells = [(0, 1), (0, 1), (0, 1), (7, 1), (7, 1), (7, 1)]
    x = [10.0, 0.0, 10.0, 40.0, 40.0, 40.0]
    y = [0.0, 10.0, 10.0, 0.0, 20.0, 40.0]
    nets = [(12, [4, 0, 2]), (1, [6]), (3, [8]), (5, [10]), (7, []), (9, []), (11, [])]
    nl, _ = handnets.build(cells, 1, nets, x, y, port_xy=[(0.0, 0.0)], clock_period=100.0)
    par = ref.rc_tree(nl)
    # pin 4 at (10, 10), pin 0 at (10, 0), pin 2 at (0, 10)
    assert par[0] == 12 and par[4] == 0 and par[2] == 12


def _first_moment_of_tree(edges, lengths, caps, r, c, m):
    """First moments of the impulse response (Elmore delays) at the tree's
    nodes by a linear solve of the discretised network: node 0 is the driver,
    an ideal source; each edge (parent, child) of length L is m equal RC
    segments, each segment's capacitance split between its ends, and a node's
    pin capacitance sits at the node.  With G the conductance matrix of the
    non-source nodes and C their capacitances, the first moments solve
    G m1 = C 1."""
    n_nodes = len(caps)
    idx = {0: -1}
    for v in range(1, n_nodes):
        idx[v] = v - 1
    n = n_nodes - 1 + len(edges) * (m - 1)
    G = np.zeros((n, n))
    C = np.zeros(n)
    nxt = n_nodes - 1

    def conn(a, b, g):
        if a >= 0:
            G[a, a] += g
        if b >= 0:
            G[b, b] += g
        if a >= 0 and b >= 0:
            G[a, b] -= g
            G[b, a] -= g

    def cap(a, v):
        if a >= 0:
            C[a] += v

    for (p, v), L in zip(edges, lengths):
        chain = [idx[p]]
        for _ in range(m - 1):
            chain.append(nxt)
            nxt += 1
        chain.append(idx[v])
        g = m / (r * L)
        for a, b in zip(chain[:-1], chain[1:]):
            conn(a, b, g)
            cap(a, 0.5 * c * L / m)
            cap(b, 0.5 * c * L / m)
    for v in range(1, n_nodes):
        C[idx[v]] += caps[v]
    m1 = np.linalg.solve(G, C)
    return np.array([m1[idx[v]] for v in range(1, n_nodes)])


@pytest.mark.parametrize("m", [1, 3, 8])
def test_tree_elmore_delay_is_the_first_moment_of_the_rc_network(c1, library, m):
    lib = _lib(library)
    st = ref.sta(c1, lib)
    par = ref.rc_tree(c1)
    r, c, scale = (float(np.float32(lib[k])) for k in ("r_per_um", "c_per_um", "delay_scale"))
    pin_cap = np.asarray(lib["pin_cap"], np.float64)
    deep = 0
    for pins in _nets(c1):
        if len(pins) < 4:
            continue
        idx = {p: i for i, p in enumerate(pins)}
        parent = [idx[int(par[p])] for p in pins[1:]]
        depth = 0
        for i in range(1, len(pins)):
            d, u = 0, i
            while u != 0:
                u, d = parent[u - 1], d + 1
            depth = max(depth, d)
        if depth < 3:
            continue
        xy = [_pin_xy(c1, p) for p in pins]
        lengths = [abs(xy[i][0] - xy[parent[i - 1]][0]) + abs(xy[i][1] - xy[parent[i - 1]][1])
                   for i in range(1, len(pins))]
        if min(lengths) < 1e-3:
            continue
        caps = [0.0] + [float(pin_cap[c1["cell_type"][c1["pin_cell"][p]]]) for p in pins[1:]]
        edges = [(parent[i - 1], i) for i in range(1, len(pins))]
        want = scale * _first_moment_of_tree(edges, lengths, caps, r, c, m)
        got = st["dnet"][pins[1:]]
        assert np.allclose(got, want, rtol=1e-10, atol=0), (pins, got, want)
        # the driver's load is the net's total capacitance
        assert math.isclose(st["load"][pins[0]], sum(caps) + c * sum(lengths), rel_tol=1e-12)
        deep += 1
        if deep == 40:
            break
    assert deep == 40  # nets three or more wires deep


def test_two_pin_nets_and_stars_match_the_star_model(c1, library):
    st1 = ref.sta(c1, _lib(library, 1))
    st2 = ref.sta(c1, _lib(library, 2))
    par = ref.rc_tree(c1)
    n2 = nstar = 0
    for pins in _nets(c1):
        if len(pins) < 2:
            continue
        if all(par[p] == pins[0] for p in pins[1:]):
            s = pins[1:]
            assert np.allclose(st2["dnet"][s], st1["dnet"][s], rtol=1e-14, atol=0)
            assert math.isclose(st2["load"][pins[0]], st1["load"][pins[0]], rel_tol=1e-14)
            n2 += len(pins) == 2
            nstar += len(pins) > 2
    assert n2 > 200 and nstar > 50


def test_tree_is_never_longer_than_the_star(c1, library):
    # the star is a spanning tree too: the minimum one has no more wire, so
    # no driver sees more load; somewhere it is strictly less
    st1 = ref.sta(c1, _lib(library, 1))
    st2 = ref.sta(c1, _lib(library, 2))
    drv = np.asarray([pins[0] for pins in _nets(c1) if len(pins) > 1])
    assert np.all(st2["load"][drv] <= st1["load"][drv] * (1 + 1e-12))
    assert np.sum(st2["load"][drv] < st1["load"][drv] * (1 - 1e-6)) > 100
    # the transitions are degraded by the tree's delays (PERI, as in the star)
    sinks = np.nonzero(st2["dnet"] > 0)[0]
    assert not np.allclose(st2["dnet"][sinks], st1["dnet"][sinks])


def test_stns_gradient_under_the_tree_model_matches_finite_differences(c1, library):
    lib = _lib(library)
    st = ref.sta(c1, lib)
    g = 10.0
    v, gx, gy = ref.stns(c1, lib, st, gamma=g)
    E = ref.endpoint_pins(c1)
    assert v <= np.minimum(st["slack"][E], 0).sum() + 1e-9
    h = 2.0 ** -10
    x = np.asarray(c1["x"], np.float64)
    y = np.asarray(c1["y"], np.float64)
    par0 = ref.rc_tree(c1)
    net_of = {}
    for n, pins in enumerate(_nets(c1)):
        for p in pins:
            net_of[p] = pins

    def near_kink(cell):
        # a pin of the cell level with its tree neighbours in x or y (the
        # |dx| kink), or a move that changes a tree's topology
        for p in np.nonzero(c1["pin_cell"] == cell)[0]:
            pins = net_of.get(int(p), [])
            px, py = _pin_xy(c1, p)
            for q in pins:
                if q == p or (par0[q] != p and par0[p] != q):
                    continue
                qx, qy = _pin_xy(c1, q)
                if abs(px - qx) < 10 * h or abs(py - qy) < 10 * h:
                    return True
        for axis in (0, 1):
            for d in (h, -h):
                a = (x if axis == 0 else y).copy()
                a[cell] += d
                pp = ref.rc_tree(c1, *((a, y) if axis == 0 else (x, a)))
                if not np.array_equal(pp, par0):
                    return True
        return False

    # the cells with the largest gradients, on nets whose tree is not a star
    nonstar = set()
    for pins in _nets(c1):
        if any(par0[p] != pins[0] for p in pins[1:]):
            nonstar.update(int(c1["pin_cell"][p]) for p in pins if c1["pin_cell"][p] >= 0)
    order = np.argsort(-(np.abs(gx) + np.abs(gy)))
    cells = [int(cc) for cc in order[:200] if int(cc) in nonstar and not near_kink(int(cc))][:10]
    assert len(cells) == 10 and abs(gx[cells[-1]]) + abs(gy[cells[-1]]) > 1e-3
    for cc in cells:
        for axis, a0 in ((0, x), (1, y)):
            a = a0.copy()
            a[cc] += h
            vp = ref.stns(c1, lib, st, g, *((a, y) if axis == 0 else (x, a)))[0]
            a[cc] -= 2 * h
            vm = ref.stns(c1, lib, st, g, *((a, y) if axis == 0 else (x, a)))[0]
            fd = (vp - vm) / (2 * h)
            gr = (gx if axis == 0 else gy)[cc]
            assert abs(fd - gr) <= 1e-5 * max(1e-3, abs(gr)), (cc, axis, fd, gr)


def test_stns_gradient_on_a_deep_tree_matches_finite_differences(library):
    # a chain of sinks off one port: every wire's length enters the delays of
    # all sinks below it (the C_below terms of the adjoint)
    from tests import handnets
    n = 5
    cells = [(0, 1)] * n + [(7, 1)] * n
    x = [12.0 * (i + 1) for i in range(n)] + [12.0 * (i + 1) + 3.0 for i in range(n)]
    y = [1.5 * i * i for i in range(n)] + [40.0 + 1.5 * i * i for i in range(n)]
    port = 4 * n
    nets = [(port, [2 * i for i in range(n)])] + [(2 * i + 1, [2 * n + 2 * i]) for i in range(n)] + \
        [(2 * n + 2 * i + 1, []) for i in range(n)]
    nl, _ = handnets.build(cells, 1, nets, x, y, port_xy=[(0.0, 0.0)], clock_period=1.0)
    par = ref.rc_tree(nl)
    assert [int(par[2 * i]) for i in range(n)] == [port] + [2 * i for i in range(n - 1)]  # a chain
    lib = _lib(library)
    st = ref.sta(nl, lib)
    v, gx, gy = ref.stns(nl, lib, st, gamma=5.0)
    h = 2.0 ** -12
    xs = np.asarray(nl["x"], np.float64)
    ys = np.asarray(nl["y"], np.float64)
    for cc in range(n):
        for axis, a0 in ((0, xs), (1, ys)):
            a = a0.copy()
            a[cc] += h
            vp = ref.stns(nl, lib, st, 5.0, *((a, ys) if axis == 0 else (xs, a)))[0]
            a[cc] -= 2 * h
            vm = ref.stns(nl, lib, st, 5.0, *((a, ys) if axis == 0 else (xs, a)))[0]
            fd = (vp - vm) / (2 * h)
            gr = (gx if axis == 0 else gy)[cc]
            assert abs(fd - gr) <= 1e-5 * max(1e-2, abs(gr)), (cc, axis, fd, gr)
        assert abs(gx[cc]) + abs(gy[cc]) > 1e-4


def test_dyadic_hand_tree_by_hand():
    """A port at the origin drives sinks at (8, 0), (16, 0), (16, 8) and
    (24, 0) under the dyadic library (r = 1/16, c = 1/4, pin capacitance 2,
    scale 1).  The tree is port -> A(8, 0) -> B(16, 0) -> {C(16, 8), D(24, 0)}
    (C and D tie at distance 8 from B; C, listed first, joins first, and D
    still hangs from B, which reached it first).  By hand, every wire 8 um
    (c L = 2, r L = 1/2): C_below(C) = C_below(D) = 2, C_below(B) = 2 + (2 + 2)
    + (2 + 2) = 10, C_below(A) = 2 + 2 + 10 = 14; delays
    A = 1/2 (1 + 14) = 7.5, B = 7.5 + 1/2 (1 + 10) = 13,
    C = D = 13 + 1/2 (1 + 2) = 14.5; load 4 x 2 + 32 / 4 = 16."""
    from tests import handnets
    lib = dict(handnets.dyadic_library(), net_model=2)
    sx, sy = [8.0, 16.0, 16.0, 24.0], [0.0, 0.0, 8.0, 0.0]
    n = 4
    cells = [(0, 1)] * n + [(netgen.FF_TYPE, 1)] * n
    port = 4 * n
    nets = [(port, [2 * i for i in range(n)])] + [(2 * i + 1, [2 * n + 2 * i]) for i in range(n)] + \
        [(2 * n + 2 * i + 1, []) for i in range(n)]
    nl, _ = handnets.build(cells, 1, nets, sx + [v + 4.0 for v in sx], sy + sy, port_xy=[(0.0, 0.0)],
                           clock_period=400.0)
    par = ref.rc_tree(nl)
    assert [int(par[2 * i]) for i in range(n)] == [port, 0, 2, 2]
    st = ref.sta(nl, lib)
    assert st["dnet"][[0, 2, 4, 6]].tolist() == [7.5, 13.0, 14.5, 14.5]
    assert st["load"][port] == 16.0
    # each two-pin net from a cell to its flip-flop is a 4 um wire: 1/4 (1/2 + 2)
    assert st["dnet"][[2 * n + 2 * i for i in range(n)]].tolist() == [0.625] * n
