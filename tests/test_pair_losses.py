"""Pins of the oracle's other pair losses (Sec. III-C compares the quadratic
PP with the Manhattan distance, which is a two-pin pair's HPWL, and with the
linear Euclidean distance).  CPU only."""
import math

import numpy as np
import pytest

from oracle import ref
from paper_2503_11674_amd import netgen
from tests import handnets
from tests.conftest import with_clock


def _chain(xs, fixed_ends=True):
    """Buffers 0..n-1 in a chain from a port at x = xs[0] to a fixed
    flip-flop at xs[-1]; buffer i sits at xs[i + 1] (y = 0).  Returns the
    netlist and the sink pins of the chain's pairs."""
    n = len(xs) - 2
    # buffer i: input pin 2i, output 2i + 1; a fixed flip-flop at the right
    # end (D = 2n, Q = 2n + 1); the left end is the port, pin 2n + 2
    cells = [(0, 1)] * n + [(7, 1)]
    ff_d, ff_q = 2 * n, 2 * n + 1
    nets = [(2 * n + 2, [0])] + [(2 * i + 1, [2 * (i + 1)]) for i in range(n - 1)] + [(2 * n - 1, [ff_d]),
                                                                                       (ff_q, [])]
    x = list(xs[1:-1]) + [xs[-1]]
    y = [0.0] * (n + 1)
    fixed = [0] * n + [1]
    nl, ids = handnets.build(cells, 1, nets, x, y, port_xy=[(xs[0], 0.0)], fixed=fixed)
    sinks = np.array([0] + [2 * (i + 1) for i in range(n - 1)] + [ff_d], np.int32)
    return nl, sinks


def test_single_pair_relations():
    """One pair: the Euclidean loss squared is PP (w = 1), the Manhattan loss
    lies between the Euclidean one and sqrt(2) times it, and both scale
    linearly with w while PP does."""
    for dx, dy in ((3.0, 4.0), (-7.5, 0.25), (0.0, -2.0)):
        nl, sinks = _chain([0.0, dx, 10.0])
        one = sinks[:1]
        nl["y"] = np.array([dy, 0.0], np.float32)
        pp = ref.p2p(nl, one, [1.0])[0]
        eu = ref.pair_loss(nl, 2, one, [1.0])[0]
        mh = ref.pair_loss(nl, 1, one, [1.0])[0]
        assert math.isclose(eu * eu, pp, rel_tol=1e-12)
        assert eu <= mh * (1 + 1e-12) and mh <= math.sqrt(2) * eu * (1 + 1e-12)
        assert math.isclose(ref.pair_loss(nl, 2, one, [3.0])[0], 3 * eu, rel_tol=1e-12)
        assert math.isclose(ref.pair_loss(nl, 1, one, [3.0])[0], 3 * mh, rel_tol=1e-12)


def test_manhattan_loss_is_two_pin_hpwl(library):
    """Over two-pin nets with unit weights the Manhattan pair loss is the
    HPWL, i.e. the weighted-average wirelength in the limit gamma -> 0."""
    nl, sinks = _chain([0.0, 1.5, 4.0, 9.25, 10.0])
    nl["y"] = np.array([0.5, -1.0, 2.0, 0.0], np.float32)
    mh = ref.pair_loss(nl, 1, sinks, np.ones(len(sinks)))[0]
    wa = ref.wa(nl, 1e-4)[0]
    assert abs(mh - wa) <= 1e-9 * mh


@pytest.mark.parametrize("kind", [1, 2])
def test_pair_loss_gradients_by_differences(library, kind):
    nl = with_clock(netgen.make_netlist(netgen.CONFIGS["C1"]), library)
    st = ref.sta(nl, library)
    rp = ref.extract(nl, library, st, n=-1, k=10, K=100)
    ps = ref.PairState(nl["num_pins"])
    ref.pairs_update(ps, rp, st["wns"], rule=1)
    sinks, w = ps.pairs()
    rng = np.random.default_rng(5)
    # dyadic positions keep the differences exact
    x = (np.round(nl["x"].astype(np.float64) * 64) / 64).astype(np.float32)
    y = (np.round(nl["y"].astype(np.float64) * 64) / 64).astype(np.float32)
    v, gx, gy = ref.pair_loss(nl, kind, sinks, w, x, y)
    h = 2.0 ** -12
    touched = np.unique(nl["pin_cell"][np.concatenate([sinks])])
    for c in rng.choice(touched[touched >= 0], 8, replace=False):
        for arr, g in ((x, gx), (y, gy)):
            a = arr.copy()
            a[c] += h
            vp = ref.pair_loss(nl, kind, sinks, w, *(((a, y) if arr is x else (x, a))))[0]
            a[c] -= 2 * h
            vm = ref.pair_loss(nl, kind, sinks, w, *(((a, y) if arr is x else (x, a))))[0]
            assert abs((vp - vm) / (2 * h) - g[c]) <= 1e-6 * max(1.0, abs(g[c]))


def test_quadratic_loss_spaces_a_chain_uniformly():
    """Sec. III-C: on a chain of movable cells between fixed ends, the
    quadratic loss's gradient vanishes only at equal spacing, while the
    linear losses give every interior cell a zero gradient for any monotone
    spacing (direction without magnitude)."""
    even = [0.0, 2.0, 4.0, 6.0, 8.0, 10.0]
    skew = [0.0, 0.5, 1.0, 1.5, 9.0, 10.0]
    for xs in (even, skew):
        nl, sinks = _chain(xs)
        w = np.ones(len(sinks))
        _, gq, _ = ref.p2p(nl, sinks, w)
        _, g1, _ = ref.pair_loss(nl, 1, sinks, w)
        _, g2, _ = ref.pair_loss(nl, 2, sinks, w)
        movable = np.arange(len(xs) - 2)
        assert np.all(g1[movable] == 0.0) and np.all(g2[movable] == 0.0)
        if xs is even:
            assert np.all(gq[movable] == 0.0)
        else:
            assert np.any(np.abs(gq[movable]) > 1.0)
