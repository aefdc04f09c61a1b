"""Pins for the oracle's placement-loop pieces: the bin density (against
numerical integration of the Gaussian over each bin, the window's mass from
the normal distribution function, translation and mirror symmetry, finite
differences) and the Nesterov step (the Lipschitz prediction lands exactly on
the minimiser of an isotropic quadratic; bounds and frozen cells)."""
import math

import numpy as np
import pytest
from scipy import integrate
from scipy.stats import norm

from oracle import ref


def _grid(**kw):
    g = dict(x0=0.0, y0=0.0, bw=10.0, bh=7.0, gx=12, gy=20, R=3)
    g.update(kw)
    return g


def test_density_of_one_cell_is_its_gaussian_integrated_over_each_bin():
    g = _grid()
    xc, yc, a = 37.3, 81.9, 2.5
    r = ref.density([xc], [yc], [a], [0], g)
    D = r["dens"]
    bx, by = int(xc // g["bw"]), int(yc // g["bh"])
    xc32, yc32 = float(np.float32(xc)), float(np.float32(yc))
    for j in range(g["gy"]):
        for i in range(g["gx"]):
            if abs(i - bx) > g["R"] or abs(j - by) > g["R"]:
                assert D[j, i] == 0.0
                continue
            want, _ = integrate.dblquad(
                lambda yy, xx: norm.pdf(xx, xc32, g["bw"]) * norm.pdf(yy, yc32, g["bh"]),
                i * g["bw"], (i + 1) * g["bw"], j * g["bh"], (j + 1) * g["bh"], epsabs=1e-13, epsrel=1e-11)
            assert math.isclose(D[j, i], a * want, rel_tol=1e-8, abs_tol=1e-14), (i, j, D[j, i], a * want)


@pytest.mark.parametrize("pos", [(60.0, 70.0), (3.0, 2.0), (119.5, 139.0)])
def test_density_mass_is_the_window_mass(pos):
    # the cell's area times the normal mass over its whole window: what falls
    # off the die is reflected back in, none is lost
    g = _grid()
    xc, yc = pos
    a = 1.75
    r = ref.density([xc], [yc], [a], [0], g)
    bx = min(max(int(xc // g["bw"]), 0), g["gx"] - 1)
    by = min(max(int(yc // g["bh"]), 0), g["gy"] - 1)
    lo_x, hi_x = (bx - g["R"]) * g["bw"], (bx + g["R"] + 1) * g["bw"]
    lo_y, hi_y = (by - g["R"]) * g["bh"], (by + g["R"] + 1) * g["bh"]
    mx = norm.cdf(hi_x, xc, g["bw"]) - norm.cdf(lo_x, xc, g["bw"])
    my = norm.cdf(hi_y, yc, g["bh"]) - norm.cdf(lo_y, yc, g["bh"])
    assert math.isclose(r["dens"].sum(), a * mx * my, rel_tol=1e-12)
    assert r["overflow"] == 0.0 and r["value"] == 0.0  # one cell never fills a bin of capacity 70


def test_density_reflects_at_the_die_edges():
    # near a corner each bin holds the Gaussian plus its mirror image in the
    # edge (integrated over the bin), the image counting where its source bin
    # lies inside the window
    g = _grid()
    xc, yc, a = 4.25, 9.5, 3.0
    r = ref.density([xc], [yc], [a], [0], g)
    bx, by, R = int(xc // g["bw"]), int(yc // g["bh"]), g["R"]

    def axis(i, c, w, b):
        m = integrate.quad(lambda t: norm.pdf(t, c, w), i * w, (i + 1) * w, epsabs=1e-14)[0]
        if -1 - i >= b - R:  # the mirrored bin -1 - i is in the window
            m += integrate.quad(lambda t: norm.pdf(t, -c, w), i * w, (i + 1) * w, epsabs=1e-14)[0]
        return m if abs(i - b) <= R else 0.0

    for j in range(g["gy"]):
        for i in range(g["gx"]):
            want = a * axis(i, xc, g["bw"], bx) * axis(j, yc, g["bh"], by)
            assert math.isclose(r["dens"][j, i], want, rel_tol=1e-9, abs_tol=1e-14), (i, j, r["dens"][j, i], want)
    assert r["dens"][0, 0] > r["dens"][0, 1]  # the corner bin gains the most


def _cluster(n, seed, g, spread=12.0):
    rng = np.random.default_rng(seed)
    cx, cy = 0.5 * g["gx"] * g["bw"], 0.5 * g["gy"] * g["bh"]
    # on a 2^-10 grid, so that shifts by whole bins and mirrors stay exact
    x = (np.round((cx + spread * rng.standard_normal(n)) * 1024) / 1024).astype(np.float32)
    y = (np.round((cy + spread * rng.standard_normal(n)) * 1024) / 1024).astype(np.float32)
    # off the bin edges, where a mirror image would change bins
    x[np.mod(x, np.float32(g["bw"])) == 0] += np.float32(1 / 1024)
    y[np.mod(y, np.float32(g["bh"])) == 0] += np.float32(1 / 1024)
    area = (1.0 + rng.random(n)).astype(np.float32) * 8.0
    return x, y, area


def test_density_is_translation_and_mirror_symmetric():
    g = _grid()
    x, y, area = _cluster(300, 1, g)
    base = ref.density(x, y, area, np.zeros(300), g)
    # translate cells and grid together by whole numbers of bins
    g2 = _grid(x0=30.0, y0=-14.0)
    sh = ref.density(x + np.float32(30.0), y - np.float32(14.0), area, np.zeros(300), g2)
    assert np.array_equal(sh["dens"], base["dens"])
    assert sh["value"] == base["value"]
    # mirror in x about the die's centre: the map mirrors
    W = g["gx"] * g["bw"]
    mir = ref.density(np.float32(W) - x, y, area, np.zeros(300), g)
    inside = (x > 1e-3) & (x < W - 1e-3)
    assert inside.all()
    assert np.allclose(mir["dens"], base["dens"][:, ::-1], rtol=1e-9, atol=1e-12)
    assert np.allclose(mir["grad_x"], -base["grad_x"], rtol=1e-7, atol=1e-9)
    assert np.allclose(mir["grad_y"], base["grad_y"], rtol=1e-7, atol=1e-9)


def test_density_penalty_and_overflow_and_gradient():
    g = _grid()
    n = 300
    x, y, area = _cluster(n, 2, g)
    fixed = np.zeros(n, np.uint8)
    fixed[:10] = 1
    r = ref.density(x, y, area, fixed, g, target=0.9)
    cap = 0.9 * g["bw"] * g["bh"]
    o = np.maximum(r["dens"] - cap, 0)
    assert (o > 0).sum() > 5  # the cluster overflows
    assert math.isclose(r["value"], float((o ** 2).sum()), rel_tol=1e-12)
    assert math.isclose(r["overflow"], float(o.sum() / area.astype(np.float64).sum()), rel_tol=1e-12)
    assert np.all(r["grad_x"][:10] == 0) and np.all(r["grad_y"][:10] == 0)
    # fixed cells still count in the map
    r2 = ref.density(x, y, area, np.zeros(n, np.uint8), g, target=0.9)
    assert np.array_equal(r2["dens"], r["dens"])
    # central differences on movable cells away from bin edges
    h = 2.0 ** -8
    rng = np.random.default_rng(3)
    checked = 0
    for c in rng.permutation(np.arange(10, n)):
        fx = (x[c] / g["bw"]) % 1.0
        fy = (y[c] / g["bh"]) % 1.0
        if min(fx, 1 - fx) * g["bw"] < 4 * h or min(fy, 1 - fy) * g["bh"] < 4 * h:
            continue
        if abs(r["grad_x"][c]) + abs(r["grad_y"][c]) < 1e-3:
            continue
        for axis in (0, 1):
            a = (x if axis == 0 else y).astype(np.float64)
            ap, am = a.copy(), a.copy()
            ap[c] += h
            am[c] -= h
            vp = ref.density(*((ap, y) if axis == 0 else (x, ap)), area, fixed, g, target=0.9)["value"]
            vm = ref.density(*((am, y) if axis == 0 else (x, am)), area, fixed, g, target=0.9)["value"]
            fd = (vp - vm) / (2 * h)
            gr = (r["grad_x"] if axis == 0 else r["grad_y"])[c]
            assert abs(fd - gr) <= 1e-4 * max(1.0, abs(gr)), (c, axis, fd, gr)
        checked += 1
        if checked == 12:
            break
    assert checked == 12


def _state(v0x, v0y):
    z = np.zeros_like(v0x)
    return {"vx": v0x.copy(), "vy": v0y.copy(), "ux": v0x.copy(), "uy": v0y.copy(),
            "vpx": v0x.copy(), "vpy": v0y.copy(), "gpx": z.copy(), "gpy": z.copy()}


def test_nesterov_lipschitz_step_solves_an_isotropic_quadratic():
    # f = k/2 |v - c|^2 preconditioned by a uniform divisor s is isotropic
    # with curvature k/s: the predicted step |dv|/|dg| is s/k, and the second
    # step lands on c
    rng = np.random.default_rng(0)
    n, k, s = 50, 3.0, 4.0
    cx, cy = rng.uniform(10, 90, n), rng.uniform(10, 90, n)
    st = _state(rng.uniform(0, 100, n), rng.uniform(0, 100, n))
    pdiv = np.full(n, s)
    frozen = np.zeros(n, np.uint8)
    bounds = (-1e9, 1e9, -1e9, 1e9)
    a_k = 1.0
    alphas = []
    for it in range(2):
        gx, gy = k * (st["vx"] - cx), k * (st["vy"] - cy)
        a_n = (1 + math.sqrt(4 * a_k * a_k + 1)) / 2
        alphas.append(ref.nesterov(st, gx, gy, pdiv, frozen, (a_k - 1) / a_n, 0.01, it == 0, bounds))
        a_k = a_n
    assert alphas[0] == 0.01
    assert math.isclose(alphas[1], s / k, rel_tol=1e-12)
    assert np.allclose(st["ux"], cx, rtol=0, atol=1e-10)
    assert np.allclose(st["uy"], cy, rtol=0, atol=1e-10)


def test_nesterov_bounds_frozen_cells_and_state_shift():
    rng = np.random.default_rng(1)
    n = 40
    st = _state(rng.uniform(0, 10, n), rng.uniform(0, 10, n))
    v0x, v0y = st["vx"].copy(), st["vy"].copy()
    frozen = np.zeros(n, np.uint8)
    frozen[::5] = 1
    gx, gy = rng.standard_normal(n) * 50, rng.standard_normal(n) * 50
    pdiv = rng.uniform(0.2, 5.0, n)
    bounds = (1.0, 9.0, 2.0, 8.0)
    alpha = ref.nesterov(st, gx, gy, pdiv, frozen, 0.3, 0.5, True, bounds)
    assert alpha == 0.5
    m = frozen == 0
    q = np.maximum(pdiv, 1.0)
    want_ux = np.clip(v0x - 0.5 * gx / q, 1.0, 9.0)
    assert np.allclose(st["ux"][m], want_ux[m], rtol=0, atol=1e-12)
    assert np.all((st["vx"][m] >= 1.0) & (st["vx"][m] <= 9.0) & (st["vy"][m] >= 2.0) & (st["vy"][m] <= 8.0))
    # u_0 = v_0 here, so v_1 = clamp(u_1 + 0.3 (u_1 - v_0))
    assert np.allclose(st["vx"][m], np.clip(st["ux"][m] + 0.3 * (st["ux"][m] - v0x[m]), 1.0, 9.0), atol=1e-12)
    assert np.array_equal(st["vx"][~m], v0x[~m]) and np.array_equal(st["ux"][~m], v0x[~m])
    assert np.array_equal(st["vpx"], v0x) and np.array_equal(st["vpy"], v0y)
    assert np.allclose(st["gpx"][m], (gx / q)[m], rtol=1e-15) and np.all(st["gpx"][~m] == 0)
