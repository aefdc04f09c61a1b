"""Parity of the placement-loop pieces with the FP64 oracle: the bin density
(map, penalty, overflow, gradient), the Nesterov step and the L1 norm; the
loop itself runs deterministically and spreads a clustered placement.

Tolerances: the map is a sum of at most (2R+1)^2 * (cells per bin) FP32
products of FP32 error-function differences (about 1e-6 relative each), so
1e-5 of the largest bin value; the penalty and overflow 1e-4 relative; the
gradient 1e-4 of the largest component plus 1e-3 relative (bins near the
capacity carry an overflow whose FP32 value is a difference of nearby
numbers).  The Nesterov step: 1e-6 of the coordinate range."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import ref  # noqa: E402
from paper_2503_11674_amd import netgen  # noqa: E402
from tests.conftest import with_clock  # noqa: E402

pytestmark = pytest.mark.gpu


def _tdp():
    from paper_2503_11674_amd import tdp
    return tdp


def _dev():
    return torch.device("cuda", 0)


def _t(a):
    return torch.tensor(np.asarray(a, np.float32), device=_dev())


def _design(name, library, fixed_every=0):
    nl = netgen.make_netlist(netgen.CONFIGS[name])
    if fixed_every:
        f = np.zeros(nl["num_cells"], np.uint8)
        f[::fixed_every] = 1
        nl["cell_fixed"] = f
    return nl


def _check_density(g, nl, x, y, area, grid, target):
    gx = torch.zeros(nl["num_cells"], dtype=torch.float32, device=_dev())
    gy = torch.zeros_like(gx)
    val, ovf, mp = g.density(_t(x), _t(y), 1.0, gx, gy, want_map=True)
    r = ref.density(x, y, area, nl["cell_fixed"], grid, target)
    D = mp.cpu().numpy().reshape(grid["gy"], grid["gx"])
    assert np.allclose(D, r["dens"], rtol=0, atol=1e-5 * r["dens"].max()), np.abs(D - r["dens"]).max()
    assert abs(float(val) - r["value"]) <= 1e-4 * r["value"]
    assert abs(float(ovf) - r["overflow"]) <= 1e-4 * r["overflow"]
    for a, b in ((gx, r["grad_x"]), (gy, r["grad_y"])):
        a = a.cpu().numpy()
        sc = np.abs(b).max()
        assert np.allclose(a, b, rtol=1e-3, atol=1e-4 * sc), np.abs(a - b).max() / sc
    return r, D, gx.cpu().numpy(), gy.cpu().numpy()


@pytest.mark.parametrize("name,bins,R", [("C1", 64, 3), ("C2", 512, 3), ("C1", 33, 0), ("C1", 40, 8)])
def test_density_parity(name, bins, R, library):
    tdp = _tdp()
    nl = _design(name, library, fixed_every=7)
    die = netgen.CONFIGS[name].die
    N = nl["num_cells"]
    # utilisation 0.5 over the die: the clustered C2 placement overflows
    area = np.full(N, 0.5 * die * die / N, np.float32)
    area[::3] *= 2.0
    grid = dict(x0=0.0, y0=0.0, bw=die / bins, bh=die / bins, gx=bins, gy=bins, R=R, target=0.9)
    g = tdp.TimingGraph(nl, library, max_paths=16, max_k=1)
    g.density_setup(grid, area)
    print(f"[density] {name} bins={bins} R={R}", flush=True)
    r, D, gx, gy = _check_density(g, nl, nl["x"], nl["y"], area, grid, 0.9)
    if name == "C2":
        assert r["overflow"] > 0.05 and (np.abs(gx) > 0).sum() > 1000
    assert np.all(gx[::7] == 0) and np.all(gy[::7] == 0)  # fixed cells
    # bitwise reproducible
    gx2 = torch.zeros(N, dtype=torch.float32, device=_dev())
    gy2 = torch.zeros_like(gx2)
    v2, o2, mp2 = g.density(_t(nl["x"]), _t(nl["y"]), 1.0, gx2, gy2, want_map=True)
    assert np.array_equal(mp2.cpu().numpy().reshape(D.shape), D)
    assert np.array_equal(gx2.cpu().numpy(), gx) and np.array_equal(gy2.cpu().numpy(), gy)
    g.close()


def test_density_edge_cases(library):
    """Cells off the die (clamped bins), all cells in one bin, a 1 x 1 grid,
    a non-square grid with its origin off zero, and a scale on the gradient."""
    tdp = _tdp()
    nl = _design("C1", library)
    N = nl["num_cells"]
    rng = np.random.default_rng(4)
    g = tdp.TimingGraph(nl, library, max_paths=16, max_k=1)
    area = np.full(N, 30.0, np.float32)
    cases = [
        ("off-die", dict(x0=100.0, y0=-50.0, bw=20.0, bh=13.0, gx=40, gy=70, R=3),
         rng.uniform(-200, 1200, N), rng.uniform(-300, 1100, N)),
        ("one bin", dict(x0=0.0, y0=0.0, bw=10.0, bh=10.0, gx=100, gy=100, R=2),
         np.full(N, 503.0) + rng.uniform(0, 4, N), np.full(N, 498.0) + rng.uniform(0, 1.5, N)),
        ("1x1", dict(x0=0.0, y0=0.0, bw=1000.0, bh=1000.0, gx=1, gy=1, R=1), nl["x"], nl["y"]),
    ]
    for what, grid, x, y in cases:
        print(f"[density] {what}", flush=True)
        g.density_setup(grid, area)
        _check_density(g, nl, np.asarray(x, np.float32), np.asarray(y, np.float32), area, grid, 1.0)
    # the scale multiplies the added gradient
    gxa = torch.zeros(N, dtype=torch.float32, device=_dev())
    gya = torch.zeros_like(gxa)
    gxb, gyb = torch.ones_like(gxa), torch.ones_like(gxa)
    x, y = _t(nl["x"]), _t(nl["y"])
    g.density(x, y, 1.0, gxa, gya)
    g.density(x, y, 0.25, gxb, gyb)
    assert torch.allclose(gxb - 1, 0.25 * gxa, rtol=1e-6, atol=1e-6 * float(gxa.abs().max()))
    g.close()


def test_density_and_nesterov_refuse_without_setup(library):
    tdp = _tdp()
    nl = _design("C1", library)
    g = tdp.TimingGraph(nl, library, max_paths=16, max_k=1)
    x, y = _t(nl["x"]), _t(nl["y"])
    with pytest.raises(tdp.TdpError):
        g.density(x, y)
    with pytest.raises(tdp.TdpError):
        g.density_setup(dict(x0=0, y0=0, bw=10, bh=10, gx=0, gy=10, R=3), np.ones(nl["num_cells"]))
    with pytest.raises(tdp.TdpError):
        g.density_setup(dict(x0=0, y0=0, bw=10, bh=10, gx=10, gy=10, R=9), np.ones(nl["num_cells"]))
    g.close()


def test_nesterov_step_parity(library):
    tdp = _tdp()
    nl = _design("C1", library, fixed_every=5)
    N = nl["num_cells"]
    g = tdp.TimingGraph(nl, library, max_paths=16, max_k=1)
    g.density_setup(dict(x0=0, y0=0, bw=10, bh=10, gx=100, gy=100, R=1), np.ones(N, np.float32))
    rng = np.random.default_rng(7)
    v = {k: rng.uniform(0, 1000, N).astype(np.float32) for k in ("vx", "vy", "ux", "uy", "vpx", "vpy")}
    v["gpx"] = rng.standard_normal(N).astype(np.float32)
    v["gpy"] = rng.standard_normal(N).astype(np.float32)
    pdiv = rng.uniform(0.5, 8, N).astype(np.float32)
    bounds = (0.0, 1000.0, 0.0, 1000.0)
    fixed = nl["cell_fixed"]
    dev_st = {k: _t(a) for k, a in v.items()}
    ora_st = {k: a.astype(np.float64) for k, a in v.items()}
    alpha = torch.zeros(1, dtype=torch.float64, device=_dev())
    for step, (first, coef) in enumerate([(True, 0.0), (False, 0.28), (False, 0.43)]):
        gxs = (rng.standard_normal(N) * 30).astype(np.float32)
        gys = (rng.standard_normal(N) * 30).astype(np.float32)
        g.nesterov_step(dev_st, _t(gxs), _t(gys), _t(pdiv), coef, 0.7, first, bounds, alpha_out=alpha)
        a_ref = ref.nesterov(ora_st, gxs, gys, pdiv, fixed, coef, 0.7, first, bounds)
        assert abs(float(alpha) - a_ref) <= 1e-6 * a_ref, (step, float(alpha), a_ref)
        for k in dev_st:
            got = dev_st[k].cpu().numpy().astype(np.float64)
            scale = 1000.0 if k[0] in "uv" else max(1.0, np.abs(ora_st[k]).max())
            assert np.allclose(got, ora_st[k], rtol=0, atol=2e-6 * scale), (step, k, np.abs(got - ora_st[k]).max())
            # carry the device state on to the next step in both
            ora_st[k] = got.copy()
    assert np.all(dev_st["vx"].cpu().numpy()[::5] == v["vx"][::5])  # fixed cells do not move
    # the L1 norm
    s = g.abs_sum(_t(v["gpx"]), _t(v["gpy"]))
    want = np.abs(v["gpx"].astype(np.float64)).sum() + np.abs(v["gpy"].astype(np.float64)).sum()
    assert abs(float(s) - want) <= 1e-12 * want
    g.close()


def test_placement_loop_spreads_and_is_deterministic(library):
    """A short timing-driven loop on 2,000 cells: overflow falls, timing and
    pairs come on at the start iteration, and two runs agree bitwise."""
    from paper_2503_11674_amd.placer import GlobalPlacer, LoopConfig
    nl = netgen.make_netlist(netgen.CONFIGS["C1"])
    # start from a crowded centre so that the density term has work to do
    rng = np.random.default_rng(11)
    nl["x"] = (500 + 40 * rng.standard_normal(nl["num_cells"])).astype(np.float32)
    nl["y"] = (500 + 40 * rng.standard_normal(nl["num_cells"])).astype(np.float32)
    nl["clock_period"] = np.float32(0.0)  # the placer sets 5 % failing at this start
    cfg = LoopConfig(die=1000.0, bins=64, max_iters=120, timing_start=40, timing_every=15, beta=1e-3,
                     lambda_init=1.0, record_every=20, stop_overflow=0.0)
    runs = []
    for rep in range(2):
        print(f"[loop] run {rep}", flush=True)
        p = GlobalPlacer(nl, library, cfg)
        hist = p.run()
        ux, uy = p.positions()
        runs.append((ux.cpu().numpy(), uy.cpu().numpy(), hist))
        p.g.close()
    (x0, y0, h0), (x1, y1, h1) = runs
    assert np.array_equal(x0, x1) and np.array_equal(y0, y1)
    assert [r.overflow for r in h0] == [r.overflow for r in h1]
    assert h0[-1].overflow < 0.5 * h0[0].overflow
    assert all(np.isfinite(r.hpwl) and np.isfinite(r.tns) for r in h0)
    assert h0[0].pairs == 0 and h0[-1].pairs > 0
    assert np.all((x0 >= 0) & (x0 <= 1000) & (y0 >= 0) & (y0 <= 1000))


def test_loop_trajectory_matches_the_oracle_composition(library):
    """Three iterations of the placer (timing off) against the same loop
    composed from the oracle's WA, density and Nesterov step: lambda_0 from
    the gradients' L1 norms, the growth rule, the preconditioner and the
    Nesterov coefficients all enter."""
    import math

    from paper_2503_11674_amd.placer import GlobalPlacer, LoopConfig
    nl = netgen.make_netlist(netgen.CONFIGS["C1"])
    nl["clock_period"] = np.float32(1e9)
    cfg = LoopConfig(die=1000.0, bins=32, beta=0.0, record_every=1 << 30)
    p = GlobalPlacer(nl, library, cfg)
    p.run(iters=3)
    gpu_x, gpu_y = (t.cpu().numpy().astype(np.float64) for t in p.positions())
    alpha_gpu = float(p.alpha)
    p.g.close()
    # the oracle composition
    N = nl["num_cells"]
    grid = dict(x0=0.0, y0=0.0, bw=1000.0 / 32, bh=1000.0 / 32, gx=32, gy=32, R=3)
    area = np.full(N, np.float32(0.5 * 1000.0 * 1000.0 / N), np.float32)
    fixed = np.asarray(nl["cell_fixed"], np.uint8)
    pins = np.bincount(np.asarray(nl["pin_cell"])[np.asarray(nl["pin_cell"]) >= 0], minlength=N)
    pdiv = np.maximum(pins, 1).astype(np.float32).astype(np.float64)
    x0, y0 = np.asarray(nl["x"], np.float64), np.asarray(nl["y"], np.float64)
    st = {"vx": x0.copy(), "vy": y0.copy(), "ux": x0.copy(), "uy": y0.copy(), "vpx": x0.copy(), "vpy": y0.copy(),
          "gpx": np.zeros(N), "gpy": np.zeros(N)}
    _, wgx, wgy = ref.wa(nl, cfg.wa_gamma, st["vx"], st["vy"])
    d = ref.density(st["vx"], st["vy"], area, fixed, grid, cfg.target)
    lam = cfg.lambda_init * (np.abs(wgx).sum() + np.abs(wgy).sum()) / (np.abs(d["grad_x"]).sum() + np.abs(d["grad_y"]).sum())
    a_k, wl_prev, wl_ref = 1.0, None, None
    for it in range(3):
        wl, wgx, wgy = ref.wa(nl, cfg.wa_gamma, st["vx"], st["vy"])
        d = ref.density(st["vx"], st["vy"], area, fixed, grid, cfg.target)
        gx, gy = wgx + lam * d["grad_x"], wgy + lam * d["grad_y"]
        a_n = (1 + math.sqrt(4 * a_k * a_k + 1)) / 2
        alpha = ref.nesterov(st, gx, gy, pdiv, fixed, (a_k - 1) / a_n, cfg.alpha0, it == 0,
                             (0.0, 1000.0, 0.0, 1000.0))
        a_k = a_n
        if wl_prev is None:
            mu, wl_ref = cfg.mu_max, cfg.wl_ref_frac * abs(wl)
        else:
            mu = min(cfg.mu_max, max(cfg.mu_min, cfg.mu_max ** (1 - (wl - wl_prev) / wl_ref)))
        wl_prev = wl
        lam *= mu
    # the step length divides by the change of the gradient between two
    # nearby points, about 1 % of the gradient here: FP32 rounding of the
    # two gradients reaches it amplified a hundredfold
    assert abs(alpha_gpu - alpha) <= 1e-2 * alpha, (alpha_gpu, alpha)
    # positions: within 1 % of each cell's own move (the step length's
    # relative error carries into the move) plus FP32 rounding of the position
    moved = np.abs(st["ux"] - x0) + np.abs(st["uy"] - y0)
    assert np.median(moved) > 0.1  # the cells did move
    err = np.abs(gpu_x - st["ux"]) + np.abs(gpu_y - st["uy"])
    assert np.all(err <= 1e-2 * moved + 1e-3), (err.max(), moved[err.argmax()])


def test_loop_with_timing_matches_the_oracle_composition(library):
    """Six iterations of the timing-driven placer (timing every second
    iteration from iteration 1) against the same loop composed from the
    oracle: at each refresh the oracle times the current placement, extracts
    report_timing_endpoint(n_fail, 1) and applies Eq. 9 to its own pair set,
    and its PP gradient (beta-scaled) joins WA and density in every later
    step.  Refresh, extraction, pair update and loss all enter the
    trajectory."""
    import math

    from paper_2503_11674_amd.placer import GlobalPlacer, LoopConfig
    nl = with_clock(netgen.make_netlist(netgen.CONFIGS["C1"]), library)
    E = int(np.count_nonzero(nl["cell_is_ff"]))
    cfg = LoopConfig(die=1000.0, bins=32, beta=1e-2, timing_start=1, timing_every=2, record_every=1 << 30)
    p = GlobalPlacer(nl, library, cfg)
    p.run(iters=6)
    gpu_x, gpu_y = (t.cpu().numpy().astype(np.float64) for t in p.positions())
    gpu_pairs = p.g.pairs_count()
    p.g.close()
    N = nl["num_cells"]
    grid = dict(x0=0.0, y0=0.0, bw=1000.0 / 32, bh=1000.0 / 32, gx=32, gy=32, R=3)
    area = np.full(N, np.float32(0.5 * 1000.0 * 1000.0 / N), np.float32)
    fixed = np.asarray(nl["cell_fixed"], np.uint8)
    pins = np.bincount(np.asarray(nl["pin_cell"])[np.asarray(nl["pin_cell"]) >= 0], minlength=N)
    pdiv = np.maximum(pins, 1).astype(np.float32).astype(np.float64)
    x0, y0 = np.asarray(nl["x"], np.float64), np.asarray(nl["y"], np.float64)
    st = {"vx": x0.copy(), "vy": y0.copy(), "ux": x0.copy(), "uy": y0.copy(), "vpx": x0.copy(), "vpy": y0.copy(),
          "gpx": np.zeros(N), "gpy": np.zeros(N)}
    _, wgx, wgy = ref.wa(nl, cfg.wa_gamma, st["vx"], st["vy"])
    d = ref.density(st["vx"], st["vy"], area, fixed, grid, cfg.target)
    lam = cfg.lambda_init * (np.abs(wgx).sum() + np.abs(wgy).sum()) / (np.abs(d["grad_x"]).sum() + np.abs(d["grad_y"]).sum())
    ps = ref.PairState(nl["num_pins"])
    timing_on = False
    a_k, wl_prev, wl_ref = 1.0, None, None
    for it in range(6):
        if it >= 1 and (it - 1) % 2 == 0:  # refresh at the current placement u
            sta = ref.sta(nl, library, x=st["ux"].astype(np.float32), y=st["uy"].astype(np.float32))
            paths = ref.extract(nl, library, sta, n=-1, k=1, K=E)
            ref.pairs_update(ps, paths, sta["wns"], rule=0, w0=cfg.w0, w1=cfg.w1)
            timing_on = True
        wl, wgx, wgy = ref.wa(nl, cfg.wa_gamma, st["vx"], st["vy"])
        d = ref.density(st["vx"], st["vy"], area, fixed, grid, cfg.target)
        gx, gy = wgx + lam * d["grad_x"], wgy + lam * d["grad_y"]
        if timing_on:
            sinks, w = ps.pairs()
            _, pgx, pgy = ref.p2p(nl, sinks, w, st["vx"], st["vy"])
            gx, gy = gx + cfg.beta * pgx, gy + cfg.beta * pgy
        a_n = (1 + math.sqrt(4 * a_k * a_k + 1)) / 2
        ref.nesterov(st, gx, gy, pdiv, fixed, (a_k - 1) / a_n, cfg.alpha0, it == 0, (0.0, 1000.0, 0.0, 1000.0))
        a_k = a_n
        if wl_prev is None:
            mu, wl_ref = cfg.mu_max, cfg.wl_ref_frac * abs(wl)
        else:
            mu = min(cfg.mu_max, max(cfg.mu_min, cfg.mu_max ** (1 - (wl - wl_prev) / wl_ref)))
        wl_prev = wl
        lam *= mu
    sinks, _ = ps.pairs()
    assert gpu_pairs == len(sinks) > 0
    # the same bound as the loop without timing: 1 % of each cell's own move
    # plus FP32 rounding of the position
    moved = np.abs(st["ux"] - x0) + np.abs(st["uy"] - y0)
    assert np.median(moved) > 0.1
    err = np.abs(gpu_x - st["ux"]) + np.abs(gpu_y - st["uy"])
    assert np.all(err <= 1e-2 * moved + 1e-3), (err.max(), moved[err.argmax()])
    # and timing moved the placement: the loop without it ends elsewhere
    cfg0 = LoopConfig(die=1000.0, bins=32, beta=0.0, record_every=1 << 30)
    p0 = GlobalPlacer(nl, library, cfg0)
    p0.run(iters=6)
    x_off = p0.positions()[0].cpu().numpy().astype(np.float64)
    p0.g.close()
    assert np.abs(x_off - gpu_x).max() > 10 * err.max()
