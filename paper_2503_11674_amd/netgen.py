"""Seeded synthetic netlists, cell libraries and placements.

This module only builds *inputs*: a timing-graph topology, a cell library of
7x7 slew-by-load tables and cell positions.  It contains no timing, path or
loss arithmetic; both the HIP path and the CPU checker consume what it makes.

The paper evaluates on the ICCAD-2015 superblue designs, which are not
available here.  The workloads below are synthetic stand-ins shaped like the
evaluation's netlists: a levelised combinational DAG between flip-flops and
primary inputs, 8 cell types, RC wires whose delay grows with the square of
the wire length (Sec. III-C, Eq. 7) and cell arcs looked up in slew x load
tables.

Netlist model (all arrays numpy, int32 indices / float32 values):
  * cells 0..N-1, randomly numbered.  Types 0..6 are combinational with
    1..4 (or 2..4) input pins and one output pin; type 7 is a flip-flop with
    one D pin (a timing endpoint) and one Q pin (a timing startpoint).
  * primary-input ports (pin_cell == -1) are extra startpoints fixed on the
    die boundary; there are no primary outputs.
  * every output pin / port drives exactly one net; every input pin is a sink
    of exactly one net.  Pins are numbered cell by cell (inputs, then the
    output), ports last.
  * combinational cells sit on levels 1..D; the first input of a level-l cell
    is driven from level l-1, the others from any level below l.  Drivers are
    chosen with probability proportional to a per-driver Exp(1) weight, which
    makes fan-out a mixture of Poissons over an exponential rate, i.e.
    geometric in shape, capped at `fanout_cap`.
  * flip-flop D pins first take dangling combinational outputs from levels
    >= D/2 (deepest first), then drivers from levels >= 3D/4.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional, Tuple

import numpy as np

N_TYPES = 8
FF_TYPE = 7
SLEW_AXIS = np.array([5, 10, 20, 30, 45, 60, 80], dtype=np.float32)          # ps
LOAD_AXIS = np.array([2, 8, 32, 128, 512, 2048, 8192], dtype=np.float32)     # fF
LIB_SEED = 2503


@dataclasses.dataclass
class NetlistConfig:
    name: str
    num_cells: int
    ff_frac: float = 0.10
    pi_frac: float = 0.10
    depth: int = 20
    fanin_lo: int = 1
    fanin_hi: int = 4
    fanout_cap: int = 16
    die: float = 1000.0
    placement: str = "uniform"          # "uniform" | "gmm"
    gmm_clusters: int = 64
    gmm_sigma: float = 30.0
    seed: int = 0
    # per-path selection used by the workload: K paths in total
    top_k_paths: int = 100


# The five workloads (sizes and distributions of the evaluation's stand-ins).
CONFIGS: Dict[str, NetlistConfig] = {
    "C1": NetlistConfig("C1", 2000, depth=20, fanout_cap=16, die=1000.0,
                        placement="uniform", top_k_paths=100),
    "C2": NetlistConfig("C2", 200_000, depth=60, fanout_cap=32, die=4000.0,
                        placement="gmm", top_k_paths=10_000),
    "C3": NetlistConfig("C3", 1_000_000, depth=80, fanout_cap=32, die=7000.0,
                        placement="gmm", top_k_paths=50_000),
    "C5": NetlistConfig("C5", 2_000_000, ff_frac=0.12, depth=100, fanin_lo=2,
                        fanin_hi=4, fanout_cap=32, die=10000.0,
                        placement="gmm", top_k_paths=100_000),
}


def batch_configs() -> List[NetlistConfig]:
    """The uneven batch: 32 netlists of 10k-300k cells and depth 20-80 (seeds
    0-31); size and depth are drawn from each instance's own seed."""
    out = []
    for i in range(32):
        r = np.random.default_rng(10_000 + i)
        u, v = r.random(), r.random()
        n = int(round(10_000 * 30.0 ** u))
        d = min(80, 20 + int(61 * v))
        die = 1000.0 * math.sqrt(n / 62_500.0)
        out.append(NetlistConfig(f"B{i}", n, depth=d, fanout_cap=32, die=die,
                                 placement="gmm", seed=i, top_k_paths=5000))
    return out


# the snapshot netlist of the batch: 500k cells, depth 60, 10 % flip-flops,
# die side scaled with sqrt(N) like the uneven netlists
SNAPSHOT_CONFIG = NetlistConfig("S500k", 500_000, depth=60, fanout_cap=32, die=1000.0 * math.sqrt(8.0),
                                placement="gmm", seed=100, top_k_paths=5000)


def batch_workload(num_snapshots: int = 8, sigma: float = 5.0,
                   snapshot_cells: Optional[int] = None) -> List[Dict[str, np.ndarray]]:
    """The batched workload: the 32 uneven netlists of batch_configs(), then
    num_snapshots placement snapshots of one netlist (positions + N(0, sigma^2),
    jitter seeds 1001, 1002, ...; the snapshots share every other array).  A
    snapshot also carries the unperturbed positions as x_base / y_base: its
    clock period is the one of the unperturbed placement.  Clock periods are
    left to the caller."""
    out = [make_netlist(c) for c in batch_configs()]
    cfg = SNAPSHOT_CONFIG if snapshot_cells is None else scaled(SNAPSHOT_CONFIG, snapshot_cells)
    base = make_netlist(cfg)
    for i in range(num_snapshots):
        snap = dict(base)
        snap["x"], snap["y"] = jitter_positions(base, sigma, seed=1001 + i)
        snap["x_base"], snap["y_base"] = base["x"], base["y"]
        out.append(snap)
    return out


def scaled(cfg: NetlistConfig, num_cells: int, depth: Optional[int] = None,
           seed: Optional[int] = None) -> NetlistConfig:
    c = dataclasses.replace(cfg)
    c.num_cells = num_cells
    if depth is not None:
        c.depth = depth
    if seed is not None:
        c.seed = seed
    c.die = cfg.die * math.sqrt(num_cells / cfg.num_cells)
    return c


# --------------------------------------------------------------------------
# cell library
# --------------------------------------------------------------------------
def make_library(seed: int = LIB_SEED) -> Dict[str, np.ndarray]:
    """8 types, each one 7x7 table indexed [slew][load], monotone
    non-decreasing along both axes and rescaled onto 5..80 ps.  The same table
    serves as the output-transition table.  Input-pin capacitance per type is
    U(1, 5) fF."""
    rng = np.random.default_rng(seed)
    tables = np.zeros((N_TYPES, 7, 7), dtype=np.float64)
    for t in range(N_TYPES):
        a = np.concatenate([[0.0], np.cumsum(rng.random(6))])
        b = np.concatenate([[0.0], np.cumsum(rng.random(6))])
        c = rng.random()
        raw = a[:, None] + b[None, :] + c * a[:, None] * b[None, :]
        lo, hi = raw.min(), raw.max()
        tables[t] = 5.0 + (raw - lo) * (75.0 / (hi - lo))
    pin_cap = 1.0 + 4.0 * rng.random(N_TYPES)
    delay = tables.astype(np.float32)
    return {
        "num_types": N_TYPES,
        "slew_axis": np.tile(SLEW_AXIS, (N_TYPES, 1)).astype(np.float32),
        "load_axis": np.tile(LOAD_AXIS, (N_TYPES, 1)).astype(np.float32),
        "delay_lut": delay,
        "slew_lut": delay.copy(),
        "pin_cap": pin_cap.astype(np.float32),
        "r_per_um": np.float32(0.1),
        "c_per_um": np.float32(0.2),
        # ohm * fF = 1e-3 ps
        "delay_scale": np.float32(1e-3),
    }


RF_SEED = 2504


def make_rf_library(lib: Dict, seed: int = RF_SEED) -> Dict[str, np.ndarray]:
    """Rise / fall form of a library: its tables become the output-rise
    tables; the output-fall tables follow the same recipe from another seed
    (monotone, 5..80 ps; the transition table again equals the delay table);
    arc unateness per type: types 0-2 positive, 3-5 negative, 6 non-unate (the
    flip-flop, type 7, rises and falls by its own tables)."""
    fall = make_library(seed)
    out = dict(lib)
    out["delay_fall"] = fall["delay_lut"].copy()
    out["slew_fall"] = fall["delay_lut"].copy()
    unate = np.zeros(int(lib["num_types"]), np.int32)
    unate[3:6] = 1
    unate[6] = 2
    out["unate"] = unate
    return out


# --------------------------------------------------------------------------
# netlist topology
# --------------------------------------------------------------------------
def _sample_prop(rng, cum: np.ndarray, lo: np.ndarray, hi: np.ndarray) -> np.ndarray:
    """Draw one index from [lo, hi) for every row, with probability
    proportional to the weights whose inclusive prefix sum is `cum`."""
    base = np.where(lo > 0, cum[np.maximum(lo - 1, 0)], 0.0)
    top = cum[hi - 1]
    u = base + rng.random(lo.shape[0]) * (top - base)
    idx = np.searchsorted(cum, u, side="right")
    return np.clip(idx, lo, hi - 1)


def make_netlist(cfg: NetlistConfig) -> Dict[str, np.ndarray]:
    rng = np.random.default_rng(cfg.seed)
    N = int(cfg.num_cells)
    D = int(cfg.depth)
    n_ff = int(round(cfg.ff_frac * N))
    n_comb = N - n_ff
    n_pi = int(round(cfg.pi_frac * N))
    if n_comb < D or n_ff < 1:
        raise ValueError("too few cells for the requested depth")

    # generation-order objects: comb g in [0, n_comb), ff f in [0, n_ff)
    comb_level = 1 + (np.arange(n_comb, dtype=np.int64) * D) // n_comb
    comb_type = rng.integers(0, 7, n_comb)
    fanin = rng.integers(cfg.fanin_lo, cfg.fanin_hi + 1, n_comb)

    # drivers in level order: [PI ports][FF Q][comb outputs by generation]
    n_drv = n_pi + n_ff + n_comb
    drv_level = np.concatenate([np.zeros(n_pi + n_ff, np.int64), comb_level])
    lvl_end = np.searchsorted(drv_level, np.arange(D + 1), side="right")  # drivers with level <= l
    weight = rng.exponential(1.0, n_drv)
    cum = np.cumsum(weight)
    fanout = np.zeros(n_drv, np.int64)
    cap = int(cfg.fanout_cap)

    in_ptr = np.concatenate([[0], np.cumsum(fanin)])
    in_drv = np.full(int(in_ptr[-1]), -1, np.int64)
    comb_start = np.searchsorted(comb_level, np.arange(1, D + 2), side="left")

    def resolve_overflow(picks: np.ndarray, lo: np.ndarray, hi: np.ndarray) -> np.ndarray:
        """Commit picks to `fanout`; picks that would push a driver above the
        cap are re-drawn among drivers still under it (within their range)."""
        picks = picks.copy()
        pending = np.arange(picks.shape[0])
        for _ in range(64):
            p = picks[pending]
            order = np.argsort(p, kind="stable")
            sp = p[order]
            rank = np.arange(sp.shape[0]) - np.searchsorted(sp, sp, side="left")
            bad_sorted = rank >= (cap - fanout[sp])
            good = pending[order[~bad_sorted]]
            np.add.at(fanout, picks[good], 1)
            pending = pending[order[bad_sorted]]
            if pending.shape[0] == 0:
                return picks
            ok_cum = np.cumsum(np.where(fanout < cap, weight, 0.0))
            picks[pending] = _sample_prop(rng, ok_cum, lo[pending], hi[pending])
        raise RuntimeError("could not satisfy the fan-out cap")

    for lvl in range(1, D + 1):
        g0, g1 = comb_start[lvl - 1], comb_start[lvl]
        if g1 <= g0:
            continue
        cells = np.arange(g0, g1)
        slot_cell = np.repeat(cells, fanin[cells])
        first = np.zeros(slot_cell.shape[0], bool)
        first[in_ptr[cells] - in_ptr[g0]] = True
        lo = np.where(first, lvl_end[lvl - 2] if lvl >= 2 else 0, 0)
        hi = np.full(slot_cell.shape[0], lvl_end[lvl - 1])
        picks = _sample_prop(rng, cum, lo, hi)
        picks = resolve_overflow(picks, lo, hi)
        in_drv[in_ptr[g0]:in_ptr[g1]] = picks

    # flip-flop D pins
    comb_drv0 = n_pi + n_ff
    dangling = np.nonzero((fanout[comb_drv0:] == 0) & (comb_level >= max(1, D // 2)))[0] + comb_drv0
    dangling = dangling[np.lexsort((dangling, -drv_level[dangling]))]
    d_drv = np.full(n_ff, -1, np.int64)
    take = min(n_ff, dangling.shape[0])
    d_drv[:take] = dangling[:take]
    fanout[dangling[:take]] += 1
    rest = n_ff - take
    if rest > 0:
        lo_l = max(1, (3 * D) // 4)
        lo = np.full(rest, lvl_end[lo_l - 1])
        hi = np.full(rest, n_drv)
        picks = _sample_prop(rng, cum, lo, hi)
        picks = resolve_overflow(picks, lo, hi)
        d_drv[take:] = picks
    # shuffle which FF gets which driver so FF numbering carries no depth order
    d_drv = d_drv[rng.permutation(n_ff)]

    # ------------------------------------------------------------------
    # external numbering: cells randomly permuted, pins cell by cell
    # ------------------------------------------------------------------
    cell_of_obj = rng.permutation(N)             # obj 0..n_comb-1 comb, then FFs
    comb_cell = cell_of_obj[:n_comb]
    ff_cell = cell_of_obj[n_comb:]
    npins_cell = np.empty(N, np.int64)
    npins_cell[comb_cell] = fanin + 1
    npins_cell[ff_cell] = 2
    cell_pin0 = np.concatenate([[0], np.cumsum(npins_cell)])[:-1]
    n_cell_pins = int(npins_cell.sum())
    P = n_cell_pins + n_pi

    pin_cell = np.empty(P, np.int64)
    pin_cell[:n_cell_pins] = np.repeat(np.arange(N), npins_cell)
    pin_cell[n_cell_pins:] = -1

    cell_type = np.empty(N, np.int64)
    cell_type[comb_cell] = comb_type
    cell_type[ff_cell] = FF_TYPE
    cell_is_ff = np.zeros(N, np.uint8)
    cell_is_ff[ff_cell] = 1
    cell_nin = np.empty(N, np.int64)
    cell_nin[comb_cell] = fanin
    cell_nin[ff_cell] = 1
    cell_in_ptr = np.concatenate([[0], np.cumsum(cell_nin)])
    # input pins are the first nin pins of each cell, in arc order
    cell_in_pins = np.repeat(cell_pin0, cell_nin) + (np.arange(int(cell_in_ptr[-1])) - np.repeat(cell_in_ptr[:-1], cell_nin))
    cell_out_pin = cell_pin0 + cell_nin

    # driver pin of each driver object
    drv_pin = np.empty(n_drv, np.int64)
    drv_pin[:n_pi] = n_cell_pins + np.arange(n_pi)
    drv_pin[n_pi:n_pi + n_ff] = cell_out_pin[ff_cell]
    drv_pin[comb_drv0:] = cell_out_pin[comb_cell]

    # sinks: comb inputs then FF D pins
    comb_in_pin = (np.repeat(cell_pin0[comb_cell], fanin)
                   + (np.arange(int(in_ptr[-1])) - np.repeat(in_ptr[:-1], fanin)))
    ff_d_pin = cell_pin0[ff_cell]
    sink_pin = np.concatenate([comb_in_pin, ff_d_pin])
    sink_drv = np.concatenate([in_drv, d_drv])
    assert (sink_drv >= 0).all()

    # nets: one per driver; numbered by driver pin id; sinks by pin id
    net_of_drv = np.argsort(drv_pin, kind="stable")   # net id -> driver obj
    drv_net = np.empty(n_drv, np.int64)
    drv_net[net_of_drv] = np.arange(n_drv)
    s_net = drv_net[sink_drv]
    order = np.lexsort((sink_pin, s_net))
    s_net_sorted = s_net[order]
    counts = np.bincount(s_net_sorted, minlength=n_drv)
    net_ptr = np.zeros(n_drv + 1, np.int64)
    net_ptr[1:] = np.cumsum(counts + 1)
    net_pins = np.empty(int(net_ptr[-1]), np.int64)
    net_pins[net_ptr[:-1]] = drv_pin[net_of_drv]
    pos_in_net = np.arange(order.shape[0]) - np.searchsorted(s_net_sorted, s_net_sorted, side="left")
    net_pins[net_ptr[s_net_sorted] + 1 + pos_in_net] = sink_pin[order]

    # ------------------------------------------------------------------
    # placement: cell centres, pin offsets, boundary ports
    # ------------------------------------------------------------------
    W = float(cfg.die)
    if cfg.placement == "uniform":
        x = rng.random(N) * W
        y = rng.random(N) * W
    elif cfg.placement == "gmm":
        centres = rng.random((cfg.gmm_clusters, 2)) * W
        which = rng.integers(0, cfg.gmm_clusters, N)
        x = centres[which, 0] + rng.normal(0.0, cfg.gmm_sigma, N)
        y = centres[which, 1] + rng.normal(0.0, cfg.gmm_sigma, N)
        x = np.clip(x, 0.0, W)
        y = np.clip(y, 0.0, W)
    else:
        raise ValueError(cfg.placement)
    off_x = rng.random(P) - 0.5
    off_y = rng.random(P) - 0.5
    # ports: uniform along the perimeter; their offsets are absolute positions
    per = rng.random(n_pi) * 4.0 * W
    side = np.minimum((per // W).astype(np.int64), 3)
    t = per - side * W
    px = np.select([side == 0, side == 1, side == 2, side == 3], [t, np.full_like(t, W), W - t, np.zeros_like(t)])
    py = np.select([side == 0, side == 1, side == 2, side == 3], [np.zeros_like(t), t, np.full_like(t, W), W - t])
    off_x[n_cell_pins:] = px
    off_y[n_cell_pins:] = py

    i32 = lambda a: np.ascontiguousarray(a, dtype=np.int32)
    f32 = lambda a: np.ascontiguousarray(a, dtype=np.float32)
    return {
        "name": cfg.name,
        "num_cells": N,
        "num_pins": P,
        "num_nets": n_drv,
        "pin_cell": i32(pin_cell),
        "pin_off_x": f32(off_x),
        "pin_off_y": f32(off_y),
        "net_ptr": i32(net_ptr),
        "net_pins": i32(net_pins),
        "cell_type": i32(cell_type),
        "cell_in_ptr": i32(cell_in_ptr),
        "cell_in_pins": i32(cell_in_pins),
        "cell_out_pin": i32(cell_out_pin),
        "cell_is_ff": np.ascontiguousarray(cell_is_ff, dtype=np.uint8),
        "cell_fixed": np.zeros(N, np.uint8),
        "x": f32(x),
        "y": f32(y),
        "depth": D,
        "clock_period": np.float32(0.0),   # set by the caller from a timing run
        "setup": np.float32(0.0),
        "input_slew": np.float32(10.0),
        "clock_slew": np.float32(10.0),
    }


def clock_period_for_fail_fraction(endpoint_arrivals: np.ndarray, fail_frac: float = 0.05) -> float:
    """Clock period that makes floor(fail_frac * E) endpoints fail: the midpoint
    between the q-th and (q+1)-th smallest endpoint arrival, q = ceil((1-f) E).
    Endpoint arrival times do not depend on the clock period, so any timing
    run at the initial placement supplies them."""
    a = np.sort(np.asarray(endpoint_arrivals, dtype=np.float64))
    E = a.shape[0]
    q = int(math.ceil((1.0 - fail_frac) * E))
    q = min(max(q, 1), E)
    if q >= E:
        return float(a[-1] + 1.0)
    return float(0.5 * (a[q - 1] + a[q]))


def jitter_positions(nl: Dict[str, np.ndarray], sigma: float, seed: int) -> Tuple[np.ndarray, np.ndarray]:
    """A perturbed placement snapshot: positions + N(0, sigma^2), clamped to the
    bounding box of the original placement."""
    rng = np.random.default_rng(seed)
    x = nl["x"].astype(np.float64)
    y = nl["y"].astype(np.float64)
    lo_x, hi_x, lo_y, hi_y = x.min(), x.max(), y.min(), y.max()
    x = np.clip(x + rng.normal(0, sigma, x.shape[0]), lo_x, hi_x)
    y = np.clip(y + rng.normal(0, sigma, y.shape[0]), lo_y, hi_y)
    return x.astype(np.float32), y.astype(np.float32)


def netlist_stats(nl: Dict[str, np.ndarray]) -> Dict[str, float]:
    ptr = nl["net_ptr"]
    fo = np.diff(ptr) - 1
    cin = np.diff(nl["cell_in_ptr"])
    comb = nl["cell_is_ff"] == 0
    return {
        "cells": int(nl["num_cells"]),
        "pins": int(nl["num_pins"]),
        "nets": int(nl["num_nets"]),
        "ff": int((~comb).sum()),
        "mean_fanout": float(fo.mean()),
        "max_fanout": int(fo.max()),
        "dangling_nets": int((fo == 0).sum()),
        "mean_fanin": float(cin[comb].mean()),
    }
