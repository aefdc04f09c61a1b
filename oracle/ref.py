"""Python face of the plain FP64 CPU oracle (``tdp_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the test suite, by the package's smoke
check and by the benchmark's CPU-baseline leg, never by the product path.

Every array is in the netlist's own (external) pin and cell numbering.  The
C library is compiled by ``build_oracle()`` (gcc, -O2, IEEE double).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Dict, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tdp_oracle.c")
# TDP_ORACLE_LIB: a separately built copy of the same source (the sanitizer
# test builds one); it is loaded as it is, never rebuilt here
_LIB_PATH = os.environ.get("TDP_ORACLE_LIB") or os.path.join(_HERE, "libtdp_oracle.so")
_lib = None


def build_oracle() -> str:
    cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-o", _LIB_PATH, _SRC, "-lm"]
    subprocess.check_call(cmd)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.environ.get("TDP_ORACLE_LIB") and (not os.path.exists(_LIB_PATH) or
                                                     os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC)):
            build_oracle()
        _lib = ctypes.CDLL(_LIB_PATH)
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _netlist_args(nl) -> list:
    keep = [_i32(nl["pin_cell"]), _f32(nl["pin_off_x"]), _f32(nl["pin_off_y"]),
            _i32(nl["net_ptr"]), _i32(nl["net_pins"]), _i32(nl["cell_type"]),
            _i32(nl["cell_in_ptr"]), _i32(nl["cell_in_pins"]), _i32(nl["cell_out_pin"]),
            np.ascontiguousarray(nl["cell_is_ff"], dtype=np.uint8)]
    args = [ctypes.c_int(int(nl["num_cells"])), ctypes.c_int(int(nl["num_pins"])),
            ctypes.c_int(int(nl["num_nets"]))] + [_p(a) for a in keep]
    return args, keep


def _lib_args(lib) -> list:
    nt = int(lib["num_types"])
    keep = [_f32(lib["slew_axis"]).reshape(nt, -1), _f32(lib["load_axis"]).reshape(nt, -1),
            _f32(lib["delay_lut"]), _f32(lib["slew_lut"]), _f32(lib["pin_cap"])]
    n_slew = keep[0].shape[1]
    n_load = keep[1].shape[1]
    args = [ctypes.c_int(nt), ctypes.c_int(n_slew), ctypes.c_int(n_load)] + [_p(a) for a in keep] + [
        ctypes.c_double(float(np.float32(lib["r_per_um"]))),
        ctypes.c_double(float(np.float32(lib["c_per_um"]))),
        ctypes.c_double(float(np.float32(lib["delay_scale"]))),
        ctypes.c_int(int(lib.get("net_model", 0)))]
    return args, keep


def lut_eval(slew_axis, load_axis, table, slew, load) -> np.ndarray:
    """Bilinear table lookup with clamping (one table)."""
    L = _load()
    sa, la, tb = _f32(slew_axis), _f32(load_axis), _f32(table)
    s, l = _f64(slew), _f64(load)
    out = np.empty(s.shape[0], np.float64)
    L.ora_lut_eval(ctypes.c_int(sa.shape[0]), ctypes.c_int(la.shape[0]), _p(sa), _p(la), _p(tb),
                   ctypes.c_int(s.shape[0]), _p(s), _p(l), _p(out))
    return out


def sta(nl, lib, x=None, y=None, clock_period: Optional[float] = None) -> Dict[str, np.ndarray]:
    """Full static timing analysis.  Returns per-pin arrays and WNS/TNS."""
    L = _load()
    x = _f32(nl["x"] if x is None else x)
    y = _f32(nl["y"] if y is None else y)
    T = float(nl["clock_period"] if clock_period is None else clock_period)
    P, N = int(nl["num_pins"]), int(nl["num_cells"])
    out = {k: np.empty(P, np.float64) for k in ("at", "slew", "rat", "slack", "dnet", "load", "darc")}
    crit = np.empty(N, np.int32)
    summ = np.zeros(3, np.float64)
    na, k1 = _netlist_args(nl)
    la, k2 = _lib_args(lib)
    rc = L.ora_sta(*na, *la, _p(x), _p(y), ctypes.c_double(T), ctypes.c_double(float(nl["setup"])),
                   ctypes.c_double(float(nl["input_slew"])), ctypes.c_double(float(nl["clock_slew"])),
                   _p(out["at"]), _p(out["slew"]), _p(out["rat"]), _p(out["slack"]), _p(out["dnet"]),
                   _p(out["load"]), _p(out["darc"]), _p(crit), _p(summ))
    if rc != 0:
        raise ValueError("timing graph has a cycle")
    out["crit"] = crit
    out["wns"], out["tns"], out["n_fail"] = float(summ[0]), float(summ[1]), int(summ[2])
    out["clock_period"] = T
    return out


def rc_tree(nl, x=None, y=None) -> np.ndarray:
    """Topology of net model 2: the parent of every sink pin in its net's
    spanning tree (-1 at drivers and at pins on no net)."""
    L = _load()
    x = _f32(nl["x"] if x is None else x)
    y = _f32(nl["y"] if y is None else y)
    parent = np.empty(int(nl["num_pins"]), np.int32)
    na, k1 = _netlist_args(nl)
    if L.ora_rc_tree(*na, _p(x), _p(y), _p(parent)) != 0:
        raise MemoryError("oracle: allocation failed")
    return parent


def sta_rf(nl, lib, x=None, y=None, clock_period: Optional[float] = None) -> Dict[str, np.ndarray]:
    """Rise / fall timing.  `lib` carries, beside the single-transition
    library (its tables are the rise tables), delay_fall / slew_fall and
    unate[num_types] (0 positive, 1 negative, 2 non-unate).  Per-pin arrays
    are [P, 2] (rise, fall); crit [N, 2] = 2 j + y per output transition;
    ep_slack [P] at D pins (+inf elsewhere)."""
    L = _load()
    x = _f32(nl["x"] if x is None else x)
    y = _f32(nl["y"] if y is None else y)
    T = float(nl["clock_period"] if clock_period is None else clock_period)
    P, N = int(nl["num_pins"]), int(nl["num_cells"])
    out = {k: np.empty(2 * P, np.float64) for k in ("at", "slew", "rat", "slack")}
    ep = np.empty(P, np.float64)
    crit = np.empty(2 * N, np.int32)
    summ = np.zeros(3, np.float64)
    na, k1 = _netlist_args(nl)
    la, k2 = _lib_args(lib)
    df, sf, un = _f32(lib["delay_fall"]), _f32(lib["slew_fall"]), _i32(lib["unate"])
    rc = L.ora_sta_rf(*na, *la, _p(df), _p(sf), _p(un), _p(x), _p(y), ctypes.c_double(T),
                      ctypes.c_double(float(nl["setup"])), ctypes.c_double(float(nl["input_slew"])),
                      ctypes.c_double(float(nl["clock_slew"])), _p(out["at"]), _p(out["slew"]), _p(out["rat"]),
                      _p(out["slack"]), _p(ep), _p(crit), _p(summ))
    if rc != 0:
        raise ValueError("timing graph has a cycle")
    res = {k: v.reshape(P, 2) for k, v in out.items()}
    res["ep_slack"] = ep
    res["crit"] = crit.reshape(N, 2)
    res["wns"], res["tns"], res["n_fail"] = float(summ[0]), float(summ[1]), int(summ[2])
    res["clock_period"] = T
    return res


def extract_rf(nl, st, n: int = -1, K: int = 1 << 30) -> Dict[str, np.ndarray]:
    """report_timing_endpoint(n, 1) under rise / fall timing (from sta_rf's
    results): paths with their pins' transitions (0 rise, 1 fall)."""
    L = _load()
    P = int(nl["num_pins"])
    E = int(np.count_nonzero(np.asarray(nl["cell_is_ff"])))
    cap = min(K, E)
    depth = int(nl.get("depth", 0)) or P
    ptr = np.zeros(cap + 1, np.int32)
    pins = np.zeros(max(1, cap * min(P, 2 * depth + 2)), np.int32)
    tran = np.zeros_like(pins)
    slack = np.zeros(max(1, cap), np.float64)
    eps = np.zeros(max(1, cap), np.int32)
    na, keep = _netlist_args(nl)
    sl, es, cr = _f64(st["slack"].reshape(-1)), _f64(st["ep_slack"]), _i32(st["crit"].reshape(-1))
    m = L.ora_extract_rf(*na, _p(sl), _p(es), _p(cr), ctypes.c_int(n), ctypes.c_int(cap), _p(ptr), _p(pins),
                         _p(tran), _p(slack), _p(eps))
    if m < 0:
        raise ValueError("timing graph has a cycle")
    w = int(ptr[m])
    return {"num_paths": int(m), "path_ptr": ptr[:m + 1].copy(), "path_pins": pins[:w].copy(),
            "path_tran": tran[:w].copy(), "path_slack": slack[:m].copy(), "path_ep": eps[:m].copy(),
            "path_rank": np.zeros(m, np.int32)}


def endpoint_pins(nl) -> np.ndarray:
    ff = np.nonzero(np.asarray(nl["cell_is_ff"]) != 0)[0]
    ptr = np.asarray(nl["cell_in_ptr"])
    return np.asarray(nl["cell_in_pins"])[ptr[ff]]


def extract(nl, lib, st, n: int = -1, k: int = 1, K: int = 1 << 30,
            slack_limit: float = float("inf")) -> Dict[str, np.ndarray]:
    """report_timing_endpoint(n, k): up to k worst paths at each of the n
    worst endpoints (n < 0: the violated ones), ordered by (slack, endpoint
    pin, rank) and cut to K."""
    L = _load()
    P = int(nl["num_pins"])
    E = int(np.count_nonzero(nl["cell_is_ff"]))
    nsel_max = E
    max_paths = max(1, min(K, nsel_max * k))
    pin_cap = max(16, max_paths * (2 * int(nl.get("depth", 64)) + 8))
    # the longest possible path is bounded by the pin count; grow on demand
    while True:
        path_ptr = np.zeros(max_paths + 1, np.int32)
        path_pins = np.zeros(pin_cap, np.int32)
        path_ep = np.zeros(max_paths, np.int32)
        path_rank = np.zeros(max_paths, np.int32)
        path_slack = np.zeros(max_paths, np.float64)
        sel_ep = np.zeros(max(1, E), np.int32)
        ep_next = np.zeros(max(1, E), np.float64)
        num_sel = np.zeros(1, np.int32)
        na, k1 = _netlist_args(nl)
        arrs = [_f64(st["at"]), _f64(st["rat"]), _f64(st["dnet"]), _f64(st["darc"]), _i32(st["crit"])]
        rc = L.ora_extract(*na, *[_p(a) for a in arrs], ctypes.c_int(n), ctypes.c_int(k),
                           ctypes.c_int(min(K, max_paths)), ctypes.c_double(slack_limit), _p(path_ptr),
                           _p(path_pins), ctypes.c_int(pin_cap), _p(path_ep), _p(path_rank),
                           _p(path_slack), _p(sel_ep), _p(ep_next), _p(num_sel))
        if rc == -2:
            pin_cap *= 2
            continue
        if rc < 0:
            raise ValueError("timing graph has a cycle")
        break
    m = rc
    ns = int(num_sel[0])
    return {"num_paths": m, "path_ptr": path_ptr[:m + 1].copy(),
            "path_pins": path_pins[:path_ptr[m]].copy(), "path_ep": path_ep[:m].copy(),
            "path_rank": path_rank[:m].copy(), "path_slack": path_slack[:m].copy(),
            "sel_ep": sel_ep[:ns].copy(), "ep_next": ep_next[:ns].copy(), "k": k}


def report_timing(nl, lib, st, K: int, slack_limit: float = float("inf")) -> Dict[str, np.ndarray]:
    """report_timing(K): the K worst paths over all endpoints together,
    ordered by (slack, endpoint pin, rank); ``next_slack`` is the slack key
    of the next path after the K-th (+inf when there is none)."""
    L = _load()
    max_paths = max(1, int(K))
    pin_cap = max(16, max_paths * (2 * int(nl.get("depth", 64)) + 8))
    while True:
        path_ptr = np.zeros(max_paths + 1, np.int32)
        path_pins = np.zeros(pin_cap, np.int32)
        path_ep = np.zeros(max_paths, np.int32)
        path_rank = np.zeros(max_paths, np.int32)
        path_slack = np.zeros(max_paths, np.float64)
        nxt = np.zeros(1, np.float64)
        na, k1 = _netlist_args(nl)
        arrs = [_f64(st["at"]), _f64(st["rat"]), _f64(st["dnet"]), _f64(st["darc"]), _i32(st["crit"])]
        rc = L.ora_report_timing(*na, *[_p(a) for a in arrs], ctypes.c_int(int(K)), ctypes.c_double(slack_limit),
                                 _p(path_ptr), _p(path_pins), ctypes.c_int(pin_cap), _p(path_ep), _p(path_rank),
                                 _p(path_slack), _p(nxt))
        if rc == -2:
            pin_cap *= 2
            continue
        if rc < 0:
            raise ValueError("timing graph has a cycle")
        break
    m = rc
    return {"num_paths": m, "path_ptr": path_ptr[:m + 1].copy(),
            "path_pins": path_pins[:path_ptr[m]].copy(), "path_ep": path_ep[:m].copy(),
            "path_rank": path_rank[:m].copy(), "path_slack": path_slack[:m].copy(),
            "next_slack": float(nxt[0])}


def path_list(paths) -> list:
    ptr, pins = paths["path_ptr"], paths["path_pins"]
    return [pins[ptr[i]:ptr[i + 1]].tolist() for i in range(paths["num_paths"])]


class PairState:
    """The maintained pin-pair set P with its weights (dense over pin ids)."""

    def __init__(self, num_pins: int):
        self.in_p = np.zeros(num_pins, np.uint8)
        self.w = np.zeros(num_pins, np.float64)

    def pairs(self):
        sinks = np.nonzero(self.in_p)[0].astype(np.int32)
        return sinks, self.w[sinks].copy()


def pairs_update(state: PairState, paths, wns: float, rule: int = 0, w0: float = 10.0,
                 w1: float = 0.2) -> PairState:
    L = _load()
    m = int(paths["num_paths"])
    ptr, pins, sl = _i32(paths["path_ptr"]), _i32(paths["path_pins"]), _f64(paths["path_slack"])
    if ptr.shape[0] == 0:
        ptr = np.zeros(1, np.int32)
    if pins.shape[0] == 0:
        pins = np.zeros(1, np.int32)
    if sl.shape[0] == 0:
        sl = np.zeros(1, np.float64)
    L.ora_pairs(ctypes.c_int(state.w.shape[0]), ctypes.c_int(m), _p(ptr), _p(pins), _p(sl),
                ctypes.c_double(wns), ctypes.c_int(rule), ctypes.c_double(w0), ctypes.c_double(w1),
                _p(state.in_p), _p(state.w))
    return state


def p2p(nl, pair_sink, pair_w, x=None, y=None):
    """PP = sum w * ((X_s - X_t)^2 + (Y_s - Y_t)^2) and its cell gradient."""
    L = _load()
    x = _f32(nl["x"] if x is None else x)
    y = _f32(nl["y"] if y is None else y)
    N = int(nl["num_cells"])
    gx, gy = np.empty(N, np.float64), np.empty(N, np.float64)
    loss = np.zeros(1, np.float64)
    ps, pw = _i32(pair_sink), _f64(pair_w)
    if ps.shape[0] == 0:
        ps, pw = np.zeros(1, np.int32), np.zeros(1, np.float64)
    na, keep = _netlist_args(nl)
    fixed = np.ascontiguousarray(nl["cell_fixed"], dtype=np.uint8)
    L.ora_p2p(*na, _p(fixed), _p(x), _p(y), ctypes.c_int(len(pair_sink)), _p(ps), _p(pw),
              _p(loss), _p(gx), _p(gy))
    return float(loss[0]), gx, gy


def pair_loss(nl, kind, pair_sink, pair_w, x=None, y=None):
    """Sec. III-C's other pair losses: kind 1 = sum w (|dX| + |dY|),
    kind 2 = sum w sqrt(dX^2 + dY^2); value and cell gradient."""
    L = _load()
    x = _f32(nl["x"] if x is None else x)
    y = _f32(nl["y"] if y is None else y)
    N = int(nl["num_cells"])
    gx, gy = np.empty(N, np.float64), np.empty(N, np.float64)
    loss = np.zeros(1, np.float64)
    ps, pw = _i32(pair_sink), _f64(pair_w)
    if ps.shape[0] == 0:
        ps, pw = np.zeros(1, np.int32), np.zeros(1, np.float64)
    na, keep = _netlist_args(nl)
    fixed = np.ascontiguousarray(nl["cell_fixed"], dtype=np.uint8)
    rc = L.ora_pair_loss(*na, _p(fixed), _p(x), _p(y), ctypes.c_int(kind), ctypes.c_int(len(pair_sink)), _p(ps),
                         _p(pw), _p(loss), _p(gx), _p(gy))
    if rc != 0:
        raise ValueError(f"pair loss kind {kind} failed ({rc})")
    return float(loss[0]), gx, gy


def stns(nl, lib, st, gamma: float = 10.0, x=None, y=None, with_abs: bool = False):
    """Smoothed TNS (frozen cell arcs and start-point arrivals from `st`)
    (with_abs: also, per cell, the summed magnitudes of the net-arc terms of
    its gradient, the scale of the rounding error)."""
    L = _load()
    x = _f32(nl["x"] if x is None else x)
    y = _f32(nl["y"] if y is None else y)
    N = int(nl["num_cells"])
    gx, gy = np.empty(N, np.float64), np.empty(N, np.float64)
    ax, ay = np.empty(N, np.float64), np.empty(N, np.float64)
    val = np.zeros(1, np.float64)
    na, k1 = _netlist_args(nl)
    la, k2 = _lib_args(lib)
    fixed = np.ascontiguousarray(nl["cell_fixed"], dtype=np.uint8)
    at0, darc = _f64(st["at"]), _f64(st["darc"])
    rc = L.ora_stns(*na, *la, _p(fixed), _p(x), _p(y), _p(at0), _p(darc),
                    ctypes.c_double(float(st["clock_period"])), ctypes.c_double(float(nl["setup"])),
                    ctypes.c_double(gamma), _p(val), _p(gx), _p(gy), _p(ax), _p(ay))
    if rc != 0:
        raise ValueError("timing graph has a cycle")
    if with_abs:
        return float(val[0]), gx, gy, ax, ay
    return float(val[0]), gx, gy


def wa(nl, gamma: float = 5.0, x=None, y=None, with_abs: bool = False):
    """Weighted-average wirelength over all nets, both axes, and its gradient
    (with_abs: also, per cell, the summed magnitudes of the summands of its
    pins' derivatives, the scale of the rounding error)."""
    L = _load()
    x = _f32(nl["x"] if x is None else x)
    y = _f32(nl["y"] if y is None else y)
    N = int(nl["num_cells"])
    gx, gy = np.empty(N, np.float64), np.empty(N, np.float64)
    ax, ay = np.empty(N, np.float64), np.empty(N, np.float64)
    val = np.zeros(1, np.float64)
    na, keep = _netlist_args(nl)
    fixed = np.ascontiguousarray(nl["cell_fixed"], dtype=np.uint8)
    L.ora_wa(*na, _p(fixed), _p(x), _p(y), ctypes.c_double(gamma), _p(val), _p(gx), _p(gy), _p(ax), _p(ay))
    if with_abs:
        return float(val[0]), gx, gy, ax, ay
    return float(val[0]), gx, gy


def density(x, y, area, fixed, grid, target: float = 1.0):
    """Bin density, squared-overflow penalty, overflow and gradient.
    grid = dict(x0, y0, bw, bh, gx, gy, R).  Returns a dict with dens
    [gy, gx] (area per bin), value, overflow, grad_x, grad_y."""
    L = _load()
    x, y, area = _f32(x), _f32(y), _f32(area)
    n = int(x.shape[0])
    fixed = np.ascontiguousarray(fixed, dtype=np.uint8)
    gx_, gy_ = int(grid["gx"]), int(grid["gy"])
    dens = np.empty(gx_ * gy_, np.float64)
    val, ovf = np.zeros(1, np.float64), np.zeros(1, np.float64)
    grx, gry = np.empty(n, np.float64), np.empty(n, np.float64)
    d = ctypes.c_double
    L.ora_density(ctypes.c_int(n), _p(x), _p(y), _p(area), _p(fixed), d(float(grid["x0"])), d(float(grid["y0"])),
                  d(float(grid["bw"])), d(float(grid["bh"])), ctypes.c_int(gx_), ctypes.c_int(gy_),
                  ctypes.c_int(int(grid["R"])), d(float(target)), _p(dens), _p(val), _p(ovf), _p(grx), _p(gry))
    return {"dens": dens.reshape(gy_, gx_), "value": float(val[0]), "overflow": float(ovf[0]),
            "grad_x": grx, "grad_y": gry}


def nesterov(state, gx, gy, pdiv, frozen, coef: float, alpha0: float, first: bool, bounds):
    """One Nesterov step.  state: dict of float64 arrays vx, vy, ux, uy, vpx,
    vpy, gpx, gpy (updated in place); bounds = (xlo, xhi, ylo, yhi).
    Returns the step length used."""
    L = _load()
    n = int(state["vx"].shape[0])
    for k in ("vx", "vy", "ux", "uy", "vpx", "vpy", "gpx", "gpy"):
        assert state[k].dtype == np.float64 and state[k].flags.c_contiguous
    gx, gy, pdiv = _f64(gx), _f64(gy), _f64(pdiv)
    frozen = np.ascontiguousarray(frozen, dtype=np.uint8)
    alpha = np.zeros(1, np.float64)
    d = ctypes.c_double
    L.ora_nesterov(ctypes.c_int(n), _p(frozen), _p(pdiv), _p(gx), _p(gy), _p(state["vx"]), _p(state["vy"]),
                   _p(state["ux"]), _p(state["uy"]), _p(state["vpx"]), _p(state["vpy"]), _p(state["gpx"]),
                   _p(state["gpy"]), d(coef), d(alpha0), ctypes.c_int(1 if first else 0),
                   *[d(float(b)) for b in bounds], _p(alpha))
    return float(alpha[0])


def sta_early(nl, lib, hold: float = 0.0, x=None, y=None) -> Dict[str, np.ndarray]:
    """Early arrivals, transitions and arc delays, hold slack at D pins, and
    {whs, ths, n_hold_fail}."""
    L = _load()
    x = _f32(nl["x"] if x is None else x)
    y = _f32(nl["y"] if y is None else y)
    P = int(nl["num_pins"])
    out = {k: np.empty(P, np.float64) for k in ("at", "slew", "darc", "hold_slack")}
    summ = np.zeros(3, np.float64)
    na, k1 = _netlist_args(nl)
    la, k2 = _lib_args(lib)
    rc = L.ora_sta_early(*na, *la, _p(x), _p(y), ctypes.c_double(float(hold)),
                         ctypes.c_double(float(nl["input_slew"])), ctypes.c_double(float(nl["clock_slew"])),
                         _p(out["at"]), _p(out["slew"]), _p(out["darc"]), _p(out["hold_slack"]), _p(summ))
    if rc != 0:
        raise ValueError("timing graph has a cycle")
    out["whs"], out["ths"], out["n_hold_fail"] = float(summ[0]), float(summ[1]), int(summ[2])
    return out
