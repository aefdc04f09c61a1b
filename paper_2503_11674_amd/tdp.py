"""Python binding of the HIP timing library (``libtdp.so``, ``include/tdp.h``).

Argument marshalling only: every step runs in the library's HIP kernels.
PyTorch supplies device memory and the current stream.  Importing this module
fails loudly if the compiled library is missing; there is no CPU fallback.

Module-level functions carry the C names (``tdp_sta_build`` ...).
``TimingGraph`` owns a graph handle; ``P2PLoss`` and ``SmoothTNS`` are the
autograd Functions for the pin-to-pin loss (Eqs. 8, 10) and the smoothed TNS.
"""
from __future__ import annotations

import ctypes
import math
import os
from typing import Dict, Optional, Sequence

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtdp.so")
if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2503_11674_amd.build_lib`")
_lib = ctypes.CDLL(LIB_PATH)

TDP_F32, TDP_F64 = 0, 1
STAGES = ["netpass", "forward", "endpoint", "backward", "select", "search", "order", "walk", "pairs",
          "p2p_fwd", "p2p_bwd", "stns", "wa", "density"]
_STATUS = {0: "ok", 1: "invalid argument", 2: "combinational cycle", 3: "out of memory", 4: "device error",
           5: "capacity exceeded", 6: "call out of order", 7: "unsupported"}

_p = ctypes.c_void_p
_i32 = ctypes.c_int32
_f32 = ctypes.c_float


class tdp_netlist(ctypes.Structure):
    _fields_ = [("num_cells", _i32), ("num_pins", _i32), ("num_nets", _i32), ("pin_cell", _p),
                ("pin_off_x", _p), ("pin_off_y", _p), ("net_ptr", _p), ("net_pins", _p), ("cell_type", _p),
                ("cell_in_ptr", _p), ("cell_in_pins", _p), ("cell_out_pin", _p), ("cell_is_ff", _p),
                ("cell_fixed", _p), ("clock_period_ps", _f32), ("setup_ps", _f32), ("input_slew_ps", _f32),
                ("clock_slew_ps", _f32)]


class tdp_library(ctypes.Structure):
    _fields_ = [("num_types", _i32), ("n_slew", _i32), ("n_load", _i32), ("slew_axis", _p), ("load_axis", _p),
                ("delay_lut", _p), ("slew_lut", _p), ("pin_cap", _p), ("r_per_um", _f32), ("c_per_um", _f32),
                ("delay_scale", _f32), ("net_model", _i32)]


class tdp_density_grid(ctypes.Structure):
    _fields_ = [("x0", _f32), ("y0", _f32), ("bin_w", _f32), ("bin_h", _f32), ("bins_x", _i32), ("bins_y", _i32),
                ("radius", _i32), ("target", _f32)]


class tdp_paths(ctypes.Structure):
    _fields_ = [("max_paths", _i32), ("d_num_paths", _p), ("path_ptr", _p), ("path_pins", _p), ("path_ep", _p),
                ("path_rank", _p), ("path_slack", _p)]


def _sig(name, *args):
    f = getattr(_lib, name)
    f.restype = ctypes.c_int
    f.argtypes = list(args)
    return f


_P = ctypes.POINTER
tdp_sta_build = _sig("tdp_sta_build", _P(tdp_netlist), _P(tdp_library), ctypes.c_int, _i32, _i32, ctypes.c_int,
                     _P(_p))
tdp_batch_build = _sig("tdp_batch_build", _P(_P(tdp_netlist)), _i32, _P(tdp_library), ctypes.c_int, _i32, _i32,
                       ctypes.c_int, _P(_p))
tdp_batch_offsets = _sig("tdp_batch_offsets", _p, _p, _p)
tdp_destroy = _lib.tdp_destroy
tdp_destroy.restype = None
tdp_destroy.argtypes = [_p]
tdp_sta_set_clock = _sig("tdp_sta_set_clock", _p, _f32, _f32)
tdp_sta_update = _sig("tdp_sta_update", _p, _p, _p, _p)
tdp_sta_update_arrivals = _sig("tdp_sta_update_arrivals", _p, _p, _p, _p)
tdp_sta_update_required = _sig("tdp_sta_update_required", _p, _p)
tdp_sta_summary = _sig("tdp_sta_summary", _p, _P(ctypes.c_double), _P(ctypes.c_double), _P(_i32), _p)
tdp_batch_summary = _sig("tdp_batch_summary", _p, _p, _p, _p, _p)
tdp_sta_export = _sig("tdp_sta_export", _p, _p, _p, _p, _p, _p, _p, _p, _p)
tdp_sta_export_crit = _sig("tdp_sta_export_crit", _p, _p, _p)
tdp_extract_paths = _sig("tdp_extract_paths", _p, _i32, _i32, _i32, _f32, _p, _P(tdp_paths))
tdp_report_timing = _sig("tdp_report_timing", _p, _i32, _f32, _p, _P(tdp_paths))
class tdp_rf_tables(ctypes.Structure):
    _fields_ = [("delay_fall", _p), ("slew_fall", _p), ("unate", _p)]


tdp_rf_setup = _sig("tdp_rf_setup", _p, _P(tdp_rf_tables))
tdp_sta_update_rf = _sig("tdp_sta_update_rf", _p, _p, _p, _p)
tdp_sta_rf_summary = _sig("tdp_sta_rf_summary", _p, _P(ctypes.c_double), _P(ctypes.c_double), _P(_i32), _p)
tdp_sta_rf_export = _sig("tdp_sta_rf_export", _p, _p, _p, _p, _p, _p)
tdp_extract_paths_rf = _sig("tdp_extract_paths_rf", _p, _i32, _i32, _p, _P(tdp_paths), _P(_p))
tdp_sta_update_arrivals_incremental = _sig("tdp_sta_update_arrivals_incremental", _p, _p, _p, _p, _i32, _p)
tdp_sta_views = _sig("tdp_sta_views", _p, _P(_p), _P(_p), _P(_p))
tdp_report_timing_noalloc = _sig("tdp_report_timing_noalloc", _p, _i32, _f32, _p, _P(tdp_paths))
tdp_paths_count = _sig("tdp_paths_count", _p, _P(_i32), _P(_i32), _p)
tdp_pairs_update = _sig("tdp_pairs_update", _p, _i32, _f32, _f32, _p)
tdp_pairs_reset = _sig("tdp_pairs_reset", _p, _p)
tdp_pairs_export = _sig("tdp_pairs_export", _p, _p, _p, _p)
tdp_pairs_import = _sig("tdp_pairs_import", _p, _p, _p, _p)
tdp_pairs_count = _sig("tdp_pairs_count", _p, _P(_i32), _p)
tdp_p2p_loss_fwd = _sig("tdp_p2p_loss_fwd", _p, _p, _p, _p, _p)
tdp_p2p_loss_bwd = _sig("tdp_p2p_loss_bwd", _p, _p, _p, _p, _p, _p, _p)
tdp_pair_loss_fwd = _sig("tdp_pair_loss_fwd", _p, _i32, _p, _p, _p, _p)
tdp_pair_loss_bwd = _sig("tdp_pair_loss_bwd", _p, _i32, _p, _p, _p, _p, _p, _p)
tdp_stns_fwd = _sig("tdp_stns_fwd", _p, _p, _p, _f32, _p, _p)
tdp_stns_bwd = _sig("tdp_stns_bwd", _p, _p, _p, _p, _p)
tdp_wa_fwd_bwd = _sig("tdp_wa_fwd_bwd", _p, _p, _p, _f32, _p, _p, _p, _p)
tdp_wa_fwd_bwd_at_update = _sig("tdp_wa_fwd_bwd_at_update", _p, _f32, _p, _p, _p, _p)
tdp_sta_update_early = _sig("tdp_sta_update_early", _p, _f32, _p)
tdp_sta_early_summary = _sig("tdp_sta_early_summary", _p, _P(ctypes.c_double), _P(ctypes.c_double), _P(_i32), _p)
tdp_sta_early_export = _sig("tdp_sta_early_export", _p, _p, _p, _p, _p, _p)
tdp_density_setup = _sig("tdp_density_setup", _p, _P(tdp_density_grid), _p)
tdp_density_fwd_bwd = _sig("tdp_density_fwd_bwd", _p, _p, _p, _f32, _p, _p, _p, _p, _p, _p)
tdp_nesterov_step = _sig("tdp_nesterov_step", _p, _p, _p, _p, _p, _p, _p, _p, _p, _p, _p, _p, ctypes.c_double,
                         ctypes.c_double, _i32, _f32, _f32, _f32, _f32, _p, _p)
tdp_abs_sum = _sig("tdp_abs_sum", _p, _p, _p, _p, _p)
tdp_profile_enable = _sig("tdp_profile_enable", _p, _i32)
tdp_profile_read = _sig("tdp_profile_read", _p, _p, _p)
tdp_set_tuning = _sig("tdp_set_tuning", _p, _i32, _i32, _i32, _i32)
tdp_autotune = _sig("tdp_autotune", _p, _p, _p, _i32, _i32, _i32, _i32, _p, _p)
tdp_graph_info = _sig("tdp_graph_info", _p, _p)
tdp_status_str = _lib.tdp_status_str
tdp_status_str.restype = ctypes.c_char_p
tdp_status_str.argtypes = [ctypes.c_int]
tdp_last_error = _lib.tdp_last_error
tdp_last_error.restype = ctypes.c_char_p
tdp_last_error.argtypes = [_p]

EXPORTED = ["tdp_sta_build", "tdp_batch_build", "tdp_batch_offsets", "tdp_destroy", "tdp_sta_set_clock",
            "tdp_sta_update", "tdp_sta_update_arrivals", "tdp_sta_update_required", "tdp_sta_update_arrivals_incremental", "tdp_sta_summary", "tdp_batch_summary", "tdp_sta_export", "tdp_sta_export_crit", "tdp_sta_views",
            "tdp_extract_paths", "tdp_report_timing", "tdp_report_timing_noalloc", "tdp_rf_setup", "tdp_sta_update_rf",
            "tdp_sta_rf_summary", "tdp_sta_rf_export", "tdp_extract_paths_rf", "tdp_paths_count", "tdp_pairs_update", "tdp_pairs_reset", "tdp_pairs_export",
            "tdp_pairs_import", "tdp_pairs_count", "tdp_p2p_loss_fwd", "tdp_p2p_loss_bwd",
            "tdp_pair_loss_fwd", "tdp_pair_loss_bwd", "tdp_stns_fwd",
            "tdp_stns_bwd", "tdp_wa_fwd_bwd", "tdp_wa_fwd_bwd_at_update", "tdp_sta_update_early",
            "tdp_sta_early_summary", "tdp_sta_early_export", "tdp_density_setup",
            "tdp_density_fwd_bwd", "tdp_nesterov_step", "tdp_abs_sum", "tdp_profile_enable", "tdp_profile_read", "tdp_set_tuning",
            "tdp_autotune", "tdp_graph_info", "tdp_status_str", "tdp_last_error"]


class TdpError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{_STATUS.get(status, status)}: {message}")
        self.status = status


def _check(st: int, g=None):
    if st != 0:
        msg = tdp_last_error(g)
        raise TdpError(st, msg.decode() if msg else "")


def _ptr(t) -> int:
    if t is None:
        return None
    if isinstance(t, np.ndarray):
        return t.ctypes.data
    return t.data_ptr()


def _stream(stream=None) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


def _cuda_f32(t: torch.Tensor, n: Optional[int] = None) -> torch.Tensor:
    """A contiguous float32 CUDA tensor, of n elements when n is given (the
    kernels index it by cell and would otherwise read or write past its end)."""
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
        raise ValueError("expected a contiguous float32 CUDA tensor")
    if n is not None and t.numel() != n:
        raise ValueError(f"expected {n} elements (one per cell), got {t.numel()}")
    return t


class _NetlistHolder:
    """Keeps the numpy arrays of a netlist alive behind a tdp_netlist."""

    def __init__(self, nl: Dict):
        a = lambda k, dt: np.ascontiguousarray(nl[k], dtype=dt)
        self.keep = {
            "pin_cell": a("pin_cell", np.int32), "pin_off_x": a("pin_off_x", np.float32),
            "pin_off_y": a("pin_off_y", np.float32), "net_ptr": a("net_ptr", np.int32),
            "net_pins": a("net_pins", np.int32), "cell_type": a("cell_type", np.int32),
            "cell_in_ptr": a("cell_in_ptr", np.int32), "cell_in_pins": a("cell_in_pins", np.int32),
            "cell_out_pin": a("cell_out_pin", np.int32), "cell_is_ff": a("cell_is_ff", np.uint8),
            "cell_fixed": np.ascontiguousarray(nl.get("cell_fixed", np.zeros(int(nl["num_cells"]), np.uint8)),
                                               dtype=np.uint8),
        }
        k = self.keep
        self.s = tdp_netlist(int(nl["num_cells"]), int(nl["num_pins"]), int(nl["num_nets"]),
                             *[k[n].ctypes.data for n in ("pin_cell", "pin_off_x", "pin_off_y", "net_ptr",
                                                          "net_pins", "cell_type", "cell_in_ptr", "cell_in_pins",
                                                          "cell_out_pin", "cell_is_ff", "cell_fixed")],
                             float(nl["clock_period"]), float(nl["setup"]), float(nl["input_slew"]),
                             float(nl["clock_slew"]))


class _LibraryHolder:
    def __init__(self, lib: Dict):
        nt = int(lib["num_types"])
        self.keep = [np.ascontiguousarray(lib[k], dtype=np.float32) for k in
                     ("slew_axis", "load_axis", "delay_lut", "slew_lut", "pin_cap")]
        ns = self.keep[0].reshape(nt, -1).shape[1]
        nl = self.keep[1].reshape(nt, -1).shape[1]
        self.s = tdp_library(nt, ns, nl, *[a.ctypes.data for a in self.keep], float(lib["r_per_um"]),
                             float(lib["c_per_um"]), float(lib["delay_scale"]), int(lib.get("net_model", 0)))


class TimingGraph:
    """A timing graph on one GPU: STA, top-K path extraction, the pin-pair set
    and the differentiable losses over it."""

    def __init__(self, netlist, lib: Dict, precision: str = "f32", max_paths: int = 1 << 16, max_k: int = 1,
                 device: int = 0):
        self.prec = TDP_F64 if precision == "f64" else TDP_F32
        self.device = device
        self._lib_h = _LibraryHolder(lib)
        h = ctypes.c_void_p()
        if isinstance(netlist, (list, tuple)):
            self._nl_h = [_NetlistHolder(n) for n in netlist]
            arr = (_P(tdp_netlist) * len(self._nl_h))(*[ctypes.pointer(n.s) for n in self._nl_h])
            _check(tdp_batch_build(arr, len(self._nl_h), ctypes.byref(self._lib_h.s), self.prec, max_paths, max_k,
                                   device, ctypes.byref(h)))
            self.num_inst = len(self._nl_h)
        else:
            self._nl_h = [_NetlistHolder(netlist)]
            _check(tdp_sta_build(ctypes.byref(self._nl_h[0].s), ctypes.byref(self._lib_h.s), self.prec, max_paths,
                                 max_k, device, ctypes.byref(h)))
            self.num_inst = 1
        self.h = h.value
        info = np.zeros(8, np.int32)
        _check(tdp_graph_info(self.h, info.ctypes.data), self.h)
        (self.num_cells, self.num_pins, self.num_nets, self.depth, self.num_endpoints, self.num_startpoints,
         self.num_comb, self.num_sinks) = [int(v) for v in info]
        self.max_paths = max_paths
        self.max_k = max_k
        self._paths = None
        self._dn_grid = None

    def close(self):
        if getattr(self, "h", None):
            tdp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _cells(self, t, optional: bool = False):
        """A per-cell float32 device tensor of this graph (positions, gradients)."""
        if t is None and optional:
            return None
        return _cuda_f32(t, self.num_cells)

    # ------------------------------------------------------------- STA
    def set_clock(self, period: float, setup: float = 0.0):
        _check(tdp_sta_set_clock(self.h, period, setup), self.h)

    def sta_update(self, x: torch.Tensor, y: torch.Tensor, stream=None):
        _check(tdp_sta_update(self.h, _ptr(self._cells(x)), _ptr(self._cells(y)), _stream(stream)), self.h)

    def sta_update_arrivals(self, x: torch.Tensor, y: torch.Tensor, stream=None):
        _check(tdp_sta_update_arrivals(self.h, _ptr(self._cells(x)), _ptr(self._cells(y)), _stream(stream)), self.h)

    def sta_update_arrivals_incremental(self, x: torch.Tensor, y: torch.Tensor, cells: torch.Tensor, stream=None):
        """Arrival pass re-timing only what the listed (moved) cells change;
        `cells` is a device int32 tensor of external cell ids."""
        if not cells.is_cuda or cells.dtype != torch.int32:
            raise ValueError("cells must be an int32 tensor on the GPU")
        cells = cells.contiguous()
        _check(tdp_sta_update_arrivals_incremental(self.h, _ptr(self._cells(x)), _ptr(self._cells(y)),
                                                   _ptr(cells), int(cells.numel()), _stream(stream)), self.h)

    def sta_update_required(self, stream=None):
        _check(tdp_sta_update_required(self.h, _stream(stream)), self.h)

    def summary(self, stream=None):
        w, t, n = ctypes.c_double(), ctypes.c_double(), _i32()
        _check(tdp_sta_summary(self.h, ctypes.byref(w), ctypes.byref(t), ctypes.byref(n), _stream(stream)), self.h)
        return w.value, t.value, n.value

    def batch_summary(self, stream=None):
        w = np.zeros(self.num_inst)
        t = np.zeros(self.num_inst)
        n = np.zeros(self.num_inst, np.int32)
        _check(tdp_batch_summary(self.h, w.ctypes.data, t.ctypes.data, n.ctypes.data, _stream(stream)), self.h)
        return w, t, n

    def batch_offsets(self):
        pb = np.zeros(self.num_inst + 1, np.int32)
        cb = np.zeros(self.num_inst + 1, np.int32)
        _check(tdp_batch_offsets(self.h, pb.ctypes.data, cb.ctypes.data), self.h)
        return pb, cb

    def export(self, stream=None) -> Dict[str, torch.Tensor]:
        dev = torch.device("cuda", self.device)
        out = {k: torch.empty(self.num_pins, dtype=torch.float64, device=dev)
               for k in ("at", "rat", "slack", "slew", "dnet", "load", "darc")}
        _check(tdp_sta_export(self.h, *[_ptr(out[k]) for k in ("at", "rat", "slack", "slew", "dnet", "load", "darc")],
                              _stream(stream)), self.h)
        crit = torch.empty(self.num_cells, dtype=torch.int32, device=dev)
        _check(tdp_sta_export_crit(self.h, _ptr(crit), _stream(stream)), self.h)
        out["crit"] = crit
        return out

    def views(self) -> Dict[str, torch.Tensor]:
        """Zero-copy tensors over the graph's own arrival and required times
        (graph precision, device pin order) and the map from external pin id
        to that order (int32): at[pin_index[p]] is pin p's arrival.  They
        hold the next update's values once it runs; do not use them after
        close(), and do not write to them (torch's import of a device array
        has no read-only flag)."""
        at, rat, idx = _p(), _p(), _p()
        _check(tdp_sta_views(self.h, ctypes.byref(at), ctypes.byref(rat), ctypes.byref(idx)), self.h)
        ts = "<f8" if self.prec == TDP_F64 else "<f4"
        dev = torch.device("cuda", self.device)
        return {"at": torch.as_tensor(_DeviceView(at.value, self.num_pins, ts, self), device=dev),
                "rat": torch.as_tensor(_DeviceView(rat.value, self.num_pins, ts, self), device=dev),
                "pin_index": torch.as_tensor(_DeviceView(idx.value, self.num_pins, "<i4", self), device=dev)}

    # ----------------------------------------------------------- paths
    def extract_paths(self, n: int = -1, k: int = 1, K: Optional[int] = None,
                      slack_limit: float = math.inf, stream=None) -> tdp_paths:
        p = tdp_paths()
        K = self.max_paths if K is None else K
        _check(tdp_extract_paths(self.h, n, k, K, slack_limit, _stream(stream), ctypes.byref(p)), self.h)
        self._paths = p
        return p

    def report_timing(self, K: int, slack_limit: float = math.inf, stream=None) -> tdp_paths:
        """report_timing(K): the K worst paths over the whole design (per
        instance of a batched graph); replaces the last extraction's paths.
        Synchronises the stream."""
        p = tdp_paths()
        _check(tdp_report_timing(self.h, K, slack_limit, _stream(stream), ctypes.byref(p)), self.h)
        self._paths = p
        return p

    # ----------------------------------------------------- rise / fall
    def rf_setup(self, lib: Dict):
        """Rise / fall tables (delay_fall, slew_fall, unate) of a library; its
        main tables are the rise tables."""
        df = np.ascontiguousarray(lib["delay_fall"], np.float32)
        sf = np.ascontiguousarray(lib["slew_fall"], np.float32)
        un = np.ascontiguousarray(lib["unate"], np.int32)
        t = tdp_rf_tables(df.ctypes.data, sf.ctypes.data, un.ctypes.data)
        _check(tdp_rf_setup(self.h, ctypes.byref(t)), self.h)

    def sta_update_rf(self, x: torch.Tensor, y: torch.Tensor, stream=None):
        _check(tdp_sta_update_rf(self.h, _ptr(self._cells(x)), _ptr(self._cells(y)), _stream(stream)), self.h)

    def rf_summary(self, stream=None):
        w, t, n = ctypes.c_double(), ctypes.c_double(), ctypes.c_int32()
        _check(tdp_sta_rf_summary(self.h, ctypes.byref(w), ctypes.byref(t), ctypes.byref(n), _stream(stream)), self.h)
        return w.value, t.value, n.value

    def rf_export(self, stream=None) -> Dict[str, torch.Tensor]:
        """[num_pins, 2] double tensors (rise, fall) in external pin order."""
        dev = torch.device("cuda", self.device)
        out = {k: torch.empty(2 * self.num_pins, dtype=torch.float64, device=dev)
               for k in ("at", "rat", "slack", "slew")}
        _check(tdp_sta_rf_export(self.h, *[_ptr(out[k]) for k in ("at", "rat", "slack", "slew")], _stream(stream)),
               self.h)
        return {k: v.view(self.num_pins, 2) for k, v in out.items()}

    def extract_paths_rf(self, n: int = -1, K: Optional[int] = None, stream=None) -> tdp_paths:
        K = self.max_paths if K is None else K
        p = tdp_paths()
        tran = _p()
        _check(tdp_extract_paths_rf(self.h, n, K, _stream(stream), ctypes.byref(p), ctypes.byref(tran)), self.h)
        self._paths = p
        self._path_tran = tran.value
        return p

    def paths_rf(self, stream=None) -> Dict[str, np.ndarray]:
        """paths() of the last rise / fall extraction, with path_tran."""
        out = self.paths(stream)
        n = int(out["path_ptr"][-1]) if len(out["path_ptr"]) else 0
        tr = torch.empty(max(n, 1), dtype=torch.uint8, device=torch.device("cuda", self.device))
        if n:
            _copy_dev(tr, self._path_tran, n)
        out["path_tran"] = tr[:n].cpu().numpy().astype(np.int32)
        return out

    def report_timing_noalloc(self, K: int, slack_limit: float = math.inf, stream=None) -> tdp_paths:
        """report_timing(K) with its node store in the library's fixed device
        array (no device allocation); TdpError (capacity) when the graph's
        store does not fit it."""
        p = tdp_paths()
        _check(tdp_report_timing_noalloc(self.h, K, slack_limit, _stream(stream), ctypes.byref(p)), self.h)
        self._paths = p
        return p

    def paths_count(self, stream=None):
        n, pins = _i32(), _i32()
        _check(tdp_paths_count(self.h, ctypes.byref(n), ctypes.byref(pins), _stream(stream)), self.h)
        return n.value, pins.value

    def paths(self, stream=None) -> Dict[str, np.ndarray]:
        """Host copy of the last extraction (synchronises)."""
        m, npins = self.paths_count(stream)
        p = self._paths
        dev = torch.device("cuda", self.device)

        def grab(ptr, n, dt):
            t = torch.empty(max(n, 1), dtype=dt, device=dev)
            if n > 0:
                _copy_dev(t, ptr, n * t.element_size())
            return t[:n].cpu().numpy()

        sdt = torch.float64 if self.prec == TDP_F64 else torch.float32
        return {"num_paths": m,
                "path_ptr": grab(p.path_ptr, m + 1, torch.int32),
                "path_pins": grab(p.path_pins, npins, torch.int32),
                "path_ep": grab(p.path_ep, m, torch.int32),
                "path_rank": grab(p.path_rank, m, torch.int32),
                "path_slack": grab(p.path_slack, m, sdt).astype(np.float64)}

    # ----------------------------------------------------------- pairs
    def pairs_update(self, rule: int = 0, w0: float = 10.0, w1: float = 0.2, stream=None):
        _check(tdp_pairs_update(self.h, rule, w0, w1, _stream(stream)), self.h)

    def pairs_reset(self, stream=None):
        _check(tdp_pairs_reset(self.h, _stream(stream)), self.h)

    def pairs_export(self, stream=None):
        w = np.zeros(self.num_pins, np.float32)
        m = np.zeros(self.num_pins, np.uint8)
        _check(tdp_pairs_export(self.h, w.ctypes.data, m.ctypes.data, _stream(stream)), self.h)
        return w, m

    def pairs_import(self, w: np.ndarray, in_p: np.ndarray, stream=None):
        w = np.ascontiguousarray(w, dtype=np.float32)
        m = np.ascontiguousarray(in_p, dtype=np.uint8)
        _check(tdp_pairs_import(self.h, w.ctypes.data, m.ctypes.data, _stream(stream)), self.h)

    def pairs_count(self, stream=None) -> int:
        n = _i32()
        _check(tdp_pairs_count(self.h, ctypes.byref(n), _stream(stream)), self.h)
        return n.value

    # ----------------------------------------------------------- losses
    def p2p_loss_fwd(self, x, y, out=None, stream=None) -> torch.Tensor:
        out = _scalar_out(out, x.device)
        _check(tdp_p2p_loss_fwd(self.h, _ptr(self._cells(x)), _ptr(self._cells(y)), _ptr(out), _stream(stream)), self.h)
        return out

    def p2p_loss_bwd(self, x, y, gout, gx, gy, stream=None):
        _check(tdp_p2p_loss_bwd(self.h, _ptr(self._cells(x)), _ptr(self._cells(y)), _ptr(_f64_scalar(gout)),
                                _ptr(self._cells(gx)), _ptr(self._cells(gy)), _stream(stream)), self.h)

    def pair_loss_fwd(self, kind: int, x, y, out=None, stream=None) -> torch.Tensor:
        """kind 0: PP (quadratic); 1: Manhattan; 2: linear Euclidean."""
        out = _scalar_out(out, x.device)
        _check(tdp_pair_loss_fwd(self.h, kind, _ptr(self._cells(x)), _ptr(self._cells(y)), _ptr(out),
                                 _stream(stream)), self.h)
        return out

    def pair_loss_bwd(self, kind: int, x, y, gout, gx, gy, stream=None):
        _check(tdp_pair_loss_bwd(self.h, kind, _ptr(self._cells(x)), _ptr(self._cells(y)), _ptr(_f64_scalar(gout)),
                                 _ptr(self._cells(gx)), _ptr(self._cells(gy)), _stream(stream)), self.h)

    def stns_fwd(self, x, y, gamma: float = 10.0, out=None, stream=None) -> torch.Tensor:
        out = _scalar_out(out, x.device)
        _check(tdp_stns_fwd(self.h, _ptr(self._cells(x)), _ptr(self._cells(y)), gamma, _ptr(out), _stream(stream)),
               self.h)
        return out

    def stns_bwd(self, gout, gx, gy, stream=None):
        _check(tdp_stns_bwd(self.h, _ptr(_f64_scalar(gout)), _ptr(self._cells(gx)), _ptr(self._cells(gy)),
                            _stream(stream)), self.h)

    def wa_fwd_bwd(self, x, y, gamma: float, gx, gy, out=None, stream=None) -> torch.Tensor:
        out = _scalar_out(out, x.device)
        _check(tdp_wa_fwd_bwd(self.h, _ptr(self._cells(x)), _ptr(self._cells(y)), gamma, _ptr(out),
                              _ptr(self._cells(gx)), _ptr(self._cells(gy)), _stream(stream)), self.h)
        return out

    def wa_fwd_bwd_at_update(self, gamma: float, gx, gy, out=None, stream=None) -> torch.Tensor:
        """WA at the positions of the last sta_update (unchanged since)."""
        out = _scalar_out(out, gx.device)
        _check(tdp_wa_fwd_bwd_at_update(self.h, gamma, _ptr(out), _ptr(self._cells(gx)), _ptr(self._cells(gy)),
                                        _stream(stream)), self.h)
        return out

    # ------------------------------------------------ early (hold) analysis
    def sta_update_early(self, hold: float = 0.0, stream=None):
        """Early arrivals and hold slacks from the last sta_update's net delays."""
        _check(tdp_sta_update_early(self.h, float(hold), _stream(stream)), self.h)

    def early_summary(self, stream=None):
        """(WHS, THS, number of D pins with negative hold slack)."""
        w, t, n = ctypes.c_double(), ctypes.c_double(), _i32()
        _check(tdp_sta_early_summary(self.h, ctypes.byref(w), ctypes.byref(t), ctypes.byref(n), _stream(stream)),
               self.h)
        return w.value, t.value, n.value

    def early_export(self, stream=None) -> Dict[str, torch.Tensor]:
        dev = torch.device("cuda", self.device)
        out = {k: torch.empty(self.num_pins, dtype=torch.float64, device=dev)
               for k in ("at", "slew", "darc", "hold_slack")}
        _check(tdp_sta_early_export(self.h, *[_ptr(out[k]) for k in ("at", "slew", "darc", "hold_slack")],
                                    _stream(stream)), self.h)
        return out

    # ------------------------------------------------ placement loop pieces
    def density_setup(self, grid: Dict, area):
        """grid: x0, y0, bw, bh, gx, gy, R, target; area: [num_cells] host."""
        a = np.ascontiguousarray(area, dtype=np.float32)
        if a.shape[0] != self.num_cells:
            raise ValueError("one area per cell")
        q = tdp_density_grid(float(grid["x0"]), float(grid["y0"]), float(grid["bw"]), float(grid["bh"]),
                             int(grid["gx"]), int(grid["gy"]), int(grid["R"]), float(grid.get("target", 1.0)))
        _check(tdp_density_setup(self.h, ctypes.byref(q), a.ctypes.data), self.h)
        self._dn_grid = int(grid["gx"]) * int(grid["gy"])

    def density(self, x, y, scale: float = 1.0, gx=None, gy=None, want_map: bool = False, stream=None):
        """(value, overflow[, map]) as device tensors; adds scale * gradient
        to gx, gy when given."""
        val = torch.zeros(2, dtype=torch.float64, device=x.device)
        mp = None
        if want_map:
            mp = torch.empty(int(self._grid_bins()), dtype=torch.float32, device=x.device)
        _check(tdp_density_fwd_bwd(self.h, _ptr(self._cells(x)), _ptr(self._cells(y)), float(scale), _ptr(val),
                                   val.data_ptr() + 8, _ptr(self._cells(gx, True)), _ptr(self._cells(gy, True)),
                                   _ptr(mp), _stream(stream)), self.h)
        return (val[0], val[1], mp) if want_map else (val[0], val[1])

    def abs_sum(self, a, b, out=None, stream=None) -> torch.Tensor:
        """sum |a| + |b| over cells (device double)."""
        out = _scalar_out(out, a.device)
        _check(tdp_abs_sum(self.h, _ptr(self._cells(a)), _ptr(self._cells(b)), _ptr(out), _stream(stream)), self.h)
        return out

    def _grid_bins(self):
        if self._dn_grid is None:
            raise RuntimeError("density_setup first")
        return self._dn_grid

    def nesterov_step(self, st: Dict, gx, gy, pdiv, coef: float, alpha0: float, first: bool, bounds,
                      alpha_out=None, stream=None):
        """One Nesterov step on the state tensors st (vx, vy, ux, uy, vpx, vpy,
        gpx, gpy; updated in place); bounds = (xlo, xhi, ylo, yhi)."""
        for k in ("vx", "vy", "ux", "uy", "vpx", "vpy", "gpx", "gpy"):
            self._cells(st[k])
        _check(tdp_nesterov_step(self.h, _ptr(self._cells(gx)), _ptr(self._cells(gy)), _ptr(self._cells(pdiv)),
                                 *[_ptr(st[k]) for k in ("vx", "vy", "ux", "uy", "vpx", "vpy", "gpx", "gpy")],
                                 float(coef), float(alpha0), 1 if first else 0, *[float(b) for b in bounds],
                                 _ptr(alpha_out), _stream(stream)), self.h)

    # ----------------------------------------------------------- tooling
    def profile(self, on=True):
        """on: True (every stage), False, or a collection of stage names."""
        if on is True:
            mask = (1 << len(STAGES)) - 1
        elif not on:
            mask = 0
        else:
            mask = sum(1 << STAGES.index(s) for s in on)
        _check(tdp_profile_enable(self.h, mask), self.h)

    def profile_read(self) -> Dict[str, tuple]:
        ms = np.zeros(len(STAGES), np.float64)
        calls = np.zeros(len(STAGES), np.int32)
        _check(tdp_profile_read(self.h, ms.ctypes.data, calls.ctypes.data), self.h)
        return {s: (float(ms[i]), int(calls[i])) for i, s in enumerate(STAGES)}

    def set_tuning(self, flow_waves: int = 0, spin_log2: int = 0, sweep_mode: int = 1, flow_per_cu: int = 0):
        """sweep_mode 0: one launch per level; 1: dataflow sweeps on a resident
        grid; 2: self-test of the dataflow sweeps' bounded waits; 3: the
        backward sweep as a dataflow grid, the forward one per level.  flow_waves:
        waves per workgroup of the resident grids (1, 2, 4; 0 keeps);
        flow_per_cu: their workgroups per compute unit (1..4; 0 keeps)."""
        _check(tdp_set_tuning(self.h, flow_waves, flow_per_cu, spin_log2, sweep_mode), self.h)

    def autotune(self, x, y, n: int = -1, k: int = 1, K: Optional[int] = None, reps: int = 3,
                 stream=None) -> Dict[str, int]:
        """Pick the fastest sweep configuration for update + extraction; a
        graph of a signature tuned before in this process takes the kept
        choice (and its measured time) without trials."""
        K = self.max_paths if K is None else K
        ch = np.zeros(4, np.int32)
        _check(tdp_autotune(self.h, _ptr(self._cells(x)), _ptr(self._cells(y)), n, k, K, reps, ch.ctypes.data,
                            _stream(stream)), self.h)
        return {"sweep_mode": int(ch[0]), "flow_waves": int(ch[1]), "flow_per_cu": int(ch[2]),
                "us_per_run": int(ch[3])}


class _DeviceView:
    """A device array owned by a graph, exposed through the CUDA array
    interface (which torch imports without a copy); keeps the graph alive."""

    def __init__(self, ptr: int, n: int, typestr: str, owner):
        self.__cuda_array_interface__ = {"shape": (n,), "typestr": typestr, "data": (ptr, False), "version": 2,
                                         "strides": None}
        self._owner = owner


def _scalar_out(out, device) -> torch.Tensor:
    """Loss values are single device doubles."""
    if out is None:
        return torch.empty((), dtype=torch.float64, device=device)
    if out.dtype != torch.float64 or not out.is_cuda:
        raise ValueError("loss output must be a float64 tensor on the GPU")
    return out


def _f64_scalar(t: torch.Tensor) -> torch.Tensor:
    """Upstream gradients are single device doubles."""
    if t.dtype != torch.float64 or not t.is_contiguous():
        t = t.to(torch.float64).contiguous()
    if not t.is_cuda or t.numel() != 1:
        raise ValueError("upstream gradient must be one value on the GPU")
    return t


def _copy_dev(dst: torch.Tensor, src_ptr: int, nbytes: int):
    """Device-to-device copy from a library-owned buffer into a tensor."""
    hip = _hip()
    rc = hip.hipMemcpy(ctypes.c_void_p(dst.data_ptr()), ctypes.c_void_p(src_ptr), ctypes.c_size_t(nbytes),
                       ctypes.c_int(3))
    if rc != 0:
        raise TdpError(4, f"hipMemcpy failed ({rc})")


_hip_lib = None


def _hip():
    global _hip_lib
    if _hip_lib is None:
        _hip_lib = ctypes.CDLL("libamdhip64.so")
        _hip_lib.hipMemcpy.restype = ctypes.c_int
        _hip_lib.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    return _hip_lib


def _zero_grads(x: torch.Tensor, y: torch.Tensor):
    """Fresh contiguous gradient buffers (the kernels accumulate into them)."""
    return (torch.zeros(x.shape, dtype=torch.float32, device=x.device),
            torch.zeros(y.shape, dtype=torch.float32, device=y.device))


class P2PLoss(torch.autograd.Function):
    """PP(x, y) over the graph's current pin-pair set (Eqs. 8, 10)."""

    @staticmethod
    def forward(ctx, x, y, graph: TimingGraph):
        ctx.graph = graph
        x, y = x.contiguous(), y.contiguous()
        ctx.save_for_backward(x, y)
        return graph.p2p_loss_fwd(x, y)

    @staticmethod
    def backward(ctx, gout):
        x, y = ctx.saved_tensors
        gx, gy = _zero_grads(x, y)
        ctx.graph.p2p_loss_bwd(x, y, gout, gx, gy)
        return gx, gy, None


class PairLoss(torch.autograd.Function):
    """A pair distance loss over the graph's pin-pair set: kind 0 quadratic
    (PP), 1 Manhattan, 2 linear Euclidean (the comparison of Sec. III-C)."""

    @staticmethod
    def forward(ctx, x, y, graph: TimingGraph, kind: int = 0):
        ctx.graph, ctx.kind = graph, kind
        x, y = x.contiguous(), y.contiguous()
        ctx.save_for_backward(x, y)
        return graph.pair_loss_fwd(kind, x, y)

    @staticmethod
    def backward(ctx, gout):
        x, y = ctx.saved_tensors
        gx, gy = _zero_grads(x, y)
        ctx.graph.pair_loss_bwd(ctx.kind, x, y, gout, gx, gy)
        return gx, gy, None, None


class SmoothTNS(torch.autograd.Function):
    """Log-sum-exp smoothed TNS with frozen cell arcs (hand-written adjoint)."""

    @staticmethod
    def forward(ctx, x, y, graph: TimingGraph, gamma: float = 10.0):
        ctx.graph = graph
        x, y = x.contiguous(), y.contiguous()
        ctx.save_for_backward(x, y)
        return graph.stns_fwd(x, y, gamma)

    @staticmethod
    def backward(ctx, gout):
        x, y = ctx.saved_tensors
        gx, gy = _zero_grads(x, y)
        ctx.graph.stns_bwd(gout, gx, gy)
        return gx, gy, None, None
