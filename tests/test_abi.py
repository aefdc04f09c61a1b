"""The C-ABI library loads and exports every declared entry point; the host
side validates netlists (status codes, no device work needed)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2503_11674_amd import netgen
from tests import handnets

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tdp.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(tdp_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    from paper_2503_11674_amd import tdp
    lib = ctypes.CDLL(tdp.LIB_PATH)
    names = _declared()
    assert len(names) >= 25
    missing = [n for n in names if not hasattr(lib, n)]
    assert missing == []
    assert set(names) <= set(tdp.EXPORTED)


def test_status_strings():
    from paper_2503_11674_amd import tdp
    assert tdp.tdp_status_str(0) == b"ok"
    assert tdp.tdp_status_str(2) == b"combinational cycle"


def _build_status(nl, lib=None):
    from paper_2503_11674_amd import tdp
    lib = lib or handnets.dyadic_library()
    nh = tdp._NetlistHolder(nl)
    lh = tdp._LibraryHolder(lib)
    h = ctypes.c_void_p()
    st = tdp.tdp_sta_build(ctypes.byref(nh.s), ctypes.byref(lh.s), 0, 4, 1, 0, ctypes.byref(h))
    msg = tdp.tdp_last_error(None)
    if st == 0:
        tdp.tdp_destroy(h.value)
    return st, (msg.decode() if msg else "")


def test_cycle_is_rejected():
    # two buffers feeding each other
    cells = [(0, 1), (0, 1)]
    nets = [(1, [2]), (3, [0])]
    nl, _ = handnets.build(cells, 0, nets, [0.0, 1.0], [0.0, 0.0])
    st, msg = _build_status(nl)
    assert st == 2, msg


@pytest.mark.parametrize("mutation,expect", [
    ("sink_in_two_nets", "input pin in two nets"),
    ("driver_is_input", "net driver is not an output pin"),
    ("dangling_input", "an input pin is in no net"),
    ("ff_two_inputs", "exactly one input"),
    ("bad_type", "cell_type out of range"),
    ("pin_out_of_range", "out of range"),
])
def test_invalid_netlists(mutation, expect):
    nl = handnets.invalid_chain(mutation)
    st, msg = _build_status(nl)
    assert st == 1 and expect in msg, (st, msg)


def test_bad_library_axis():
    nl, _ = handnets.chain_netlist()
    lib = handnets.dyadic_library()
    lib["slew_axis"] = lib["slew_axis"].copy()
    lib["slew_axis"][0, 3] = lib["slew_axis"][0, 2]
    st, msg = _build_status(nl, lib)
    assert st == 1 and "slew axis" in msg


def test_valid_netlist_reaches_the_device_check():
    # on a machine without a GPU a valid netlist gets as far as device lookup
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    nl = netgen.make_netlist(netgen.CONFIGS["C1"])
    st, msg = _build_status(nl, netgen.make_library())
    assert st == 4 and "device" in msg


def test_path_capacity_that_overflows_32_bits_is_rejected():
    # path pins are addressed with 32-bit offsets: max_paths * (2 D + 2) must fit
    from paper_2503_11674_amd import tdp
    nl, _ = handnets.chain_netlist()
    nh = tdp._NetlistHolder(nl)
    lh = tdp._LibraryHolder(handnets.dyadic_library())
    h = ctypes.c_void_p()
    st = tdp.tdp_sta_build(ctypes.byref(nh.s), ctypes.byref(lh.s), 0, 1 << 30, 1, 0, ctypes.byref(h))
    msg = tdp.tdp_last_error(None).decode()
    assert st == 1 and "max_paths" in msg, (st, msg)
    assert h.value is None
