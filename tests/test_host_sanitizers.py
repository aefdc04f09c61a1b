"""The oracle's C code and the library's host-side graph build (netlist
checks, levelisation, 64-lane chunk layout) under the address and
undefined-behaviour sanitizers, on the CPU.  Both are compiled with gcc
-fsanitize=address,undefined into a temporary folder; a child Python with
the sanitizer runtime preloaded runs every oracle function on the small
workload and the builder on valid designs (single and batched) and on each
invalid netlist the build must reject.  Any sanitizer report, or a status
other than the expected one, fails the test."""
import os
import shutil
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
FLAGS = ["-O1", "-g", "-fPIC", "-shared", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
         "-fno-omit-frame-pointer"]

CHILD = textwrap.dedent("""
    import ctypes, os, sys
    import numpy as np
    sys.path.insert(0, os.environ["TDP_ROOT"])
    from oracle import ref
    from paper_2503_11674_amd import netgen
    from paper_2503_11674_amd.tdp import _NetlistHolder, _LibraryHolder
    from tests import handnets
    from tests.conftest import with_clock

    lib = netgen.make_library()
    for net_model in (0, 1):
        lb = dict(lib, net_model=net_model)
        nl = with_clock(netgen.make_netlist(netgen.CONFIGS["C1"]), lb)
        st = ref.sta(nl, lb)
        paths = ref.extract(nl, lb, st, n=-1, k=4, K=400)
        ref.report_timing(nl, lb, st, K=300)
        ps = ref.PairState(nl["num_pins"])
        ref.pairs_update(ps, paths, st["wns"], rule=0)
        sinks, w = ps.pairs()
        ref.p2p(nl, sinks, w)
        for kind in (1, 2):
            ref.pair_loss(nl, kind, sinks, w)
        ref.stns(nl, lb, st, 10.0, with_abs=True)
        ref.wa(nl, 5.0, with_abs=True)
        ref.sta_early(nl, lb, hold=5.0)
        rl = netgen.make_rf_library(lb)
        rf = ref.sta_rf(nl, rl)
        ref.extract_rf(nl, rf, n=-1)
    n = int(nl["num_cells"])
    x, y = np.asarray(nl["x"], np.float32), np.asarray(nl["y"], np.float32)
    grid = dict(x0=0.0, y0=0.0, bw=25.0, bh=25.0, gx=40, gy=40, R=2)
    d = ref.density(x, y, np.ones(n, np.float32), nl["cell_fixed"], grid, 0.9)
    state = {k: np.zeros(n, np.float64) for k in ("vx", "vy", "ux", "uy", "vpx", "vpy", "gpx", "gpy")}
    state["vx"][:], state["vy"][:] = x, y
    ref.nesterov(state, d["grad_x"], d["grad_y"], np.ones(n), nl["cell_fixed"], 0.0, 0.5, True,
                 (0.0, 1000.0, 0.0, 1000.0))
    print("oracle ok", flush=True)

    hb = ctypes.CDLL(os.environ["TDP_HOST_SHIM"])
    hb.tdp_host_build_check.restype = ctypes.c_int32

    def build(nls, lb):
        hs = [_NetlistHolder(a) for a in nls]
        arr = (ctypes.c_void_p * len(hs))(*[ctypes.addressof(h.s) for h in hs])
        lh = _LibraryHolder(lb)
        err = ctypes.create_string_buffer(256)
        sizes = (ctypes.c_int64 * 4)()
        stt = hb.tdp_host_build_check(arr, len(hs), ctypes.byref(lh.s), err, 256, sizes)
        return stt, err.value.decode(), list(sizes)

    c1 = netgen.make_netlist(netgen.CONFIGS["C1"])
    stt, msg, sz = build([c1], lib)
    assert stt == 0 and sz[0] > 0 and sz[1] > 0, (stt, msg, sz)
    stt, msg, sz = build([c1, handnets.chain_netlist()[0], c1], lib)
    assert stt == 0, (stt, msg)
    dy = handnets.dyadic_library()
    for m in ("sink_in_two_nets", "driver_is_input", "dangling_input", "ff_two_inputs", "bad_type",
              "pin_out_of_range"):
        stt, msg, _ = build([handnets.invalid_chain(m)], dy)
        assert stt == 1, (m, stt, msg)
    cyc, _ = handnets.build([(0, 1), (0, 1)], 0, [(1, [2]), (3, [0])], [0.0, 1.0], [0.0, 0.0])
    stt, msg, _ = build([cyc], dy)
    assert stt == 2, (stt, msg)
    print("builder ok", flush=True)
""")


def _runtime(name):
    r = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True)
    p = r.stdout.strip()
    return p if r.returncode == 0 and os.path.isabs(p) and os.path.exists(p) else None


def test_oracle_and_host_build_under_sanitizers(tmp_path):
    if shutil.which("gcc") is None or shutil.which("g++") is None:
        pytest.skip("no gcc")
    asan = _runtime("libasan.so")
    if asan is None:
        pytest.skip("no gcc address-sanitizer runtime")
    ora = str(tmp_path / "libtdp_oracle_san.so")
    subprocess.check_call(["gcc", "-std=c99", *FLAGS, "-o", ora, os.path.join(ROOT, "oracle", "tdp_oracle.c"),
                           "-lm"])
    shim = str(tmp_path / "libtdp_host_build_san.so")
    csrc = os.path.join(ROOT, "paper_2503_11674_amd", "csrc")
    subprocess.check_call(["g++", "-std=c++17", *FLAGS, "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
                           "-I" + os.path.join(ROOT, "include"), "-I" + csrc, "-o", shim,
                           os.path.join(ROOT, "tests", "host_build_shim.cpp"), os.path.join(csrc, "tdp_build.cpp")])
    env = dict(os.environ, LD_PRELOAD=asan, ASAN_OPTIONS="detect_leaks=0", UBSAN_OPTIONS="print_stacktrace=1",
               TDP_ORACLE_LIB=ora, TDP_HOST_SHIM=shim, TDP_ROOT=ROOT)
    r = subprocess.run([sys.executable, "-c", CHILD], env=env, capture_output=True, text=True, timeout=600)
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
    assert "oracle ok" in r.stdout and "builder ok" in r.stdout
