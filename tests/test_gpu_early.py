"""Parity of the early (hold) analysis on the GPU with the FP64 oracle:
arrivals, transitions, arc delays and hold slacks at 2k and 200k cells, both
net models, FP64 graphs to 1e-12, the hand diamond bit-exact in FP32, and the
summary.  Tolerances as in test_gpu_parity.py; the hold time sits midway
between two early D arrivals, so that no slack is within rounding of 0 and
the count of violations compares exactly."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import ref  # noqa: E402
from paper_2503_11674_amd import netgen  # noqa: E402
from tests import handnets  # noqa: E402
from tests.comparator import timing_close  # noqa: E402
from tests.conftest import with_clock  # noqa: E402

pytestmark = pytest.mark.gpu


def _tdp():
    from paper_2503_11674_amd import tdp
    return tdp


def _xy(nl):
    d = torch.device("cuda", 0)
    return (torch.tensor(np.asarray(nl["x"], np.float32), device=d),
            torch.tensor(np.asarray(nl["y"], np.float32), device=d))


def _hold_between(arrivals, frac=0.05):
    a = np.sort(arrivals[np.isfinite(arrivals)])
    q = max(1, int(frac * len(a)))
    return float(0.5 * (a[q - 1] + a[q]))


@pytest.mark.parametrize("name,net_model,prec", [("C1", 0, "f32"), ("C1", 1, "f32"), ("C1", 2, "f32"),
                                                 ("C2", 0, "f32"), ("C2", 1, "f64")])
def test_early_parity(name, net_model, prec, library):
    tdp = _tdp()
    lib = dict(library, net_model=net_model)
    nl = with_clock(netgen.make_netlist(netgen.CONFIGS[name]), lib)
    D = ref.endpoint_pins(nl)
    e0 = ref.sta_early(nl, lib)
    # the library takes the hold time as a float, like the clock and setup
    hold = float(np.float32(_hold_between(e0["at"][D])))
    e = ref.sta_early(nl, lib, hold=hold)
    print(f"[early] {name} model {net_model} {prec} hold {hold:.2f}", flush=True)
    g = tdp.TimingGraph(nl, lib, precision=prec, max_paths=16, max_k=1)
    g.sta_update(*_xy(nl))
    g.sta_update_early(hold)
    o = {k: v.cpu().numpy() for k, v in g.early_export().items()}
    rtol = 1e-12 if prec == "f64" else 1e-4
    inf_ok, bad, worst = timing_close(o["at"], e["at"], rtol=rtol)
    assert inf_ok and bad == 0, ("at", bad, worst)
    for key in ("slew", "darc"):
        inf_ok, bad, worst = timing_close(o[key], e[key], rtol=1e-12 if prec == "f64" else 2e-5)
        assert inf_ok and bad == 0, (key, bad, worst)
    scale = np.maximum(np.abs(np.where(np.isfinite(e["at"]), e["at"], 0)), abs(hold))
    inf_ok, bad, worst = timing_close(o["hold_slack"], e["hold_slack"], rtol=rtol, scale=scale)
    assert inf_ok and bad == 0, ("hold", bad, worst)
    whs, ths, nf = g.early_summary()
    assert nf == e["n_hold_fail"] > 0
    assert abs(whs - e["whs"]) <= rtol * max(abs(e["whs"]), abs(hold))
    assert abs(ths - e["ths"]) <= rtol * max(abs(e["ths"]), 1.0) * 10
    # early <= late wherever both are finite (the tables grow with the transition)
    late = {k: v.cpu().numpy() for k, v in g.export().items()}
    fin = np.isfinite(late["at"])
    assert np.all(o["at"][fin] <= late["at"][fin] * (1 + 1e-6) + 1e-6)
    # bitwise reproducible
    g.sta_update_early(hold)
    o2 = {k: v.cpu().numpy() for k, v in g.early_export().items()}
    for k in o:
        assert np.array_equal(o[k], o2[k]), k
    g.close()


def test_early_hand_diamond_bit_exact():
    tdp = _tdp()
    nl, _ = handnets.diamond_netlist()
    lib = handnets.dyadic_library()
    g = tdp.TimingGraph(nl, lib, max_paths=4, max_k=1)
    g.sta_update(*_xy(nl))
    g.sta_update_early(50.0)
    o = {k: v.cpu().numpy() for k, v in g.early_export().items()}
    e = ref.sta_early(nl, lib, hold=50.0)
    for k in ("at", "slew", "darc", "hold_slack"):
        assert np.array_equal(o[k], e[k]), (k, o[k], e[k])
    assert g.early_summary() == (-7.75, -7.75, 1)
    g.close()


def test_early_needs_an_update(library):
    tdp = _tdp()
    nl = with_clock(netgen.make_netlist(netgen.CONFIGS["C1"]), library)
    g = tdp.TimingGraph(nl, library, max_paths=16, max_k=1)
    with pytest.raises(tdp.TdpError):
        g.sta_update_early(0.0)
    g.sta_update(*_xy(nl))
    with pytest.raises(tdp.TdpError):
        g.early_summary()
    with pytest.raises(tdp.TdpError):
        g.sta_update_early(float("nan"))
    g.sta_update_early(0.0)
    assert g.early_summary() == (0.0, 0.0, 0)  # arrivals are positive: nothing fails a zero hold
    # a new timing update makes the hold results stale until the next early update
    g.sta_update(*_xy(nl))
    with pytest.raises(tdp.TdpError):
        g.early_summary()
    with pytest.raises(tdp.TdpError):
        g.early_export()
    g.sta_update_arrivals(*_xy(nl))
    with pytest.raises(tdp.TdpError):
        g.early_summary()
    g.sta_update_early(0.0)
    assert g.early_summary() == (0.0, 0.0, 0)
    g.close()
