"""Rise / fall timing on the GPU against the oracle: arrival, required time,
slack and transition of both transitions at every pin, WNS / TNS / count,
report_timing_endpoint(n, 1) paths with their transitions (every path a
chain of arcs its cells' unateness allows, ending in its endpoint's worse
transition, with the oracle's slack; at least 98 % pin-for-pin identical to
the oracle's in single precision, all of them in double), the pair update
and the loss on those paths, double precision to 1e-12, and the state rules
between the two timers."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import ref  # noqa: E402
from paper_2503_11674_amd import netgen  # noqa: E402
from tests.comparator import timing_close  # noqa: E402

pytestmark = pytest.mark.gpu


def _tdp():
    from paper_2503_11674_amd import tdp
    return tdp


def _dev():
    return torch.device("cuda", 0)


def _case(name, library, net_model=0):
    lib = netgen.make_rf_library(dict(library, net_model=net_model))
    nl = netgen.make_netlist(netgen.CONFIGS[name])
    nl["clock_period"] = np.float32(0.0)
    rf0 = ref.sta_rf(nl, lib)
    ep = ref.endpoint_pins(nl)
    nl["clock_period"] = np.float32(netgen.clock_period_for_fail_fraction(np.max(rf0["at"][ep], axis=1), 0.05))
    return nl, lib, ref.sta_rf(nl, lib), ep


def _xy(nl):
    return torch.tensor(nl["x"], device=_dev()), torch.tensor(nl["y"], device=_dev())


def _arc_ok(nl, lib, a, ta, b, tb, role_of):
    """(a, ta) -> (b, tb) is a net arc (same transition) or a cell arc the
    type's unateness allows."""
    if role_of[b] in ("cin", "ffd"):
        return ta == tb
    ty = int(nl["cell_type"][nl["pin_cell"][b]])
    u = int(lib["unate"][ty])
    return u == 2 or (u == 0 and ta == tb) or (u == 1 and ta != tb)


def _roles(nl):
    P = int(nl["num_pins"])
    role = np.array(["port"] * P, dtype=object)
    for c in range(int(nl["num_cells"])):
        ff = bool(nl["cell_is_ff"][c])
        for p in nl["cell_in_pins"][nl["cell_in_ptr"][c]:nl["cell_in_ptr"][c + 1]]:
            role[p] = "ffd" if ff else "cin"
        role[nl["cell_out_pin"][c]] = "ffq" if ff else "cout"
    return role


@pytest.mark.parametrize("name,net_model", [("C1", 0), ("C2", 0), ("C2", 1), ("C2", 2)])
def test_rise_fall_timing_and_paths(name, net_model, library):
    tdp = _tdp()
    nl, lib, rf, ep = _case(name, library, net_model)
    g = tdp.TimingGraph(nl, lib, max_paths=len(ep), max_k=1)
    g.rf_setup(lib)
    g.sta_update_rf(*_xy(nl))
    o = {k: v.cpu().numpy() for k, v in g.rf_export().items()}
    scale = np.maximum(np.abs(np.where(np.isfinite(rf["at"]), rf["at"], 0)),
                       np.abs(np.where(np.isfinite(rf["rat"]), rf["rat"], 0)))
    scale = np.maximum(scale, abs(float(nl["clock_period"])))
    for key in ("at", "rat", "slack"):
        inf_ok, bad, worst = timing_close(o[key].reshape(-1), rf[key].reshape(-1),
                                          scale=scale.reshape(-1) if key != "at" else None)
        print(name, key, "worst", worst)
        assert inf_ok and bad == 0, (key, bad, worst)
    inf_ok, bad, worst = timing_close(o["slew"].reshape(-1), rf["slew"].reshape(-1), rtol=2e-5)
    assert inf_ok and bad == 0, ("slew", bad, worst)
    wns, tns, nf = g.rf_summary()
    assert nf == rf["n_fail"] == len(ep) // 20
    assert abs(wns - rf["wns"]) <= 1e-4 * abs(rf["wns"]) and abs(tns - rf["tns"]) <= 1e-4 * abs(rf["tns"])
    # report_timing_endpoint(n_fail, 1)
    g.extract_paths_rf(n=-1)
    gp = g.paths_rf()
    rp = ref.extract_rf(nl, rf, n=-1)
    assert gp["num_paths"] == rp["num_paths"] == nf
    tol = 1e-4 * max(abs(float(nl["clock_period"])), abs(rf["wns"]))
    assert np.all(np.abs(gp["path_slack"] - rp["path_slack"]) <= tol)
    role = _roles(nl)
    same = 0
    for i in range(gp["num_paths"]):
        pins = gp["path_pins"][gp["path_ptr"][i]:gp["path_ptr"][i + 1]]
        tr = gp["path_tran"][gp["path_ptr"][i]:gp["path_ptr"][i + 1]]
        assert role[pins[0]] in ("port", "ffq") and role[pins[-1]] == "ffd" and pins[-1] == gp["path_ep"][i]
        for j in range(len(pins) - 1):
            assert _arc_ok(nl, lib, pins[j], tr[j], pins[j + 1], tr[j + 1], role)
        # it ends in the endpoint's worse transition
        e, te = pins[-1], tr[-1]
        assert abs(rf["slack"][e, te] - rf["ep_slack"][e]) <= tol
        rps = rp["path_pins"][rp["path_ptr"][i]:rp["path_ptr"][i + 1]]
        rtr = rp["path_tran"][rp["path_ptr"][i]:rp["path_ptr"][i + 1]]
        same += int(np.array_equal(pins, rps) and np.array_equal(tr, rtr))
    print(name, "identical paths", same, "of", gp["num_paths"])
    assert same >= 0.98 * gp["num_paths"]
    # pairs and the loss on those paths
    g.pairs_reset()
    g.pairs_update(rule=0)
    w, inp = g.pairs_export()
    ps = ref.PairState(nl["num_pins"])
    ref.pairs_update(ps, gp, wns, rule=0)
    assert np.array_equal(inp.astype(bool), ps.in_p.astype(bool))
    np.testing.assert_allclose(w[inp.astype(bool)], ps.w[inp.astype(bool)], rtol=1e-4)
    x, y = _xy(nl)
    loss = float(g.p2p_loss_fwd(x, y))
    sinks, wr = ps.pairs()
    l_ref, _, _ = ref.p2p(nl, sinks, wr)
    assert abs(loss - l_ref) <= 1e-4 * abs(l_ref)
    g.close()


def test_rise_fall_double_precision_and_state(library):
    tdp = _tdp()
    nl, lib, rf, ep = _case("C1", library)
    g = tdp.TimingGraph(nl, lib, precision="f64", max_paths=len(ep), max_k=1)
    with pytest.raises(tdp.TdpError):
        g.sta_update_rf(*_xy(nl))  # before setup
    g.rf_setup(lib)
    g.sta_update_rf(*_xy(nl))
    o = {k: v.cpu().numpy() for k, v in g.rf_export().items()}
    for key in ("at", "rat", "slack", "slew"):
        inf_ok, bad, worst = timing_close(o[key].reshape(-1), rf[key].reshape(-1), rtol=1e-12)
        assert inf_ok and bad == 0, (key, bad, worst)
    g.extract_paths_rf(n=-1)
    gp = g.paths_rf()
    rp = ref.extract_rf(nl, rf, n=-1)
    for key in ("path_ptr", "path_pins", "path_tran", "path_ep"):
        assert np.array_equal(gp[key], rp[key]), key
    # the single-transition results read as stale until its own update
    with pytest.raises(tdp.TdpError) as e:
        g.summary()
    assert e.value.status == 6
    g.sta_update(*_xy(nl))
    g.summary()
    with pytest.raises(tdp.TdpError) as e:
        g.extract_paths_rf(n=-1)
    assert e.value.status == 6
    g.close()
    gb = tdp.TimingGraph([nl, nl], lib, max_paths=10, max_k=1)
    with pytest.raises(tdp.TdpError) as e:
        gb.rf_setup(lib)
    assert e.value.status == 7
    gb.close()


@pytest.mark.parametrize("net_model", [0, 1, 2])
def test_rise_fall_nets_wider_than_a_chunk(net_model, library):
    """Two nets of more than 63 sinks take the one-thread-per-net path of the
    backward pass: both transitions' arrival, required time and slack match
    the oracle, in double precision to 1e-12."""
    from tests.test_gpu_net_model import _fanout_design
    tdp = _tdp()
    lib = netgen.make_rf_library(dict(library, net_model=net_model))
    nl = _fanout_design()
    assert (np.diff(nl["net_ptr"]) - 1 > 63).sum() == 2
    nl["clock_period"] = np.float32(0.0)
    rf0 = ref.sta_rf(nl, lib)
    ep = ref.endpoint_pins(nl)
    nl["clock_period"] = np.float32(netgen.clock_period_for_fail_fraction(np.max(rf0["at"][ep], axis=1), 0.3))
    rf = ref.sta_rf(nl, lib)
    for precision, rtol in (("f64", 1e-12), ("f32", None)):
        g = tdp.TimingGraph(nl, lib, precision=precision, max_paths=len(ep), max_k=1)
        g.rf_setup(lib)
        g.sta_update_rf(*_xy(nl))
        o = {k: v.cpu().numpy() for k, v in g.rf_export().items()}
        for key in ("at", "rat", "slack"):
            if rtol is None:  # single precision: relative to the pin's timing magnitudes, as above
                scale = np.maximum(np.abs(np.where(np.isfinite(rf["at"]), rf["at"], 0)),
                                   np.abs(np.where(np.isfinite(rf["rat"]), rf["rat"], 0)))
                scale = np.maximum(scale, abs(float(nl["clock_period"])))
                inf_ok, bad, worst = timing_close(o[key].reshape(-1), rf[key].reshape(-1),
                                                  scale=scale.reshape(-1) if key != "at" else None)
            else:
                inf_ok, bad, worst = timing_close(o[key].reshape(-1), rf[key].reshape(-1), rtol=rtol)
            assert inf_ok and bad == 0, (precision, key, bad, worst)
        g.close()
