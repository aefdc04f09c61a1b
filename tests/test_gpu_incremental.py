"""Incremental arrival updates: after moving a subset of cells, re-timing
only what they change gives, bitwise, what a full update at the new
positions gives (every pin's timing, critical inputs, WNS / TNS, and the k
worst paths per endpoint, which read the deviation lists, hop records and
chain depths), over several rounds of moves, in single and double
precision, at 200k and 2M cells; an empty move list changes nothing; a bad
id is reported."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2503_11674_amd import netgen  # noqa: E402
from tests.conftest import with_clock  # noqa: E402

pytestmark = pytest.mark.gpu


def _tdp():
    from paper_2503_11674_amd import tdp
    return tdp


def _state(g, k, K):
    g.sta_update_required()
    o = {key: v.cpu().numpy() for key, v in g.export().items()}
    g.extract_paths(n=-1, k=k, K=K)
    return o, g.paths(), g.summary()


def _same(a, b):
    (oa, pa, sa), (ob, pb, sb) = a, b
    for key in oa:
        assert np.array_equal(oa[key], ob[key]), key
    for key in ("path_ptr", "path_pins", "path_ep", "path_rank", "path_slack"):
        assert np.array_equal(pa[key], pb[key]), key
    assert sa == sb


# sweep forms of the incremental graph and of the full-update graph (0: per
# level, 1: both sweeps as dataflow grids, 3: the backward one only)
@pytest.mark.parametrize("name,precision,moves,modes", [("C2", "f32", (1, 100, 5000), (1, 3)),
                                                        ("C2", "f64", (300,), (0, 0)),
                                                        ("C5", "f32", (1000,), (3, 0))])
def test_incremental_equals_full(name, precision, moves, modes, library):
    tdp = _tdp()
    cfg = netgen.CONFIGS[name]
    nl = with_clock(netgen.make_netlist(cfg), library)
    E = int(np.count_nonzero(nl["cell_is_ff"]))
    k = 4
    K = min(cfg.top_k_paths, E * k)
    dev = torch.device("cuda", 0)
    x = torch.tensor(nl["x"], device=dev)
    y = torch.tensor(nl["y"], device=dev)
    gi = tdp.TimingGraph(nl, library, precision=precision, max_paths=K, max_k=k)
    gf = tdp.TimingGraph(nl, library, precision=precision, max_paths=K, max_k=k)
    if precision == "f32":
        gi.set_tuning(sweep_mode=modes[0])
        gf.set_tuning(sweep_mode=modes[1])
    gi.sta_update(x, y)
    # a second required pass over the same arrivals gives the same results
    _same(_state(gi, k, K), _state(gi, k, K))
    rng = np.random.default_rng(7)
    movable = np.nonzero(np.asarray(nl["cell_fixed"]) == 0)[0]
    for rnd, m in enumerate(moves):
        cells = rng.choice(movable, m, replace=False).astype(np.int32)
        dx = rng.normal(0, 20.0, m).astype(np.float32)
        dy = rng.normal(0, 20.0, m).astype(np.float32)
        xn, yn = x.clone(), y.clone()
        ct = torch.tensor(cells, device=dev, dtype=torch.long)
        xn[ct] += torch.tensor(dx, device=dev)
        yn[ct] += torch.tensor(dy, device=dev)
        # the list may repeat cells and comes in any order
        lst = torch.tensor(np.concatenate([cells, cells[: m // 3]])[::-1].copy(), device=dev, dtype=torch.int32)
        gi.sta_update_arrivals_incremental(xn, yn, lst)
        gf.sta_update(xn, yn)
        _same(_state(gi, k, K), _state(gf, k, K))
        print(f"{name} {precision} round {rnd}: {m} cells moved, incremental == full", flush=True)
        x, y = xn, yn
    # nothing moved: nothing changes
    before = _state(gi, k, K)
    gi.sta_update_arrivals_incremental(x, y, torch.zeros(0, dtype=torch.int32, device=dev))
    _same(before, _state(gi, k, K))
    # an id outside the design is reported
    gi.sta_update_arrivals_incremental(x, y, torch.tensor([int(nl["num_cells"])], dtype=torch.int32, device=dev))
    gi.sta_update_required()
    with pytest.raises(tdp.TdpError) as e:
        gi.summary()
    assert e.value.status == 4
    gi.close()
    gf.close()
