"""report_timing(K) without device allocation: the entry point whose node
store lives in the library's fixed device array, against report_timing on
the same graphs (bitwise), on two calls in a row with the second on a
smaller input, and its refusal of a graph whose store does not fit."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2503_11674_amd import netgen  # noqa: E402
from tests.conftest import with_clock  # noqa: E402

pytestmark = pytest.mark.gpu

KEYS = ("path_ptr", "path_pins", "path_ep", "path_rank", "path_slack")


def _graph(name, library, max_paths, max_k):
    from paper_2503_11674_amd import tdp
    nl = with_clock(netgen.make_netlist(netgen.CONFIGS[name]), library)
    g = tdp.TimingGraph(nl, library, max_paths=max_paths, max_k=max_k)
    dev = torch.device("cuda", 0)
    g.sta_update(torch.tensor(nl["x"], device=dev), torch.tensor(nl["y"], device=dev))
    return g


def _same(a, b):
    assert a["num_paths"] == b["num_paths"] and a["num_paths"] > 0
    for key in KEYS:
        assert np.array_equal(a[key], b[key]), key


def test_report_timing_without_allocation_matches(library):
    from paper_2503_11674_amd import tdp
    big = _graph("C2", library, 10000, 10)
    small = _graph("C1", library, 200, 10)
    print("C2 then C1 (smaller), each against report_timing", flush=True)
    for g, K in ((big, 10000), (small, 150)):
        g.report_timing(K)
        want = g.paths()
        g.report_timing_noalloc(K)
        got = g.paths()
        _same(want, got)
        # the lists the pair update reads follow the same paths
        g.pairs_reset()
        g.pairs_update(rule=0)
        w_a, in_a = g.pairs_export()
        g.report_timing(K)
        g.pairs_reset()
        g.pairs_update(rule=0)
        w_b, in_b = g.pairs_export()
        assert np.array_equal(w_a, w_b) and np.array_equal(in_a, in_b)
    # a graph whose node store exceeds the fixed array is refused with the
    # size it needs
    big.close()
    huge = _graph("C2", library, 400000, 10)
    with pytest.raises(tdp.TdpError) as e:
        huge.report_timing_noalloc(1000)
    assert e.value.status == 5 and "bytes" in str(e.value)
    huge.close()
    small.close()
