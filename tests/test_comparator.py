"""The vectorised comparator used at full sizes agrees with the plain one,
and both catch planted mistakes (oracle output against a modified copy of
itself, CPU only)."""
import copy

import numpy as np

from oracle import ref
from paper_2503_11674_amd import netgen
from tests.bruteforce import Graph
from tests.comparator import arc_tables, compare_paths, compare_paths_fast, pair_sinks, pairs_of, valid_paths
from tests.conftest import with_clock


def _case(library):
    nl = with_clock(netgen.make_netlist(netgen.CONFIGS["C1"]), library)
    st = ref.sta(nl, library)
    k = 10
    rp = ref.extract(nl, library, st, n=-1, k=k, K=100)
    return nl, st, rp, k


def _both(gp, rp, st, nl, k):
    slow = compare_paths(gp, rp, st, Graph(nl), k)
    fast, pinned = compare_paths_fast(gp, rp, st, arc_tables(nl), k)
    for key in ("missing", "extra", "pinned", "pinned_ok", "unpinned", "unpinned_ok"):
        assert slow[key] == fast[key], (key, slow[key], fast[key])
    keys = {(int(rp["path_ep"][i]), int(rp["path_rank"][i])) for i in np.nonzero(pinned)[0]}
    assert keys == slow["pinned_keys"]
    return fast


def test_fast_comparator_agrees_on_identical_output(library):
    nl, st, rp, k = _case(library)
    c = _both(rp, rp, st, nl, k)
    assert c["missing"] == 0 and c["extra"] == 0
    assert c["pinned_ok"] == c["pinned"] > 0 and c["unpinned_ok"] == c["unpinned"]
    assert valid_paths(rp, arc_tables(nl)).all()


def test_fast_comparator_catches_planted_mistakes(library):
    nl, st, rp, k = _case(library)
    # a path with one pin replaced by another sink of the same net is invalid
    # and, if pinned, not equal
    bad = copy.deepcopy(rp)
    bad["path_pins"][bad["path_ptr"][0] + 1] = bad["path_pins"][bad["path_ptr"][1] + 1]
    c = _both(bad, rp, st, nl, k)
    assert c["pinned_ok"] + c["unpinned_ok"] == c["pinned"] + c["unpinned"] - 1
    assert not valid_paths(bad, arc_tables(nl))[0]
    # a dropped path is missing
    drop = copy.deepcopy(rp)
    m = drop["num_paths"] - 1
    drop["num_paths"] = m
    drop["path_ptr"] = drop["path_ptr"][:m + 1]
    drop["path_pins"] = drop["path_pins"][:drop["path_ptr"][m]]
    for key in ("path_ep", "path_rank", "path_slack"):
        drop[key] = drop[key][:m]
    c = _both(drop, rp, st, nl, k)
    assert c["missing"] == 1
    # a slack off by more than the tolerance fails its path
    off = copy.deepcopy(rp)
    off["path_slack"] = off["path_slack"].copy()
    off["path_slack"][3] += 1.0
    c = _both(off, rp, st, nl, k)
    assert c["pinned_ok"] + c["unpinned_ok"] == c["pinned"] + c["unpinned"] - 1


def test_pair_sinks_matches_pairs_of(library):
    nl, st, rp, k = _case(library)
    assert set(pair_sinks(rp).tolist()) == pairs_of(rp)
    mask = rp["path_slack"] < np.median(rp["path_slack"])
    keys = {(int(rp["path_ep"][i]), int(rp["path_rank"][i])) for i in np.nonzero(mask)[0]}
    assert set(pair_sinks(rp, mask).tolist()) == pairs_of(rp, keys)


def test_compare_global_accepts_the_oracle_and_flags_mistakes(library):
    from tests.comparator import compare_global, path_slacks
    nl, st, _, _ = _case(library)
    tables = arc_tables(nl)
    rp = ref.report_timing(nl, library, st, 100)
    assert np.allclose(path_slacks(rp, st), rp["path_slack"], rtol=0, atol=1e-9)

    def ok(r):
        return (r["count_ok"] and r["valid"] == r["num"] and r["slack_ok"] == r["num"] and r["distinct"]
                and r["sorted"] and r["order_stat_ok"] and r["ranks_ok"] and r["pinned_found"] == r["pinned"])

    gp = copy.deepcopy(rp)
    gp["path_slack"] = gp["path_slack"].astype(np.float32).astype(np.float64)
    res = compare_global(gp, rp, st, tables)
    assert ok(res) and res["pinned"] > 50
    # the (K+1)-th path in place of a pinned one: the order statistics move
    more = ref.report_timing(nl, library, st, 101)
    i = int(np.nonzero(np.diff(rp["path_slack"]) > 1.0)[0][0])
    lists = ref.path_list(more)
    keep = [j for j in range(101) if j != i]
    bad = {"num_paths": 100, "path_ep": more["path_ep"][keep], "path_rank": more["path_rank"][keep],
           "path_slack": more["path_slack"][keep]}
    sel = [lists[j] for j in keep]
    bad["path_ptr"] = np.concatenate([[0], np.cumsum([len(p) for p in sel])]).astype(np.int32)
    bad["path_pins"] = np.concatenate(sel).astype(np.int32)
    r = compare_global(bad, rp, st, tables)
    assert not ok(r)
    # a wrong rank, a corrupt pin, a duplicated path
    g2 = copy.deepcopy(gp)
    g2["path_rank"][0] += 1
    assert not compare_global(g2, rp, st, tables)["ranks_ok"]
    g3 = copy.deepcopy(gp)
    g3["path_pins"][g3["path_ptr"][3] + 1] = g3["path_pins"][g3["path_ptr"][3] + 3]
    assert compare_global(g3, rp, st, tables)["valid"] < 100
    g4 = copy.deepcopy(gp)
    a, b = g4["path_ptr"][0], g4["path_ptr"][1]
    c_, d_ = g4["path_ptr"][1], g4["path_ptr"][2]
    if b - a == d_ - c_:
        g4["path_pins"][c_:d_] = g4["path_pins"][a:b]
        assert not compare_global(g4, rp, st, tables)["distinct"]
