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
