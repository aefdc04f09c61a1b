"""Tolerance-aware comparison of the HIP results against the CPU oracle.

Timing values: |v - ref| <= 1e-4 * max(|ref|, 1 ps) for arrival and required
times; for slack the scale is max(|AT_ref|, |RAT_ref|, 1 ps).  Infinities must
match exactly.

Paths: at each selected endpoint the oracle's rank-r path (slacks
s_0 <= s_1 <= ... and s_k, the next one) is *pinned* when it is separated from
its neighbours by more than a threshold thr:
    (r == 0 or s_r - s_{r-1} > thr) and s_{r+1} - s_r > thr.
A pinned path must be pin-for-pin identical; an unpinned one must be a valid
path whose slack matches the oracle's rank-r slack within tolerance.

thr is 1e-3 ps in double precision.  In single precision the arrival times
themselves carry rounding error, bounded for a path of L arcs by
gamma_L * sum|terms| with gamma_L = L u / (1 - L u), u = 2^-24 (recursive
summation), sum|terms| = |AT(start)| + sum |arc delays| + |RAT(end)|; twice
that bound (both paths of a pair move) is the single-precision threshold.
"""
import math

import numpy as np

U32 = 2.0 ** -24


def timing_close(v, ref, scale=None, rtol=1e-4):
    v = np.asarray(v, np.float64)
    ref = np.asarray(ref, np.float64)
    inf_ok = np.array_equal(np.isposinf(v), np.isposinf(ref)) and np.array_equal(np.isneginf(v), np.isneginf(ref))
    fin = np.isfinite(ref)
    sc = np.maximum(np.abs(ref[fin]) if scale is None else np.asarray(scale)[fin], 1.0)
    err = np.abs(v[fin] - ref[fin])
    bad = err > rtol * sc
    return inf_ok, int(bad.sum()), float((err / sc).max()) if err.size else 0.0


def fp32_threshold(path, st, nl_roles=None):
    """Rounding bound on a single-precision path slack (see module doc)."""
    L = len(path) - 1
    g = L * U32 / (1 - L * U32)
    terms = abs(st["at"][path[0]]) + abs(st["rat"][path[-1]])
    for a, b in zip(path[:-1], path[1:]):
        terms += abs(st["at"][b] - st["at"][a]) if np.isfinite(st["at"][b]) else 0.0
    return max(1e-3, 2.0 * g * terms)


def compare_paths(gpu, ref, st, graph, k, fp32=True):
    """gpu / ref: dicts from TimingGraph.paths() / oracle.extract().
    Returns counts (pinned, pinned_ok, unpinned, unpinned_ok, missing)."""
    ref_by_ep = {}
    plist = [ref["path_pins"][ref["path_ptr"][i]:ref["path_ptr"][i + 1]].tolist() for i in range(ref["num_paths"])]
    for i in range(ref["num_paths"]):
        ref_by_ep.setdefault(int(ref["path_ep"][i]), {})[int(ref["path_rank"][i])] = (ref["path_slack"][i], plist[i])
    nxt = dict(zip(ref["sel_ep"].tolist(), ref["ep_next"].tolist()))
    gl = [gpu["path_pins"][gpu["path_ptr"][i]:gpu["path_ptr"][i + 1]].tolist() for i in range(gpu["num_paths"])]
    gpu_by = {(int(gpu["path_ep"][i]), int(gpu["path_rank"][i])): (gpu["path_slack"][i], gl[i])
              for i in range(gpu["num_paths"])}
    c = dict(pinned=0, pinned_ok=0, unpinned=0, unpinned_ok=0, missing=0, extra=0)
    pinned_keys = set()
    for e, ranks in ref_by_ep.items():
        n = len(ranks)
        sl = [ranks[r][0] for r in range(n)]
        sl_next = nxt.get(e, math.inf) if n == k else math.inf
        for r in range(n):
            s_r, pl = ranks[r]
            thr = fp32_threshold(pl, st) if fp32 else 1e-3
            lo = r == 0 or s_r - sl[r - 1] > thr
            hi = (sl[r + 1] if r + 1 < n else sl_next) - s_r > thr
            got = gpu_by.get((e, r))
            if got is None:
                c["missing"] += 1
                continue
            tol = 1e-4 * max(abs(st["at"][pl[-1]]), abs(st["rat"][pl[-1]]), 1.0)
            if lo and hi:
                c["pinned"] += 1
                pinned_keys.add((e, r))
                if got[1] == pl and abs(got[0] - s_r) <= tol:
                    c["pinned_ok"] += 1
            else:
                c["unpinned"] += 1
                if abs(got[0] - s_r) <= tol and graph.is_path(got[1]):
                    c["unpinned_ok"] += 1
    c["extra"] = sum(1 for key in gpu_by if key[0] not in ref_by_ep or key[1] not in ref_by_ep[key[0]])
    c["pinned_keys"] = pinned_keys
    return c


def pairs_of(paths_dict, keys=None):
    """Sink pins of the net arcs on the given paths (all if keys is None)."""
    out = set()
    ptr, pins = paths_dict["path_ptr"], paths_dict["path_pins"]
    for i in range(paths_dict["num_paths"]):
        if keys is not None and (int(paths_dict["path_ep"][i]), int(paths_dict["path_rank"][i])) not in keys:
            continue
        out.update(pins[ptr[i] + 1:ptr[i + 1]:2].tolist())
    return out
