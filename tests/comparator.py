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


# ------------------------------------------------------------------
# Vectorised forms for the full-size workloads (millions of path pins).
def _segments(ptr):
    """For a CSR pointer array: path index and position in the path of every
    element."""
    ptr = np.asarray(ptr, np.int64)
    lens = np.diff(ptr)
    pid = np.repeat(np.arange(lens.shape[0]), lens)
    pos = np.arange(ptr[-1]) - ptr[pid]
    return pid, pos, lens


def arc_tables(nl):
    """driver_of[sink pin], out_of[combinational input pin], is_start[pin],
    is_end[pin] (-1 / False where not applicable)."""
    P = int(nl["num_pins"])
    net_ptr, net_pins = np.asarray(nl["net_ptr"]), np.asarray(nl["net_pins"])
    driver_of = np.full(P, -1, np.int64)
    nlen = np.diff(net_ptr)
    drv = np.repeat(net_pins[net_ptr[:-1]], nlen)
    first = np.zeros(net_pins.shape[0], bool)
    first[net_ptr[:-1][nlen > 0]] = True
    driver_of[net_pins[~first]] = drv[~first]
    out_of = np.full(P, -1, np.int64)
    ff = np.asarray(nl["cell_is_ff"]) != 0
    cptr, cins = np.asarray(nl["cell_in_ptr"]), np.asarray(nl["cell_in_pins"])
    clen = np.diff(cptr)
    owner = np.repeat(np.arange(int(nl["num_cells"])), clen)
    comb_in = ~ff[owner]
    out_of[cins[comb_in]] = np.asarray(nl["cell_out_pin"])[owner[comb_in]]
    is_start = np.asarray(nl["pin_cell"]) < 0
    is_start[np.asarray(nl["cell_out_pin"])[ff]] = True
    is_end = np.zeros(P, bool)
    is_end[cins[ff[owner]]] = True
    return driver_of, out_of, is_start, is_end


def valid_paths(paths, tables):
    """Per path: a start point, then alternately a net arc into a sink and a
    cell arc to that cell's output, ending at its endpoint pin."""
    driver_of, out_of, is_start, is_end = tables
    pins = np.asarray(paths["path_pins"], np.int64)
    ptr = np.asarray(paths["path_ptr"], np.int64)
    m = int(paths["num_paths"])
    if m == 0:
        return np.zeros(0, bool)
    pid, pos, lens = _segments(ptr)
    ok = np.ones(pins.shape[0], bool)
    odd = pos % 2 == 1
    ok[odd] = driver_of[pins[odd]] == pins[np.nonzero(odd)[0] - 1]
    ev = (pos % 2 == 0) & (pos > 0)
    ok[ev] = out_of[pins[np.nonzero(ev)[0] - 1]] == pins[ev]
    ok[pos == 0] = is_start[pins[pos == 0]]
    good = np.ones(m, bool)
    np.logical_and.at(good, pid, ok)
    last = pins[ptr[1:] - 1]
    good &= (lens % 2 == 0) & is_end[last] & (last == np.asarray(paths["path_ep"], np.int64))
    return good


def compare_paths_fast(gpu, ref, st, tables, k, fp32=True):
    """compare_paths for large outputs.  Returns the same counts and the
    boolean mask of pinned oracle paths that the GPU output also has (in the
    oracle's output order)."""
    m = int(ref["num_paths"])
    at, rat = np.asarray(st["at"]), np.asarray(st["rat"])
    r_ep = np.asarray(ref["path_ep"], np.int64)
    r_rk = np.asarray(ref["path_rank"], np.int64)
    r_sl = np.asarray(ref["path_slack"], np.float64)
    r_ptr = np.asarray(ref["path_ptr"], np.int64)
    r_pins = np.asarray(ref["path_pins"], np.int64)
    key_r = r_ep * (k + 1) + r_rk
    g_key = np.asarray(gpu["path_ep"], np.int64) * (k + 1) + np.asarray(gpu["path_rank"], np.int64)
    # thresholds (module doc): rounding bound of each oracle path's slack
    lens = np.diff(r_ptr)
    if fp32:
        d = np.abs(np.diff(at[r_pins])) if r_pins.shape[0] > 1 else np.zeros(0)
        cs = np.concatenate([[0.0], np.cumsum(d)])
        inner = cs[r_ptr[1:] - 1] - cs[r_ptr[:-1]]
        terms = np.abs(at[r_pins[r_ptr[:-1]]]) + np.abs(rat[r_pins[r_ptr[1:] - 1]]) + inner
        L = (lens - 1).astype(np.float64)
        gam = L * U32 / (1 - L * U32)
        thr = np.maximum(1e-3, 2.0 * gam * terms)
    else:
        thr = np.full(m, 1e-3)
    # neighbours in (endpoint, rank) order
    o = np.argsort(key_r, kind="stable")
    ep_o, sl_o, rk_o = r_ep[o], r_sl[o], r_rk[o]
    same_prev = np.zeros(m, bool)
    same_prev[1:] = ep_o[1:] == ep_o[:-1]
    same_next = np.zeros(m, bool)
    same_next[:-1] = same_prev[1:]
    nxt = dict(zip(np.asarray(ref["sel_ep"]).tolist(), np.asarray(ref["ep_next"]).tolist()))
    cnt = np.bincount(np.searchsorted(np.unique(ep_o), ep_o))
    count_of = np.repeat(cnt, cnt)
    s_next = np.full(m, np.inf)
    s_next[:-1] = np.where(same_next[:-1], sl_o[1:], np.inf)
    tail = ~same_next & (count_of == k)
    s_next[tail] = [nxt.get(int(e), np.inf) for e in ep_o[tail]]
    s_prev = np.full(m, -np.inf)
    s_prev[1:] = np.where(same_prev[1:], sl_o[:-1], -np.inf)
    thr_o = thr[o]
    lo = (rk_o == 0) | (sl_o - s_prev > thr_o)
    hi = s_next - sl_o > thr_o
    pinned_o = lo & hi
    pinned = np.zeros(m, bool)
    pinned[o] = pinned_o
    # match GPU paths by key
    g_sort = np.argsort(g_key, kind="stable")
    pos = np.searchsorted(g_key[g_sort], key_r)
    pos = np.minimum(pos, max(0, g_key.shape[0] - 1))
    found = (g_key.shape[0] > 0) & (g_key[g_sort][pos] == key_r) if g_key.shape[0] else np.zeros(m, bool)
    gi = g_sort[pos]
    c = dict(missing=int((~found).sum()), extra=int((~np.isin(g_key, key_r)).sum()))
    g_ptr = np.asarray(gpu["path_ptr"], np.int64)
    g_pins = np.asarray(gpu["path_pins"], np.int64)
    g_sl = np.asarray(gpu["path_slack"], np.float64)
    last = r_pins[r_ptr[1:] - 1]
    tol = 1e-4 * np.maximum(np.maximum(np.abs(at[last]), np.abs(rat[last])), 1.0)
    slack_ok = found & (np.abs(g_sl[gi] - r_sl) <= tol)
    # pin-for-pin equality for pinned paths of equal length
    g_len = np.diff(g_ptr)[gi]
    same_len = found & (g_len == lens)
    cand = np.nonzero(pinned & same_len)[0]
    eq = np.zeros(m, bool)
    if cand.shape[0]:
        ln = lens[cand]
        seg = np.repeat(np.arange(cand.shape[0]), ln)
        off = np.arange(ln.sum()) - np.repeat(np.cumsum(ln) - ln, ln)
        a = r_pins[r_ptr[cand][seg] + off]
        b = g_pins[g_ptr[gi[cand]][seg] + off]
        bad = np.zeros(cand.shape[0], np.int64)
        np.add.at(bad, seg, (a != b).astype(np.int64))
        eq[cand] = bad == 0
    gvalid = valid_paths(gpu, tables)
    c["pinned"] = int((pinned & found).sum())
    c["pinned_ok"] = int((pinned & eq & slack_ok).sum())
    unp = ~pinned & found
    c["unpinned"] = int(unp.sum())
    c["unpinned_ok"] = int((unp & slack_ok & gvalid[gi]).sum())
    c["gpu_valid"] = int(gvalid.sum())
    return c, pinned & found


def pair_sinks(paths, mask=None):
    """Sink pins of the net arcs on the paths selected by mask (all if None),
    one entry per occurrence."""
    pid, pos, _ = _segments(paths["path_ptr"])
    pins = np.asarray(paths["path_pins"], np.int64)
    sel = pos % 2 == 1
    if mask is not None:
        sel &= np.asarray(mask)[pid]
    return pins[sel]


def path_slacks(paths, st):
    """FP64 slack of every path from the oracle's arc delays:
    RAT(end) - (AT(start) + net delays into its sinks + cell-arc delays)."""
    m = int(paths["num_paths"])
    if m == 0:
        return np.zeros(0)
    pid, pos, _ = _segments(paths["path_ptr"])
    pins = np.asarray(paths["path_pins"], np.int64)
    ptr = np.asarray(paths["path_ptr"], np.int64)
    d = np.zeros(pins.shape[0])
    odd = pos % 2 == 1
    d[odd] = np.asarray(st["dnet"])[pins[odd]]
    ev = (pos % 2 == 0) & (pos > 0)
    d[ev] = np.asarray(st["darc"])[pins[np.nonzero(ev)[0] - 1]]
    arr = np.zeros(m)
    np.add.at(arr, pid, d)
    arr += np.asarray(st["at"])[pins[ptr[:-1]]]
    return np.asarray(st["rat"])[pins[ptr[1:] - 1]] - arr


def _fp32_thresholds(paths, st):
    """Per path: the single-precision rounding bound of the module doc."""
    at, rat = np.asarray(st["at"]), np.asarray(st["rat"])
    ptr = np.asarray(paths["path_ptr"], np.int64)
    pins = np.asarray(paths["path_pins"], np.int64)
    d = np.abs(np.diff(at[pins])) if pins.shape[0] > 1 else np.zeros(0)
    cs = np.concatenate([[0.0], np.cumsum(d)])
    inner = cs[ptr[1:] - 1] - cs[ptr[:-1]]
    terms = np.abs(at[pins[ptr[:-1]]]) + np.abs(rat[pins[ptr[1:] - 1]]) + inner
    L = (np.diff(ptr) - 1).astype(np.float64)
    gam = L * U32 / (1 - L * U32)
    return np.maximum(1e-3, 2.0 * gam * terms)


def compare_global(gpu, ref, st, tables, fp32=True):
    """report_timing(K): the GPU's paths against the oracle's.

    Several answers are correct where slacks tie within rounding, so the
    checks are: every GPU path is a valid, distinct path whose reported slack
    matches its FP64 recomputation; the sorted FP64 slacks of the two answers
    agree within the rounding bound (the K order statistics are unique); an
    oracle path whose slack is separated by more than that bound from its
    neighbours in the global order (and, for the last one, from the next path
    after it) is in the GPU answer pin for pin; ranks count the earlier paths
    of the same endpoint."""
    m = int(ref["num_paths"])
    n = int(gpu["num_paths"])
    res = {"num": n, "count_ok": n == m}
    at, rat = np.asarray(st["at"]), np.asarray(st["rat"])
    g_ptr = np.asarray(gpu["path_ptr"], np.int64)
    g_pins = np.asarray(gpu["path_pins"], np.int64)
    g_sl = np.asarray(gpu["path_slack"], np.float64)
    rec = path_slacks(gpu, st)
    last = g_pins[g_ptr[1:] - 1] if n else np.zeros(0, np.int64)
    tol = 1e-4 * np.maximum(np.maximum(np.abs(at[last]), np.abs(rat[last])), 1.0)
    res["valid"] = int(valid_paths(gpu, tables).sum())
    res["slack_ok"] = int((np.abs(g_sl - rec) <= tol).sum())
    g_list = [tuple(g_pins[g_ptr[i]:g_ptr[i + 1]].tolist()) for i in range(n)]
    res["distinct"] = len(set(g_list)) == n
    res["sorted"] = bool(np.all(np.diff(g_sl) >= 0))
    thr = _fp32_thresholds(ref, st) if fp32 else np.full(m, 1e-3)
    thr_all = float(thr.max()) if m else 1e-3
    r_sl = np.asarray(ref["path_slack"], np.float64)
    k = min(n, m)
    res["order_stat_ok"] = bool(np.all(np.abs(np.sort(rec)[:k] - np.sort(r_sl)[:k]) <= 2 * thr_all + tol[:k].max()
                                       if k else True))
    # pinned oracle paths
    nxt = float(ref.get("next_slack", np.inf))
    prev = np.concatenate([[-np.inf], r_sl[:-1]])
    after = np.concatenate([r_sl[1:], [nxt]])
    pinned = ((r_sl - prev) > thr) & ((after - r_sl) > thr)
    r_ptr = np.asarray(ref["path_ptr"], np.int64)
    r_pins = np.asarray(ref["path_pins"], np.int64)
    gset = set(g_list)
    found = [tuple(r_pins[r_ptr[i]:r_ptr[i + 1]].tolist()) in gset for i in np.nonzero(pinned)[0]]
    res["pinned"] = int(pinned.sum())
    res["pinned_found"] = int(sum(found))
    seen = {}
    ok = True
    for i, e in enumerate(np.asarray(gpu["path_ep"]).tolist()):
        ok &= int(gpu["path_rank"][i]) == seen.get(e, 0)
        seen[e] = seen.get(e, 0) + 1
    res["ranks_ok"] = bool(ok)
    res["endpoints"] = len(seen)
    return res
