"""Throughput of the timing-driven placement hot path on one MI355X.

One step = static timing analysis (net delays, forward arrivals, endpoint
WNS/TNS, backward required times and slack), report_timing_endpoint(n_fail, k)
with k = K // n_fail, the Eq. 9 pin-pair update, weighted-average wirelength
forward+backward and the pin-to-pin loss forward+backward, on the 2M-cell
synthetic workload (clustered placement, depth 100, 12 % flip-flops, K = 100k
paths).  Cell positions are fixed across steps, so every step does the same
work.  Prints one JSON line.

  python bench.py [--steps K] [--warmup W] [--workload C5|C3|C2|C1] [--no-cpu]

--workload C4 measures the batched form instead: timing update + extraction
(k = 10, K = 5,000 per instance) over 32 uneven netlists and 8 placement
snapshots of a 500k-cell netlist, as one union graph replayed from a captured
HIP graph, against the same 40 instances launched one graph at a time.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_2m_cells.md")
# the kernel that carries each stage's work (per-level sweeps launch it once
# per level, the dataflow sweeps once)
STAGE_KERNEL = {
    "netpass": ("tdp::k_netpass<float, false>", "tdp::k_netpass<float, true>"), "forward": ("tdp::k_forward<float, 8>", "tdp::k_forward_flow<8>"),
    "backward": ("tdp::k_backward<float>", "tdp::k_backward_flow"), "walk": ("tdp::k_walk<float>",),
    "pairs": ("tdp::k_pairs_acc_lds<float>",), "wa": ("tdp::k_wa_net",), "search": ("tdp::k_search<float, 8>",),
}


def source_digest() -> str:
    """sha1 over the library's sources: counters taken from another version
    of the kernels do not apply."""
    import hashlib
    h = hashlib.sha1()
    csrc = os.path.join(ROOT, "paper_2503_11674_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()


def measured_traffic(kernel: str):
    """HBM bytes per dispatch of `kernel` from the committed counter summary,
    or None when it is missing or was taken from other sources."""
    try:
        text = open(TRAFFIC_FILE).read()
    except OSError:
        return None
    if f"Source digest: {source_digest()}" not in text:
        return None
    for line in text.splitlines():
        cells = [c.strip() for c in line.strip().strip("|").split("|")]
        if len(cells) == 5 and cells[0] == kernel:
            return int(float(cells[4]) * 1e6)
    return None
STATS_FILE = os.path.join(ROOT, "profiles", "kernel_stats_2m_cells.md")


def rocprof_avg_us(kernel: str):
    """Average dispatch duration of `kernel` in the committed rocprofv3
    statistics of the 2M-cell step, or None when missing or taken from other
    sources."""
    try:
        text = open(STATS_FILE).read()
    except OSError:
        return None
    if f"Source digest: {source_digest()}" not in text:
        return None
    for line in text.splitlines():
        cells = [c.strip() for c in line.strip().strip("|").split("|")]
        if len(cells) >= 3 and cells[0] == kernel:
            try:
                return float(cells[2])
            except ValueError:
                return None
    return None


BETA = 2.5e-5          # weight of the pin-to-pin term in the objective (Sec. IV)
WA_GAMMA = 5.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    # about a second of timed GPU work at 2M cells, long enough for an
    # outside sampler of GPU activity to see it
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="C5")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched (40-instance) leg of the default run")
    ap.add_argument("--graph", action="store_true", help="replay the step as a captured HIP graph")
    ap.add_argument("--no-tune", action="store_true", help="skip the autotuner (default launch configuration)")
    ap.add_argument("--step-only", action="store_true",
                    help="skip the legs after the timed steps (pair-loss variants, early analysis, rise / fall, "
                         "incremental arrivals), e.g. for a profile of the step alone")
    ap.add_argument("--sweep-mode", type=int, default=-1, help="force a sweep form (0 per level, 1 dataflow)")
    ap.add_argument("--serial", action="store_true", help="run the whole step on one stream")
    ap.add_argument("--table1", action="store_true",
                    help="extraction statistics of report_timing(K) against report_timing_endpoint(n, k) "
                         "(paths, endpoints, pin pairs, time) instead of the step benchmark")
    ap.add_argument("--loop", action="store_true",
                    help="the placement loop around the step (Sec. IV, Fig. 5 analogue): wirelength-driven "
                         "against timing-driven runs, and the time per iteration")
    ap.add_argument("--loop-beta", type=float, default=2e-3,
                    help="PP weight of the timing-driven runs of --loop (um^-2 scale of these designs)")
    ap.add_argument("--net-model", type=int, default=0, choices=(0, 1, 2),
                    help="0: lumped RC wires (Eq. 7); 1: Elmore star nets with degraded sink transitions; "
                         "2: Elmore delays on each net's rectilinear minimum spanning tree, degraded transitions")
    ap.add_argument("--configs", action="store_true",
                    help="one line per workload (2k, 200k, 1M and 2M cells, and the batched union), each from its "
                         "own run of this script, with the oracle's rate where it finishes in seconds")
    ap.add_argument("--copy-calib", type=int, default=0, metavar="MB",
                    help="after timing, run one plain device copy of MB MiB (counter calibration)")
    return ap.parse_args()


def algo_bytes(info, counts):
    """Algorithmic bytes per stage of one step: what the method itself must
    move (float32 values, int32 ids; an array element counts once per pass, a
    gather counts its element size).  S sink arcs, M nets (drivers), A
    combinational input pins, N_c combinational cells, E endpoints (= flip-
    flops), PI primary inputs, K_out paths of Lbar cells (Lbar measured: half
    the pins per path), Q unique pairs, T touched cells.
      net pass 28 S + 28 M; forward 24 A + 18 N_c + 16 (E + FF + PI);
      endpoint / select 12 E; backward 28 S + 16 M;
      extraction 13 K_out Lbar + 12 K_out; p2p forward + backward 36 Q + 8 T;
      WA forward + backward 16 P + 4 M + 8 N.
    The pair update has no such figure; its bytes follow the kernels' reads
    and writes of the occurrences and of the pair tables."""
    N, P, M, D, E, n_start, n_comb, S = info
    A = S - E
    PI = n_start - E
    npaths, npins = counts["paths"], counts["path_pins"]
    lbar = npins / (2.0 * npaths) if npaths else 0.0
    b = {}
    b["netpass"] = 28 * S + 28 * M
    b["forward"] = 24 * A + 18 * n_comb + 16 * (E + E + PI)
    b["endpoint"] = 12 * E
    b["backward"] = 28 * S + 16 * M
    ext = 13 * npaths * lbar + 12 * npaths
    # extraction as one figure, spread over its kernels by what each touches
    b["select"] = 0
    b["search"] = 0
    b["order"] = 12 * npaths
    b["walk"] = int(13 * npaths * lbar)
    occ = npins // 2
    b["pairs"] = 2 * (12 * occ + 8 * npaths) + 9 * S + 76 * counts["pairs"]
    b["p2p_fwd"] = 36 * counts["pairs"]
    b["p2p_bwd"] = 8 * counts["touched"]
    b["wa"] = 16 * P + 4 * M + 8 * N
    b["_extraction"] = int(ext)
    return b


def design_overhead(info, side_k):
    """Bytes per step that this design moves beyond the method's own: the
    forward sweep's per-cell deviation lists (cost and sink per entry) and
    four-hop walk records and the per-input arrivals it keeps for them; the
    backward sweep's second copy of the net delays in net-chunk order."""
    N, P, M, D, E, n_start, n_comb, S = info
    A = S - E
    km = side_k if side_k > 1 else 0
    return {"forward": n_comb * (8 * km + 64 + 4) + 4 * A, "backward": 4 * S}


def build_step(g, x, y, k, K, gx, gy, wl, pp, beta, overlap=True):
    """One step of the hot path on graph g at positions (x, y): timing update,
    report_timing_endpoint(n_fail, k) cut to K, the Eq. 9 pair update, WA
    forward+backward and the p2p loss forward+backward (beta-scaled into the
    same gradient).  With overlap, the two stages that nothing later in the
    step reads run on side streams: the required-time pass beside extraction
    and pairs, WA beside them too (it needs only the positions); both join
    the calling stream before the step returns.  Every call launches on the
    stream current at call time (the capture stream under a HIP graph)."""
    import torch
    side_req = torch.cuda.Stream()
    side_wa = torch.cuda.Stream()
    ev_arr, ev_req, ev_wa = torch.cuda.Event(), torch.cuda.Event(), torch.cuda.Event()

    def step():
        main = torch.cuda.current_stream()
        if not overlap:
            g.sta_update(x, y)
            g.extract_paths(n=-1, k=k, K=K)
            g.pairs_update(rule=0, w0=10.0, w1=0.2)
            gx.zero_()
            gy.zero_()
            g.wa_fwd_bwd_at_update(WA_GAMMA, gx, gy, out=wl)  # positions of this step's update
            g.p2p_loss_fwd(x, y, out=pp)
            g.p2p_loss_bwd(x, y, beta, gx, gy)
            return
        # submission order matters as much as the streams: the host enqueues
        # the main stream's extraction before the 101 launches of the
        # required-time pass, so the main stream never waits for the host
        g.sta_update_arrivals(x, y)
        ev_arr.record(main)
        side_wa.wait_event(ev_arr)
        with torch.cuda.stream(side_wa):
            gx.zero_()
            gy.zero_()
            g.wa_fwd_bwd_at_update(WA_GAMMA, gx, gy, out=wl)
        ev_wa.record(side_wa)
        g.extract_paths(n=-1, k=k, K=K)
        g.pairs_update(rule=0, w0=10.0, w1=0.2)
        g.p2p_loss_fwd(x, y, out=pp)
        side_req.wait_event(ev_arr)
        g.sta_update_required(stream=side_req)
        ev_req.record(side_req)
        main.wait_event(ev_wa)  # the p2p gradient adds to WA's
        g.p2p_loss_bwd(x, y, beta, gx, gy)
        main.wait_event(ev_req)

    return step


def bench_table1(a):
    """Sec. III-B / Table I on a synthetic design: the K worst paths of the
    whole design (report_timing(K), K = n_fail and 10 n_fail) against the
    worst paths per failing endpoint (report_timing_endpoint(n_fail, 1) and
    (n_fail, 10)): number of paths, of distinct endpoints and of distinct pin
    pairs (net arcs) on them, and the GPU time of the call."""
    import torch

    from paper_2503_11674_amd import netgen
    from paper_2503_11674_amd.tdp import TimingGraph

    cfg = netgen.CONFIGS[a.workload]
    nl = netgen.make_netlist(cfg)
    lib = netgen.make_library()
    dev = torch.device("cuda", 0)
    x = torch.tensor(nl["x"], device=dev)
    y = torch.tensor(nl["y"], device=dev)
    E = int(np.count_nonzero(nl["cell_is_ff"]))
    nf = E // 20
    g = TimingGraph(nl, lib, max_paths=10 * nf, max_k=10)
    g.sta_update(x, y)
    at = g.export()["at"].cpu().numpy()
    ep = nl["cell_in_pins"][nl["cell_in_ptr"][np.nonzero(nl["cell_is_ff"])[0]]]
    g.set_clock(netgen.clock_period_for_fail_fraction(at[ep], 0.05))
    g.sta_update(x, y)
    wns, tns, n_fail = g.summary()
    cmds = [(f"report_timing({n_fail})", lambda: g.report_timing(n_fail)),
            (f"report_timing({10 * n_fail})", lambda: g.report_timing(10 * n_fail)),
            (f"report_timing_endpoint({n_fail},1)", lambda: g.extract_paths(n=-1, k=1, K=n_fail)),
            (f"report_timing_endpoint({n_fail},10)", lambda: g.extract_paths(n=-1, k=10, K=10 * n_fail))]
    rows = []
    for name, call in cmds:
        print(f"[table1] {name}", file=sys.stderr, flush=True)
        call()
        torch.cuda.synchronize()
        ts = []
        for _ in range(max(1, a.steps)):
            t0 = time.perf_counter()
            call()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        p = g.paths()
        ptr, pins = p["path_ptr"], p["path_pins"]
        lens = np.diff(ptr)
        pos = np.arange(pins.shape[0]) - np.repeat(ptr[:-1], lens)
        rows.append({"command": name, "paths": int(p["num_paths"]),
                     "endpoints": int(np.unique(p["path_ep"]).shape[0]),
                     "pin_pairs": int(np.unique(pins[pos % 2 == 1]).shape[0]),
                     "ms": round(1e3 * float(np.median(ts)), 3),
                     "worst_slack": float(p["path_slack"][0]) if p["num_paths"] else None,
                     "last_slack": float(p["path_slack"][-1]) if p["num_paths"] else None})
        print(f"[table1] {rows[-1]}", file=sys.stderr, flush=True)
    print(json.dumps({"table": "extraction statistics (Sec. III-B, Table I analogue)",
                      "workload": f"{a.workload}: {nl['num_cells']} cells, {nl['num_pins']} pins, "
                                  f"{E} endpoints", "n_fail": n_fail, "wns": wns, "tns": tns,
                      "runs": max(1, a.steps), "rows": rows}), flush=True)


def bench_loop(a):
    """The placement loop (Sec. IV) in three parts.

    Global placement: the wirelength-driven schedule from the generated
    placement to overflow < 0.1 (history of HPWL, overflow every 15
    iterations, iterations and wall time; its final WNS / TNS at the clock
    below).

    The paper's schedule: the same run from the same start with timing from
    half its iteration count, every 15 iterations, lambda growing and
    momentum on, to the same stopping rule (HPWL, overflow, WNS, TNS every 15
    iterations).

    Timing phase (the part of the paper's flow after timing starts): from that
    converged placement, with the clock at which 5 % of its endpoints fail and
    lambda frozen at its final value, 150 more iterations of the same
    optimiser state with beta = 0 and with timing every 15 iterations (report_timing_endpoint(n_fail, 1),
    Eq. 9, PP); HPWL, overflow, WNS, TNS every 15 iterations (a Fig. 5
    analogue).  Also the GPU time per iteration with and without a timing
    refresh."""
    import torch

    from paper_2503_11674_amd import netgen
    from paper_2503_11674_amd.placer import GlobalPlacer, LoopConfig

    cfg_n = netgen.CONFIGS[a.workload]
    nl = netgen.make_netlist(cfg_n)
    lib = dict(netgen.make_library(), net_model=a.net_model)
    N = int(nl["num_cells"])
    bins = 1
    while bins * bins < N // 2:
        bins *= 2
    die = float(cfg_n.die)

    def log(tag):
        return lambda r: print(f"[loop] {tag} it={r.it} hpwl={r.hpwl:.4g} ovf={r.overflow:.3f} "
                               f"wns={r.wns:.1f} tns={r.tns:.4g} pairs={r.pairs}", file=sys.stderr, flush=True)

    def rows(hist):
        return [[r.it, round(r.hpwl, 1), round(r.overflow, 4), round(r.wns, 1), round(r.tns, 1), r.n_fail, r.pairs]
                for r in hist]

    # global placement, wirelength-driven, to convergence
    nl["clock_period"] = np.float32(1e9)
    # (timing_start 0: the stopping rule applies from the start)
    p = GlobalPlacer(nl, lib, LoopConfig(die=die, bins=bins, beta=0.0, record_every=15, timing_start=0))
    t0 = time.perf_counter()
    hist = p.run(log=log("global"))
    torch.cuda.synchronize()
    glob = {"iterations": p.it, "wall_s": round(time.perf_counter() - t0, 3),
            "history": [[r.it, round(r.hpwl, 1), round(r.overflow, 4)] for r in hist]}
    ux, uy = (t.cpu().numpy().copy() for t in p.positions())
    lam = float(p.lam)
    snap = p.snapshot()
    p.g.sta_update(*p.positions())
    at = p.g.export()["at"].cpu().numpy()
    ff = np.nonzero(np.asarray(nl["cell_is_ff"]))[0]
    ep = np.asarray(nl["cell_in_pins"])[np.asarray(nl["cell_in_ptr"])[ff]]
    T = netgen.clock_period_for_fail_fraction(at[ep], 0.05)
    p.g.set_clock(T)
    p.g.sta_update(*p.positions())
    w_, t_, n_ = p.g.summary()
    glob["final_at_clock"] = [glob["iterations"], round(hist[-1].hpwl, 1),
                              round(hist[-1].overflow, 4), round(w_, 1), round(t_, 1), n_, 0]
    p.g.close()
    print(f"[loop] converged after {glob['iterations']} iterations; clock {T:.1f} ps; lambda {lam:.4g}",
          file=sys.stderr, flush=True)

    # the paper's schedule in one run from the same start: timing from the
    # middle of the wirelength-driven run (the paper starts at iteration 500
    # of about a thousand), every 15 iterations, with lambda's growth and
    # Nesterov's momentum live, to the same stopping rule
    t_start = max(1, glob["iterations"] // 2)
    nl3 = dict(nl, clock_period=np.float32(T))
    p = GlobalPlacer(nl3, lib, LoopConfig(die=die, bins=bins, beta=a.loop_beta, timing_start=t_start,
                                          record_every=15))
    t0 = time.perf_counter()
    hist = p.run(log=log("paper schedule"))
    torch.cuda.synchronize()
    sched = {"timing_start": t_start, "timing_every": 15, "beta": a.loop_beta, "iterations": p.it,
             "wall_s": round(time.perf_counter() - t0, 3), "history": rows(hist)}
    p.g.close()

    # the timing phase: both runs continue the converged run's optimiser state
    # (positions, previous point and gradient) with lambda frozen and without
    # momentum (the predicted step alone: past convergence the momentum
    # coefficient, near 1, carries the placement away)
    nl2 = dict(nl, x=ux.astype(np.float32), y=uy.astype(np.float32), clock_period=np.float32(T))
    runs = []
    for beta in (0.0, a.loop_beta):
        cfg = LoopConfig(die=die, bins=bins, beta=beta, lambda_fixed=lam, timing_start=snap["it"], max_iters=150,
                         record_every=15, stop_overflow=-1.0, momentum=False)
        p = GlobalPlacer(nl2, lib, cfg)
        p.resume(snap)
        start = p.metrics()
        t0 = time.perf_counter()
        hist = p.run(log=log(f"beta={beta}"))
        torch.cuda.synchronize()
        runs.append({"beta": beta, "iterations": p.it, "wall_s": round(time.perf_counter() - t0, 3),
                     "start": rows([start])[0], "history": rows(hist)})
        if beta > 0:
            # GPU time per iteration (HIP events on the default stream): plain
            # iterations, and a timing refresh (every 15th iteration)
            n_it = max(10, a.steps)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            p.cfg.timing_start = 1 << 30  # no refresh inside this segment
            torch.cuda.synchronize()
            e0.record()
            for _ in range(n_it):
                p.step()
            e1.record()
            torch.cuda.synchronize()
            it_ms = e0.elapsed_time(e1) / n_it
            e0.record()
            for _ in range(3):
                p.timing_refresh()
            e1.record()
            torch.cuda.synchronize()
            runs[-1]["ms_per_iteration"] = round(it_ms, 4)
            runs[-1]["ms_per_timing_refresh"] = round(e0.elapsed_time(e1) / 3, 4)
        p.g.close()
    out = {"table": "placement loop (Sec. IV): global placement, then the timing phase (Fig. 5 analogue)",
           "workload": f"{a.workload}: {N} cells, {int(nl['num_pins'])} pins, die {die:.0f} um, {bins}x{bins} "
                       f"bins, utilisation 0.5, clock {T:.1f} ps (5 % failing at the converged placement)",
           "global": glob,
           "columns": ["iteration", "hpwl_um", "overflow", "wns_ps", "tns_ps", "n_fail", "pairs"],
           "paper_schedule": sched,
           "timing_phase": runs}
    print(json.dumps(out))


def after_step_legs(g, nl, lib, x, y, gx, gy, pp, ep, dev):
    """The legs timed after the step on the same graph: the three pair
    distances, the smoothed TNS and its adjoint, the early (hold) analysis,
    rise / fall timing and incremental arrival updates; leaves the graph in
    the step's single-transition state."""
    import torch

    from paper_2503_11674_amd import netgen

    # the three pair distances of Sec. III-C on the step's pair set, forward
    # and backward, after the timed region (events on the current stream)
    pair_ms = {}
    one = torch.ones((), dtype=torch.float64, device=dev)
    for kind, name in ((0, "quadratic"), (1, "manhattan"), (2, "euclidean")):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        g.pair_loss_fwd(kind, x, y, out=pp)
        g.pair_loss_bwd(kind, x, y, one, gx, gy)
        e0.record()
        for _ in range(20):
            g.pair_loss_fwd(kind, x, y, out=pp)
            g.pair_loss_bwd(kind, x, y, one, gx, gy)
        e1.record()
        e1.synchronize()
        pair_ms[name] = round(e0.elapsed_time(e1) / 20, 4)
    # the smoothed TNS (gamma 10 ps) at the step's positions, forward and
    # adjoint
    st_v = torch.zeros((), dtype=torch.float64, device=dev)
    g.stns_fwd(x, y, 10.0, out=st_v)
    g.stns_bwd(one, gx, gy)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    ev[0].record()
    for _ in range(10):
        g.stns_fwd(x, y, 10.0, out=st_v)
    ev[1].record()
    for _ in range(10):
        g.stns_bwd(one, gx, gy)
    ev[2].record()
    ev[2].synchronize()
    stns = {"fwd_ms": round(ev[0].elapsed_time(ev[1]) / 10, 4), "bwd_ms": round(ev[1].elapsed_time(ev[2]) / 10, 4),
            "value": round(float(st_v), 1)}

    # the early (hold) analysis on the same update, outside the step: the hold
    # time at which 5 % of the D pins fail
    g.sta_update_early(0.0)
    at_e = g.early_export()["at"].cpu().numpy()
    hold = float(np.quantile(at_e[ep], 0.05))
    g.sta_update_early(hold)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        g.sta_update_early(hold)
    e1.record()
    e1.synchronize()
    whs, ths, n_hold = g.early_summary()
    early = {"ms": round(e0.elapsed_time(e1) / 10, 4), "hold_ps": round(hold, 1), "whs": round(whs, 1),
             "ths": round(ths, 1), "n_hold_fail": n_hold}

    # rise / fall timing on the same positions, outside the step: the update
    # and report_timing_endpoint(n_fail, 1) on it
    rf_lib = netgen.make_rf_library(lib)
    g.rf_setup(rf_lib)
    g.sta_update_rf(x, y)
    g.extract_paths_rf(n=-1)
    torch.cuda.synchronize()
    e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    e0.record()
    for _ in range(5):
        g.sta_update_rf(x, y)
    e1.record()
    for _ in range(5):
        g.extract_paths_rf(n=-1)
    e2.record()
    e2.synchronize()
    rf_w, rf_t, rf_n = g.rf_summary()
    rise_fall = {"update_ms": round(e0.elapsed_time(e1) / 5, 4), "extract_k1_ms": round(e1.elapsed_time(e2) / 5, 4),
                 "wns": round(rf_w, 1), "tns": round(rf_t, 1), "n_fail": rf_n, "paths": g.paths_count()[0]}
    g.sta_update(x, y)  # back to the single-transition state
    torch.cuda.synchronize()

    # incremental arrival updates against the full arrival pass: m cells move
    # (seeded jitter), and the positions alternate between the two placements
    # so that every call is a genuine update of m moved cells
    incremental = {}
    rng = np.random.default_rng(11)
    movable = np.nonzero(np.asarray(nl["cell_fixed"]) == 0)[0]
    for m in (100, 1000, 10_000, 100_000):
        if m > len(movable) // 2:
            break
        cells = np.sort(rng.choice(movable, m, replace=False)).astype(np.int32)
        ct = torch.tensor(cells, device=dev, dtype=torch.long)
        xn, yn = x.clone(), y.clone()
        xn[ct] += torch.tensor(rng.normal(0, 5.0, m).astype(np.float32), device=dev)
        yn[ct] += torch.tensor(rng.normal(0, 5.0, m).astype(np.float32), device=dev)
        cl = torch.tensor(cells, device=dev, dtype=torch.int32)
        pos = ((xn, yn), (x, y))
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        g.sta_update_arrivals(x, y)
        ev[0].record()
        for i in range(10):
            g.sta_update_arrivals(*pos[i & 1])
        ev[1].record()
        for i in range(10):
            g.sta_update_arrivals_incremental(*pos[i & 1], cl)
        ev[2].record()
        ev[2].synchronize()
        incremental[str(m)] = {"full_arrivals_ms": round(ev[0].elapsed_time(ev[1]) / 10, 4),
                               "incremental_ms": round(ev[1].elapsed_time(ev[2]) / 10, 4)}
    g.sta_update(x, y)
    torch.cuda.synchronize()

    return pair_ms, stns, early, rise_fall, incremental


def tree_net_leg(nl, lib, x, y, k, K, ep, tune, dev, steps=20):
    """The same step on a graph built with the spanning-tree net model
    (net_model 2: Elmore delays on each net's rectilinear minimum spanning
    tree), its clock again failing 5 % of the endpoints under this model, in
    the sweep form the step chose; outside the timed region."""
    import time

    import torch

    from paper_2503_11674_amd import netgen
    from paper_2503_11674_amd.tdp import TimingGraph

    g2 = TimingGraph(nl, dict(lib, net_model=2), max_paths=K, max_k=k)
    g2.sta_update(x, y)
    at = g2.export()["at"].cpu().numpy()
    g2.set_clock(netgen.clock_period_for_fail_fraction(at[ep], 0.05))
    if tune and "sweep_mode" in tune:
        g2.set_tuning(sweep_mode=tune["sweep_mode"])
    gx, gy = torch.zeros_like(x), torch.zeros_like(y)
    wl = torch.zeros((), dtype=torch.float64, device=dev)
    pp = torch.zeros((), dtype=torch.float64, device=dev)
    beta = torch.full((), BETA, dtype=torch.float64, device=dev)
    step = build_step(g2, x, y, k, K, gx, gy, wl, pp, beta)
    for _ in range(3):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    ms = 1000.0 * (time.perf_counter() - t0) / steps
    w, t, n = g2.summary()
    out = {"ms_per_step": round(ms, 4), "pins_per_s": round(g2.num_pins / (ms * 1e-3), 1), "wns": round(w, 1),
           "tns": round(t, 1), "n_fail": n}
    g2.close()
    torch.cuda.synchronize()
    return out


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {a.gpus}): independent designs or placement snapshots would "
              f"shard one per GPU, and that layout is not built.", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2503_11674_amd import netgen
    from paper_2503_11674_amd.tdp import TimingGraph, STAGES, TdpError

    if a.configs:
        return bench_configs(a)
    if a.workload == "C4":
        return bench_batch(a)
    if a.table1:
        return bench_table1(a)
    if a.loop:
        return bench_loop(a)
    cfg = netgen.CONFIGS[a.workload]
    t0 = time.time()
    nl = netgen.make_netlist(cfg)
    lib = dict(netgen.make_library(), net_model=a.net_model)
    print(f"[bench] generated {a.workload}: {nl['num_cells']} cells {nl['num_pins']} pins "
          f"({time.time() - t0:.1f}s)", file=sys.stderr, flush=True)
    dev = torch.device("cuda", 0)
    x = torch.tensor(nl["x"], device=dev)
    y = torch.tensor(nl["y"], device=dev)
    K = cfg.top_k_paths
    E = int(np.count_nonzero(nl["cell_is_ff"]))
    n_fail_target = E // 20
    k = max(1, K // max(1, n_fail_target))
    g = TimingGraph(nl, lib, max_paths=K, max_k=k)
    # clock period: floor(5 %) of the endpoints fail at the initial placement
    # (arrival times do not depend on the period)
    g.sta_update(x, y)
    at = g.export()["at"].cpu().numpy()
    ep = nl["cell_in_pins"][nl["cell_in_ptr"][np.nonzero(nl["cell_is_ff"])[0]]]
    T = netgen.clock_period_for_fail_fraction(at[ep], 0.05)
    g.set_clock(T)
    nl["clock_period"] = np.float32(T)
    info = (g.num_cells, g.num_pins, g.num_nets, g.depth, g.num_endpoints, g.num_startpoints, g.num_comb,
            g.num_sinks)

    gx = torch.zeros_like(x)
    gy = torch.zeros_like(y)
    wl = torch.zeros((), dtype=torch.float64, device=dev)
    pp = torch.zeros((), dtype=torch.float64, device=dev)
    beta = torch.full((), BETA, dtype=torch.float64, device=dev)

    step = build_step(g, x, y, k, K, gx, gy, wl, pp, beta, overlap=not a.serial)

    tune = None
    if a.sweep_mode >= 0:
        g.set_tuning(sweep_mode=a.sweep_mode)
        tune = {"forced_sweep_mode": a.sweep_mode}
    elif not a.no_tune:
        tune = g.autotune(x, y, n=-1, k=k, K=K, reps=3)
        # the library's autotuner times the update and extraction on one
        # stream; the step overlaps the required-time pass and WA with them,
        # so the sweep form is settled on the step itself among the
        # autotuner's pick and two that leave more of the GPU to the main
        # stream
        cands = [(tune["sweep_mode"], tune["flow_waves"], tune["flow_per_cu"]), (3, 1, 1), (0, 4, 1)]
        step_ms = {}
        for c in dict.fromkeys(cands):
            try:
                g.set_tuning(sweep_mode=c[0], flow_waves=c[1], flow_per_cu=c[2])
            except TdpError:  # no resident grids for this graph
                continue
            for _ in range(2):
                step()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(5):
                step()
            torch.cuda.synchronize()
            step_ms[c] = (time.perf_counter() - t0) / 5 * 1e3
        best = min(step_ms, key=step_ms.get)
        g.set_tuning(sweep_mode=best[0], flow_waves=best[1], flow_per_cu=best[2])
        tune = dict(tune, step_choice={"sweep_mode": best[0], "flow_waves": best[1], "flow_per_cu": best[2]},
                    step_ms={f"{c[0]}/{c[1]}/{c[2]}": round(v, 4) for c, v in step_ms.items()})
        tune["sweep_mode"] = best[0]
    if tune:
        print(f"[bench] autotuner: {tune}", file=sys.stderr, flush=True)
    for _ in range(a.warmup):
        step()
    torch.cuda.synchronize()
    # per-stage times from a profiled pass of the same step on one stream
    # (side-stream stages overlap others, so their event times would include
    # the other streams' work)
    serial = build_step(g, x, y, k, K, gx, gy, wl, pp, beta, overlap=False)
    g.profile(True)
    for _ in range(2):
        serial()
    prof_all = g.profile_read()
    g.profile(False)
    g.pairs_reset()
    for _ in range(a.warmup):
        step()
    torch.cuda.synchronize()
    wns, tns, nfail = g.summary()
    npaths, npins = g.paths_count()
    counts = {"paths": npaths, "path_pins": npins, "pairs": g.pairs_count(), "k": k,
              "nsel": nfail, "nslots": nfail * k, "touched": 0}
    counts["touched"] = 2 * counts["pairs"]
    side_k = g.max_k if g.max_k == 1 else 1 << (g.max_k - 1).bit_length()
    sb = algo_bytes(info, counts)
    ov = design_overhead(info, side_k)
    stages = {}
    for s_ in STAGES:
        ms, calls = prof_all.get(s_, (0.0, 0))
        if calls:
            per = ms / calls
            stages[s_] = {"ms": round(per, 4)}
            if sb.get(s_):
                stages[s_]["GBps"] = round(sb[s_] / (per * 1e-3) / 1e9, 1)
    # the dominant kernel: the longest stage on the step's critical path (the
    # calling stream; with overlap the required-time pass and WA run beside it)
    side = () if a.serial else ("backward", "wa")
    dom = max((s_ for s_ in stages if s_ not in side), key=lambda s_: stages[s_]["ms"]) if stages else None
    graph = None
    if a.graph:
        step()
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            step()
        torch.cuda.synchronize()
    print(f"[bench] T={T:.1f} ps wns={wns:.1f} tns={tns:.1f} n_fail={nfail} k={k}; timing {a.steps} steps",
          file=sys.stderr, flush=True)
    # timed region; in eager mode the dominant stage's events ride on its stream
    g.profile([dom] if (graph is None and dom) else False)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(a.steps):
        if graph is not None:
            graph.replay()
        else:
            step()
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    prof = g.profile_read() if graph is None else {}
    g.profile(False)
    ms_step = 1000.0 * t_total / a.steps
    if a.copy_calib > 0:
        # a copy of known size: its FETCH_SIZE / WRITE_SIZE counters scale the
        # hardware counters of the library's kernels to bytes
        src = torch.empty(a.copy_calib << 20, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()

    pair_ms, stns, early, rise_fall, incremental, tree_nets = {}, None, None, None, {}, None
    if not a.step_only:
        pair_ms, stns, early, rise_fall, incremental = after_step_legs(g, nl, lib, x, y, gx, gy, pp, ep, dev)
        if a.net_model == 0:
            tree_nets = tree_net_leg(nl, lib, x, y, k, K, ep, tune, dev)

    sta_ms = sum(stages[s]["ms"] for s in ("netpass", "forward", "endpoint", "backward") if s in stages)
    ext_ms = sum(stages[s]["ms"] for s in ("select", "search", "order", "walk") if s in stages)
    loss_ms = sum(stages[s]["ms"] for s in ("p2p_fwd", "p2p_bwd") if s in stages)
    pins = g.num_pins
    step_gb = sum(v for k_, v in sb.items() if k_ not in ("select", "search", "order", "walk")) / 1e9
    roof = None
    if dom and prof.get(dom, (0.0, 0))[1]:
        # the sweeps launch their kernel once per non-empty level in the
        # per-level form, once in the resident form; the stage time over its
        # launches is the average launch duration (with the gaps between the
        # launches of a per-level sweep)
        mode = (tune or {}).get("sweep_mode", (tune or {}).get("forced_sweep_mode", 0))
        flow_dom = (dom == "forward" and mode in (1, 2)) or (dom == "backward" and mode >= 1)
        per_level = dom in ("forward", "backward") and not flow_dom
        launches = g.depth + 1 if per_level else 1  # forward: D levels + the last level's lists
        names = STAGE_KERNEL.get(dom, (dom,))
        kname = names[1] if flow_dom and len(names) > 1 else names[0]
        per_launch = sb[dom] / launches
        ms_dom, calls_dom = prof[dom]
        dur = ms_dom / calls_dom * 1e-3 / launches
        ach = per_launch / dur / 1e9
        rp_us = rocprof_avg_us(kname)
        roof = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBPS, 4), "traffic": measured_traffic(kname),
                "kernel": kname, "stage": dom, "launches_per_step": launches,
                "avg_launch_us": round(dur * 1e6, 3), "algorithmic_bytes_per_launch": int(per_launch),
                "design_overhead_bytes_per_launch": int(ov.get(dom, 0) / launches),
                "rocprof_avg_us": rp_us,
                "frac_at_rocprof_duration": (round(per_launch / (rp_us * 1e-6) / 1e9 / HBM_PEAK_GBPS, 4)
                                             if rp_us else None)}
    out = {
        "metric": "timing-graph pins/s for STA+top-K extraction; p2p loss fwd+bwd GB/s",
        "value": round(pins / (ms_step * 1e-3), 1),
        "unit": "pins/s",
        "n_gpus": 1, "steps": a.steps, "warmup": a.warmup, "ms_per_step": round(ms_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{a.workload}: {nl['num_cells']} cells, {pins} pins, depth {g.depth}, "
                               f"{E} endpoints, (n_fail, k, K) = ({nfail}, {k}, {K}), clustered placement "
                               f"in {cfg.die:.0f} um die; step = STA + extraction + Eq. 9 pairs + WA + p2p "
                               f"fwd/bwd" + {0: "", 1: "; Elmore star nets",
                                             2: "; Elmore spanning-tree nets"}[a.net_model],
                   "parallelism": "none"},
        "sta_extract_pins_per_s": round(pins / ((sta_ms + ext_ms) * 1e-3), 1) if sta_ms else None,
        "p2p_fwd_bwd_GBps": round((sb["p2p_fwd"] + sb["p2p_bwd"]) / (loss_ms * 1e-3) / 1e9, 2) if loss_ms else None,
        "step_algorithmic_GB": round(step_gb, 4),
        "step_hbm_frac": round(step_gb / (ms_step * 1e-3) / HBM_PEAK_GBPS, 4),
        "stages": stages,
        "pair_losses_ms": pair_ms,
        "early_analysis": early,
        "rise_fall": rise_fall,
        "incremental_arrivals": incremental,
        "smoothed_tns": stns,
        "spanning_tree_nets": tree_nets,
        "roofline": roof,
        "graph_replay": bool(graph is not None),
        "streams": 1 if a.serial else 3,
        "tuning": tune,
        "timing": {"wns": wns, "tns": tns, "n_fail": nfail, "paths": npaths, "path_pins": npins,
                   "pairs": counts["pairs"]},
    }
    if not a.no_batch:
        # the batched workload on the same GPU, after the headline's timed
        # region: the union against per-instance launches
        b = measure_batch(a, 10, 2, a.no_tune)
        out["batched_C4"] = {key: b[key] for key in (
            "value", "ms_per_step", "batched_graph_ms", "batched_eager_ms", "per_instance_graph_ms",
            "per_instance_eager_ms", "speedup_vs_per_instance_eager", "speedup_vs_per_instance_graph", "paths",
            "n_fail")}
        out["batched_C4"]["workload"] = b["config"]["workload"]
        out["batched_C4"]["unit"] = "pins/s"
    if not a.no_cpu:
        out["cpu_baseline"] = cpu_baseline(nl, lib, k, K, pins)
    print(json.dumps(out))


def bench_configs(a):
    """The step on every workload: each in a child run of this script (its
    own autotuning and timing), summarised in one JSON line."""
    import subprocess
    rows = {}
    for w in ("C1", "C2", "C3", "C5", "C4"):
        cmd = [sys.executable, os.path.abspath(__file__), "--workload", w, "--steps", str(a.steps), "--warmup",
               str(a.warmup), "--no-batch"]
        if w in ("C5", "C4") or a.no_cpu:  # the default run carries the 2M-cell oracle rate
            cmd.append("--no-cpu")
        print(f"[bench] workload {w}", file=sys.stderr, flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True, timeout=1200)
        if r.returncode != 0:
            sys.stderr.write(r.stderr[-3000:])
            raise SystemExit(f"the run for {w} failed ({r.returncode})")
        d = json.loads(r.stdout.strip().splitlines()[-1])
        row = {"workload": d["config"]["workload"], "pins_per_s": d["value"], "ms_per_step": d["ms_per_step"]}
        for key in ("sta_extract_pins_per_s", "p2p_fwd_bwd_GBps", "step_hbm_frac", "batched_graph_ms",
                    "per_instance_eager_ms", "per_instance_graph_ms", "speedup_vs_per_instance_eager",
                    "speedup_vs_per_instance_graph"):
            if d.get(key) is not None:
                row[key] = d[key]
        if d.get("roofline"):
            row["roofline"] = {k: d["roofline"][k] for k in ("kernel", "achieved", "frac")}
        if d.get("cpu_baseline"):
            cb = d["cpu_baseline"]
            row["oracle_pins_per_s"] = cb["value"]
            row["oracle_sta_extract_pins_per_s"] = cb["sta_extract_pins_per_s"]
            row["oracle_cores"] = cb["cores"]
        rows[w] = row
        print(f"[bench] {w}: {json.dumps(row)}", file=sys.stderr, flush=True)
    print(json.dumps({"metric": "timing-graph pins/s for STA+top-K extraction; p2p loss fwd+bwd GB/s, per workload",
                      "unit": "pins/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup, "dtype": "f32",
                      "data": "synthetic", "per_config": rows}))


def bench_batch(a):
    """Batched timing update + extraction against per-instance launches."""
    print(json.dumps(measure_batch(a, a.steps, a.warmup, a.no_tune)))


def measure_batch(a, steps, warmup, no_tune):
    """The 40-instance batched workload: one union graph replayed from a
    captured HIP graph against the same instances one graph at a time."""
    import torch

    from paper_2503_11674_amd import netgen
    from paper_2503_11674_amd.tdp import TimingGraph

    t0 = time.time()
    nls = netgen.batch_workload()
    lib = netgen.make_library()
    k, K = 10, 5000
    dev = torch.device("cuda", 0)
    print(f"[bench] generated {len(nls)} instances, {sum(n['num_cells'] for n in nls)} cells "
          f"({time.time() - t0:.1f}s)", file=sys.stderr, flush=True)
    singles = []
    for nl in nls:
        x = torch.tensor(nl["x"], device=dev)
        y = torch.tensor(nl["y"], device=dev)
        g = TimingGraph(nl, lib, max_paths=K, max_k=k)
        # a snapshot keeps the clock period of the unperturbed placement
        g.sta_update(torch.tensor(nl.get("x_base", nl["x"]), device=dev),
                     torch.tensor(nl.get("y_base", nl["y"]), device=dev))
        at = g.export()["at"].cpu().numpy()
        ep = nl["cell_in_pins"][nl["cell_in_ptr"][np.nonzero(nl["cell_is_ff"])[0]]]
        T = netgen.clock_period_for_fail_fraction(at[ep], 0.05)
        g.set_clock(T)
        nl["clock_period"] = np.float32(T)
        singles.append((g, x, y))
    gb = TimingGraph(nls, lib, max_paths=K, max_k=k)
    xb = torch.cat([s[1] for s in singles])
    yb = torch.cat([s[2] for s in singles])
    pins = gb.num_pins
    print(f"[bench] union graph: {gb.num_cells} cells, {pins} pins", file=sys.stderr, flush=True)
    tune_b = None if no_tune else gb.autotune(xb, yb, n=-1, k=k, K=K, reps=3)
    tune_s = None if no_tune else [g.autotune(x, y, n=-1, k=k, K=K, reps=2) for g, x, y in singles]

    def batched():
        gb.sta_update(xb, yb)
        gb.extract_paths(n=-1, k=k, K=K)

    def per_instance():
        for g, x, y in singles:
            g.sta_update(x, y)
            g.extract_paths(n=-1, k=k, K=K)

    def timed(fn, steps):
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / steps

    def captured(fn):
        fn()
        torch.cuda.synchronize()
        gr = torch.cuda.CUDAGraph()
        with torch.cuda.graph(gr):
            fn()
        torch.cuda.synchronize()
        return gr

    for _ in range(warmup):
        batched()
        per_instance()
    gr_b = captured(batched)
    gr_s = captured(per_instance)
    print(f"[bench] timing {steps} steps of each form", file=sys.stderr, flush=True)
    t_b = timed(gr_b.replay, steps)
    t_s_graph = timed(gr_s.replay, steps)
    t_s_eager = timed(per_instance, steps)
    t_b_eager = timed(batched, steps)
    # the union's selections are the instances' own: same path counts
    nb = gb.paths_count()
    ns = [g.paths_count() for g, _, _ in singles]
    wb, _, fb = gb.batch_summary()
    out = {
        "metric": "timing-graph pins/s for STA+top-K extraction; p2p loss fwd+bwd GB/s",
        "value": round(pins / t_b, 1), "unit": "pins/s",
        "n_gpus": 1, "steps": steps, "warmup": warmup, "ms_per_step": round(1000 * t_b, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"C4: {len(nls)} instances (32 netlists of 10k-300k cells, depth 20-80, and 8 "
                               f"jittered snapshots of a 500k-cell netlist), {gb.num_cells} cells, {pins} pins; "
                               f"step = timing update + extraction (n_fail, k={k}, K={K} per instance)",
                   "parallelism": "none"},
        "batched_graph_ms": round(1000 * t_b, 4),
        "batched_eager_ms": round(1000 * t_b_eager, 4),
        "per_instance_graph_ms": round(1000 * t_s_graph, 4),
        "per_instance_eager_ms": round(1000 * t_s_eager, 4),
        "speedup_vs_per_instance_eager": round(t_s_eager / t_b, 3),
        "speedup_vs_per_instance_graph": round(t_s_graph / t_b, 3),
        "paths": {"batched": nb[0], "per_instance": int(sum(n[0] for n in ns))},
        "n_fail": {"batched": int(fb.sum()), "min_instance": int(fb.min())},
        "tuning": {"batched": tune_b, "per_instance": tune_s[:3] if tune_s else None},
    }
    gr_b = gr_s = None
    for g, _, _ in singles:
        g.close()
    gb.close()
    return out


def host_cpu() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(nl, lib, k, K, pins, runs=3):
    """The FP64 CPU oracle, single threaded, on the same workload: one step
    (STA, extraction, pairs, WA and p2p forward+backward), once to warm up,
    then the median of `runs` timed steps."""
    from oracle import ref

    def one():
        t0 = time.perf_counter()
        st = ref.sta(nl, lib)
        pa = ref.extract(nl, lib, st, n=-1, k=k, K=K)
        t1 = time.perf_counter()
        ps = ref.PairState(nl["num_pins"])
        ref.pairs_update(ps, pa, st["wns"])
        s, w = ps.pairs()
        ref.wa(nl, WA_GAMMA)
        ref.p2p(nl, s, w)
        t2 = time.perf_counter()
        return t2 - t0, t1 - t0

    one()
    times = sorted(one() for _ in range(runs))
    t_step, t_sta = times[len(times) // 2]
    return {"value": round(pins / t_step, 1), "unit": "pins/s", "cores": 1, "kind": "oracle",
            "sample": f"one full step of the same workload (STA + extraction + pairs + WA + p2p fwd/bwd), FP64; "
                      f"one warm-up, median of {runs}",
            "seconds": round(t_step, 3), "seconds_all": [round(t[0], 3) for t in times],
            "sta_extract_pins_per_s": round(pins / t_sta, 1),
            "host_cpu": host_cpu(), "host_threads_available": os.cpu_count()}


if __name__ == "__main__":
    main()
