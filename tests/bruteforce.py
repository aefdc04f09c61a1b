"""Brute-force path enumeration on tiny timing graphs (test helper).

Independent of the oracle's sweeps: it lists every start-to-end path by
depth-first search and takes maxima / minima / sorted orders over whole paths.
It needs the per-arc delays (net delay into each sink pin, cell-arc delay from
each combinational input pin) and the start-point arrivals, which the tests pin
separately (hand chains, lookup-table identities).
"""
import numpy as np


class Graph:
    def __init__(self, nl):
        P = int(nl["num_pins"])
        self.P = P
        self.role = ["port"] * P
        self.driver = [-1] * P
        self.sinks = {}
        self.cell_inputs = {}
        pin_cell = nl["pin_cell"]
        for c in range(int(nl["num_cells"])):
            ins = list(nl["cell_in_pins"][nl["cell_in_ptr"][c]:nl["cell_in_ptr"][c + 1]])
            ff = bool(nl["cell_is_ff"][c])
            for p in ins:
                self.role[p] = "ffd" if ff else "cin"
            o = int(nl["cell_out_pin"][c])
            self.role[o] = "ffq" if ff else "cout"
            self.cell_inputs[o] = [int(p) for p in ins]
        for n in range(int(nl["num_nets"])):
            pins = nl["net_pins"][nl["net_ptr"][n]:nl["net_ptr"][n + 1]]
            d = int(pins[0])
            self.sinks[d] = [int(t) for t in pins[1:]]
            for t in pins[1:]:
                self.driver[int(t)] = d
        self.pin_cell = pin_cell

    def preds(self, v):
        r = self.role[v]
        if r in ("cin", "ffd"):
            return [self.driver[v]] if self.driver[v] >= 0 else []
        if r == "cout":
            return self.cell_inputs[v]
        return []

    def succs(self, v):
        r = self.role[v]
        if r in ("port", "cout", "ffq"):
            return self.sinks.get(v, [])
        if r == "cin":
            return [int(self.cell_out_of(v))]
        return []

    def cell_out_of(self, v):
        for o, ins in self.cell_inputs.items():
            if v in ins:
                return o
        raise KeyError(v)

    def is_start(self, v):
        return self.role[v] in ("port", "ffq")

    def is_path(self, pl):
        """pl is a start-point-to-endpoint chain of timing arcs."""
        if not pl or not self.is_start(pl[0]) or self.role[pl[-1]] != "ffd":
            return False
        return all(a in self.preds(b) for a, b in zip(pl[:-1], pl[1:]))

    def paths_to(self, v):
        """All start -> v paths, as pin lists in start -> v order."""
        if self.is_start(v):
            return [[v]]
        out = []
        for u in self.preds(v):
            for p in self.paths_to(u):
                out.append(p + [v])
        return out

    def paths_from(self, v):
        """All v -> endpoint paths (v first)."""
        if self.role[v] == "ffd":
            return [[v]]
        out = []
        for w in self.succs(v):
            for p in self.paths_from(w):
                out.append([v] + p)
        return out

    def arc_delay(self, u, v, dnet, darc):
        if self.role[v] in ("cin", "ffd"):
            return dnet[v]
        return darc[u]

    def path_delay(self, path, dnet, darc):
        return sum(self.arc_delay(path[i], path[i + 1], dnet, darc) for i in range(len(path) - 1))


def brute_sta(nl, st):
    """AT(v) = max over start->v paths; RAT(v) = min over v->endpoint paths."""
    g = Graph(nl)
    dnet, darc = st["dnet"], st["darc"]
    T = float(st["clock_period"]) - float(nl["setup"])
    at = np.full(g.P, -np.inf)
    rat = np.full(g.P, np.inf)
    for v in range(g.P):
        ps = g.paths_to(v)
        if ps:
            at[v] = max(st["at"][p[0]] + g.path_delay(p, dnet, darc) for p in ps)
        qs = g.paths_from(v)
        if qs:
            rat[v] = min(T - g.path_delay(q, dnet, darc) for q in qs)
    return at, rat


def brute_endpoint_paths(nl, st, e):
    """Every path into endpoint e with its slack, sorted by slack."""
    g = Graph(nl)
    T = float(st["clock_period"]) - float(nl["setup"])
    out = []
    for p in g.paths_to(e):
        arr = st["at"][p[0]] + g.path_delay(p, st["dnet"], st["darc"])
        out.append((T - arr, p))
    out.sort(key=lambda t: t[0])
    return out
