"""Small hand-built netlists and libraries for exact tests.

Netlists use the same array layout as ``paper_2503_11674_amd.netgen``: pins are
numbered cell by cell (input pins in arc order, then the output pin), ports
last; every net lists its driver first.
"""
import numpy as np

from paper_2503_11674_amd import netgen


def build(cells, n_ports, nets, x, y, off_x=None, off_y=None, port_xy=None,
          clock_period=0.0, setup=0.0, input_slew=10.0, clock_slew=10.0, fixed=None):
    """cells: list of (type, n_inputs); type 7 is a flip-flop (1 input = D).
    nets: list of (driver_pin, [sink pins]).  Returns a netlist dict and the
    pin ids as {"in": [[...] per cell], "out": [...], "port": [...]}."""
    N = len(cells)
    pin = 0
    ins, outs = [], []
    pin_cell = []
    for c, (ty, nin) in enumerate(cells):
        ins.append(list(range(pin, pin + nin)))
        pin_cell += [c] * (nin + 1)
        outs.append(pin + nin)
        pin += nin + 1
    ports = list(range(pin, pin + n_ports))
    pin_cell += [-1] * n_ports
    P = pin + n_ports
    ox = np.zeros(P, np.float32) if off_x is None else np.asarray(off_x, np.float32)
    oy = np.zeros(P, np.float32) if off_y is None else np.asarray(off_y, np.float32)
    if port_xy is not None:
        for p, (px, py) in zip(ports, port_xy):
            ox[p], oy[p] = px, py
    net_ptr = [0]
    net_pins = []
    for d, sinks in nets:
        net_pins += [d] + list(sinks)
        net_ptr.append(len(net_pins))
    cell_in_ptr = np.concatenate([[0], np.cumsum([nin for _, nin in cells])])
    nl = {
        "name": "hand",
        "num_cells": N, "num_pins": P, "num_nets": len(nets),
        "pin_cell": np.asarray(pin_cell, np.int32),
        "pin_off_x": ox, "pin_off_y": oy,
        "net_ptr": np.asarray(net_ptr, np.int32), "net_pins": np.asarray(net_pins, np.int32),
        "cell_type": np.asarray([ty for ty, _ in cells], np.int32),
        "cell_in_ptr": np.asarray(cell_in_ptr, np.int32),
        "cell_in_pins": np.asarray([p for l in ins for p in l], np.int32),
        "cell_out_pin": np.asarray(outs, np.int32),
        "cell_is_ff": np.asarray([1 if ty == netgen.FF_TYPE else 0 for ty, _ in cells], np.uint8),
        "cell_fixed": np.zeros(N, np.uint8) if fixed is None else np.asarray(fixed, np.uint8),
        "x": np.asarray(x, np.float32), "y": np.asarray(y, np.float32),
        "depth": 8,
        "clock_period": np.float32(clock_period), "setup": np.float32(setup),
        "input_slew": np.float32(input_slew), "clock_slew": np.float32(clock_slew),
    }
    return nl, {"in": ins, "out": outs, "port": ports}


def dyadic_library():
    """A library whose lookups at grid points and whose wires give exact
    binary fractions:
      delay(type t, slew s, load l) = (4 + t) + s/4 + l/64   (comb types 0..6)
      clock-to-Q (type 7)           = 20 + s/2 + l/32
      output slew                   = 10 (every type)
      pin capacitance               = 2 fF (every type)
      r = 1/16 ohm/um, c = 1/4 fF/um, scale 1  ->  net delay L^2 / 64,
      load = sum over sinks of (2 + L/4).
    The tables are affine in (slew, load), so bilinear interpolation
    reproduces them exactly between grid points as well."""
    sa = netgen.SLEW_AXIS.astype(np.float64)
    la = netgen.LOAD_AXIS.astype(np.float64)
    delay = np.zeros((8, 7, 7))
    for t in range(7):
        delay[t] = (4 + t) + sa[:, None] / 4 + la[None, :] / 64
    delay[7] = 20 + sa[:, None] / 2 + la[None, :] / 32
    return {
        "num_types": 8,
        "slew_axis": np.tile(netgen.SLEW_AXIS, (8, 1)).astype(np.float32),
        "load_axis": np.tile(netgen.LOAD_AXIS, (8, 1)).astype(np.float32),
        "delay_lut": delay.astype(np.float32),
        "slew_lut": np.full((8, 7, 7), 10.0, np.float32),
        "pin_cap": np.full(8, 2.0, np.float32),
        "r_per_um": np.float32(1.0 / 16),
        "c_per_um": np.float32(0.25),
        "delay_scale": np.float32(1.0),
    }


def chain_netlist():
    """PI port -> BUF1 -> BUF2 -> FF.D, every wire 24 um long, zero pin
    offsets.  Cells: 0 = BUF1 (type 0), 1 = BUF2 (type 0), 2 = FF (type 7).
    Clock period 32 ps, setup 0."""
    cells = [(0, 1), (0, 1), (7, 1)]
    # pins: BUF1 in 0 out 1; BUF2 in 2 out 3; FF D 4 Q 5; port 6
    nets = [(6, [0]), (1, [2]), (3, [4]), (5, [])]
    x = [24.0, 48.0, 72.0]
    y = [0.0, 0.0, 0.0]
    return build(cells, 1, nets, x, y, port_xy=[(0.0, 0.0)], clock_period=32.0)


def diamond_netlist():
    """Two paths into a 2-input cell:
        port A (0,0) -> BUF (cell 0 at (24,0)) -> AND.in0
        port A       -> AND.in1 directly (48 um)
        AND (cell 1, type 2, at (48,0)) -> FF (cell 2 at (72,0)).D
    Pins: BUF in 0 out 1; AND in0 2 in1 3 out 4; FF D 5 Q 6; port 7.
    Clock period 50 ps, setup 0."""
    cells = [(0, 1), (2, 2), (7, 1)]
    nets = [(7, [0, 3]), (1, [2]), (4, [5]), (6, [])]
    x = [24.0, 48.0, 72.0]
    y = [0.0, 0.0, 0.0]
    return build(cells, 1, nets, x, y, port_xy=[(0.0, 0.0)], clock_period=50.0)


def invalid_chain(mutation: str):
    """The hand chain with one fault the build must reject (TDP_E_INVALID):
    sink_in_two_nets, driver_is_input, dangling_input, ff_two_inputs,
    bad_type, pin_out_of_range."""
    nl, _ = chain_netlist()
    nl = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in nl.items()}
    if mutation == "sink_in_two_nets":
        nl["net_pins"] = np.array([6, 0, 1, 2, 0, 3, 4, 5], np.int32)
        nl["net_ptr"] = np.array([0, 2, 5, 7, 8], np.int32)
    elif mutation == "driver_is_input":
        nl["net_pins"][0] = 0
    elif mutation == "dangling_input":
        nl["net_pins"] = np.array([6, 1, 2, 3, 4, 5], np.int32)
        nl["net_ptr"] = np.array([0, 1, 3, 5, 6], np.int32)
    elif mutation == "ff_two_inputs":
        cells = [(0, 1), (7, 2)]
        nets = [(5, [0]), (1, [2, 3]), (4, [])]
        nl, _ = build(cells, 1, nets, [1.0, 2.0], [0.0, 0.0])
    elif mutation == "bad_type":
        nl["cell_type"][0] = 99
    elif mutation == "pin_out_of_range":
        nl["net_pins"][1] = 1000
    else:
        raise KeyError(mutation)
    return nl
