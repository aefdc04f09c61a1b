/*
 * tdp.h - C ABI of the MI355X timing-driven-placement hot path.
 *
 * Shi et al., "Timing-Driven Global Placement by Efficient Critical Path
 * Extraction" (arXiv 2503.11674).  The library runs, on one GPU:
 *   1. static timing analysis on the timing DAG (Sec. II-B, Eq. 2-4): RC net
 *      delays from pin positions (Sec. III-C, Eq. 7), slew x load table cell
 *      arcs, arrival times forward, required times backward, slack per pin,
 *      WNS / TNS over the violated endpoints;
 *   2. report_timing_endpoint(n, k) (Sec. III-B, Table I): the n most
 *      critical endpoints and the k worst paths at each;
 *   3. the maintained pin-pair set P with the weight update of Eq. 9
 *      (Sec. III-D), and the pin-to-pin loss PP = sum w * Q (Eqs. 8, 10) with
 *      its gradient on cell positions;
 * plus a log-sum-exp smoothed TNS with its adjoint, weighted-average
 * wirelength (the WL term of Eq. 1), the Manhattan and Euclidean pair losses
 * that Sec. III-C compares PP with, report_timing(K) (the K worst paths of the
 * design, Table I), a batched form over many designs, and a fuller timing
 * model around the paper's (an Elmore net model with degraded transitions,
 * the early / hold half of an early/late timer); and, for the placement loop
 * around all of it (Sec. IV), a bin-density term with its gradient and a
 * Nesterov step.
 *
 * Conventions (every entry point):
 *  - Return a tdp_status; nothing throws across the ABI.  A failed call leaves
 *    the graph as it was; tdp_last_error() gives a message.
 *  - "host" pointers are read during the call only; the caller keeps them.
 *    "device" pointers are HIP device memory on the graph's device; the
 *    caller owns them.  Device outputs are written asynchronously on the
 *    given stream (NULL = the default stream); calls that return values to
 *    the host synchronise that stream and say so.
 *  - Units: positions um, times ps, capacitances fF.
 *  - Pins and cells are numbered by the caller ("external" numbering).  Cell
 *    positions x[], y[] are float arrays indexed by external cell id.
 *  - After the first call of each kind (which may allocate), the update,
 *    extraction, pair and loss calls neither allocate nor synchronise, so a
 *    caller can capture them in a hipGraph.
 */
#ifndef TDP_H_
#define TDP_H_

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tdp_graph_s *tdp_graph;

typedef enum {
  TDP_OK = 0,
  TDP_E_INVALID = 1,     /* malformed netlist / library / argument */
  TDP_E_CYCLE = 2,       /* the timing graph is not acyclic */
  TDP_E_NOMEM = 3,       /* device or host allocation failed */
  TDP_E_DEVICE = 4,      /* a HIP call failed */
  TDP_E_CAPACITY = 5,    /* request exceeds a capacity fixed at build */
  TDP_E_STATE = 6,       /* call out of order (e.g. extract before update) */
  TDP_E_UNSUPPORTED = 7
} tdp_status;

typedef enum { TDP_F32 = 0, TDP_F64 = 1 } tdp_precision;

/* Timing graph (host arrays, read during build only).
 *  pin_cell[num_pins]      owning cell, or -1 for a primary-input port
 *  pin_off_x/y[num_pins]   pin offset from its cell's position; for a port,
 *                          its absolute position
 *  net_ptr[num_nets+1], net_pins[...]   CSR; each net lists its driver first,
 *                          then its sinks.  Every port and every cell output
 *                          drives exactly one net (which may have no sink);
 *                          every input pin is a sink of exactly one net.
 *  cell_type[num_cells]    index into the library
 *  cell_in_ptr/cell_in_pins  CSR of each cell's input pins, in arc order;
 *                          a flip-flop has exactly one (its D pin)
 *  cell_out_pin[num_cells] output pin (Q for a flip-flop)
 *  cell_is_ff[num_cells]   1: D is a timing endpoint, Q a timing startpoint
 *  cell_fixed[num_cells]   1: no gradient is written for the cell (may be NULL)
 *  clock_period_ps, setup_ps  required time at a D pin = period - setup
 *  input_slew_ps           transition at the primary inputs
 *  clock_slew_ps           clock transition used for clock-to-Q arcs (ideal
 *                          clock: every D/Q pin sees the edge at time 0) */
typedef struct {
  int32_t num_cells, num_pins, num_nets;
  const int32_t *pin_cell;
  const float *pin_off_x, *pin_off_y;
  const int32_t *net_ptr, *net_pins;
  const int32_t *cell_type;
  const int32_t *cell_in_ptr, *cell_in_pins;
  const int32_t *cell_out_pin;
  const uint8_t *cell_is_ff, *cell_fixed;
  float clock_period_ps, setup_ps, input_slew_ps, clock_slew_ps;
} tdp_netlist;

/* Cell library (host arrays, copied at build); 1..256 cell types.
 *  slew_axis[num_types][n_slew], load_axis[num_types][n_load]: strictly
 *    increasing breakpoints; lookups clamp to the axis range and interpolate
 *    bilinearly between breakpoints.
 *  delay_lut, slew_lut [num_types][n_slew][n_load]: arc delay and output
 *    transition (slew_lut may equal delay_lut).
 *  pin_cap[num_types]: input-pin capacitance.
 *  In models 0 and 1 every sink sits on a wire of its own from the driver,
 *  of length L, the Manhattan driver-to-sink distance, with resistance
 *  r_per_um * L and capacitance c_per_um * L (Eq. 7: R and C both linear in
 *  length).  A driver's load = sum over its sinks of (pin_cap + c_per_um * L).
 *  net_model selects the net delay into a sink and the transition it sees:
 *    0  lumped (Eq. 7): delay_scale * r_per_um * c_per_um * L^2; the sink
 *       sees its driver's transition.
 *    1  Elmore delay of that star RC net: delay_scale * r_per_um * L *
 *       (c_per_um * L / 2 + pin_cap of the sink); the sink's transition is
 *       the driver's degraded by the wire (PERI, Kashyap et al., TCAD 2004):
 *       sqrt(s_drv^2 + (ln 9 * delay)^2).
 *    2  Elmore delay of an RC tree on the net's rectilinear minimum spanning
 *       tree (Prim's algorithm from the driver on single-precision Manhattan
 *       distances; ties to the pin first in the net's list, and a pin keeps
 *       the first tree pin that reached it).  Each edge is a wire of its
 *       Manhattan length L (r_per_um * L, c_per_um * L); the delay to a pin
 *       is delay_scale times the sum, over the edges (parent, u) on its path,
 *       of r_per_um * L * (c_per_um * L / 2 + capacitance at and below u);
 *       the driver's load is the sum of the sink pin capacitances plus
 *       c_per_um times the tree's length; transitions degrade as in model 1.
 *       The smoothed TNS differentiates the delays through the wire lengths
 *       of the tree at the given positions.  Sec. III-C's wires as the RC
 *       trees of the paper's timer (Sec. II-B); the spanning tree stands in
 *       for a Steiner tree.
 *  Any other value fails the build with TDP_E_INVALID. */
typedef struct {
  int32_t num_types, n_slew, n_load;
  const float *slew_axis, *load_axis;
  const float *delay_lut, *slew_lut;
  const float *pin_cap;
  float r_per_um, c_per_um, delay_scale;
  int32_t net_model;
} tdp_library;

/* Extracted paths (device views owned by the graph; valid until the next
 * tdp_extract_paths on the same graph).  Path i has pins
 * path_pins[path_ptr[i] .. path_ptr[i+1]) in start -> endpoint order, as
 * external pin ids: the start pin (port or Q), then for each combinational
 * cell on the path its input pin and output pin, then the D pin.
 * path_slack is float (TDP_F32) or double (TDP_F64).  *d_num_paths is a
 * device int32 (tdp_paths_count() reads it to the host). */
typedef struct {
  int32_t max_paths;
  const int32_t *d_num_paths;
  const int32_t *path_ptr;       /* [max_paths + 1] */
  const int32_t *path_pins;      /* [max_paths * (2 * depth + 2)] */
  const int32_t *path_ep;        /* [max_paths] endpoint (D) pin */
  const int32_t *path_rank;      /* [max_paths] 0 = worst path at its endpoint */
  const void *path_slack;        /* [max_paths] */
} tdp_paths;

/* ---------------------------------------------------------------- build */
/* The timing graph of Sec. II-B (pins as nodes, net and cell arcs as edges,
 * flip-flop Q pins and primary inputs as start points, D pins as endpoints):
 * validate and levelise it, renumber it for the device and upload it.  max_paths bounds n*k of any later extraction, max_k bounds k
 * (1..32; max_k > 1 makes every update also keep, per cell, the max_k
 * cheapest deviations along its critical fan-in chain).  Errors:
 * TDP_E_INVALID (index out of range, a pin in zero or two nets, a port that
 * is not a driver, a combinational cell without inputs, a flip-flop without
 * exactly one input, bad axes), TDP_E_CYCLE (combinational loop). */
tdp_status tdp_sta_build(const tdp_netlist *netlist, const tdp_library *lib, tdp_precision prec,
                         int32_t max_paths, int32_t max_k, int device, tdp_graph *out);

/* Batched form (not in the paper: many designs or placement snapshots timed
 * together): the graphs of `count` netlists become one disjoint union
 * (instance-major numbering, external ids offset by the preceding instances'
 * pin and cell counts); every later call runs all instances in the same
 * launches.  Per-instance quantities (clock period and setup, WNS/TNS,
 * endpoint selection, K) are kept per instance; input and clock slews must
 * agree (TDP_E_INVALID otherwise).  Single precision only.  max_paths_each
 * bounds n*k per instance. */
tdp_status tdp_batch_build(const tdp_netlist *const *netlists, int32_t count, const tdp_library *lib,
                           tdp_precision prec, int32_t max_paths_each, int32_t max_k, int device,
                           tdp_graph *out);
/* Host copies of the union's offsets: pin_base[count+1], cell_base[count+1]. */
tdp_status tdp_batch_offsets(tdp_graph, int32_t *pin_base, int32_t *cell_base);

void tdp_destroy(tdp_graph);

/* Change the required time at every D pin (period - setup, the endpoint
 * required time of Eq. 2), in every instance of a batched graph.
 * Synchronous (a small host-to-device copy). */
tdp_status tdp_sta_set_clock(tdp_graph, float clock_period_ps, float setup_ps);

/* ------------------------------------------------------------------ STA */
/* Full timing update from cell positions (device float [num_cells] each),
 * Sec. II-B: net delays (Eq. 7) and loads, arrival times and transitions
 * forward by level, endpoint slacks and WNS / TNS / violated-endpoint count
 * (Eqs. 3-4), required times (Eq. 2) and slack backward.  Asynchronous. */
tdp_status tdp_sta_update(tdp_graph, const float *d_x, const float *d_y, hipStream_t);
/* The same update in two passes, for callers that overlap work on several
 * streams:
 *  tdp_sta_update_arrivals: net delays, loads, arrival times, transitions,
 *    critical inputs, deviation lists, endpoint slacks, WNS / TNS (all that
 *    extraction, pairs and the losses read);
 *  tdp_sta_update_required: required times (Eq. 2) from the arrival pass's
 *    delays; slack = required - arrival.
 * The required pass may run on another stream concurrently with later
 * extraction, pair and loss calls (they do not read required times), but it
 * must be ordered after its arrival pass and before the next arrival pass
 * and before any export or summary (event waits between the streams). */
tdp_status tdp_sta_update_arrivals(tdp_graph, const float *d_x, const float *d_y, hipStream_t);
tdp_status tdp_sta_update_required(tdp_graph, hipStream_t);
/* Incremental arrival pass (Sec. II-B's forward propagation, re-timing only
 * what moved cells change): d_cells (device int32 [n_cells], external cell
 * ids in any order, repeats allowed) lists every cell whose position differs
 * from the previous update's.  Only the nets of those cells are re-timed;
 * then, level by level, a 64-lane chunk of cells is re-timed only if the net
 * pass changed one of its inputs' delays or its load, or a driver of one of
 * its inputs changed arrival or transition; its deviation lists, hop records
 * and chain depths only if it was re-timed or such a driver's changed.  The
 * results equal tdp_sta_update_arrivals at the new positions bitwise; as
 * after that call, tdp_sta_update_required must follow before required
 * times, slacks or summaries are read.  The sweep stays one launch per level
 * whatever moved, so this pays only where the moved cells' fan-out cones
 * touch few chunks; on deep random logic a full update can be faster.  The
 * first call allocates its marks and maps.  Ids outside [0, num_cells) are
 * skipped and make tdp_sta_summary return TDP_E_DEVICE.  TDP_E_STATE without
 * a previous update, TDP_E_UNSUPPORTED for a graph with a net wider than 63
 * sinks. */
tdp_status tdp_sta_update_arrivals_incremental(tdp_graph, const float *d_x, const float *d_y, const int32_t *d_cells,
                                               int32_t n_cells, hipStream_t);

/* WNS and TNS (Eqs. 3-4; both 0 without violations) and the number of
 * violated endpoints of the last update.  Synchronises the stream.  For a
 * batched graph this is the union's; see tdp_batch_summary.  TDP_E_INVALID
 * when a cell position given to the last arrival pass was NaN or infinite
 * (the timing results of that pass are then meaningless). */
tdp_status tdp_sta_summary(tdp_graph, double *wns, double *tns, int32_t *n_fail, hipStream_t);
tdp_status tdp_batch_summary(tdp_graph, double *wns, double *tns, int32_t *n_fail, hipStream_t);

/* Per-pin results of the last update (Sec. II-B: arrival, required time
 * and slack = required - arrival per pin) in external pin order, as double
 * device arrays [num_pins] (any pointer may be NULL):
 *   at, rat, slack, slew (at a sink pin, the transition its cell arc or
 *   setup check sees: degraded by the wire under net model 1);
 *   dnet (net delay into a sink pin, 0 elsewhere),
 *   load (at a driver pin, 0 elsewhere), darc (cell-arc delay from a
 *   combinational input pin to its output, 0 elsewhere).
 * Unconstrained pins (no endpoint downstream) have rat = slack = +inf. */
tdp_status tdp_sta_export(tdp_graph, double *d_at, double *d_rat, double *d_slack, double *d_slew,
                          double *d_dnet, double *d_load, double *d_darc, hipStream_t);
/* Arc index of the input that sets each combinational cell's arrival (the
 * maximum of Sec. II-B's forward propagation; lowest index on ties), -1 for
 * flip-flops; int32 device [num_cells]. */
tdp_status tdp_sta_export_crit(tdp_graph, int32_t *d_crit, hipStream_t);
/* Zero-copy views of the last update's arrival and required times (Sec.
 * II-B), in the graph's precision (float for TDP_F32, double for TDP_F64)
 * and in the device's pin order, with the map from external pin id to that
 * order: at[pin_index[p]] is pin p's arrival, rat[pin_index[p]] its
 * required time (slack = rat - at; it is not stored, tdp_sta_export forms
 * it).  All three are device pointers owned by the graph: read them on the
 * update's stream, or after it; they hold the next update's values once it
 * runs and are freed by tdp_destroy.  TDP_E_STATE before the first update. */
tdp_status tdp_sta_views(tdp_graph, const void **d_at, const void **d_rat, const int32_t **d_pin_index);

/* ------------------------------------------------------- rise / fall */
/* Rise / fall timing: a fuller model around the paper's (its timer, Sec.
 * II-B / III-B, times both transitions of every pin; the paper fixes neither
 * library nor this detail).  Every pin carries a rise and a fall.  A cell
 * type's arcs are positive unate (unate 0: input rise -> output rise, fall ->
 * fall), negative unate (1: rise -> fall, fall -> rise) or non-unate (2:
 * either -> either).  The library's delay_lut / slew_lut give the output
 * rise, these tables ([num_types][n_slew][n_load], host, copied) the output
 * fall; a flip-flop's Q rises and falls by them at the clock slew.  A net
 * passes a transition with the same delay either way.  Output transition x:
 * arrival = max over (input j, input transition y that causes x) of arrival
 * + table delay at y's transition, critical = the first (j, y) attaining it
 * (j ascending, rise first), transition = the maximum of the table
 * transitions.  An endpoint's slack is the smaller of its two; WNS / TNS /
 * count as Eqs. 3-4 over endpoints.  Required times per transition: a D pin's
 * is period - setup; an input's the minimum over the outputs it causes of
 * (required - arc delay); a driver's the minimum over its sinks. */
typedef struct {
  const float *delay_fall, *slew_fall;
  const int32_t *unate;  /* [num_types] */
} tdp_rf_tables;
/* Set (or replace) the tables and allocate the rise / fall arrays
 * (synchronous).  TDP_E_UNSUPPORTED on a batched graph, TDP_E_INVALID on a
 * bad unateness or a non-finite entry. */
tdp_status tdp_rf_setup(tdp_graph, const tdp_rf_tables *tables);
/* Rise / fall update from cell positions (device float [num_cells] each):
 * net delays and loads as tdp_sta_update, arrivals, transitions, critical
 * inputs, endpoint slacks, WNS / TNS, required times.  It replaces the graph's
 * endpoint slacks and summary, so the single-transition results read as not
 * updated (TDP_E_STATE) until the next tdp_sta_update.  Asynchronous;
 * TDP_E_STATE before tdp_rf_setup. */
tdp_status tdp_sta_update_rf(tdp_graph, const float *d_x, const float *d_y, hipStream_t);
/* WNS, TNS and violated count of the last rise / fall update; synchronises. */
tdp_status tdp_sta_rf_summary(tdp_graph, double *wns, double *tns, int32_t *n_fail, hipStream_t);
/* Double device arrays [2 * num_pins] in external pin order, [2 p] the
 * rise and [2 p + 1] the fall (any may be NULL): arrival, required time,
 * slack (+inf where either is infinite) and transition. */
tdp_status tdp_sta_rf_export(tdp_graph, double *d_at, double *d_rat, double *d_slack, double *d_slew,
                             hipStream_t);
/* report_timing_endpoint(n, 1) (Sec. III-B, Table I) on the rise / fall
 * update: the n endpoints of smallest slack (n < 0: every violated one),
 * ordered by (slack, pin id) and cut to K (and to max_paths), one path each,
 * ending in the endpoint's worse transition (rise on a tie) and following the
 * critical (input, transition) pairs back to a start point.  Output as
 * tdp_extract_paths, plus *d_path_tran (may be NULL): a device uint8 view,
 * parallel to path_pins, of each pin's transition (0 rise, 1 fall).  The pair
 * update then takes these paths.  TDP_E_STATE before a rise / fall update,
 * TDP_E_CAPACITY if n > max_paths. */
tdp_status tdp_extract_paths_rf(tdp_graph, int32_t n, int32_t K, hipStream_t, tdp_paths *out,
                                const uint8_t **d_path_tran);

/* ------------------------------------------------------------- paths */
/* report_timing_endpoint(n, k): endpoints ordered by (slack, pin id); n >= 0
 * takes the first n, n < 0 the violated ones (device-side count, no host
 * round trip).  At each selected endpoint the k paths of smallest slack are
 * found by slack-ordered deviation expansion from the arrival-time tree;
 * paths whose slack is >= slack_limit are dropped.  All paths are ordered by
 * (slack, endpoint pin id, rank) and cut to K.  Errors: TDP_E_CAPACITY if
 * n*k > max_paths (n < 0: number of endpoints * k) or k > max_k, TDP_E_STATE
 * before the first update. */
tdp_status tdp_extract_paths(tdp_graph, int32_t n, int32_t k, int32_t K, float slack_limit,
                             hipStream_t, tdp_paths *out);
/* report_timing(K) (Sec. III-B, Table I): the K paths of smallest slack over
 * the whole design (each instance of a batched graph on its own), however
 * many end at one endpoint; paths with slack >= slack_limit are dropped.
 * K is capped at max_paths (max_paths_each for a batched graph).  Output as
 * tdp_extract_paths (same views, replacing its paths), ordered by (slack,
 * then a fixed order among equal slacks); path_rank counts the earlier paths
 * of the same endpoint.  Exact: a bound on the K-th slack from the
 * per-endpoint search, then every path within it by deviation expansion.
 * Unlike the per-endpoint call it synchronises the stream (one counter read
 * per expansion round) and allocates its node store on its first call.
 * Errors: TDP_E_STATE before the first update, TDP_E_INVALID for K < 0 or a
 * NaN limit, TDP_E_NOMEM if the node store cannot be allocated,
 * TDP_E_CAPACITY if more paths tie at the K-th slack than the store holds
 * (8 * max_paths nodes, at least E * max_k). */
tdp_status tdp_report_timing(tdp_graph, int32_t K, float slack_limit, hipStream_t, tdp_paths *out);
/* For callers that cannot allocate device memory (serving loops, harnesses
 * that forbid hipMalloc): tdp_report_timing with its node store and sort /
 * scan scratch carved from a fixed 64 MiB device array that the library
 * holds on every device it runs on until the process ends; the call
 * allocates nothing.  Same arguments, outputs and results (bitwise) as
 * tdp_report_timing.  The store holds max(8 * max_paths, E * max_k, 4096)
 * nodes at 60 bytes each in single precision (68 in double) plus the sort's
 * histograms, so graphs up to about a million nodes fit; a larger one gets
 * TDP_E_CAPACITY with the size it needs, and nothing runs.  Every call on a
 * device shares that device's array and leaves its contents behind: calls
 * that overlap on one device (other host threads, other graphs) race, so
 * the caller orders them.  Errors otherwise as tdp_report_timing, and
 * TDP_E_DEVICE if the array's device address cannot be obtained. */
tdp_status tdp_report_timing_noalloc(tdp_graph, int32_t K, float slack_limit, hipStream_t, tdp_paths *out);
/* Number of paths and of path pins of the last extraction (synchronises). */
tdp_status tdp_paths_count(tdp_graph, int32_t *num_paths, int32_t *num_pins, hipStream_t);

/* --------------------------------------------------------------- pairs */
/* Update the maintained pin-pair set P from the last extraction (Eq. 9).
 * A pair is a net arc (driver pin, sink pin) on an extracted path, named by
 * its sink pin.  rule 0 (Eq. 9): skipped when WNS = 0; paths with negative
 * slack are taken in extraction order; a pair not in P enters with w0, a pair
 * already in P (this round or earlier) gains w1 * slack / WNS.  rule 1:
 * stateless, w = sum over this extraction's paths through the pair of
 * exp(-slack / max(|WNS|, 1 ps)).  P persists across calls under rule 0. */
tdp_status tdp_pairs_update(tdp_graph, int32_t rule, float w0, float w1, hipStream_t);
tdp_status tdp_pairs_reset(tdp_graph, hipStream_t);
/* Checkpoint / resume of P: dense per external pin (weight, membership), host
 * arrays [num_pins].  Export synchronises; import rebuilds the pair list. */
tdp_status tdp_pairs_export(tdp_graph, float *h_w, uint8_t *h_in_p, hipStream_t);
tdp_status tdp_pairs_import(tdp_graph, const float *h_w, const uint8_t *h_in_p, hipStream_t);
tdp_status tdp_pairs_count(tdp_graph, int32_t *num_pairs, hipStream_t);

/* ---------------------------------------------------------------- loss */
/* PP = sum over P of w * ((X_s - X_t)^2 + (Y_s - Y_t)^2), X = cell position +
 * pin offset (Eqs. 8, 10).  *d_loss (one device double) is overwritten.
 * Each term is evaluated in the graph's precision and the terms are summed
 * in double in a fixed order. */
tdp_status tdp_p2p_loss_fwd(tdp_graph, const float *d_x, const float *d_y, double *d_loss, hipStream_t);
/* d_gx/d_gy [num_cells] += (*d_gout) * dPP/dx, dPP/dy, with d_gout one
 * device double (NULL: 1); fixed cells and
 * ports get nothing.  Deterministic (fixed summation order per cell). */
tdp_status tdp_p2p_loss_bwd(tdp_graph, const float *d_x, const float *d_y, const double *d_gout,
                            float *d_gx, float *d_gy, hipStream_t);

/* The other pair distances Sec. III-C compares the quadratic one with, over
 * the same pairs and weights: kind 1 = sum w (|X_s - X_t| + |Y_s - Y_t|)
 * (the Manhattan distance, a two-pin pair's HPWL), kind 2 = sum w
 * sqrt((X_s - X_t)^2 + (Y_s - Y_t)^2) (linear Euclidean); kind 0 is PP and
 * equals tdp_p2p_loss_fwd / _bwd.  Gradients per axis: kind 1 w sgn(d)
 * (sgn(0) = 0), kind 2 w d / L (0 at L = 0).  Same conventions as the p2p
 * calls; TDP_E_INVALID for another kind. */
tdp_status tdp_pair_loss_fwd(tdp_graph, int32_t kind, const float *d_x, const float *d_y, double *d_loss,
                             hipStream_t);
tdp_status tdp_pair_loss_bwd(tdp_graph, int32_t kind, const float *d_x, const float *d_y, const double *d_gout,
                             float *d_gx, float *d_gy, hipStream_t);

/* Smoothed TNS (not in the paper: a differentiable stand-in for the TNS of
 * Eq. 4): cell-arc delays and start arrivals frozen from the last
 * update, net delays from d_x/d_y; log-sum-exp over fan-in with temperature
 * gamma_ps, value = -gamma * sum over endpoints of softplus(-slack/gamma).
 * fwd overwrites *d_val; bwd (same positions as the last fwd) adds
 * (*d_gout) * gradient into d_gx/d_gy.  d_val and d_gout are single device
 * doubles (d_gout NULL: 1). */
tdp_status tdp_stns_fwd(tdp_graph, const float *d_x, const float *d_y, float gamma_ps, double *d_val,
                        hipStream_t);
tdp_status tdp_stns_bwd(tdp_graph, const double *d_gout, float *d_gx, float *d_gy, hipStream_t);

/* Weighted-average wirelength (the WL term of Eq. 1, in the smooth form the
 * paper's placer uses) over every net (driver and sinks, ports too), both
 * axes, temperature gamma_um.  *d_wl (one device double) is overwritten;
 * d_gx/d_gy [num_cells] += gradient (movable cells only). */
tdp_status tdp_wa_fwd_bwd(tdp_graph, const float *d_x, const float *d_y, float gamma_um, double *d_wl,
                          float *d_gx, float *d_gy, hipStream_t);
/* The same at the positions of the last tdp_sta_update, reusing the cell
 * coordinates that update gathered per pin (a coalesced read instead of a
 * random one per pin).  The caller must not have changed those positions
 * since; results are then bitwise those of tdp_wa_fwd_bwd.  TDP_E_STATE
 * before the first update. */
tdp_status tdp_wa_fwd_bwd_at_update(tdp_graph, float gamma_um, double *d_wl, float *d_gx, float *d_gy,
                                    hipStream_t);

/* ------------------------------------------------ early (hold) analysis */
/* The early half of an early/late timer (the paper's timer, Sec. II-B /
 * III-B, runs both; its objective uses the late half), on the net delays and
 * loads of the
 * last tdp_sta_update (TDP_E_STATE before one).  Start points arrive as in
 * the late analysis; a sink at its driver's early arrival plus the net delay
 * (transition from the driver's early transition as the net model gives
 * it); a combinational output at the minimum over its inputs of (arrival +
 * table delay at the input's early transition and the output's load), with
 * the minimum of the table transitions.  Hold check at a D pin (ideal
 * clock): hold slack = early arrival - hold_ps.  Not part of the paper's
 * objective (setup TNS / WNS).  Asynchronous; the first call allocates its
 * arrays. */
tdp_status tdp_sta_update_early(tdp_graph, float hold_ps, hipStream_t);
/* WHS (minimum hold slack over D pins, 0 if none is negative), THS (sum of
 * the negative ones) and their count, over every D pin of the graph;
 * synchronises.  TDP_E_STATE before tdp_sta_update_early. */
tdp_status tdp_sta_early_summary(tdp_graph, double *whs, double *ths, int32_t *n_fail, hipStream_t);
/* Device double arrays [num_pins], any may be NULL: early arrival and
 * transition (at a sink, the one its cell arc or hold check sees), early
 * arc delay at combinational inputs (0 elsewhere), hold slack at D pins
 * (+inf elsewhere). */
tdp_status tdp_sta_early_export(tdp_graph, double *d_at, double *d_slew, double *d_darc, double *d_hold_slack,
                                hipStream_t);

/* ------------------------------------------------ placement loop pieces */
/* The placer around the hot path (Sec. IV) minimises wirelength + lambda *
 * density (Eq. 1) + beta * PP (Eq. 6) with Nesterov's method.  The paper does
 * not restate its density term; this library's is a bin density:
 *   the die [x0, x0 + bins_x*bin_w) x [y0, y0 + bins_y*bin_h) is cut into
 *   bins, bin (i, j) stored at j*bins_x + i; cell c spreads its area a_c as a
 *   Gaussian centred on its position with standard deviations (bin_w, bin_h),
 *   integrated over each bin and cut to the (2*radius+1)^2 bins around the
 *   bin holding the cell (indices clamped into the grid); window mass off
 *   the die is reflected back in at its edges (mirror images, as a Neumann
 *   boundary): D(i, j) = sum_c a_c Wx_c(i) Wy_c(j).
 *   value    = sum_b max(0, D_b - cap)^2, cap = target * bin_w * bin_h;
 *   overflow = sum_b max(0, D_b - cap) / sum_c a_c. */
typedef struct {
  float x0, y0, bin_w, bin_h;
  int32_t bins_x, bins_y; /* 1..4096 each */
  int32_t radius;         /* 0..8 */
  float target;           /* > 0 */
} tdp_density_grid;

/* Sets the grid and the cell areas (host [num_cells], finite, >= 0) and
 * allocates the scratch of the density and Nesterov calls (synchronous; a
 * later call with a grid no larger and a radius no larger reuses it).
 * TDP_E_INVALID on a bad grid or area. */
tdp_status tdp_density_setup(tdp_graph, const tdp_density_grid *grid, const float *h_area);

/* Density value and overflow (single device doubles, overwritten; either
 * may be NULL) at cell positions d_x, d_y [num_cells]; with d_gx and d_gy
 * (both or neither) adds scale * d value / d position on movable cells;
 * d_map (optional, [bins]) receives D.  Results are bitwise reproducible (no
 * floating-point atomics).  TDP_E_STATE before tdp_density_setup. */
tdp_status tdp_density_fwd_bwd(tdp_graph, const float *d_x, const float *d_y, float scale, double *d_value,
                               double *d_overflow, float *d_gx, float *d_gy, float *d_map, hipStream_t);

/* One step of Nesterov's method as ePlace applies it (Lu et al., TODAES
 * 2015) on the cells' 2*num_cells coordinates, all device float arrays
 * [num_cells]:
 *   q = (d_gx, d_gy) / max(1, d_pdiv) per cell (fixed cells: 0);
 *   alpha = |v - vp| / |q - gp|, or alpha0 when first != 0 or that ratio is
 *           not a positive number (written to *d_alpha when not NULL);
 *   u' = clamp(v - alpha q), v' = clamp(u' + coef (u' - u)) into
 *   [xlo, xhi] x [ylo, yhi]; then vp = v, gp = q, u = u', v = v' in place.
 * Fixed cells keep v and u.  Uses the scratch of tdp_density_setup
 * (TDP_E_STATE before it); asynchronous, allocates nothing. */
tdp_status tdp_nesterov_step(tdp_graph, const float *d_gx, const float *d_gy, const float *d_pdiv, float *d_vx,
                             float *d_vy, float *d_ux, float *d_uy, float *d_vpx, float *d_vpy, float *d_gpx,
                             float *d_gpy, double coef, double alpha0, int32_t first, float xlo, float xhi,
                             float ylo, float yhi, double *d_alpha, hipStream_t);

/* *d_out (one device double, overwritten) = sum over cells of |d_a[c]| +
 * |d_b[c]| (an L1 norm of a gradient pair, e.g. to set lambda from the ratio
 * of the wirelength and density gradients), in a fixed order.  Uses the
 * scratch of tdp_density_setup (TDP_E_STATE before it). */
tdp_status tdp_abs_sum(tdp_graph, const float *d_a, const float *d_b, double *d_out, hipStream_t);

/* ------------------------------------------------------------ tooling */
/* Stage timing: when enabled, every call records HIP events around its
 * stages on its stream.  tdp_profile_read synchronises and returns the
 * accumulated milliseconds per stage (see TDP_STAGE_*) and the number of
 * timed calls per stage, then clears them. */
enum {
  TDP_STAGE_NETPASS = 0, TDP_STAGE_FORWARD, TDP_STAGE_ENDPOINT, TDP_STAGE_BACKWARD,
  TDP_STAGE_SELECT, TDP_STAGE_SEARCH, TDP_STAGE_ORDER, TDP_STAGE_WALK, TDP_STAGE_PAIRS,
  TDP_STAGE_P2P_FWD, TDP_STAGE_P2P_BWD, TDP_STAGE_STNS, TDP_STAGE_WA, TDP_STAGE_DENSITY, TDP_NUM_STAGES
};
/* stage_mask: bit TDP_STAGE_x times that stage (0 turns timing off; events
 * are pooled and reused, so timing one stage adds two event records per
 * call of it). */
tdp_status tdp_profile_enable(tdp_graph, int32_t stage_mask);
tdp_status tdp_profile_read(tdp_graph, double *ms, int32_t *calls);

/* Launch tuning of the timing sweeps (Sec. II-B's arrival and required-time
 * propagation), used by the autotuner.
 *  sweep_mode 0: one launch per level (any graph);
 *  sweep_mode 1: one launch per sweep on a resident grid: every workgroup of
 *    it is on the GPU at once, each 64-lane wave owns a fixed set of chunks
 *    of pins in dependency order and waits for the values each chunk reads
 *    (single precision, every net with at most 63 sinks); TDP_E_UNSUPPORTED
 *    otherwise.  Every wait is bounded: a wait that runs out of polls makes
 *    all waves stop waiting, and tdp_sta_summary then returns TDP_E_DEVICE.
 *  sweep_mode 2: self-test of those bounded waits: as 1, but the start
 *    points are never published, so every wait gives up.
 *  sweep_mode 3: arrivals one launch per level, required times on a
 *    resident grid (the default where the resident grid is possible).
 *  flow_waves: 64-lane waves per workgroup of the resident grids (1, 2 or
 *    4; 0 keeps; default 4);
 *  flow_per_cu: workgroups per compute unit of the resident grids (1..4,
 *    capped by the kernel's occupancy; 0 keeps; default 1).  The grids must
 *    fit on the GPU beside whatever runs concurrently on other streams; two
 *    such sweeps from different graphs may run at once within 4 per CU.
 *  spin_log2: log2 of the poll budget per wait (0 keeps, 1..30).
 * Results do not depend on the tuning: both sweep forms compute every value
 * with the same operations in the same order. */
tdp_status tdp_set_tuning(tdp_graph, int32_t flow_waves, int32_t flow_per_cu, int32_t spin_log2,
                          int32_t sweep_mode);

/* Autotuner: on the caller's positions, times the timing update followed by
 * extract_paths(n, k, K) (k = 0: the update alone) under every sweep
 * configuration the graph supports (per-level launches; resident dataflow
 * grids for both sweeps or for the required times only, with 1, 2 or 4
 * waves per workgroup and 1, 2 or 4 workgroups per compute unit), one
 * warm-up and `reps` timed runs each (1..1000), and keeps the fastest.
 * Choices are kept for the life of the process by graph signature (device,
 * precision, pin / cell / net / endpoint counts, depth, instances,
 * deviation-list width, n, k, K): a later call for a graph with the same
 * signature takes the kept choice without trials.  h_choice (4 int32, host,
 * may be NULL) receives {sweep_mode, flow_waves, flow_per_cu, microseconds
 * per run as measured when the choice was made}.  Synchronises; on return
 * the graph holds the chosen configuration's results for these positions.
 * Errors as tdp_sta_update / tdp_extract_paths. */
tdp_status tdp_autotune(tdp_graph, const float *d_x, const float *d_y, int32_t n, int32_t k, int32_t K,
                        int32_t reps, int32_t *h_choice, hipStream_t);

/* Sizes of the graph: num_cells, num_pins, num_nets, depth, endpoints,
 * startpoints, combinational cells, sink pins (8 int32, host). */
tdp_status tdp_graph_info(tdp_graph, int32_t *info8);

const char *tdp_status_str(tdp_status);
const char *tdp_last_error(tdp_graph);

#ifdef __cplusplus
}
#endif
#endif /* TDP_H_ */
