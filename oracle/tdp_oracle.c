/*
 * Plain FP64 CPU oracle for the timing-driven placement hot path of
 * "Timing-Driven Global Placement by Efficient Critical Path Extraction"
 * (Shi et al., arXiv 2503.11674).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the package's smoke check
 * and the benchmark's CPU-baseline leg may load this library.  It shares no
 * code, header or table with the HIP implementation: it takes the same
 * netlist arrays (external pin / cell numbering) and computes everything with
 * straightforward loops in double precision, single threaded.
 *
 * What it computes, and where the paper defines it:
 *   ora_sta      - static timing analysis on the timing DAG (Sec. II-B, Eq. 2):
 *                  arrival times forward, required times backward,
 *                  slack = required - arrival at every pin; WNS and TNS over
 *                  violated endpoints, both 0 when none violates (Eqs. 3-4).
 *                  Net delay is R*C, with R and C linear in wire length
 *                  (Sec. III-C, Eq. 7), i.e. r*c*L^2 with L the Manhattan
 *                  distance, or, as a fuller model of the same wires, the
 *                  Elmore delay of a star RC net or of a spanning-tree RC
 *                  net, with degraded sink transitions (net model section
 *                  below); cell arcs come from slew x load tables.
 *   ora_sta_early - the early half of an early/late timer: earliest
 *                  arrivals at best-case transitions and the hold check at
 *                  the D pins (not used by the paper's objective, which is
 *                  setup TNS / WNS; a fuller timing model around it).
 *   ora_sta_rf   - rise / fall timing: both transitions of every pin, cell
 *                  arcs by unateness, with report_timing_endpoint(n, 1) on it
 *                  (ora_extract_rf); a fuller timing model around the paper's.
 *   ora_extract  - report_timing_endpoint(n, k) (Sec. III-B, Table I): the n
 *                  most critical endpoints, and the k worst paths at each.
 *                  Reached by deviation (sidetrack) enumeration from the
 *                  arrival-time tree, in order of path slack.
 *   ora_report_timing - report_timing(K) (Sec. III-B, Table I): the K worst
 *                  paths over the whole design, by one best-first deviation
 *                  enumeration across all endpoints.
 *   ora_pairs    - the maintained pin-pair set P and the weight rule of
 *                  Eq. 9 (Sec. III-D), or the stateless exponential rule.
 *   ora_p2p      - PP = sum w * Q(i, j), Q the squared Euclidean pin distance
 *                  (Eqs. 8 and 10), with its gradient on cell positions.
 *   ora_pair_loss - the two distance losses the paper compares PP with
 *                  (Sec. III-C): the Manhattan distance (a two-pin pair's
 *                  HPWL) and the linear Euclidean distance, with gradients.
 *   ora_stns     - a log-sum-exp smoothed TNS with its adjoint (not in the
 *                  paper; definition below).
 *   ora_wa       - weighted-average wirelength (the WL_e of Eq. 1, the
 *                  published weighted-average model) with its gradient.
 *   ora_density  - a bin-density penalty and overflow for the placement loop
 *                  around the hot path (the density term of Eq. 1; its
 *                  definition is below), with its gradient.
 *   ora_nesterov - one Nesterov step with the Lipschitz step prediction
 *                  ePlace uses (the optimiser of the paper's placer).
 *
 * Pin roles: a port (pin_cell == -1) is a primary input and drives a net;
 * a combinational cell has input pins (net sinks) and one output pin (a net
 * driver); a flip-flop has a D pin (net sink, timing endpoint) and a Q pin
 * (net driver, timing startpoint).  The clock is ideal: a flip-flop's
 * clock-to-Q arc is looked up at the clock slew and the Q pin's load.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ROLE_PORT 0
#define ROLE_CIN 1
#define ROLE_COUT 2
#define ROLE_FFD 3
#define ROLE_FFQ 4

typedef struct {
  int num_cells, num_pins, num_nets;
  const int32_t *pin_cell;
  const float *pin_off_x, *pin_off_y;
  const int32_t *net_ptr, *net_pins;
  const int32_t *cell_type, *cell_in_ptr, *cell_in_pins, *cell_out_pin;
  const uint8_t *cell_is_ff;
} onl;

typedef struct {
  int num_types, n_slew, n_load;
  const float *slew_axis, *load_axis, *delay_lut, *slew_lut, *pin_cap;
  double r, c, scale;
  int model; /* net model: 0 lumped (Eq. 7), 1 Elmore star, 2 Elmore spanning tree; 1 and 2
                degrade the sink transitions */
} olib;

/* ------------------------------------------------------------------------ */
/* derived connectivity                                                      */
/* ------------------------------------------------------------------------ */
typedef struct {
  int *role;       /* [P] */
  int *driver;     /* [P] driver pin of a sink pin, -1 otherwise */
  int *net_of;     /* [P] net the pin belongs to */
  int *in_index;   /* [P] arc index of a comb input pin within its cell */
  int *topo;       /* [P] pins in a topological order */
} oconn;

static void conn_free(oconn *c) {
  free(c->role); free(c->driver); free(c->net_of); free(c->in_index); free(c->topo);
}

/* returns 0, or -1 if the timing graph has a cycle / dangling structure */
static int conn_build(const onl *n, oconn *c) {
  int P = n->num_pins, N = n->num_cells, M = n->num_nets;
  c->role = (int *)malloc(sizeof(int) * P);
  c->driver = (int *)malloc(sizeof(int) * P);
  c->net_of = (int *)malloc(sizeof(int) * P);
  c->in_index = (int *)malloc(sizeof(int) * P);
  c->topo = (int *)malloc(sizeof(int) * P);
  for (int p = 0; p < P; ++p) { c->role[p] = ROLE_PORT; c->driver[p] = -1; c->net_of[p] = -1; c->in_index[p] = -1; }
  for (int cell = 0; cell < N; ++cell) {
    int ff = n->cell_is_ff[cell];
    for (int k = n->cell_in_ptr[cell]; k < n->cell_in_ptr[cell + 1]; ++k) {
      int p = n->cell_in_pins[k];
      c->role[p] = ff ? ROLE_FFD : ROLE_CIN;
      c->in_index[p] = k - n->cell_in_ptr[cell];
    }
    c->role[n->cell_out_pin[cell]] = ff ? ROLE_FFQ : ROLE_COUT;
  }
  for (int net = 0; net < M; ++net) {
    int d = n->net_pins[n->net_ptr[net]];
    c->net_of[d] = net;
    for (int k = n->net_ptr[net] + 1; k < n->net_ptr[net + 1]; ++k) {
      c->driver[n->net_pins[k]] = d;
      c->net_of[n->net_pins[k]] = net;
    }
  }
  /* Kahn's algorithm over pins.  Arcs: driver -> sink (net arcs) and comb
   * input -> comb output (cell arcs). */
  int *indeg = (int *)calloc(P, sizeof(int));
  for (int p = 0; p < P; ++p) {
    if (c->driver[p] >= 0) indeg[p] += 1;
    if (c->role[p] == ROLE_COUT) {
      int cell = n->pin_cell[p];
      indeg[p] += n->cell_in_ptr[cell + 1] - n->cell_in_ptr[cell];
    }
  }
  int head = 0, tail = 0;
  for (int p = 0; p < P; ++p) if (indeg[p] == 0) c->topo[tail++] = p;
  while (head < tail) {
    int p = c->topo[head++];
    int r = c->role[p];
    if (r == ROLE_PORT || r == ROLE_COUT || r == ROLE_FFQ) {
      int net = c->net_of[p];
      if (net >= 0)
        for (int k = n->net_ptr[net] + 1; k < n->net_ptr[net + 1]; ++k) {
          int t = n->net_pins[k];
          if (--indeg[t] == 0) c->topo[tail++] = t;
        }
    } else if (r == ROLE_CIN) {
      int o = n->cell_out_pin[n->pin_cell[p]];
      if (--indeg[o] == 0) c->topo[tail++] = o;
    }
  }
  free(indeg);
  return tail == P ? 0 : -1;
}

/* ------------------------------------------------------------------------ */
/* lookup table: clamp to the axis range, bilinear in (slew, load)          */
/* ------------------------------------------------------------------------ */
static double lut_eval(const olib *L, const float *tables, int type, double slew, double load) {
  const float *sa = L->slew_axis + (size_t)type * L->n_slew;
  const float *la = L->load_axis + (size_t)type * L->n_load;
  const float *T = tables + (size_t)type * L->n_slew * L->n_load;
  double s = slew, l = load;
  if (s < sa[0]) s = sa[0];
  if (s > sa[L->n_slew - 1]) s = sa[L->n_slew - 1];
  if (l < la[0]) l = la[0];
  if (l > la[L->n_load - 1]) l = la[L->n_load - 1];
  int i = 0;
  while (i + 1 < L->n_slew - 1 && sa[i + 1] <= s) ++i;
  int j = 0;
  while (j + 1 < L->n_load - 1 && la[j + 1] <= l) ++j;
  double tau = (s - sa[i]) / ((double)sa[i + 1] - sa[i]);
  double ups = (l - la[j]) / ((double)la[j + 1] - la[j]);
  double t00 = T[i * L->n_load + j], t10 = T[(i + 1) * L->n_load + j];
  double t01 = T[i * L->n_load + j + 1], t11 = T[(i + 1) * L->n_load + j + 1];
  return (1 - tau) * (1 - ups) * t00 + tau * (1 - ups) * t10 + (1 - tau) * ups * t01 + tau * ups * t11;
}

int ora_lut_eval(int n_slew, int n_load, const float *slew_axis, const float *load_axis,
                 const float *table, int count, const double *slew, const double *load, double *out) {
  olib L;
  memset(&L, 0, sizeof L);
  L.num_types = 1; L.n_slew = n_slew; L.n_load = n_load;
  L.slew_axis = slew_axis; L.load_axis = load_axis;
  for (int q = 0; q < count; ++q) out[q] = lut_eval(&L, table, 0, slew[q], load[q]);
  return 0;
}

static void pin_xy(const onl *n, const float *x, const float *y, int p, double *px, double *py) {
  int cell = n->pin_cell[p];
  double bx = cell >= 0 ? (double)x[cell] : 0.0;
  double by = cell >= 0 ? (double)y[cell] : 0.0;
  *px = bx + (double)n->pin_off_x[p];
  *py = by + (double)n->pin_off_y[p];
}

/* ------------------------------------------------------------------------ */
/* net model                                                                 */
/* ------------------------------------------------------------------------ */
/* Each sink hangs off the driver on a wire of its own whose length L is the
 * Manhattan driver-to-sink distance, with resistance r*L and capacitance c*L
 * (Eq. 7: both linear in length).  The driver's load is the total capacitance
 * of the net, sum over sinks of (pin cap + c*L), in either model.
 *   model 0 (Eq. 7 as written): the wire's lumped R times C, scale*r*c*L^2.
 *   model 1: the Elmore delay of that star RC net.  The first moment of the
 *     impulse response at a sink is the sum, over the resistances between the
 *     driver and the sink, of resistance times the capacitance downstream of
 *     it.  The sink's branch is a uniform line, so that sum is
 *     r*L*(c*L/2 + C_sink), the other branches having no resistance in common
 *     with it; scale converts to the time unit.
 * Sink transition: model 0 passes the driver's transition through unchanged;
 * model 1 degrades it by the wire with the PERI rule (Kashyap, Alpert, Liu
 * and Devgan, IEEE TCAD 2004): the root sum of squares of the input
 * transition and the wire's own step-response transition, the latter taken
 * as ln(9) times the Elmore delay (the 10-90% time of a single-pole
 * response with that time constant); model 2 does the same.
 *
 * Model 2: the net is an RC tree whose topology is a rectilinear minimum
 * spanning tree of its pins, grown from the driver by Prim's algorithm: start
 * with the driver; repeatedly add the pin outside the tree closest (Manhattan
 * distance) to any pin inside it, joined to that pin.  Ties go to the pin
 * first in the net's pin list and, for its parent, to the pin that joined
 * the tree first.  The distances that decide the topology are single
 * precision, (cell coordinate difference) + (offset difference) per axis, so
 * that a single-precision timer takes the same decisions.  Every tree edge is
 * a uniform wire of its Manhattan length L (resistance r L, capacitance c L).
 * With C_below(u) the capacitance at and below pin u (its pin capacitance and
 * the wires and pins of its subtree), the Elmore delay to a pin is the sum,
 * over the edges e = (parent, v) on its path from the driver, of
 * r L_e (c L_e / 2 + C_below(v)), times scale.  The driver's load is again the
 * net's total capacitance: the pin capacitances plus c times the tree's total
 * length.  A two-pin net gives model 1's delay. */
static double net_delay(const olib *L, double len, double sink_cap) {
  if (L->model == 1) return L->scale * L->r * len * (0.5 * L->c * len + sink_cap);
  return L->scale * L->r * L->c * len * len;
}

/* d net_delay / d len */
static double net_delay_dlen(const olib *L, double len, double sink_cap) {
  if (L->model == 1) return L->scale * L->r * (L->c * len + sink_cap);
  return 2.0 * L->scale * L->r * L->c * len;
}

static double sink_slew(const olib *L, double drv_slew, double dnet) {
  if (L->model == 0) return drv_slew;
  double w = log(9.0) * dnet;
  return sqrt(drv_slew * drv_slew + w * w);
}

/* one net's tree: node 0 is the driver, node i >= 1 the net's i-th sink */
typedef struct {
  int m;          /* number of sinks */
  int32_t *pin;   /* [m+1] pin id of each node */
  int *par;       /* [m+1] parent node, -1 at the driver */
  int *ord;       /* [m]   sink nodes in the order they join the tree */
  double *len;    /* [m+1] length of the wire from the parent */
  double *cd;     /* [m+1] capacitance at and below the node */
  double *delay;  /* [m+1] Elmore delay from the driver */
  double *aux;    /* [m+1] scratch of the adjoint */
  float *dist;    /* [m+1] Prim's distance to the tree */
  char *in;       /* [m+1] node is in the tree */
} otree;

static int otree_alloc(otree *T, int max_pins) {
  size_t k = (size_t)(max_pins > 1 ? max_pins : 1);
  T->pin = (int32_t *)malloc(sizeof(int32_t) * k);
  T->par = (int *)malloc(sizeof(int) * k);
  T->ord = (int *)malloc(sizeof(int) * k);
  T->len = (double *)malloc(sizeof(double) * k);
  T->cd = (double *)malloc(sizeof(double) * k);
  T->delay = (double *)malloc(sizeof(double) * k);
  T->aux = (double *)malloc(sizeof(double) * k);
  T->dist = (float *)malloc(sizeof(float) * k);
  T->in = (char *)malloc(k);
  return T->pin && T->par && T->ord && T->len && T->cd && T->delay && T->aux && T->dist && T->in ? 0 : -1;
}

static void otree_free(otree *T) {
  free(T->pin); free(T->par); free(T->ord); free(T->len); free(T->cd); free(T->delay); free(T->aux);
  free(T->dist); free(T->in);
}

static int max_net_pins(const int32_t *net_ptr, int num_nets) {
  int w = 1;
  for (int net = 0; net < num_nets; ++net)
    if (net_ptr[net + 1] - net_ptr[net] > w) w = net_ptr[net + 1] - net_ptr[net];
  return w;
}

/* single-precision Manhattan distance of two pins (the topology's metric) */
static float pin_fdist(const onl *n, const float *x, const float *y, int a, int b) {
  int ca = n->pin_cell[a], cb = n->pin_cell[b];
  float ax = ca >= 0 ? x[ca] : 0.0f, ay = ca >= 0 ? y[ca] : 0.0f;
  float bx = cb >= 0 ? x[cb] : 0.0f, by = cb >= 0 ? y[cb] : 0.0f;
  float dx = (ax - bx) + (n->pin_off_x[a] - n->pin_off_x[b]);
  float dy = (ay - by) + (n->pin_off_y[a] - n->pin_off_y[b]);
  return fabsf(dx) + fabsf(dy);
}

/* Prim's spanning tree of one net (model 2's topology) */
static void tree_topology(const onl *n, const float *x, const float *y, int net, otree *T) {
  int b = n->net_ptr[net], m = n->net_ptr[net + 1] - b - 1;
  T->m = m;
  for (int i = 0; i <= m; ++i) { T->pin[i] = n->net_pins[b + i]; T->par[i] = -1; T->in[i] = 0; }
  T->in[0] = 1;
  for (int i = 1; i <= m; ++i) { T->dist[i] = pin_fdist(n, x, y, T->pin[0], T->pin[i]); T->par[i] = 0; }
  for (int step = 0; step < m; ++step) {
    int j = -1;
    for (int i = 1; i <= m; ++i)
      if (!T->in[i] && (j < 0 || T->dist[i] < T->dist[j])) j = i;
    T->in[j] = 1;
    T->ord[step] = j;
    for (int i = 1; i <= m; ++i)
      if (!T->in[i]) {
        float d = pin_fdist(n, x, y, T->pin[j], T->pin[i]);
        if (d < T->dist[i]) { T->dist[i] = d; T->par[i] = j; }
      }
  }
}

/* wire lengths, capacitances below each node and Elmore delays on the tree */
static void tree_elmore(const onl *n, const olib *L, const float *x, const float *y, otree *T) {
  int m = T->m;
  T->len[0] = 0.0; T->cd[0] = 0.0; T->delay[0] = 0.0;
  for (int i = 1; i <= m; ++i) {
    double xi, yi, xp, yp;
    pin_xy(n, x, y, T->pin[i], &xi, &yi);
    pin_xy(n, x, y, T->pin[T->par[i]], &xp, &yp);
    T->len[i] = fabs(xp - xi) + fabs(yp - yi);
    T->cd[i] = (double)L->pin_cap[n->cell_type[n->pin_cell[T->pin[i]]]];
  }
  /* children join after their parents: the reverse joining order visits
   * every subtree before its root */
  for (int step = m - 1; step >= 0; --step) {
    int j = T->ord[step], p = T->par[j];
    if (p > 0) T->cd[p] += L->c * T->len[j] + T->cd[j];
  }
  for (int step = 0; step < m; ++step) {
    int j = T->ord[step];
    T->delay[j] = T->delay[T->par[j]] + L->scale * L->r * T->len[j] * (0.5 * L->c * T->len[j] + T->cd[j]);
  }
}

/* net delay into every sink and the load of every driver, in the library's
 * net model */
static void net_pass(const onl *n, const olib *L, const float *x, const float *y, double *dnet, double *load) {
  otree T;
  if (L->model == 2 && otree_alloc(&T, max_net_pins(n->net_ptr, n->num_nets)) != 0) { otree_free(&T); abort(); }
  for (int net = 0; net < n->num_nets; ++net) {
    int s = n->net_pins[n->net_ptr[net]];
    double ld = 0.0;
    if (L->model == 2) {
      tree_topology(n, x, y, net, &T);
      tree_elmore(n, L, x, y, &T);
      for (int i = 1; i <= T.m; ++i) {
        int t = T.pin[i];
        dnet[t] = T.delay[i];
        ld += (double)L->pin_cap[n->cell_type[n->pin_cell[t]]] + L->c * T.len[i];
      }
    } else {
      double xs, ys;
      pin_xy(n, x, y, s, &xs, &ys);
      for (int k = n->net_ptr[net] + 1; k < n->net_ptr[net + 1]; ++k) {
        int t = n->net_pins[k];
        double xt, yt;
        pin_xy(n, x, y, t, &xt, &yt);
        double len = fabs(xs - xt) + fabs(ys - yt);
        double cap = (double)L->pin_cap[n->cell_type[n->pin_cell[t]]];
        dnet[t] = net_delay(L, len, cap);
        ld += cap + L->c * len;
      }
    }
    load[s] = ld;
  }
  if (L->model == 2) otree_free(&T);
}

#define NETLIST_ARGS                                                                             \
  int num_cells, int num_pins, int num_nets, const int32_t *pin_cell, const float *pin_off_x,    \
      const float *pin_off_y, const int32_t *net_ptr, const int32_t *net_pins,                   \
      const int32_t *cell_type, const int32_t *cell_in_ptr, const int32_t *cell_in_pins,         \
      const int32_t *cell_out_pin, const uint8_t *cell_is_ff
#define LIB_ARGS                                                                                 \
  int num_types, int n_slew, int n_load, const float *slew_axis, const float *load_axis,         \
      const float *delay_lut, const float *slew_lut, const float *pin_cap, double r_per_um,      \
      double c_per_um, double delay_scale, int net_model

#define FILL_NETLIST(nn)                                                                         \
  onl nn;                                                                                        \
  nn.num_cells = num_cells; nn.num_pins = num_pins; nn.num_nets = num_nets;                      \
  nn.pin_cell = pin_cell; nn.pin_off_x = pin_off_x; nn.pin_off_y = pin_off_y;                    \
  nn.net_ptr = net_ptr; nn.net_pins = net_pins; nn.cell_type = cell_type;                        \
  nn.cell_in_ptr = cell_in_ptr; nn.cell_in_pins = cell_in_pins; nn.cell_out_pin = cell_out_pin;  \
  nn.cell_is_ff = cell_is_ff
#define FILL_LIB(ll)                                                                             \
  olib ll;                                                                                       \
  ll.num_types = num_types; ll.n_slew = n_slew; ll.n_load = n_load; ll.slew_axis = slew_axis;    \
  ll.load_axis = load_axis; ll.delay_lut = delay_lut; ll.slew_lut = slew_lut;                    \
  ll.pin_cap = pin_cap; ll.r = r_per_um; ll.c = c_per_um; ll.scale = delay_scale;            \
  ll.model = net_model

/* ------------------------------------------------------------------------ */
/* STA                                                                       */
/* ------------------------------------------------------------------------ */
/* Outputs (all indexed by external pin id unless noted):
 *   at, slew, rat, slack  [P]
 *   dnet  [P]  net delay into a sink pin (0 elsewhere)
 *   load  [P]  load seen by a driver pin (0 elsewhere)
 *   darc  [P]  cell-arc delay from a comb input pin to its output (0 elsewhere)
 *   crit  [N]  arc index of the input that sets a comb cell's output arrival
 *              (lowest index on ties), -1 for flip-flops
 *   summary[3] = {WNS, TNS, number of violated endpoints}
 * Returns 0, or -1 if the timing graph has a cycle. */
int ora_sta(NETLIST_ARGS, LIB_ARGS, const float *x, const float *y, double clock_period,
            double setup, double input_slew, double clock_slew, double *at, double *slew,
            double *rat, double *slack, double *dnet, double *load, double *darc, int32_t *crit,
            double *summary) {
  FILL_NETLIST(n);
  FILL_LIB(L);
  oconn c;
  if (conn_build(&n, &c) != 0) { conn_free(&c); return -1; }
  int P = num_pins, N = num_cells;
  for (int p = 0; p < P; ++p) {
    at[p] = -INFINITY; slew[p] = 0; rat[p] = INFINITY; slack[p] = INFINITY;
    dnet[p] = 0; load[p] = 0; darc[p] = 0;
  }
  for (int cell = 0; cell < N; ++cell) crit[cell] = -1;

  /* net pass: wire lengths, net delays, driver loads */
  net_pass(&n, &L, x, y, dnet, load);

  /* forward arrival times in topological order */
  for (int q = 0; q < P; ++q) {
    int p = c.topo[q];
    switch (c.role[p]) {
      case ROLE_PORT:
        at[p] = 0.0;
        slew[p] = input_slew;
        break;
      case ROLE_FFQ: {
        int type = cell_type[pin_cell[p]];
        at[p] = lut_eval(&L, delay_lut, type, clock_slew, load[p]);
        slew[p] = lut_eval(&L, slew_lut, type, clock_slew, load[p]);
        break;
      }
      case ROLE_CIN:
      case ROLE_FFD:
        if (c.driver[p] >= 0) {
          at[p] = at[c.driver[p]] + dnet[p];
          slew[p] = sink_slew(&L, slew[c.driver[p]], dnet[p]);
        }
        break;
      case ROLE_COUT: {
        int cell = pin_cell[p], type = cell_type[cell];
        double best = -INFINITY, sl = 0.0;
        int arg = -1;
        for (int k = cell_in_ptr[cell]; k < cell_in_ptr[cell + 1]; ++k) {
          int i = cell_in_pins[k];
          if (at[i] == -INFINITY) continue;
          double d = lut_eval(&L, delay_lut, type, slew[i], load[p]);
          double so = lut_eval(&L, slew_lut, type, slew[i], load[p]);
          darc[i] = d;
          double a = at[i] + d;
          if (a > best) { best = a; arg = k - cell_in_ptr[cell]; }
          if (so > sl) sl = so;
        }
        at[p] = best;
        slew[p] = sl;
        crit[cell] = arg;
        break;
      }
    }
  }

  /* endpoints: required time at a D pin is the clock period minus setup */
  double wns = 0.0, tns = 0.0;
  long nfail = 0;
  for (int p = 0; p < P; ++p)
    if (c.role[p] == ROLE_FFD) {
      rat[p] = clock_period - setup;
      double s = rat[p] - at[p];
      if (at[p] == -INFINITY) s = INFINITY;
      if (s < 0) { nfail++; tns += s; if (s < wns) wns = s; }
    }
  summary[0] = wns; summary[1] = tns; summary[2] = (double)nfail;

  /* backward required times in reverse topological order */
  for (int q = P - 1; q >= 0; --q) {
    int p = c.topo[q];
    int r = c.role[p];
    if (r == ROLE_CIN) {
      int o = cell_out_pin[pin_cell[p]];
      rat[p] = rat[o] == INFINITY ? INFINITY : rat[o] - darc[p];
    } else if (r == ROLE_PORT || r == ROLE_COUT || r == ROLE_FFQ) {
      double best = INFINITY;
      int net = c.net_of[p];
      if (net >= 0)
        for (int k = net_ptr[net] + 1; k < net_ptr[net + 1]; ++k) {
          int t = net_pins[k];
          if (rat[t] == INFINITY) continue;
          double v = rat[t] - dnet[t];
          if (v < best) best = v;
        }
      rat[p] = best;
    }
  }
  for (int p = 0; p < P; ++p)
    slack[p] = (rat[p] == INFINITY || at[p] == -INFINITY) ? INFINITY : rat[p] - at[p];
  conn_free(&c);
  return 0;
}

/* Early (hold) analysis on the same timing graph: the other half of an
 * early/late timer.  Net delays and loads are those of the net model; start
 * points arrive as in ora_sta; every other pin takes the earliest arrival:
 *   sink t:         AT_e(t) = AT_e(drv) + dnet(t), transition as ora_sta
 *                   gives a sink from its driver's (early) transition;
 *   comb output o:  AT_e(o) = min_j (AT_e(i_j) + d_e(i_j)), d_e(i_j) the
 *                   delay table at i_j's early transition and o's load;
 *                   transition = min_j of the transition table (best case).
 * Hold check at a D pin (ideal clock): hold slack = AT_e - hold.  Outputs
 * [P]: at_e, slew_e, darc_e (0 off comb inputs), hold_slack (+inf off D pins
 * and at unreachable D pins); summary = {WHS, THS, number of D pins with
 * hold slack < 0}, the first two 0 when none violates.  Returns 0, or -1 on
 * a cycle. */
int ora_sta_early(NETLIST_ARGS, LIB_ARGS, const float *x, const float *y, double hold, double input_slew,
                  double clock_slew, double *at_e, double *slew_e, double *darc_e, double *hold_slack,
                  double *summary) {
  FILL_NETLIST(n);
  FILL_LIB(L);
  oconn c;
  if (conn_build(&n, &c) != 0) { conn_free(&c); return -1; }
  int P = num_pins;
  double *dnet = (double *)calloc(P, sizeof(double)), *load = (double *)calloc(P, sizeof(double));
  for (int p = 0; p < P; ++p) { at_e[p] = INFINITY; slew_e[p] = 0; darc_e[p] = 0; hold_slack[p] = INFINITY; }
  net_pass(&n, &L, x, y, dnet, load);
  for (int q = 0; q < P; ++q) {
    int p = c.topo[q];
    switch (c.role[p]) {
      case ROLE_PORT:
        at_e[p] = 0.0;
        slew_e[p] = input_slew;
        break;
      case ROLE_FFQ: {
        int type = cell_type[pin_cell[p]];
        at_e[p] = lut_eval(&L, delay_lut, type, clock_slew, load[p]);
        slew_e[p] = lut_eval(&L, slew_lut, type, clock_slew, load[p]);
        break;
      }
      case ROLE_CIN:
      case ROLE_FFD:
        if (c.driver[p] >= 0 && at_e[c.driver[p]] != INFINITY) {
          at_e[p] = at_e[c.driver[p]] + dnet[p];
          slew_e[p] = sink_slew(&L, slew_e[c.driver[p]], dnet[p]);
        }
        break;
      case ROLE_COUT: {
        int cell = pin_cell[p], type = cell_type[cell];
        double best = INFINITY, sl = INFINITY;
        for (int k = cell_in_ptr[cell]; k < cell_in_ptr[cell + 1]; ++k) {
          int i = cell_in_pins[k];
          if (at_e[i] == INFINITY) continue;
          double d = lut_eval(&L, delay_lut, type, slew_e[i], load[p]);
          double so = lut_eval(&L, slew_lut, type, slew_e[i], load[p]);
          darc_e[i] = d;
          if (at_e[i] + d < best) best = at_e[i] + d;
          if (so < sl) sl = so;
        }
        at_e[p] = best;
        slew_e[p] = best == INFINITY ? 0.0 : sl;
        break;
      }
    }
  }
  double whs = 0.0, ths = 0.0;
  long nfail = 0;
  for (int p = 0; p < P; ++p)
    if (c.role[p] == ROLE_FFD && at_e[p] != INFINITY) {
      double h = at_e[p] - hold;
      hold_slack[p] = h;
      if (h < 0) { nfail++; ths += h; if (h < whs) whs = h; }
    }
  summary[0] = whs; summary[1] = ths; summary[2] = (double)nfail;
  free(dnet); free(load);
  conn_free(&c);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* k worst paths per endpoint                                                */
/* ------------------------------------------------------------------------ */
typedef struct { double cost; long seq; int parent; int dev; int u; } ocand;

typedef struct { ocand *a; int n, cap; } oheap;

static int cand_less(const ocand *x, const ocand *y) {
  if (x->cost != y->cost) return x->cost < y->cost;
  return x->seq < y->seq;
}
static void heap_push(oheap *h, ocand v) {
  if (h->n == h->cap) { h->cap = h->cap ? 2 * h->cap : 64; h->a = (ocand *)realloc(h->a, sizeof(ocand) * h->cap); }
  int i = h->n++;
  h->a[i] = v;
  while (i > 0) {
    int par = (i - 1) / 2;
    if (!cand_less(&h->a[i], &h->a[par])) break;
    ocand t = h->a[i]; h->a[i] = h->a[par]; h->a[par] = t;
    i = par;
  }
}
static ocand heap_pop(oheap *h) {
  ocand top = h->a[0];
  h->a[0] = h->a[--h->n];
  int i = 0;
  for (;;) {
    int l = 2 * i + 1, r = l + 1, m = i;
    if (l < h->n && cand_less(&h->a[l], &h->a[m])) m = l;
    if (r < h->n && cand_less(&h->a[r], &h->a[m])) m = r;
    if (m == i) break;
    ocand t = h->a[i]; h->a[i] = h->a[m]; h->a[m] = t;
    i = m;
  }
  return top;
}

typedef struct { double slack; int ep; int rank; int start; int len; } opath;

/* Builds the path into endpoint e that follows the arrival-time tree except at
 * the deviations devs[0..nd) (devs[nd-1] nearest the endpoint; a deviation is
 * the non-critical input pin taken at its cell), appends its pins in
 * start -> end order to the pool and records it with its slack recomputed
 * from the arc delays along it. */
static void add_path(const oconn *c, const int32_t *pin_cell, const int32_t *cell_in_ptr,
                     const int32_t *cell_in_pins, const double *at, const double *rat, const double *dnet,
                     const double *darc, const int32_t *crit, int e, int rank, const int *devs, int nd,
                     int *chain_pins, int32_t **pool, long *pool_n, long *pool_cap, opath **paths, int *npaths,
                     int *pcap) {
  int len = 0, di = nd - 1;
  chain_pins[len++] = e;
  int v = c->driver[e];
  for (;;) {
    chain_pins[len++] = v;
    if (c->role[v] != ROLE_COUT) break;
    int cell = pin_cell[v];
    int in;
    if (di >= 0 && pin_cell[devs[di]] == cell) in = devs[di--];
    else in = cell_in_pins[cell_in_ptr[cell] + crit[cell]];
    chain_pins[len++] = in;
    v = c->driver[in];
  }
  /* reverse into start -> end order and recompute the path slack */
  if (*pool_n + len > *pool_cap) {
    *pool_cap = (*pool_n + len) * 2 + 1024;
    *pool = (int32_t *)realloc(*pool, sizeof(int32_t) * *pool_cap);
  }
  int32_t *dst = *pool + *pool_n;
  int start = chain_pins[len - 1];
  double arr = at[start];
  for (int a = 0; a < len; ++a) {
    int pin = chain_pins[len - 1 - a];
    dst[a] = pin;
    if (a == 0) continue;
    int role = c->role[pin];
    if (role == ROLE_CIN || role == ROLE_FFD) arr += dnet[pin];
    else if (role == ROLE_COUT) arr += darc[chain_pins[len - a]];
  }
  if (*npaths == *pcap) {
    *pcap = *pcap ? 2 * *pcap : 1024;
    *paths = (opath *)realloc(*paths, sizeof(opath) * *pcap);
  }
  opath *o = *paths + *npaths;
  o->slack = rat[e] - arr;
  o->ep = e;
  o->rank = rank;
  o->start = (int)*pool_n;
  o->len = len;
  *npaths += 1;
  *pool_n += len;
}

static int opath_cmp(const void *a, const void *b) {
  const opath *x = (const opath *)a, *y = (const opath *)b;
  if (x->slack != y->slack) return x->slack < y->slack ? -1 : 1;
  if (x->ep != y->ep) return x->ep < y->ep ? -1 : 1;
  return x->rank < y->rank ? -1 : (x->rank > y->rank);
}

typedef struct { double slack; int pin; } oep;
static int oep_cmp(const void *a, const void *b) {
  const oep *x = (const oep *)a, *y = (const oep *)b;
  if (x->slack != y->slack) return x->slack < y->slack ? -1 : 1;
  return x->pin < y->pin ? -1 : (x->pin > y->pin);
}

/* Inputs: the STA results of ora_sta for the same netlist.
 * n_sel < 0 selects the violated endpoints.  Up to k paths per endpoint are
 * returned, ordered by (path slack, endpoint pin, rank) and cut to K; paths
 * whose slack is >= slack_limit are not expanded.  For every selected
 * endpoint, ep_next[] receives the slack of its (k+1)-th path (+inf if none),
 * so a caller can tell how far rank k sits from the next path.
 * Outputs: path_ptr[K+1], path_pins[pin_cap], path_ep[K], path_rank[K],
 * path_slack[K]; sel_ep[E] / ep_next[E] for the selected endpoints in
 * selection order.  Returns the number of paths, -1 on a cycle, -2 if an
 * output capacity is too small, -3 if k is outside 1..4000. */
int ora_extract(NETLIST_ARGS, const double *at, const double *rat, const double *dnet,
                const double *darc, const int32_t *crit, int n_sel, int k, int K,
                double slack_limit, int32_t *path_ptr, int32_t *path_pins, int pins_capacity,
                int32_t *path_ep, int32_t *path_rank, double *path_slack, int32_t *sel_ep,
                double *ep_next, int32_t *num_sel) {
  FILL_NETLIST(n);
  oconn c;
  if (k < 1 || k > 4000) return -3;
  if (conn_build(&n, &c) != 0) { conn_free(&c); return -1; }
  int P = num_pins;

  /* endpoint order: (slack, pin id) */
  int E = 0;
  for (int p = 0; p < P; ++p) if (c.role[p] == ROLE_FFD) E++;
  oep *eps = (oep *)malloc(sizeof(oep) * (E > 0 ? E : 1));
  E = 0;
  for (int p = 0; p < P; ++p)
    if (c.role[p] == ROLE_FFD) {
      double s = (at[p] == -INFINITY) ? INFINITY : rat[p] - at[p];
      eps[E].slack = s; eps[E].pin = p; E++;
    }
  qsort(eps, E, sizeof(oep), oep_cmp);
  int nsel = n_sel;
  if (nsel < 0) { nsel = 0; while (nsel < E && eps[nsel].slack < 0) nsel++; }
  if (nsel > E) nsel = E;
  *num_sel = nsel;

  int maxlen = 2 * P + 2;
  opath *paths = NULL;
  int npaths = 0, pcap = 0;
  int32_t *pool = NULL;
  long pool_n = 0, pool_cap = 0;
  int *chain_pins = (int *)malloc(sizeof(int) * maxlen);

  for (int q = 0; q < nsel; ++q) {
    int e = eps[q].pin;
    sel_ep[q] = e;
    ep_next[q] = INFINITY;
    double s_e = eps[q].slack;
    if (s_e == INFINITY) continue;
    oheap h = {0, 0, 0};
    ocand *popped = (ocand *)malloc(sizeof(ocand) * (k + 1));
    int npop = 0;
    long seq = 0;
    ocand root = {0.0, seq++, -1, -1, c.driver[e]};
    heap_push(&h, root);
    while (h.n > 0 && npop < k + 1) {
      ocand p = heap_pop(&h);
      if (s_e + p.cost >= slack_limit) break;
      if (npop == k) { ep_next[q] = s_e + p.cost; break; }
      popped[npop] = p;
      int me = npop++;
      /* children: one more deviation on the arrival-tree chain from p.u */
      int v = p.u;
      while (c.role[v] == ROLE_COUT) {
        int cell = pin_cell[v];
        int b = cell_in_ptr[cell];
        for (int j = 0; b + j < cell_in_ptr[cell + 1]; ++j) {
          if (j == crit[cell]) continue;
          int i = cell_in_pins[b + j];
          if (at[i] == -INFINITY) continue;
          double delta = at[v] - (at[i] + darc[i]);
          ocand ch = {p.cost + delta, seq++, me, i, c.driver[i]};
          heap_push(&h, ch);
        }
        v = c.driver[cell_in_pins[b + crit[cell]]];
      }
    }
    /* materialise each popped path */
    for (int r = 0; r < npop; ++r) {
      int devs[4096];
      int nd = 0;
      for (int a = r; a >= 0 && popped[a].dev >= 0; a = popped[a].parent) devs[nd++] = popped[a].dev;
      add_path(&c, pin_cell, cell_in_ptr, cell_in_pins, at, rat, dnet, darc, crit, e, r, devs, nd, chain_pins,
               &pool, &pool_n, &pool_cap, &paths, &npaths, &pcap);
    }
    free(popped);
    free(h.a);
  }
  qsort(paths, npaths, sizeof(opath), opath_cmp);
  int nout = npaths < K ? npaths : K;
  long total = 0;
  for (int a = 0; a < nout; ++a) total += paths[a].len;
  int rc = nout;
  if (total > pins_capacity) {
    rc = -2;
  } else {
    path_ptr[0] = 0;
    for (int a = 0; a < nout; ++a) {
      memcpy(path_pins + path_ptr[a], pool + paths[a].start, sizeof(int32_t) * paths[a].len);
      path_ptr[a + 1] = path_ptr[a] + paths[a].len;
      path_ep[a] = paths[a].ep;
      path_rank[a] = paths[a].rank;
      path_slack[a] = paths[a].slack;
    }
  }
  free(paths); free(pool); free(chain_pins); free(eps);
  conn_free(&c);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* K worst paths over the whole design                                       */
/* ------------------------------------------------------------------------ */
/* report_timing(K) (Sec. III-B, Table I): the K paths of smallest slack over
 * all endpoints together, however many fall on one endpoint.  Every
 * endpoint's deviation tree is searched by one best-first expansion: a
 * candidate's key is its path slack, the endpoint's slack plus its deviation
 * costs; the roots are the endpoints' critical paths, taken in (slack, pin)
 * order so that equal keys pop in that order.  The first K pops are the
 * answer.  Paths with key >= slack_limit are not reported.
 * Outputs as ora_extract: paths ordered by (recomputed slack, endpoint pin,
 * rank), rank counting the earlier pops at the same endpoint; *next_slack
 * receives the key of the (K+1)-th pop (+inf if there is none).  Returns
 * the number of paths, -1 on a cycle, -2 if pins_capacity is too small. */
typedef struct { double key, cost; long seq; int parent, dev, u, ep; } gcand;
typedef struct { gcand *a; int n, cap; } gheap;

static int gcand_less(const gcand *x, const gcand *y) {
  if (x->key != y->key) return x->key < y->key;
  return x->seq < y->seq;
}
static void gheap_push(gheap *h, gcand v) {
  if (h->n == h->cap) { h->cap = h->cap ? 2 * h->cap : 1024; h->a = (gcand *)realloc(h->a, sizeof(gcand) * h->cap); }
  int i = h->n++;
  h->a[i] = v;
  while (i > 0) {
    int par = (i - 1) / 2;
    if (!gcand_less(&h->a[i], &h->a[par])) break;
    gcand t = h->a[i]; h->a[i] = h->a[par]; h->a[par] = t;
    i = par;
  }
}
static gcand gheap_pop(gheap *h) {
  gcand top = h->a[0];
  h->a[0] = h->a[--h->n];
  int i = 0;
  for (;;) {
    int l = 2 * i + 1, r = l + 1, m = i;
    if (l < h->n && gcand_less(&h->a[l], &h->a[m])) m = l;
    if (r < h->n && gcand_less(&h->a[r], &h->a[m])) m = r;
    if (m == i) break;
    gcand t = h->a[i]; h->a[i] = h->a[m]; h->a[m] = t;
    i = m;
  }
  return top;
}

int ora_report_timing(NETLIST_ARGS, const double *at, const double *rat, const double *dnet,
                      const double *darc, const int32_t *crit, int K, double slack_limit,
                      int32_t *path_ptr, int32_t *path_pins, int pins_capacity, int32_t *path_ep,
                      int32_t *path_rank, double *path_slack, double *next_slack) {
  FILL_NETLIST(n);
  oconn c;
  if (conn_build(&n, &c) != 0) { conn_free(&c); return -1; }
  int P = num_pins;
  int E = 0;
  for (int p = 0; p < P; ++p) if (c.role[p] == ROLE_FFD) E++;
  oep *eps = (oep *)malloc(sizeof(oep) * (E > 0 ? E : 1));
  E = 0;
  for (int p = 0; p < P; ++p)
    if (c.role[p] == ROLE_FFD) {
      double s = (at[p] == -INFINITY) ? INFINITY : rat[p] - at[p];
      eps[E].slack = s; eps[E].pin = p; E++;
    }
  qsort(eps, E, sizeof(oep), oep_cmp);
  int *ep_count = (int *)calloc(P > 0 ? P : 1, sizeof(int));

  gheap h = {0, 0, 0};
  long seq = 0;
  for (int q = 0; q < E; ++q) {
    if (eps[q].slack == INFINITY) continue;
    gcand root = {eps[q].slack, 0.0, seq++, -1, -1, c.driver[eps[q].pin], eps[q].pin};
    gheap_push(&h, root);
  }
  gcand *popped = (gcand *)malloc(sizeof(gcand) * (K > 0 ? K : 1));
  int *rank_of = (int *)malloc(sizeof(int) * (K > 0 ? K : 1));
  int npop = 0;
  *next_slack = INFINITY;
  while (h.n > 0) {
    gcand p = gheap_pop(&h);
    if (p.key >= slack_limit) break;
    if (npop == K) { *next_slack = p.key; break; }
    popped[npop] = p;
    rank_of[npop] = ep_count[p.ep]++;
    int me = npop++;
    double s_e = rat[p.ep] - at[p.ep];
    /* children: one more deviation on the arrival-tree chain from p.u */
    int v = p.u;
    while (c.role[v] == ROLE_COUT) {
      int cell = pin_cell[v];
      int b = cell_in_ptr[cell];
      for (int j = 0; b + j < cell_in_ptr[cell + 1]; ++j) {
        if (j == crit[cell]) continue;
        int i = cell_in_pins[b + j];
        if (at[i] == -INFINITY) continue;
        double delta = at[v] - (at[i] + darc[i]);
        gcand ch = {s_e + (p.cost + delta), p.cost + delta, seq++, me, i, c.driver[i], p.ep};
        gheap_push(&h, ch);
      }
      v = c.driver[cell_in_pins[b + crit[cell]]];
    }
  }
  /* materialise: deviations of pop r, upstream-most first */
  int *devs = (int *)malloc(sizeof(int) * (P > 0 ? P : 1));
  int *chain_pins = (int *)malloc(sizeof(int) * (2 * P + 2));
  opath *paths = NULL;
  int npaths = 0, pcap = 0;
  int32_t *pool = NULL;
  long pool_n = 0, pool_cap = 0;
  for (int r = 0; r < npop; ++r) {
    int nd = 0;
    for (int a = r; a >= 0 && popped[a].dev >= 0; a = popped[a].parent) devs[nd++] = popped[a].dev;
    add_path(&c, pin_cell, cell_in_ptr, cell_in_pins, at, rat, dnet, darc, crit, popped[r].ep, rank_of[r], devs,
             nd, chain_pins, &pool, &pool_n, &pool_cap, &paths, &npaths, &pcap);
  }
  qsort(paths, npaths, sizeof(opath), opath_cmp);
  int rc = npaths;
  if (pool_n > pins_capacity) {
    rc = -2;
  } else {
    path_ptr[0] = 0;
    for (int a = 0; a < npaths; ++a) {
      memcpy(path_pins + path_ptr[a], pool + paths[a].start, sizeof(int32_t) * paths[a].len);
      path_ptr[a + 1] = path_ptr[a] + paths[a].len;
      path_ep[a] = paths[a].ep;
      path_rank[a] = paths[a].rank;
      path_slack[a] = paths[a].slack;
    }
  }
  free(paths); free(pool); free(chain_pins); free(devs); free(popped); free(rank_of); free(h.a);
  free(ep_count); free(eps);
  conn_free(&c);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* pin-pair set and weights (Eq. 9)                                          */
/* ------------------------------------------------------------------------ */
/* The pairs of a path are its net arcs (driver pin, sink pin); a sink pin has
 * exactly one driver, so the sink pin id names the pair.  Paths are taken in
 * the order given (ascending path slack).
 * rule 0 (Eq. 9, stateful): skipped when wns == 0; only paths with negative
 *   slack count; a pair not yet in P enters with w0, a pair already in P gains
 *   w1 * slack / WNS.  in_p[] and w[] carry P across calls.
 * rule 1 (exponential, stateless): w = sum over the paths through the pair of
 *   exp(-slack / max(|WNS|, 1 ps)); P is this call's pairs.
 * in_p[P] (uint8) and w[P] (double) are indexed by sink pin id. */
int ora_pairs(int num_pins, int num_paths, const int32_t *path_ptr, const int32_t *path_pins,
              const double *path_slack, double wns, int rule, double w0, double w1,
              uint8_t *in_p, double *w) {
  if (rule == 1) {
    for (int p = 0; p < num_pins; ++p) { in_p[p] = 0; w[p] = 0.0; }
    double scale = fabs(wns) > 1.0 ? fabs(wns) : 1.0;
    for (int a = 0; a < num_paths; ++a) {
      double contrib = exp(-path_slack[a] / scale);
      for (int q = path_ptr[a] + 1; q < path_ptr[a + 1]; q += 2) {
        int t = path_pins[q];
        in_p[t] = 1;
        w[t] += contrib;
      }
    }
    return 0;
  }
  if (wns == 0.0) return 0;
  for (int a = 0; a < num_paths; ++a) {
    double s = path_slack[a];
    if (!(s < 0)) continue;
    for (int q = path_ptr[a] + 1; q < path_ptr[a + 1]; q += 2) {
      int t = path_pins[q];
      if (!in_p[t]) { in_p[t] = 1; w[t] = w0; }
      else w[t] += w1 * (s / wns);
    }
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* PP loss (Eqs. 8, 10) and its gradient                                     */
/* ------------------------------------------------------------------------ */
/* pairs: sink pin ids pair_sink[Q] with weights pair_w[Q]; the driver is the
 * sink's net driver.  grad_x/grad_y [N] are overwritten; fixed cells and
 * ports get no gradient.  Returns PP via *loss. */
int ora_p2p(NETLIST_ARGS, const uint8_t *cell_fixed, const float *x, const float *y, int num_pairs,
            const int32_t *pair_sink, const double *pair_w, double *loss, double *grad_x,
            double *grad_y) {
  FILL_NETLIST(n);
  oconn c;
  if (conn_build(&n, &c) != 0) { conn_free(&c); return -1; }
  for (int cell = 0; cell < num_cells; ++cell) { grad_x[cell] = 0; grad_y[cell] = 0; }
  double pp = 0.0;
  for (int a = 0; a < num_pairs; ++a) {
    int t = pair_sink[a], s = c.driver[t];
    double xs, ys, xt, yt;
    pin_xy(&n, x, y, s, &xs, &ys);
    pin_xy(&n, x, y, t, &xt, &yt);
    double w = pair_w[a];
    pp += w * ((xs - xt) * (xs - xt) + (ys - yt) * (ys - yt));
    int cs = pin_cell[s], ct = pin_cell[t];
    if (cs >= 0 && !cell_fixed[cs]) { grad_x[cs] += 2 * w * (xs - xt); grad_y[cs] += 2 * w * (ys - yt); }
    if (ct >= 0 && !cell_fixed[ct]) { grad_x[ct] += 2 * w * (xt - xs); grad_y[ct] += 2 * w * (yt - ys); }
  }
  *loss = pp;
  conn_free(&c);
  return 0;
}

/* Pair losses of Sec. III-C other than the quadratic one, over the same
 * pairs: kind 1 = w (|X_s - X_t| + |Y_s - Y_t|), kind 2 = w sqrt((X_s - X_t)^2
 * + (Y_s - Y_t)^2).  Gradient on cell positions: kind 1 gives w sgn(d) per
 * axis (sgn(0) = 0), kind 2 gives w d / L (0 when L = 0). */
int ora_pair_loss(NETLIST_ARGS, const uint8_t *cell_fixed, const float *x, const float *y, int kind,
                  int num_pairs, const int32_t *pair_sink, const double *pair_w, double *loss,
                  double *grad_x, double *grad_y) {
  FILL_NETLIST(n);
  if (kind != 1 && kind != 2) return -3;
  oconn c;
  if (conn_build(&n, &c) != 0) { conn_free(&c); return -1; }
  for (int cell = 0; cell < num_cells; ++cell) { grad_x[cell] = 0; grad_y[cell] = 0; }
  double total = 0.0;
  for (int a = 0; a < num_pairs; ++a) {
    int t = pair_sink[a], s = c.driver[t];
    double xs, ys, xt, yt;
    pin_xy(&n, x, y, s, &xs, &ys);
    pin_xy(&n, x, y, t, &xt, &yt);
    double w = pair_w[a], dx = xs - xt, dy = ys - yt, gxs, gys;
    if (kind == 1) {
      total += w * (fabs(dx) + fabs(dy));
      gxs = w * (double)((dx > 0) - (dx < 0));
      gys = w * (double)((dy > 0) - (dy < 0));
    } else {
      double len = sqrt(dx * dx + dy * dy);
      total += w * len;
      gxs = len > 0 ? w * dx / len : 0.0;
      gys = len > 0 ? w * dy / len : 0.0;
    }
    int cs = pin_cell[s], ct = pin_cell[t];
    if (cs >= 0 && !cell_fixed[cs]) { grad_x[cs] += gxs; grad_y[cs] += gys; }
    if (ct >= 0 && !cell_fixed[ct]) { grad_x[ct] -= gxs; grad_y[ct] -= gys; }
  }
  *loss = total;
  conn_free(&c);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* smoothed TNS and its adjoint                                              */
/* ------------------------------------------------------------------------ */
/* Not in the paper; this is the definition.  Cell-arc delays (darc) and
 * start-point arrivals (at0 at ports and Q pins) are frozen from a hard
 * timing run; net delays follow the positions.
 *   sink t:         A(t) = A(drv) + dnet(t)
 *   comb output o:  A(o) = m + g*ln sum_j exp((a_j - m)/g), a_j = A(i_j) + darc(i_j)
 *   endpoint e:     s(e) = (T - setup) - A(e)
 *   value:          -g * sum_e softplus(-s(e)/g)
 * The gradient on cell positions goes through the net delay of the library's
 * net model as a function of L = |dx| + |dy| (sign(0) = 0).  grad_x/grad_y
 * [N] are overwritten.  gabs_x/gabs_y (optional, [N]) receive, per cell, the
 * sum of the magnitudes of the net-arc terms added into its gradient: the
 * terms of a cell's pins can cancel, so their magnitudes, not the sum, set
 * the scale of rounding error. */
int ora_stns(NETLIST_ARGS, LIB_ARGS, const uint8_t *cell_fixed, const float *x, const float *y,
             const double *at0, const double *darc, double clock_period, double setup,
             double gamma, double *value, double *grad_x, double *grad_y, double *gabs_x, double *gabs_y) {
  FILL_NETLIST(n);
  FILL_LIB(L);
  oconn c;
  if (conn_build(&n, &c) != 0) { conn_free(&c); return -1; }
  int P = num_pins;
  double *A = (double *)malloc(sizeof(double) * P);
  double *Ab = (double *)calloc(P, sizeof(double));
  double *dn = (double *)calloc(P, sizeof(double));
  double *ld = (double *)calloc(P, sizeof(double)); /* loads stay frozen; not used */
  for (int p = 0; p < P; ++p) A[p] = -INFINITY;
  net_pass(&n, &L, x, y, dn, ld);
  for (int q = 0; q < P; ++q) {
    int p = c.topo[q];
    int r = c.role[p];
    if (r == ROLE_PORT || r == ROLE_FFQ) A[p] = at0[p];
    else if (r == ROLE_CIN || r == ROLE_FFD) { if (c.driver[p] >= 0) A[p] = A[c.driver[p]] + dn[p]; }
    else {
      int cell = pin_cell[p];
      double m = -INFINITY;
      for (int k2 = cell_in_ptr[cell]; k2 < cell_in_ptr[cell + 1]; ++k2) {
        int i = cell_in_pins[k2];
        double a = A[i] + darc[i];
        if (a > m) m = a;
      }
      double sum = 0.0;
      for (int k2 = cell_in_ptr[cell]; k2 < cell_in_ptr[cell + 1]; ++k2) {
        int i = cell_in_pins[k2];
        sum += exp((A[i] + darc[i] - m) / gamma);
      }
      A[p] = m + gamma * log(sum);
    }
  }
  double val = 0.0;
  for (int p = 0; p < P; ++p)
    if (c.role[p] == ROLE_FFD && A[p] != -INFINITY) {
      double s = (clock_period - setup) - A[p];
      double z = -s / gamma;
      double sp = (z > 0 ? z : 0.0) + log1p(exp(-fabs(z)));
      val += -gamma * sp;
      Ab[p] = -1.0 / (1.0 + exp(-z));   /* d value / d A(e) = -sigmoid(z) */
    }
  *value = val;
  for (int q = P - 1; q >= 0; --q) {
    int p = c.topo[q];
    int r = c.role[p];
    if (r == ROLE_COUT) {
      int cell = pin_cell[p];
      for (int k2 = cell_in_ptr[cell]; k2 < cell_in_ptr[cell + 1]; ++k2) {
        int i = cell_in_pins[k2];
        Ab[i] += Ab[p] * exp((A[i] + darc[i] - A[p]) / gamma);
      }
    } else if (r == ROLE_CIN || r == ROLE_FFD) {
      if (c.driver[p] >= 0) Ab[c.driver[p]] += Ab[p];
    }
  }
  for (int cell = 0; cell < num_cells; ++cell) { grad_x[cell] = 0; grad_y[cell] = 0; }
  if (gabs_x && gabs_y)
    for (int cell = 0; cell < num_cells; ++cell) { gabs_x[cell] = 0; gabs_y[cell] = 0; }
  otree T;
  if (L.model == 2 && otree_alloc(&T, max_net_pins(net_ptr, num_nets)) != 0) { otree_free(&T); abort(); }
  for (int net = 0; net < num_nets; ++net) {
    if (L.model == 2) {
      /* the net's tree at these positions; the topology is piecewise
       * constant, so only the wire lengths carry the gradient.  With A(v) the
       * adjoint summed over v's subtree and B(v) the sum, over the edges on
       * v's path, of scale r L_e A(child end), the derivative of the value
       * by the length of the edge into v is
       *   scale r (c L_v + C_below(v)) A(v) + c B(parent(v)):
       * the edge's own term and, through C_below, the edges above it. */
      tree_topology(&n, x, y, net, &T);
      tree_elmore(&n, &L, x, y, &T);
      double *Asub = T.aux, *B = T.delay; /* the delays are not needed again */
      for (int i = 0; i <= T.m; ++i) Asub[i] = i > 0 ? Ab[T.pin[i]] : 0.0;
      for (int step = T.m - 1; step >= 0; --step) {
        int j = T.ord[step], p = T.par[j];
        if (p > 0) Asub[p] += Asub[j];
      }
      B[0] = 0.0;
      for (int step = 0; step < T.m; ++step) {
        int j = T.ord[step], p = T.par[j];
        double rs = L.scale * L.r;
        B[j] = B[p] + rs * T.len[j] * Asub[j];
        double gl = rs * (L.c * T.len[j] + T.cd[j]) * Asub[j] + L.c * B[p];
        double xp, yp, xj, yj;
        pin_xy(&n, x, y, T.pin[p], &xp, &yp);
        pin_xy(&n, x, y, T.pin[j], &xj, &yj);
        double dx = xp - xj, dy = yp - yj;
        double gx = gl * ((dx > 0) - (dx < 0)), gy = gl * ((dy > 0) - (dy < 0)); /* d value / d X_parent */
        int cp = pin_cell[T.pin[p]], cj = pin_cell[T.pin[j]];
        if (cp >= 0 && !cell_fixed[cp]) { grad_x[cp] += gx; grad_y[cp] += gy; }
        if (cj >= 0 && !cell_fixed[cj]) { grad_x[cj] -= gx; grad_y[cj] -= gy; }
        if (gabs_x && gabs_y) {
          if (cp >= 0 && !cell_fixed[cp]) { gabs_x[cp] += fabs(gx); gabs_y[cp] += fabs(gy); }
          if (cj >= 0 && !cell_fixed[cj]) { gabs_x[cj] += fabs(gx); gabs_y[cj] += fabs(gy); }
        }
      }
      continue;
    }
    int s = net_pins[net_ptr[net]];
    double xs, ys;
    pin_xy(&n, x, y, s, &xs, &ys);
    int cs = pin_cell[s];
    for (int k2 = net_ptr[net] + 1; k2 < net_ptr[net + 1]; ++k2) {
      int t = net_pins[k2];
      double xt, yt;
      pin_xy(&n, x, y, t, &xt, &yt);
      double len = fabs(xs - xt) + fabs(ys - yt);
      double dx = xs - xt, dy = ys - yt;
      double sx = (dx > 0) - (dx < 0), sy = (dy > 0) - (dy < 0);
      double dd = net_delay_dlen(&L, len, (double)pin_cap[cell_type[pin_cell[t]]]);
      double gx = Ab[t] * dd * sx;   /* d value / d X_s */
      double gy = Ab[t] * dd * sy;
      int ct = pin_cell[t];
      if (cs >= 0 && !cell_fixed[cs]) { grad_x[cs] += gx; grad_y[cs] += gy; }
      if (ct >= 0 && !cell_fixed[ct]) { grad_x[ct] -= gx; grad_y[ct] -= gy; }
      if (gabs_x && gabs_y) {
        if (cs >= 0 && !cell_fixed[cs]) { gabs_x[cs] += fabs(gx); gabs_y[cs] += fabs(gy); }
        if (ct >= 0 && !cell_fixed[ct]) { gabs_x[ct] += fabs(gx); gabs_y[ct] += fabs(gy); }
      }
    }
  }
  if (L.model == 2) otree_free(&T);
  free(A); free(Ab); free(dn); free(ld);
  conn_free(&c);
  return 0;
}

/* The topology of net model 2: parent[p] is the pin that p hangs from in its
 * net's spanning tree (the driver for the pins joined to it directly), -1 at
 * drivers and at pins on no net. */
int ora_rc_tree(NETLIST_ARGS, const float *x, const float *y, int32_t *parent) {
  FILL_NETLIST(n);
  otree T;
  if (otree_alloc(&T, max_net_pins(net_ptr, num_nets)) != 0) { otree_free(&T); return -1; }
  for (int p = 0; p < num_pins; ++p) parent[p] = -1;
  for (int net = 0; net < num_nets; ++net) {
    tree_topology(&n, x, y, net, &T);
    for (int i = 1; i <= T.m; ++i) parent[T.pin[i]] = T.pin[T.par[i]];
  }
  otree_free(&T);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* rise / fall timing                                                        */
/* ------------------------------------------------------------------------ */
/* A fuller timing model around the paper's (its timer, Sec. II-B / III-B,
 * times both transitions of every pin; the paper fixes neither a library nor
 * this detail, so the definition here is the contract).  Every pin carries
 * two transitions, rise (index 0) and fall (index 1).  The arcs of a cell
 * type have a unateness:
 *   0 positive: an input rise causes an output rise, a fall a fall;
 *   1 negative: an input rise causes an output fall, a fall a rise;
 *   2 non-unate: either input transition causes either output transition.
 * The output rise of type t is looked up in the rise tables (delay_lut /
 * slew_lut), the output fall in delay_fall / slew_fall; a flip-flop's Q rises
 * and falls by its clock-to-Q tables at the clock slew.  A net carries a
 * transition unchanged, with the same delay and degradation either way.
 *   sink t:           AT_y(t) = AT_y(drv) + dnet(t), slew_y(t) from slew_y(drv)
 *   comb output o, transition x:
 *     AT_x(o)   = max over inputs j and input transitions y that cause x of
 *                 AT_y(i_j) + D_x(slew_y(i_j), load(o))
 *     crit_x(o) = the first (j, y) attaining it, j ascending, rise before fall
 *     slew_x(o) = max over the same (j, y) of S_x(slew_y(i_j), load(o))
 *   D pin e:          slack_y(e) = (T - setup) - AT_y(e); the endpoint's slack
 *                     is the smaller of the two (Eqs. 3-4 over endpoints)
 *   required:         RAT_y(e) = T - setup at a D pin; RAT_y(i_j) = min over
 *                     the x that y causes of RAT_x(o) - D_x(slew_y(i_j), load);
 *                     RAT_y(drv) = min over sinks of RAT_y(t) - dnet(t)
 * Arrays indexed [2 * pin + transition]; crit [2 * cell + x] = 2 j + y (-1 for
 * flip-flops and unreached outputs); ep_slack [P] the endpoint slack at D pins
 * (+inf elsewhere); summary[3] = {WNS, TNS, violated endpoints}. */
static int rf_causes(int unate, int y, int x) {
  if (unate == 2) return 1;
  return unate == 0 ? y == x : y != x;
}

int ora_sta_rf(NETLIST_ARGS, LIB_ARGS, const float *delay_fall, const float *slew_fall, const int32_t *unate,
               const float *x, const float *y, double clock_period, double setup, double input_slew,
               double clock_slew, double *at, double *slew, double *rat, double *slack, double *ep_slack,
               int32_t *crit, double *summary) {
  FILL_NETLIST(n);
  FILL_LIB(L);
  oconn c;
  if (conn_build(&n, &c) != 0) { conn_free(&c); return -1; }
  int P = num_pins, N = num_cells;
  double *dnet = (double *)calloc(P, sizeof(double));
  double *load = (double *)calloc(P, sizeof(double));
  for (int q = 0; q < 2 * P; ++q) { at[q] = -INFINITY; slew[q] = 0.0; rat[q] = INFINITY; slack[q] = INFINITY; }
  for (int p = 0; p < P; ++p) ep_slack[p] = INFINITY;
  for (int q = 0; q < 2 * N; ++q) crit[q] = -1;
  const float *dtab[2] = {delay_lut, delay_fall}, *stab[2] = {slew_lut, slew_fall};

  net_pass(&n, &L, x, y, dnet, load);

  for (int q = 0; q < P; ++q) {
    int p = c.topo[q];
    int role = c.role[p];
    if (role == ROLE_PORT) {
      for (int tr = 0; tr < 2; ++tr) { at[2 * p + tr] = 0.0; slew[2 * p + tr] = input_slew; }
    } else if (role == ROLE_FFQ) {
      int type = cell_type[pin_cell[p]];
      for (int tr = 0; tr < 2; ++tr) {
        at[2 * p + tr] = lut_eval(&L, dtab[tr], type, clock_slew, load[p]);
        slew[2 * p + tr] = lut_eval(&L, stab[tr], type, clock_slew, load[p]);
      }
    } else if (role == ROLE_CIN || role == ROLE_FFD) {
      int d = c.driver[p];
      if (d >= 0)
        for (int tr = 0; tr < 2; ++tr) {
          at[2 * p + tr] = at[2 * d + tr] + dnet[p];
          slew[2 * p + tr] = sink_slew(&L, slew[2 * d + tr], dnet[p]);
        }
    } else { /* ROLE_COUT */
      int cell = pin_cell[p], type = cell_type[cell];
      for (int xo = 0; xo < 2; ++xo) {
        double best = -INFINITY, sl = 0.0;
        int arg = -1;
        for (int k = cell_in_ptr[cell]; k < cell_in_ptr[cell + 1]; ++k) {
          int i = cell_in_pins[k];
          for (int yi = 0; yi < 2; ++yi) {
            if (!rf_causes(unate[type], yi, xo) || at[2 * i + yi] == -INFINITY) continue;
            double a = at[2 * i + yi] + lut_eval(&L, dtab[xo], type, slew[2 * i + yi], load[p]);
            double so = lut_eval(&L, stab[xo], type, slew[2 * i + yi], load[p]);
            if (a > best) { best = a; arg = 2 * (k - cell_in_ptr[cell]) + yi; }
            if (so > sl) sl = so;
          }
        }
        at[2 * p + xo] = best;
        slew[2 * p + xo] = sl;
        crit[2 * cell + xo] = arg;
      }
    }
  }

  double req = clock_period - setup, wns = 0.0, tns = 0.0;
  int nfail = 0;
  for (int p = 0; p < P; ++p) {
    if (c.role[p] != ROLE_FFD) continue;
    double worst = INFINITY;
    for (int tr = 0; tr < 2; ++tr) {
      rat[2 * p + tr] = req;
      if (at[2 * p + tr] == -INFINITY) continue;
      double sl = req - at[2 * p + tr];
      if (sl < worst) worst = sl;
    }
    ep_slack[p] = worst;
    if (worst < 0) { ++nfail; tns += worst; if (worst < wns) wns = worst; }
  }
  summary[0] = wns; summary[1] = tns; summary[2] = nfail;

  for (int q = P - 1; q >= 0; --q) {
    int p = c.topo[q];
    int role = c.role[p];
    if (role == ROLE_FFD) continue;
    if (role == ROLE_CIN) {
      int cell = pin_cell[p], type = cell_type[cell], o = cell_out_pin[cell];
      for (int yi = 0; yi < 2; ++yi) {
        double r = INFINITY;
        for (int xo = 0; xo < 2; ++xo) {
          if (!rf_causes(unate[type], yi, xo) || rat[2 * o + xo] == INFINITY) continue;
          double v = rat[2 * o + xo] - lut_eval(&L, dtab[xo], type, slew[2 * p + yi], load[o]);
          if (v < r) r = v;
        }
        rat[2 * p + yi] = r;
      }
    } else { /* a driver: port, comb output or Q */
      int net = c.net_of[p];
      for (int tr = 0; tr < 2; ++tr) {
        double r = INFINITY;
        if (net >= 0)
          for (int k = net_ptr[net] + 1; k < net_ptr[net + 1]; ++k) {
            int t = net_pins[k];
            if (rat[2 * t + tr] == INFINITY) continue;
            double v = rat[2 * t + tr] - dnet[t];
            if (v < r) r = v;
          }
        rat[2 * p + tr] = r;
      }
    }
  }
  for (int q = 0; q < 2 * P; ++q)
    slack[q] = (rat[q] == INFINITY || at[q] == -INFINITY) ? INFINITY : rat[q] - at[q];
  free(dnet); free(load);
  conn_free(&c);
  return 0;
}

/* report_timing_endpoint(n, 1) under rise / fall timing: endpoints ordered by
 * (endpoint slack, pin id), the first n (n < 0: the violated ones) with finite
 * slack, cut to K; each endpoint's path ends in its worse transition (rise on
 * a tie) and follows crit back to a start point.  Path pins are written start
 * to end (path_ptr [K+1], path_pins / path_tran [K * (2 depth + 2)]), with
 * the endpoint pin and the path slack (= the endpoint's slack).  Returns the
 * number of paths. */
typedef struct { double slack; int pin; } orfep;
static int orfep_cmp(const void *a, const void *b) {
  const orfep *u = (const orfep *)a, *v = (const orfep *)b;
  if (u->slack < v->slack) return -1;
  if (u->slack > v->slack) return 1;
  return u->pin - v->pin;
}

int ora_extract_rf(NETLIST_ARGS, const double *rf_slack, const double *ep_slack, const int32_t *crit, int n_sel,
                   int K, int32_t *path_ptr, int32_t *path_pins, int32_t *path_tran, double *path_slack,
                   int32_t *path_ep) {
  FILL_NETLIST(n);
  oconn c;
  if (conn_build(&n, &c) != 0) { conn_free(&c); return -1; }
  int P = num_pins;
  orfep *eps = (orfep *)malloc(sizeof(orfep) * (P > 0 ? P : 1));
  int ne = 0, nviol = 0;
  for (int p = 0; p < P; ++p)
    if (c.role[p] == ROLE_FFD && ep_slack[p] != INFINITY) {
      eps[ne].slack = ep_slack[p];
      eps[ne].pin = p;
      if (ep_slack[p] < 0) ++nviol;
      ++ne;
    }
  qsort(eps, ne, sizeof(orfep), orfep_cmp);
  int m = n_sel < 0 ? nviol : (n_sel < ne ? n_sel : ne);
  if (m > K) m = K;
  int *rev = (int *)malloc(sizeof(int) * 2 * (P + 1));
  int *revt = (int *)malloc(sizeof(int) * 2 * (P + 1));
  int w = 0;
  path_ptr[0] = 0;
  for (int q = 0; q < m; ++q) {
    int e = eps[q].pin;
    int tr = rf_slack[2 * e] <= rf_slack[2 * e + 1] ? 0 : 1;
    int len = 0, p = e;
    for (;;) {
      rev[len] = p; revt[len] = tr; ++len;
      int d = c.driver[p];
      if (d < 0) break;
      rev[len] = d; revt[len] = tr; ++len;
      if (c.role[d] != ROLE_COUT) break;
      int cell = pin_cell[d];
      int cr = crit[2 * cell + tr];
      if (cr < 0) break;
      p = cell_in_pins[cell_in_ptr[cell] + cr / 2];
      tr = cr % 2;
    }
    for (int i = 0; i < len; ++i) { path_pins[w + i] = rev[len - 1 - i]; path_tran[w + i] = revt[len - 1 - i]; }
    w += len;
    path_ptr[q + 1] = w;
    path_slack[q] = eps[q].slack;
    path_ep[q] = e;
  }
  free(rev); free(revt); free(eps);
  conn_free(&c);
  return m;
}

/* ------------------------------------------------------------------------ */
/* weighted-average wirelength                                               */
/* ------------------------------------------------------------------------ */
/* Per net and axis, over all pins of the net (driver and sinks, ports too):
 *   WA = sum x e^{x/g} / sum e^{x/g} - sum x e^{-x/g} / sum e^{-x/g},
 * evaluated with the exponents shifted by the net's max (resp. min).  The
 * value is summed over nets and both axes; grad_x/grad_y [N] are overwritten
 * with d value / d cell position (fixed cells and ports get none). */
/* dabs (optional) receives |first term| + |second term| of each pin's
 * derivative: the two cancel for coincident pins, so their magnitudes, not
 * the difference, set the scale of rounding error. */
static double wa_axis(int cnt, const double *v, double g, double *dv, double *dabs) {
  double mx = v[0], mn = v[0];
  for (int i = 1; i < cnt; ++i) { if (v[i] > mx) mx = v[i]; if (v[i] < mn) mn = v[i]; }
  double sa = 0, sxa = 0, sb = 0, sxb = 0;
  for (int i = 0; i < cnt; ++i) {
    double a = exp((v[i] - mx) / g), b = exp(-(v[i] - mn) / g);
    sa += a; sxa += v[i] * a; sb += b; sxb += v[i] * b;
  }
  double fp = sxa / sa, fm = sxb / sb;
  for (int i = 0; i < cnt; ++i) {
    double a = exp((v[i] - mx) / g), b = exp(-(v[i] - mn) / g);
    double t1 = a / sa * (1.0 + (v[i] - fp) / g), t2 = b / sb * (1.0 - (v[i] - fm) / g);
    dv[i] = t1 - t2;
    /* magnitudes of the four summands a/sa, a/sa (v - fp)/g, b/sb, b/sb (v - fm)/g */
    if (dabs) dabs[i] = a / sa * (1.0 + fabs(v[i] - fp) / g) + b / sb * (1.0 + fabs(v[i] - fm) / g);
  }
  return fp - fm;
}

/* gabs_x/gabs_y (optional, [N]) receive, per cell, the sum over its pins of
 * the magnitudes of the summands of each pin's derivative: the scale of the
 * rounding error of the gradient. */
int ora_wa(NETLIST_ARGS, const uint8_t *cell_fixed, const float *x, const float *y, double gamma,
           double *value, double *grad_x, double *grad_y, double *gabs_x, double *gabs_y) {
  FILL_NETLIST(n);
  (void)cell_type; (void)cell_in_ptr; (void)cell_in_pins; (void)cell_out_pin; (void)cell_is_ff;
  int maxdeg = 1;
  for (int net = 0; net < num_nets; ++net) {
    int d = net_ptr[net + 1] - net_ptr[net];
    if (d > maxdeg) maxdeg = d;
  }
  double *vx = (double *)malloc(sizeof(double) * maxdeg), *vy = (double *)malloc(sizeof(double) * maxdeg);
  double *gx = (double *)malloc(sizeof(double) * maxdeg), *gy = (double *)malloc(sizeof(double) * maxdeg);
  double *ax = (double *)malloc(sizeof(double) * maxdeg), *ay = (double *)malloc(sizeof(double) * maxdeg);
  for (int cell = 0; cell < num_cells; ++cell) {
    grad_x[cell] = 0; grad_y[cell] = 0;
    if (gabs_x) gabs_x[cell] = 0;
    if (gabs_y) gabs_y[cell] = 0;
  }
  double total = 0.0;
  for (int net = 0; net < num_nets; ++net) {
    int b = net_ptr[net], cnt = net_ptr[net + 1] - b;
    for (int i = 0; i < cnt; ++i) pin_xy(&n, x, y, net_pins[b + i], &vx[i], &vy[i]);
    total += wa_axis(cnt, vx, gamma, gx, ax) + wa_axis(cnt, vy, gamma, gy, ay);
    for (int i = 0; i < cnt; ++i) {
      int cell = pin_cell[net_pins[b + i]];
      if (cell >= 0 && !cell_fixed[cell]) {
        grad_x[cell] += gx[i]; grad_y[cell] += gy[i];
        if (gabs_x) gabs_x[cell] += ax[i];
        if (gabs_y) gabs_y[cell] += ay[i];
      }
    }
  }
  *value = total;
  free(vx); free(vy); free(gx); free(gy); free(ax); free(ay);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* placement loop: bin density and one Nesterov step                        */
/* ------------------------------------------------------------------------ */
/* The paper's loop (Sec. IV) is DREAMPlace's: wirelength plus lambda times a
 * density term (Eq. 1) plus beta * PP (Eq. 6), minimised with Nesterov's
 * method.  The density term is not restated in the paper; this is the
 * definition used here.
 *
 * The die [x0, x0 + gx*bw) x [y0, y0 + gy*bh) is cut into gx x gy bins, bin
 * (i, j) stored at j*gx + i.  Cell c spreads its area a_c as a Gaussian
 * centred on its position with standard deviations bw and bh, integrated
 * over each bin and cut to the (2R+1) x (2R+1) bins around the bin holding
 * the cell (its indices clamped into the grid).  Mass the window puts off the
 * die is reflected back in at the die's edges (mirror images of the Gaussian,
 * as the Neumann boundary of DREAMPlace's electrostatic density does), so
 * that an edge does not look emptier than the interior:
 *   D(i, j) = sum_c a_c Wx_c(i) Wy_c(j),
 *   Wx_c(i) = sum over window bins v that fold onto i of
 *             Phi((x0 + (v+1) bw - x_c) / bw) - Phi((x0 + v bw - x_c) / bw),
 * Phi the standard normal distribution function, a bin v < 0 folding onto
 * -1 - v and a bin v >= gx onto 2 gx - 1 - v (repeatedly, for grids narrower
 * than the window).  With cap = target*bw*bh:
 *   value    = sum_b max(0, D_b - cap)^2
 *   overflow = sum_b max(0, D_b - cap) / sum_c a_c
 *   d value / d x_c = sum_b 2 max(0, D_b - cap) a_c Wx_c'(i) Wy_c(j)
 * (likewise in y), Wx_c'(i) the same fold of (phi(lower) - phi(upper)) / bw,
 * phi the standard normal density at a window bin's standardised edges; the
 * window stays put while the cell stays in its bin.  Fixed cells count in D and get
 * no gradient.  grad_x / grad_y [num_cells] are overwritten. */
static double std_cdf(double z) { return 0.5 * erfc(-z / sqrt(2.0)); }
static double std_pdf(double z) { return exp(-0.5 * z * z) / sqrt(2.0 * acos(-1.0)); }

static int fold_bin(int v, int g) {
  while (v < 0 || v >= g) v = v < 0 ? -1 - v : 2 * g - 1 - v;
  return v;
}

/* folded window weights of one axis: wt[k] and dt[k] for grid bin
 * b - R + k (0 when off the grid), from a cell at standardised position
 * (v - v0) / w relative to its window bin b */
static void axis_weights(double v, double v0, double w, int g, int b, int R, double *wt, double *dt) {
  for (int k = 0; k < 2 * R + 1; ++k) { wt[k] = 0.0; dt[k] = 0.0; }
  for (int k = 0; k < 2 * R + 1; ++k) {
    int u = b - R + k;
    double lo = (v0 + u * w - v) / w, hi = (v0 + (u + 1) * w - v) / w;
    int f = fold_bin(u, g);
    int kf = f - (b - R);
    wt[kf] += std_cdf(hi) - std_cdf(lo);
    dt[kf] += (std_pdf(lo) - std_pdf(hi)) / w;
  }
}

static int bin_of(double v, double v0, double w, int g) {
  double q = floor((v - v0) / w);
  if (q < 0) q = 0;
  if (q > g - 1) q = g - 1;
  return (int)q;
}

int ora_density(int num_cells, const float *x, const float *y, const float *area, const uint8_t *cell_fixed,
                double x0, double y0, double bw, double bh, int gx, int gy, int R, double target,
                double *dens, double *value, double *overflow, double *grad_x, double *grad_y) {
  double cap = target * bw * bh, total_area = 0.0;
  int K = 2 * R + 1;
  double *wx = (double *)malloc(sizeof(double) * K), *dx = (double *)malloc(sizeof(double) * K);
  double *wy = (double *)malloc(sizeof(double) * K), *dy = (double *)malloc(sizeof(double) * K);
  for (int b = 0; b < gx * gy; ++b) dens[b] = 0.0;
  for (int c = 0; c < num_cells; ++c) {
    int bx = bin_of(x[c], x0, bw, gx), by = bin_of(y[c], y0, bh, gy);
    total_area += area[c];
    axis_weights(x[c], x0, bw, gx, bx, R, wx, dx);
    axis_weights(y[c], y0, bh, gy, by, R, wy, dy);
    for (int kj = 0; kj < K; ++kj) {
      int j = by - R + kj;
      if (j < 0 || j >= gy) continue;
      for (int ki = 0; ki < K; ++ki) {
        int i = bx - R + ki;
        if (i < 0 || i >= gx) continue;
        dens[j * gx + i] += area[c] * wx[ki] * wy[kj];
      }
    }
  }
  double val = 0.0, ovf = 0.0;
  for (int b = 0; b < gx * gy; ++b) {
    double o = dens[b] > cap ? dens[b] - cap : 0.0;
    val += o * o;
    ovf += o;
  }
  *value = val;
  *overflow = total_area > 0 ? ovf / total_area : 0.0;
  for (int c = 0; c < num_cells; ++c) {
    grad_x[c] = 0.0; grad_y[c] = 0.0;
    if (cell_fixed && cell_fixed[c]) continue;
    int bx = bin_of(x[c], x0, bw, gx), by = bin_of(y[c], y0, bh, gy);
    axis_weights(x[c], x0, bw, gx, bx, R, wx, dx);
    axis_weights(y[c], y0, bh, gy, by, R, wy, dy);
    for (int kj = 0; kj < K; ++kj) {
      int j = by - R + kj;
      if (j < 0 || j >= gy) continue;
      for (int ki = 0; ki < K; ++ki) {
        int i = bx - R + ki;
        if (i < 0 || i >= gx) continue;
        double o = dens[j * gx + i] - cap;
        if (o <= 0) continue;
        grad_x[c] += 2.0 * o * area[c] * dx[ki] * wy[kj];
        grad_y[c] += 2.0 * o * area[c] * wx[ki] * dy[kj];
      }
    }
  }
  free(wx); free(dx); free(wy); free(dy);
  return 0;
}

/* One step of Nesterov's method as ePlace applies it to placement (Lu et
 * al., TODAES 2015), on the 2n coordinates (x then y) of n cells:
 *   g      = the gradient at v_k divided per cell by max(1, pdiv_c)
 *            (a diagonal preconditioner; frozen cells: 0),
 *   alpha  = |v_k - v_{k-1}| / |g - g_{k-1}| (the Lipschitz prediction),
 *            or alpha0 when first != 0 or that ratio is not a positive number,
 *   u_{k+1} = clamp(v_k - alpha g),
 *   v_{k+1} = clamp(u_{k+1} + coef (u_{k+1} - u_k)),
 * clamp into [xlo, xhi] x [ylo, yhi].  Frozen cells keep v and u.  The
 * arrays v, u, vp (v_{k-1}), gp (g_{k-1}) are updated in place: afterwards
 * v = v_{k+1}, u = u_{k+1}, vp = v_k, gp = g.  Returns alpha in *alpha_out. */
static double clampd(double v, double lo, double hi) { return v < lo ? lo : (v > hi ? hi : v); }

int ora_nesterov(int n, const uint8_t *frozen, const double *pdiv, const double *gx, const double *gy,
                 double *vx, double *vy, double *ux, double *uy, double *vpx, double *vpy, double *gpx,
                 double *gpy, double coef, double alpha0, int first, double xlo, double xhi, double ylo,
                 double yhi, double *alpha_out) {
  double *qx = (double *)malloc(sizeof(double) * (n > 0 ? n : 1));
  double *qy = (double *)malloc(sizeof(double) * (n > 0 ? n : 1));
  double dv = 0.0, dg = 0.0;
  for (int c = 0; c < n; ++c) {
    double s = pdiv[c] > 1.0 ? pdiv[c] : 1.0;
    qx[c] = frozen[c] ? 0.0 : gx[c] / s;
    qy[c] = frozen[c] ? 0.0 : gy[c] / s;
    if (frozen[c]) continue;
    dv += (vx[c] - vpx[c]) * (vx[c] - vpx[c]) + (vy[c] - vpy[c]) * (vy[c] - vpy[c]);
    dg += (qx[c] - gpx[c]) * (qx[c] - gpx[c]) + (qy[c] - gpy[c]) * (qy[c] - gpy[c]);
  }
  double alpha = alpha0;
  if (!first && dg > 0.0) {
    double a = sqrt(dv) / sqrt(dg);
    if (a > 0.0 && isfinite(a)) alpha = a;
  }
  for (int c = 0; c < n; ++c) {
    if (frozen[c]) { vpx[c] = vx[c]; vpy[c] = vy[c]; gpx[c] = 0.0; gpy[c] = 0.0; continue; }
    double nux = clampd(vx[c] - alpha * qx[c], xlo, xhi), nuy = clampd(vy[c] - alpha * qy[c], ylo, yhi);
    double nvx = clampd(nux + coef * (nux - ux[c]), xlo, xhi), nvy = clampd(nuy + coef * (nuy - uy[c]), ylo, yhi);
    vpx[c] = vx[c]; vpy[c] = vy[c];
    gpx[c] = qx[c]; gpy[c] = qy[c];
    ux[c] = nux; uy[c] = nuy;
    vx[c] = nvx; vy[c] = nvy;
  }
  *alpha_out = alpha;
  free(qx); free(qy);
  return 0;
}
