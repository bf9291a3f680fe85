// Stage-cell programs (Algorithm 1's nested loops, Section 6's stage
// operations): a pattern is a short list of cells, each one loop over the
// windowed neighbours of an already bound vertex (for_all), or a probe of
// the edges between two bound vertices (the intersection of a neighbour
// list with one vertex, found by binary search in the neighbour-sorted
// in-rows, as in the 4-cycle example).  A cell may skip neighbours equal to
// bound vertices (differentiate, difference with a singleton), keep each
// neighbour once (a stage's output is a vertex set), and folds what its
// inner cells return: a sum, or how many of its bindings reach a threshold
// (Section 4's threshold on how many take part); a loop whose parent only
// asks whether it reaches a threshold stops once it does.  One lane
// interprets the program for one anchor with an explicit stack of cell
// states, so a new pattern needs no new kernel.
#include "api_internal.h"

#define A_TRY(x)                    \
  do {                              \
    amlm_status st_ = (x);          \
    if (st_ != AMLM_OK) return st_; \
  } while (0)

namespace {

constexpr uint32_t kProgMaxCells = 6;
constexpr uint8_t kOpForOut = AMLM_CELL_FOR_OUT, kOpProbe = AMLM_CELL_PROBE;
constexpr uint8_t kTloWindow = AMLM_T_WINDOW, kThiIncl = AMLM_T_THROUGH;
constexpr uint8_t kAggSum = AMLM_AGG_SUM, kAggAtLeastK = AMLM_AGG_AT_LEAST_K;
constexpr uint32_t kVarU = 0, kVarV = 1;

struct CellDev {
  uint8_t op, node, peer, tlo, tref, thi, skip, distinct, agg;
  uint32_t thr;
};

struct Prog {
  CellDev c[kProgMaxCells];
  uint32_t n;
};

struct Frame {
  uint32_t pos, end;   // FOR: current position and end of the slice
  int32_t lo, hi;      // the cell's window [lo, hi]
  uint32_t acc;        // the fold so far
  int32_t t_edge;      // time of the edge bound by this cell's current iteration
};

__device__ __forceinline__ uint32_t sat_add(uint32_t a, uint32_t b, uint32_t cap) {
  const uint64_t s = (uint64_t)a + b;
  return s > cap ? cap : (uint32_t)s;
}

__global__ __launch_bounds__(256) void k_interp(GraphView g, Prog P, int64_t delta, uint32_t k, uint32_t ceil,
                                                 uint32_t *out) {
  const uint32_t e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= g.E) return;
  const uint32_t u = g.src[e], v = g.dst[e];
  if (u == v) {  // self-loops take part in nothing
    out[e] = 0;
    return;
  }
  const int32_t t = g.t[e];
  const int64_t lo64 = (int64_t)t - delta;
  const int32_t wlo = lo64 < 0 ? 0 : (int32_t)lo64;  // relative times are >= 0
  uint32_t var[2 + kProgMaxCells];
  for (uint32_t b = 0; b < 2 + kProgMaxCells; b++) var[b] = 0xffffffffu;
  var[kVarU] = u;
  var[kVarV] = v;
  Frame F[kProgMaxCells];
  // value returned by cell i for its current parent binding
  auto window = [&](const CellDev &c, int32_t &lo, int32_t &hi) {
    lo = c.tlo == kTloWindow ? wlo : F[c.tref].t_edge + 1;
    hi = c.thi == kThiIncl ? t : t - 1;
  };
  auto probe = [&](const CellDev &c) -> uint32_t {
    // edges var[node] -> var[peer] with time in the window: the peer's
    // neighbour-sorted in-row, keys (source, time)
    int32_t lo, hi;
    window(c, lo, hi);
    if (lo > hi) return 0u;
    const uint32_t a = var[c.node], b = var[c.peer];
    if (a == b) return 0u;
    const uint32_t rs = g.in_ptr[b], re = g.in_ptr[b + 1];
    const uint32_t q0 = lower_bound_u64(g.inn_key, rs, re, nbr_key(a, lo));
    const uint32_t q1 = lower_bound_u64(g.inn_key, q0, re, nbr_key(a, hi) + 1);
    const uint32_t n = q1 - q0;
    return c.distinct ? (n > 0 ? 1u : 0u) : n;
  };
  auto open = [&](uint32_t i) -> bool {
    // set up FOR cell i for the current bindings; false if its slice is empty
    const CellDev &c = P.c[i];
    Frame &f = F[i];
    window(c, f.lo, f.hi);
    f.acc = 0;
    if (f.lo > f.hi) {
      f.pos = f.end = 0;
      return false;
    }
    const uint32_t x = var[c.node];
    if (c.op == kOpForOut) {
      const uint32_t rs = g.out_ptr[x], re = g.out_ptr[x + 1];
      f.pos = lower_bound_i32(g.out_t, rs, re, f.lo);
      f.end = upper_bound_i32(g.out_t, f.pos, re, f.hi);
    } else {
      const uint32_t rs = g.in_ptr[x], re = g.in_ptr[x + 1];
      f.pos = lower_bound_i32(g.in_t, rs, re, f.lo);
      f.end = upper_bound_i32(g.in_t, f.pos, re, f.hi);
    }
    if (i + 1 == P.n && c.agg == kAggSum && !c.distinct && !c.skip) {
      // an innermost plain count: the slice's length, without walking it
      f.acc = min(f.end - f.pos, ceil);
      f.pos = f.end;
    }
    return true;
  };
  // fold one child value into cell i
  auto fold = [&](uint32_t i, uint32_t val) {
    const CellDev &c = P.c[i];
    const uint32_t thr = c.agg == kAggAtLeastK ? k : c.thr;
    if (c.agg == kAggSum) F[i].acc = sat_add(F[i].acc, val, ceil);
    else F[i].acc = sat_add(F[i].acc, val >= thr ? 1u : 0u, ceil);
  };
  // Early exit (Algorithm 1's break): every fold only grows, so once cell
  // d's value reaches the threshold its parent compares it with, more
  // bindings cannot change what the parent counts
  auto enough = [&](int d) -> bool {
    if (d == 0) return false;
    const CellDev &pc = P.c[d - 1];
    if (pc.agg == kAggSum) return false;
    const uint32_t thr = pc.agg == kAggAtLeastK ? k : pc.thr;
    return F[d].acc >= thr;
  };
  uint32_t result;
  if (P.c[0].op == kOpProbe) {
    result = probe(P.c[0]);
    out[e] = result < ceil ? result : ceil;
    return;
  }
  int d = 0;
  open(0);
  for (;;) {
    Frame &f = F[d];
    const CellDev &c = P.c[d];
    if (f.pos >= f.end) {
      // cell d is done: fold it into its parent, or finish
      if (d == 0) break;
      const uint32_t val = f.acc;
      d--;
      fold(d, val);
      F[d].pos++;
      continue;
    }
    if (enough(d)) {
      f.pos = f.end;
      continue;
    }
    const uint32_t p = f.pos;
    uint32_t w;
    bool take;
    if (c.op == kOpForOut) {
      w = g.out_nbr[p];
      f.t_edge = g.out_t[p];
      // vertex set: the neighbour's first edge inside the window
      take = !c.distinct || g.out_prv[p] < f.lo;
    } else {
      w = g.in_nbr[p];
      f.t_edge = g.in_t[p];
      // vertex set: the neighbour's last edge inside the window
      take = !c.distinct || g.in_nxt[p] > f.hi;
    }
    for (uint32_t b = 0; take && b < 2 + kProgMaxCells; b++)
      if (((c.skip >> b) & 1u) && var[b] == w) take = false;
    if (!take) {
      f.pos++;
      continue;
    }
    var[2 + d] = w;
    if ((uint32_t)d + 1 == P.n) {
      fold(d, 1u);
      f.pos++;
      continue;
    }
    const CellDev &nc = P.c[d + 1];
    if (nc.op == kOpProbe) {
      // a probe is always the last cell
      fold(d, probe(nc));
      f.pos++;
      continue;
    }
    d++;
    open(d);
  }
  result = F[0].acc;
  out[e] = result < ceil ? result : ceil;
}

}  // namespace

extern "C" amlm_status amlm_mine_program(amlm_graph *g, const amlm_cell *cells, uint32_t n_cells, int64_t delta,
                                         uint32_t k, uint32_t *out_dev, void *hip_stream) {
  if (!g || !cells) {
    set_error("null argument");
    return AMLM_E_INVALID;
  }
  if (n_cells == 0 || n_cells > kProgMaxCells) {
    set_error("a program has 1 to 6 cells");
    return AMLM_E_INVALID;
  }
  if (delta < 0 || k == 0) {
    set_error("delta must be >= 0 and k >= 1");
    return AMLM_E_INVALID;
  }
  if (g->batch.n) {
    set_error("programs run on single graphs");
    return AMLM_E_INVALID;
  }
  Prog P{};
  P.n = n_cells;
  for (uint32_t i = 0; i < n_cells; i++) {
    const amlm_cell &c = cells[i];
    const uint32_t bound = 2 + i;  // u, v and the vertices of cells 0 .. i-1
    auto fail = [&](const char *what) {
      set_error("cell " + std::to_string(i) + ": " + what);
      return AMLM_E_INVALID;
    };
    if (c.op > AMLM_CELL_PROBE) return fail("unknown operation");
    if (c.op == AMLM_CELL_PROBE && i + 1 != n_cells) return fail("a probe must be the last cell");
    if (c.node >= bound || (c.op == AMLM_CELL_PROBE && c.peer >= bound)) return fail("vertex not bound yet");
    if (c.tlo > AMLM_T_AFTER || c.thi > AMLM_T_BEFORE) return fail("unknown time bound");
    if (c.tlo == AMLM_T_AFTER && (c.tref >= i || cells[c.tref].op == AMLM_CELL_PROBE))
      return fail("the time reference must be an earlier loop cell");
    if (c.skip >> bound) return fail("skips a vertex not bound yet");
    if (c.agg > AMLM_AGG_AT_LEAST_K) return fail("unknown fold");
    P.c[i] = CellDev{c.op, c.node, c.peer, c.tlo, c.tref, c.thi, c.skip, c.distinct, c.agg, c.threshold};
  }
  A_TRY(sticky_check(g));
  if (g->E == 0) return AMLM_OK;
  if (!out_dev) {
    set_error("null output");
    return AMLM_E_INVALID;
  }
  hipStream_t s = (hipStream_t)hip_stream;
  hipLaunchKernelGGL(k_interp, dim3((uint32_t)((g->E + 255) / 256)), dim3(256), 0, s, graph_view(g), P, delta, k,
                     g->ceiling, out_dev);
  if (hipGetLastError() != hipSuccess) {
    set_error("k_interp launch failed");
    return sticky_note(g, AMLM_E_DEVICE);
  }
  return AMLM_OK;
}
