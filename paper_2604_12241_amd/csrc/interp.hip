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
// asks whether it reaches a threshold stops once it does.  The program is
// interpreted with an explicit stack of cell states, so a new pattern needs
// no new kernel: one lane per anchor for a probe or a single loop; one wave
// per anchor when the first two cells are loops (or a loop and a probe),
// with the first loop's bindings over the lanes and the second loop's
// bindings flattened over them.
#include <algorithm>

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
constexpr uint32_t kCtrInterp = 41;   // claim counter word in the mining scratch
constexpr uint32_t kInterpWaves = 16; // waves per CU in the grid of k_interp_wave

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

// One anchor's interpretation state: the bound vertices (u, v, then one per
// loop cell) and the loop cells' frames.
struct Ctx {
  uint32_t var[2 + kProgMaxCells];
  Frame F[kProgMaxCells];
  int32_t t, wlo;
};

__device__ __forceinline__ void cell_window(const CellDev &c, const Ctx &x, int32_t &lo, int32_t &hi) {
  lo = c.tlo == kTloWindow ? x.wlo : x.F[c.tref].t_edge + 1;
  hi = c.thi == kThiIncl ? x.t : x.t - 1;
}

// Blocked Bloom filter over vertex hashes (vhash): the top bits pick a word,
// four 5-bit fields of the low bits pick its bits.
constexpr uint32_t kPFiltLog2 = 9, kPFiltWords = 1u << kPFiltLog2;  // 2 KB
constexpr int kPFiltShift = 32 - (int)kPFiltLog2;
__device__ __forceinline__ uint32_t pfilt_bits(uint32_t h) {
  return (1u << (h & 31)) | (1u << ((h >> 5) & 31)) | (1u << ((h >> 10) & 31)) | (1u << ((h >> 15) & 31));
}

// edges var[node] -> var[peer] inside the cell's window: a key range of the
// peer's neighbour-sorted in-row (keys (source, time)).  filt (may be NULL):
// a filter of the peer's in-neighbours over a window containing the cell's;
// a vertex it rejects has no such edge.
__device__ uint32_t cell_probe(const GraphView &g, const CellDev &c, const Ctx &x, const uint32_t *filt) {
  int32_t lo, hi;
  cell_window(c, x, lo, hi);
  if (lo > hi) return 0u;
  const uint32_t a = x.var[c.node], b = x.var[c.peer];
  if (a == b) return 0u;
  if (filt) {
    const uint32_t h = vhash(a), fb = pfilt_bits(h);
    if ((filt[h >> kPFiltShift] & fb) != fb) return 0u;
  }
  const uint32_t rs = g.in_ptr[b], re = g.in_ptr[b + 1];
  const uint32_t q0 = lower_bound_u64(g.inn_key, rs, re, nbr_key(a, lo));
  const uint32_t q1 = lower_bound_u64(g.inn_key, q0, re, nbr_key(a, hi) + 1);
  const uint32_t n = q1 - q0;
  return c.distinct ? (n > 0 ? 1u : 0u) : n;
}

// the slice [pos, end) of loop cell i for the current bindings
__device__ void cell_slice(const GraphView &g, const CellDev &c, Ctx &x, uint32_t i) {
  Frame &f = x.F[i];
  cell_window(c, x, f.lo, f.hi);
  f.acc = 0;
  if (f.lo > f.hi) {
    f.pos = f.end = 0;
    return;
  }
  const uint32_t w = x.var[c.node];
  if (c.op == kOpForOut) {
    const uint32_t rs = g.out_ptr[w], re = g.out_ptr[w + 1];
    f.pos = lower_bound_i32(g.out_t, rs, re, f.lo);
    f.end = upper_bound_i32(g.out_t, f.pos, re, f.hi);
  } else {
    const uint32_t rs = g.in_ptr[w], re = g.in_ptr[w + 1];
    f.pos = lower_bound_i32(g.in_t, rs, re, f.lo);
    f.end = upper_bound_i32(g.in_t, f.pos, re, f.hi);
  }
}

// an innermost loop that only counts its slice
__device__ __forceinline__ bool plain_count(const Prog &P, uint32_t i) {
  const CellDev &c = P.c[i];
  return i + 1 == P.n && c.agg == kAggSum && !c.distinct && !c.skip;
}

// what a child value adds to loop cell c's fold: the value (sum) or whether
// it reaches the threshold
__device__ __forceinline__ uint32_t contribution(const CellDev &c, uint32_t val, uint32_t k) {
  if (c.agg == kAggSum) return val;
  return val >= (c.agg == kAggAtLeastK ? k : c.thr) ? 1u : 0u;
}

// the edge at position p of loop cell d: binds its neighbour (w) and time;
// false if the cell skips it
__device__ bool cell_bind(const GraphView &g, const CellDev &c, Ctx &x, uint32_t d, uint32_t p, uint32_t &w) {
  Frame &f = x.F[d];
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
    if (((c.skip >> b) & 1u) && x.var[b] == w) take = false;
  return take;
}

// The value of cell d0 for the current bindings of cells 0 .. d0 - 1, with
// an explicit stack of the deeper loop cells.  A loop whose parent only asks
// whether it reaches a threshold stops once it does (Algorithm 1's break:
// every fold only grows, so more bindings cannot change what the parent
// counts).
__device__ uint32_t run_from(const GraphView &g, const Prog &P, uint32_t k, uint32_t ceil, Ctx &x, uint32_t d0,
                             const uint32_t *filt) {
  if (P.c[d0].op == kOpProbe) return cell_probe(g, P.c[d0], x, filt);
  auto open = [&](uint32_t i) {
    cell_slice(g, P.c[i], x, i);
    if (plain_count(P, i)) {  // the slice's length, without walking it
      x.F[i].acc = min(x.F[i].end - x.F[i].pos, ceil);
      x.F[i].pos = x.F[i].end;
    }
  };
  auto fold = [&](uint32_t i, uint32_t val) { x.F[i].acc = sat_add(x.F[i].acc, contribution(P.c[i], val, k), ceil); };
  auto enough = [&](uint32_t d) -> bool {
    if (d == 0) return false;
    const CellDev &pc = P.c[d - 1];
    return pc.agg != kAggSum && x.F[d].acc >= (pc.agg == kAggAtLeastK ? k : pc.thr);
  };
  uint32_t d = d0;
  open(d0);
  for (;;) {
    Frame &f = x.F[d];
    const CellDev &c = P.c[d];
    if (f.pos >= f.end || enough(d)) {
      // cell d is done: fold it into its parent, or finish
      if (d == d0) break;
      const uint32_t val = f.acc;
      d--;
      fold(d, val);
      x.F[d].pos++;
      continue;
    }
    uint32_t w;
    if (!cell_bind(g, c, x, d, f.pos, w)) {
      f.pos++;
      continue;
    }
    x.var[2 + d] = w;
    if (d + 1 == P.n) {
      fold(d, 1u);
      f.pos++;
      continue;
    }
    if (P.c[d + 1].op == kOpProbe) {  // a probe is always the last cell
      fold(d, cell_probe(g, P.c[d + 1], x, filt));
      f.pos++;
      continue;
    }
    d++;
    open(d);
  }
  return x.F[d0].acc;
}

__device__ void ctx_init(const GraphView &g, Ctx &x, uint32_t e, int64_t delta) {
  for (uint32_t b = 0; b < 2 + kProgMaxCells; b++) x.var[b] = 0xffffffffu;
  x.var[kVarU] = g.src[e];
  x.var[kVarV] = g.dst[e];
  x.t = g.t[e];
  const int64_t lo64 = (int64_t)x.t - delta;
  x.wlo = lo64 < 0 ? 0 : (int32_t)lo64;  // relative times are >= 0
}

// One lane per anchor: programs whose first cell is a probe, or a single loop.
__global__ __launch_bounds__(256) void k_interp(GraphView g, Prog P, int64_t delta, uint32_t k, uint32_t ceil,
                                                 uint32_t *out) {
  const uint32_t e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= g.E) return;
  if (g.src[e] == g.dst[e]) {  // self-loops take part in nothing
    out[e] = 0;
    return;
  }
  Ctx x;
  ctx_init(g, x, e, delta);
  const uint32_t r = run_from(g, P, k, ceil, x, 0, nullptr);
  out[e] = r < ceil ? r : ceil;
}

// last slot j in [0, n) with pref[j] <= f (pref[0] = 0 <= f)
__device__ __forceinline__ uint32_t slot_of(const uint32_t *pref, uint32_t n, uint32_t f) {
  uint32_t lo = 0, hi = n;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (pref[mid] <= f) lo = mid; else hi = mid;
  }
  return lo;
}

constexpr uint32_t kWaveAnchors = 4;  // anchors per claim of a wave

// One wave per anchor, for programs whose first two cells are loops (or a
// loop and a probe): the first loop's bindings over the lanes, 64 at a time;
// the second loop's bindings of those 64 flattened over the lanes, each
// evaluating the deeper cells on its own; per-binding folds in LDS.  Folds
// are sums of non-negative terms saturating at the ceiling, so their order
// does not matter.
__global__ __launch_bounds__(64) void k_interp_wave(GraphView g, Prog P, int64_t delta, uint32_t k, uint32_t ceil,
                                                    uint32_t *out, uint32_t *claim) {
  __shared__ unsigned long long acc1[AMLM_WAVE];
  __shared__ uint32_t b_w0[AMLM_WAVE], b_pos1[AMLM_WAVE], b_pref[AMLM_WAVE];
  __shared__ int32_t b_t0[AMLM_WAVE], b_lo1[AMLM_WAVE], b_hi1[AMLM_WAVE];
  __shared__ uint32_t pfilt[kPFiltWords];
  const uint32_t lane = lane_id();
  const CellDev &c0 = P.c[0], &c1 = P.c[1];
  const bool probe1 = c1.op == kOpProbe;
  const bool plain1 = !probe1 && plain_count(P, 1);
  // a last probe into u or v (fixed for the anchor): filter the peer's
  // in-neighbours over the anchor's window [t - delta, t], which contains
  // every window the probe can have
  const CellDev &cl = P.c[P.n - 1];
  const bool pf = cl.op == kOpProbe && cl.peer <= kVarV;
  for (;;) {
    uint32_t e0 = 0;
    if (lane == 0) e0 = atomicAdd(claim, kWaveAnchors);
    e0 = __shfl(e0, 0, AMLM_WAVE);
    if (e0 >= g.E) return;
    const uint32_t e1 = e0 + kWaveAnchors < g.E ? e0 + kWaveAnchors : g.E;
    for (uint32_t e = e0; e < e1; e++) {
      if (g.src[e] == g.dst[e]) {
        if (lane == 0) out[e] = 0;
        continue;
      }
      Ctx x;
      ctx_init(g, x, e, delta);
      cell_slice(g, c0, x, 0);
      const uint32_t pos0 = x.F[0].pos, end0 = x.F[0].end;
      const uint32_t *filt = nullptr;
      if (pf && pos0 < end0) {
        const uint32_t peer = x.var[cl.peer], prs = g.in_ptr[peer], pre = g.in_ptr[peer + 1];
        const uint32_t f0 = lower_bound_i32(g.in_t, prs, pre, x.wlo), f1 = upper_bound_i32(g.in_t, f0, pre, x.t);
        __syncthreads();
        for (uint32_t w = lane; w < kPFiltWords; w += AMLM_WAVE) pfilt[w] = 0u;
        __syncthreads();
        for (uint32_t q = f0 + lane; q < f1; q += AMLM_WAVE) {
          const uint32_t h = g.in_h[q];
          atomicOr(&pfilt[h >> kPFiltShift], pfilt_bits(h));
        }
        __syncthreads();
        filt = pfilt;
      }
      unsigned long long acc0 = 0;  // this lane's share of cell 0's fold
      for (uint32_t b = pos0; b < end0; b += AMLM_WAVE) {
        const uint32_t p = b + lane;
        uint32_t w0 = 0;
        const bool take = p < end0 && cell_bind(g, c0, x, 0, p, w0);
        if (take) x.var[2] = w0;
        if (P.n == 1) {
          if (take) acc0 += contribution(c0, 1u, k);
          continue;
        }
        if (probe1) {
          if (take) acc0 += contribution(c0, cell_probe(g, c1, x, filt), k);
          continue;
        }
        uint32_t len1 = 0;
        if (take) {
          cell_slice(g, c1, x, 1);
          len1 = x.F[1].end - x.F[1].pos;
        }
        if (plain1) {
          if (take) acc0 += contribution(c0, min(len1, ceil), k);
          continue;
        }
        // the second loop's bindings of this group, flattened over the lanes
        const uint64_t tmask = __ballot(take);
        const uint32_t nb = (uint32_t)__popcll(tmask);
        const uint32_t slot = (uint32_t)__popcll(tmask & lanemask_lt());
        const uint32_t incl = wave_incl_scan(take ? len1 : 0u);
        const uint32_t total = __shfl(incl, AMLM_WAVE - 1, AMLM_WAVE);
        if (take) {
          b_w0[slot] = w0;
          b_t0[slot] = x.F[0].t_edge;
          b_pos1[slot] = x.F[1].pos;
          b_pref[slot] = incl - len1;
          b_lo1[slot] = x.F[1].lo;
          b_hi1[slot] = x.F[1].hi;
          acc1[slot] = 0ull;
        }
        __syncthreads();
        if (nb) {
          for (uint32_t h0 = 0; h0 < total; h0 += AMLM_WAVE) {
            const uint32_t h = h0 + lane;
            if (h >= total) continue;
            const uint32_t j = slot_of(b_pref, nb, h);
            Ctx y = x;
            y.var[2] = b_w0[j];
            y.F[0].t_edge = b_t0[j];
            y.F[1].lo = b_lo1[j];
            y.F[1].hi = b_hi1[j];
            uint32_t w1;
            if (!cell_bind(g, c1, y, 1, b_pos1[j] + (h - b_pref[j]), w1)) continue;
            y.var[3] = w1;
            const uint32_t val = P.n == 2 ? 1u : run_from(g, P, k, ceil, y, 2, filt);
            atomicAdd(&acc1[j], (unsigned long long)contribution(c1, val, k));
          }
        }
        __syncthreads();
        if (take) {
          const unsigned long long v1 = acc1[slot];
          acc0 += contribution(c0, v1 < ceil ? (uint32_t)v1 : ceil, k);
        }
        __syncthreads();
      }
      for (int o = AMLM_WAVE / 2; o > 0; o >>= 1) acc0 += __shfl_xor(acc0, o, AMLM_WAVE);
      if (lane == 0) out[e] = acc0 < ceil ? (uint32_t)acc0 : ceil;
    }
  }
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
  if (P.c[0].op != kOpProbe && n_cells >= 2) {
    // nested loops: one wave per anchor (a claim counter in the mining scratch)
    A_TRY(sticky_note(g, alloc_mine_scratch(g)));
    uint32_t *claim = g->ms.ctr + kCtrInterp;
    if (launch_fill_u32(claim, 0, 1, s) != hipSuccess) {
      set_error("k_interp_wave set-up failed");
      return sticky_note(g, AMLM_E_DEVICE);
    }
    const uint32_t blocks = (uint32_t)std::min<uint64_t>((uint64_t)device_info().num_cu * kInterpWaves,
                                                         (g->E + kWaveAnchors - 1) / kWaveAnchors);
    hipLaunchKernelGGL(k_interp_wave, dim3(blocks), dim3(AMLM_WAVE), 0, s, graph_view(g), P, delta, k, g->ceiling,
                       out_dev, claim);
  } else {
    hipLaunchKernelGGL(k_interp, dim3((uint32_t)((g->E + 255) / 256)), dim3(256), 0, s, graph_view(g), P, delta, k,
                       g->ceiling, out_dev);
  }
  if (hipGetLastError() != hipSuccess) {
    set_error("k_interp launch failed");
    return sticky_note(g, AMLM_E_DEVICE);
  }
  return AMLM_OK;
}
