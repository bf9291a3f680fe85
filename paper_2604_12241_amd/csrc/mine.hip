// Mining kernels.
//
//  k_anchor_out / k_anchor_in
//            one lane per anchor, in CSR then CSC order: window bounds by
//            galloping and binary search (Find_Starting_Edge, Algorithm 1),
//            FAN_OUT / FAN_IN, the size of the sender set S(e) when its
//            window slice is short, and the classification of the anchor into
//            the scatter-gather list (CSC order: grouped by v, time-sorted) and
//            the cycle list (edge-id order).
//  k_sg      scatter-gather / gather-scatter (Section 5 scatter-gather
//            decomposition, Section 6 compiled example).  A wave takes up to
//            64 anchors; each run of anchors into the same v is a segment
//            whose gather side (v's in-neighbours over the segment's window)
//            is staged once in an LDS Bloom filter.  Senders are found lane-
//            parallel over the anchors' sender windows; each sender's
//            out-window is scanned with lanes flattened over (sender, entry)
//            pairs; filter hits are queued and confirmed in batches by binary
//            search in the neighbour-sorted in-index.
//  k_cyc     bounded time-respecting cycle search (Section 5 cycle
//            decomposition; Section 6 4-cycle example: expansion, then the
//            closing intersection by binary search over sorted neighbour
//            lists).  A wave takes 64 anchors and searches depth first over
//            frames of up to 64 partial paths; each frame's time slices are
//            flattened over the lanes and the surviving paths are compacted
//            into the next frame with ballot + popcount.
#include "costmodel.h"
#include "mine.h"

namespace {

__device__ __forceinline__ int32_t window_lo(int32_t t, int64_t delta) {
  int64_t lo = (int64_t)t - delta;
  return lo < -1 ? -1 : (int32_t)lo;
}

__device__ __forceinline__ uint32_t rfl(uint32_t x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ uint32_t ceil_log2_u32(uint32_t x) { return x <= 1 ? 0u : 32u - (uint32_t)__clz(x - 1); }
__device__ __forceinline__ int32_t rfl(int32_t x) { return (int32_t)__builtin_amdgcn_readfirstlane((uint32_t)x); }

// ------------------------------------------------------------------ anchor passes
// Pass 1 runs over the CSR (one lane per out-entry: anchor e = (u -> v, t) in
// u's row), so neighbouring lanes search the same rows: FAN_OUT inside u's
// own row by galloping from the anchor's position, and u's sender window
// [lo, t) in u's in-row.  Pass 2 runs over the CSC: FAN_IN inside v's row,
// and v's out-window [lo, t) (the first hop of a cycle).
__global__ __launch_bounds__(256) void k_anchor_out(MineParams mp, uint8_t *flags_sg, uint4 *sg_win, uint32_t *feat) {
  const GraphView &g = mp.g;
  uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= g.Ev) return;
  uint32_t eid = g.out_eid[p];
  if (eid < mp.anchor_lo || eid >= mp.anchor_hi) return;  // context edge (incremental mining)
  uint32_t u = g.out_src[p], v = g.out_nbr[p];
  int32_t t = g.out_t[p];
  int32_t lo = window_lo(t, delta_of(mp, u));
  const uint32_t k = k_of(mp, u);
  uint32_t rs = g.out_ptr[u], re = g.out_ptr[u + 1];
  uint32_t fan_out = 0;
  if (mp.col_fo >= 0 || mp.col_do >= 0 || feat) {
    uint32_t hi = gallop_upper_right(g.out_t, p + 1, re, t);
    uint32_t lb = gallop_lower_left(g.out_t, rs, p, lo);
    fan_out = hi - lb;
    if (mp.col_fo >= 0) mp.counts[(uint64_t)mp.col_fo * mp.stride + eid] = min(fan_out, mp.ceil);
    if (mp.col_do >= 0) {
      // distinct destinations: the window's first edge of each (u, d) pair
      uint32_t nd = 0;
      for (uint32_t q = lb; q < hi; q++) nd += g.out_prv[q] < lo;
      mp.counts[(uint64_t)mp.col_do * mp.stride + eid] = min(nd, mp.ceil);
      if (mp.work) atomicAdd(&mp.work[kWorkIo * mp.stride + eid], (unsigned long long)kAlgElem * fan_out);
    }
  }
  if (mp.col_sg >= 0 || mp.col_gs >= 0) {
    uint32_t cs = g.in_ptr[u], ce = g.in_ptr[u + 1];
    uint32_t p1 = lower_bound_i32(g.in_t, cs, ce, t);
    uint32_t p0 = gallop_lower_left(g.in_t, cs, p1, lo);
    bool item = false;
    if (p1 > p0) {
      if (p1 - p0 <= kAnchorScanCap) {
        uint32_t ns = 0;
        for (uint32_t j = p0; j < p1; j++) ns += (g.in_nbr[j] != v) & (g.in_nxt[j] >= t);
        if (ns > 0) {
          if (k == 1) {
            // every sender has u as its first intermediate and v is always a
            // scatter destination after the first gather: SG_1 = GS_1 = |S|
            if (mp.col_sg >= 0) mp.counts[(uint64_t)mp.col_sg * mp.stride + eid] = min(ns, mp.ceil);
            if (mp.col_gs >= 0) mp.counts[(uint64_t)mp.col_gs * mp.stride + eid] = min(ns, mp.ceil);
          } else {
            item = true;
          }
        }
      } else {
        item = true;
      }
    }
    if (item) {
      // scatter-gather anchors are listed in CSC order: grouped by v, time-sorted
      uint32_t q = g.pos_in[eid];
      uint8_t fl = kFlagSG;
      if (mp.col_gs >= 0 && k >= 2) {
        // gather-scatter's destination side: u's first edges to each d in
        // (tau, t], tau = the earliest sender edge (senders exclude v)
        uint32_t j = p0;
        while (j < p1 && g.in_nbr[j] == v) j++;
        if (j < p1) {
          const int32_t tau = g.in_t[j];
          const uint32_t d0 = gallop_lower_left(g.out_t, rs, p, tau + 1);
          const uint32_t d1 = gallop_upper_right(g.out_t, p + 1, re, t);
          uint32_t nd = 0, c = d0;
          for (; c < d1 && nd < k; c++) nd += g.out_prv[c] <= tau;
          if (nd >= k) fl |= kFlagGsDest;
          if (mp.work) atomicAdd(&mp.work[kWorkSgImpl * mp.stride + eid], (unsigned long long)(kBytesScatterEntry * (c - d0)));
        }
      }
      flags_sg[q] = fl;
      sg_win[q].x = p0;
      sg_win[q].y = p1;
      if (feat) {
        uint32_t *o = feat + (uint64_t)q * kMlpRaw;
        o[0] = fan_out;
        o[2] = p1 - p0;
        o[4] = re - rs;
        o[5] = ce - cs;
      }
    }
  }
}

__global__ __launch_bounds__(256) void k_anchor_in(MineParams mp, uint8_t *flags_sg, uint8_t *flags_cy,
                                                   uint4 *sg_win, uint32_t *feat) {
  const GraphView &g = mp.g;
  uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= g.Ev) return;
  uint32_t eid = g.in_eid[q];
  if (eid < mp.anchor_lo || eid >= mp.anchor_hi) return;
  uint32_t v = g.in_dst[q], u = g.in_nbr[q];
  int32_t t = g.in_t[q];
  int32_t lo = window_lo(t, delta_of(mp, u));
  const bool is_sg = (mp.col_sg >= 0 || mp.col_gs >= 0) && flags_sg[q];
  if (mp.col_fi >= 0 || mp.col_di >= 0 || is_sg) {
    uint32_t rs = g.in_ptr[v], re = g.in_ptr[v + 1];
    uint32_t hi = gallop_upper_right(g.in_t, q + 1, re, t);
    uint32_t lb = gallop_lower_left(g.in_t, rs, q, lo);
    if (mp.col_fi >= 0) mp.counts[(uint64_t)mp.col_fi * mp.stride + eid] = min(hi - lb, mp.ceil);
    if (mp.col_di >= 0) {
      // distinct sources: the last edge of each (m, v) pair at or before t
      uint32_t nd = 0;
      for (uint32_t j = lb; j < hi; j++) nd += g.in_nxt[j] > t;
      mp.counts[(uint64_t)mp.col_di * mp.stride + eid] = min(nd, mp.ceil);
      if (mp.work) atomicAdd(&mp.work[kWorkIo * mp.stride + eid], (unsigned long long)kAlgElem * (hi - lb));
    }
    if (is_sg) {
      sg_win[q].z = lb;
      sg_win[q].w = hi;
      // short windows: look for an in-neighbour other than u (longer ones
      // are taken to have one)
      if (hi - lb <= kAnchorScanCap) {
        bool other = false;
        for (uint32_t j = lb; j < hi; j++) other |= g.in_nbr[j] != u;
        if (!other) flags_sg[q] |= kFlagSgNoJoin;
      }
      if (feat) {
        feat[(uint64_t)q * kMlpRaw + 1] = hi - lb;
        feat[(uint64_t)q * kMlpRaw + 7] = re - rs;
      }
    }
  }
  if ((flags_cy && mp.col_cyc >= 0) || (is_sg && feat)) {
    uint32_t vs = g.out_ptr[v], ve = g.out_ptr[v + 1];
    uint32_t q1 = lower_bound_i32(g.out_t, vs, ve, t);
    // any order: v's first hop may also leave at time t itself
    const uint32_t qc = mp.cyc_any ? upper_bound_i32(g.out_t, q1, ve, t) : q1;
    if (flags_cy && mp.col_cyc >= 0 && qc > vs && g.out_t[qc - 1] >= lo) flags_cy[eid] = kFlagCYC;
    if (is_sg && feat) {
      uint32_t q0 = gallop_lower_left(g.out_t, vs, q1, lo);
      feat[(uint64_t)q * kMlpRaw + 3] = q1 - q0;
      feat[(uint64_t)q * kMlpRaw + 6] = ve - vs;
    }
  }
}

// Cycle roots alone (the cycle search then starts before the anchor passes):
// the same test as k_anchor_in's, v has a first hop inside the window.
__global__ __launch_bounds__(256) void k_cyc_roots(MineParams mp, uint8_t *flags_cy) {
  const GraphView &g = mp.g;
  uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= g.Ev) return;
  uint32_t eid = g.in_eid[q];
  if (eid < mp.anchor_lo || eid >= mp.anchor_hi) return;
  uint32_t v = g.in_dst[q], u = g.in_nbr[q];
  int32_t t = g.in_t[q];
  int32_t lo = window_lo(t, delta_of(mp, u));
  uint32_t vs = g.out_ptr[v], ve = g.out_ptr[v + 1];
  uint32_t q1 = lower_bound_i32(g.out_t, vs, ve, t);
  const uint32_t qc = mp.cyc_any ? upper_bound_i32(g.out_t, q1, ve, t) : q1;
  if (qc > vs && g.out_t[qc - 1] >= lo) flags_cy[eid] = kFlagCYC;
}

// Phase order for one (anchor, sender) pair, scanning the sender's
// out-slice [b, b + n) in time order: every chosen scatter leg (u's
// included) must come before every chosen gather leg, the anchor being u's.
// Each intermediate m != u is tried once, at its first edge in the window
// (time f_m), against its last edge into v at or before t (time g_m, found
// in v's neighbour-sorted row [vrs, vre)); a split time tau then exists for
// the intervals seen so far iff the (k-1)-th largest g among them exceeds
// max(f of the latest interval, f_u).  The k - 1 largest g are kept in
// registers (k <= kPhaseKMax).  Returns whether the pair qualifies; *scanned
// gets the elements scanned (all of them when it does not).  `filter`
// (may be NULL) rejects m that are surely not in v's gather window.
template <class Filter>
__device__ bool sg_phase_pair(const MineParams &mp, uint32_t s, uint32_t u, int32_t lo, int32_t t, uint32_t k,
                              uint32_t b, uint32_t n, uint32_t vrs, uint32_t vre, const Filter &filter,
                              uint32_t *scanned) {
  const GraphView &g = mp.g;
  *scanned = n;
  if (k <= 1) {
    *scanned = 0;
    return true;
  }
  // f_u: the sender's first edge to u inside the window
  const uint32_t urs = g.in_ptr[u], ure = g.in_ptr[u + 1];
  const uint64_t ku = nbr_key(s, lo < 0 ? 0 : lo);
  const uint32_t qu = ku ? upper_bound_u64_interp(g.inn_key, urs, ure, ku - 1) : urs;
  int32_t f_u = t;
  if (qu < ure && (uint32_t)(g.inn_key[qu] >> 32) == s) f_u = (int32_t)(uint32_t)g.inn_key[qu];
  int32_t top[kPhaseKMax - 1];
#pragma unroll
  for (uint32_t i = 0; i < kPhaseKMax - 1; i++) top[i] = AMLM_INT_MIN;
  const uint32_t need = k - 1;
  for (uint32_t i = 0; i < n; i++) {
    const uint32_t pos = b + i;
    const uint32_t m = g.out_nbr[pos];
    if (m == u || g.out_prv[pos] >= lo) continue;  // u, or not m's first edge in the window
    if (!filter(g.out_h[pos])) continue;
    const uint32_t q = upper_bound_u64_interp(g.inn_key, vrs, vre, nbr_key(m, t));
    if (q == vrs) continue;
    const uint64_t kk = g.inn_key[q - 1];
    const int32_t gm = (int32_t)(uint32_t)kk, fm = g.out_t[pos];
    if ((uint32_t)(kk >> 32) != m || gm < lo || fm >= gm) continue;
    // insert gm into the descending list of the k - 1 largest
    int32_t x = gm;
#pragma unroll
    for (uint32_t j = 0; j < kPhaseKMax - 1; j++) {
      if (j < need && x > top[j]) {
        const int32_t y = top[j];
        top[j] = x;
        x = y;
      }
    }
    int32_t kth = top[0];
#pragma unroll
    for (uint32_t j = 1; j < kPhaseKMax - 1; j++)
      if (j == need - 1) kth = top[j];
    if (kth > max(fm, f_u)) {
      *scanned = i + 1;
      return true;
    }
  }
  return false;
}

// ------------------------------------------------------------------ algorithmic bytes
// The method's algorithmic bytes per anchor, by a canonical procedure that
// does not depend on how the kernels below organise their work (nothing is
// reused across anchors; an element is a neighbour id and a time):
//   row kWorkIo:  the edge's (src, dst, ts) and its output counts;
//   row kWorkSg:  the sender scan of u's in-window [t - delta, t); for each
//                 distinct sender s, min(n_s, |IN(v) in [t - delta, t]|)
//                 elements, n_s being how far a scan of s's out-window in
//                 (time, id) order gets before k - 1 intermediates other than
//                 u have qualified (the whole window if fewer do): the
//                 compiled scatter-gather intersection, bounded by its smaller
//                 side (Section 6's degree-ordered intersection) and ended
//                 early (Algorithm 1's break); and, for GS_k when |S| >= k, the
//                 scan of u's out-row after tau until k distinct destinations;
//   row kWorkCyc: counted by k_cyc (slices scanned at depths 0 .. L-3, one
//                 closing search at depth L-2, 8 bytes per credited edge).
// Accounting only (amlm_mine_work): one wave per anchor, one lane per sender
// edge, each lane scanning its sender's window serially.
__global__ __launch_bounds__(256) void k_alg_io(MineParams mp, uint32_t ncols) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= mp.g.E || i < mp.anchor_lo || i >= mp.anchor_hi) return;
  mp.work[kWorkIo * mp.stride + i] = kAlgEdgeRow + (unsigned long long)kAlgCount * ncols;
}

__global__ __launch_bounds__(256) void k_alg_sg(MineParams mp) {
  const GraphView &g = mp.g;
  const uint32_t lane = lane_id();
  const uint32_t nw = gridDim.x * (blockDim.x / AMLM_WAVE);
  for (uint32_t q = blockIdx.x * (blockDim.x / AMLM_WAVE) + threadIdx.x / AMLM_WAVE; q < g.Ev; q += nw) {
    const uint32_t eid = g.in_eid[q];
    if (eid < mp.anchor_lo || eid >= mp.anchor_hi) continue;
    const uint32_t v = g.in_dst[q], u = g.in_nbr[q];
    const int32_t t = g.in_t[q];
    const int32_t lo = window_lo(t, delta_of(mp, u));
    const uint32_t k = k_of(mp, u);
    const uint32_t cs = g.in_ptr[u], ce = g.in_ptr[u + 1];
    const uint32_t p1 = lower_bound_i32(g.in_t, cs, ce, t);
    const uint32_t p0 = lower_bound_i32(g.in_t, cs, p1, lo);
    const uint32_t vrs = g.in_ptr[v], vre = g.in_ptr[v + 1];
    // |IN(v) in [lo, t]|: the anchor sits at q inside v's row
    const uint32_t r = upper_bound_i32(g.in_t, q + 1, vre, t) - lower_bound_i32(g.in_t, vrs, q, lo);
    uint32_t ns = 0;
    unsigned long long join = 0;
    for (uint32_t j = p0 + lane; j < p1; j += AMLM_WAVE) {
      const uint32_t s = g.in_nbr[j];
      if (s == v || g.in_nxt[j] < t) continue;  // not the last s -> u edge before t
      ns++;
      if (mp.col_sg < 0 || k < 2) continue;
      const uint32_t rs = g.out_ptr[s], re = g.out_ptr[s + 1];
      const uint32_t b = lower_bound_i32(g.out_t, rs, re, lo);
      const uint32_t n_full = lower_bound_i32(g.out_t, b, re, t) - b;
      uint32_t n_s = min(n_full, r), found = 0;
      if (mp.sg_phase) {
        uint32_t scanned;
        auto any = [](uint32_t) { return true; };
        (void)sg_phase_pair(mp, s, u, lo, t, k, b, n_full, vrs, vre, any, &scanned);
        join += min(scanned, r);
        continue;
      }
      for (uint32_t i = 0; i < min(n_full, r); i++) {
        const uint32_t pos = b + i, m = g.out_nbr[pos];
        if (m == u || g.out_prv[pos] >= lo) continue;  // u, or not the first s -> m edge of the window
        const uint32_t qk = upper_bound_u64_interp(g.inn_key, vrs, vre, nbr_key(m, t));
        if (qk == vrs) continue;
        const uint64_t kk = g.inn_key[qk - 1];  // the last m -> v edge at or before t, if any
        const int32_t tb = (int32_t)(uint32_t)kk;
        if ((uint32_t)(kk >> 32) != m || !(mp.sg_unordered ? tb >= lo : tb > g.out_t[pos])) continue;
        if (++found == k - 1) {
          n_s = i + 1;
          break;
        }
      }
      join += n_s;
    }
    for (int o = 32; o > 0; o >>= 1) {
      ns += __shfl_xor(ns, o, AMLM_WAVE);
      join += __shfl_xor(join, o, AMLM_WAVE);
    }
    if (lane != 0 || p1 == p0) continue;
    unsigned long long w = (unsigned long long)kAlgElem * (p1 - p0) + (unsigned long long)kAlgElem * join;
    if (mp.col_gs >= 0 && ns >= k) {
      // tau: the earliest sender edge (senders exclude v); then u's
      // destinations in (tau, t] until k distinct ones
      uint32_t j = p0;
      while (g.in_nbr[j] == v) j++;
      const int32_t tau = g.in_t[j];
      const uint32_t urs = g.out_ptr[u], ure = g.out_ptr[u + 1];
      const uint32_t d0 = upper_bound_i32(g.out_t, urs, ure, tau), d1 = upper_bound_i32(g.out_t, d0, ure, t);
      uint32_t c = d0, nd = 0;
      for (; c < d1 && nd < k; c++) nd += g.out_prv[c] <= tau;
      w += (unsigned long long)kAlgElem * (c - d0);
    }
    mp.work[kWorkSg * mp.stride + eid] = w;
  }
}

// ------------------------------------------------------------------ k_sg
constexpr uint32_t kCandCap = 2 * AMLM_WAVE;

struct SgLds {
  uint32_t bloom[kBloomWordsMax];
  // anchors of the current chunk
  uint32_t i_u[kSgChunkMax], i_p0[kSgChunkMax], i_ns[kSgChunkMax], i_sg[kSgChunkMax];
  uint32_t i_work[kSgChunkMax], i_wlen[kSgChunkMax];
  uint32_t i_vk[kSgChunkMax];   // vkey of the anchor's v (pair keys: vhash(m) ^ i_vk)
  uint32_t i_hu[kSgChunkMax];   // vhash(u): u is never an intermediate
  uint32_t i_vrs[kSgChunkMax], i_vre[kSgChunkMax];  // v's in-row, for the candidate checks
  // exclusive offsets: the group's segment windows (filter build), then the
  // group's sender windows
  uint32_t seg_off[kSgChunkMax];
  int32_t i_t[kSgChunkMax], i_lo[kSgChunkMax];
  uint32_t i_r0[kSgChunkMax], i_r1[kSgChunkMax];  // its v-window [r0, r1) in v's in-row
  uint8_t i_join[kSgChunkMax];  // 1 if the anchor's senders need the join
  uint8_t i_gsd[kSgChunkMax];   // 1 if u has k scatter destinations after tau
  uint8_t grp_seg[kSgChunkMax]; // first anchor of each segment of the current group
  // (anchor, sender) pairs of one batch
  uint32_t pr_b[AMLM_WAVE], pr_cnt[AMLM_WAVE];
  // each pair's slice length until the join has read it into a register,
  // then the exclusive offsets of the slices flattened over the lanes
  union {
    uint32_t pr_n[AMLM_WAVE];
    uint32_t pr_off[AMLM_WAVE];
  };
  uint8_t pr_item[AMLM_WAVE];
  uint8_t pr_rev[AMLM_WAVE];   // 1: the pair joins from the gather side (sg_join_rev)
  // Bloom-positive candidates awaiting the exact check
  uint32_t cq_pos[kCandCap];
  uint8_t cq_pair[kCandCap];
  // (the byte-wide fields, the shared pair arrays and a filter of at most
  // 960 words keep the LDS of a wave within 6400 bytes: 24 waves per CU)
};

// Key mask of a gather vertex v: the filter of a group of segments holds the
// pairs (v, m) of their gather windows as vhash(m) ^ vkey(v), a bijection of
// vhash(m) for each v, so one filter serves segments into different vertices.
__device__ __forceinline__ uint32_t vkey(uint32_t v) { return __builtin_rotateleft32(vhash(v), 16); }

// Register-blocked Bloom filter over vertex hashes (vhash): a key selects
// one of the filter's `words` 32-bit words by its top 12 bits (scaled to the
// word count, which need not be a power of two) and sets kBloomK bits inside
// it chosen by consecutive 5-bit fields of its low bits, so a test is a
// single LDS read, a multiply and a few shifts.
struct BloomProbe {
  uint32_t word, mask;
};
__device__ __forceinline__ BloomProbe bloom_probe(uint32_t h, uint32_t words) {
  BloomProbe p;
  p.word = ((h >> 20) * words) >> 12;
  p.mask = 0;
#pragma unroll
  for (int i = 0; i < kBloomK; i++) p.mask |= 1u << ((h >> (5 * i)) & 31u);
  return p;
}
__device__ __forceinline__ bool bloom_test(const uint32_t *bloom, uint32_t words, uint32_t h) {
  BloomProbe p = bloom_probe(h, words);
  return (bloom[p.word] & p.mask) == p.mask;
}
__device__ __forceinline__ void bloom_insert(uint32_t *bloom, uint32_t words, uint32_t h) {
  BloomProbe p = bloom_probe(h, words);
  atomicOr(&bloom[p.word], p.mask);
}

// Owner of flattened index f: the largest a < n with off[a] <= f.
__device__ __forceinline__ uint32_t owner_of(const uint32_t *off, uint32_t n, uint32_t f) {
  uint32_t a = 0, b = n - 1;
  while (a < b) {
    uint32_t mid = (a + b + 1) >> 1;
    if (off[mid] <= f) a = mid; else b = mid - 1;
  }
  return a;
}

// Confirm `take` queued candidates (from the top of the queue): m must have
// an edge to v later than the (s, m) entry and no later than the anchor, and
// the entry must be the first (s, m) edge inside the window.  The search in
// v's CSC-N row comes first: it rejects the filter's false positives from
// lines that other candidates into the same v keep in cache, before any read
// of the sender's row.
__device__ void sg_verify(const MineParams &mp, SgLds &L, uint32_t cq_top, uint32_t take) {
  const GraphView &g = mp.g;
  const uint32_t lane = lane_id();
  if (lane < take) {
    uint32_t idx = cq_top - take + lane;
    uint32_t a = L.cq_pair[idx], pos = L.cq_pos[idx];
    uint32_t it = L.pr_item[a];
    int32_t lo = L.i_lo[it], t = L.i_t[it];
    const uint32_t vrs = L.i_vrs[it], vre = L.i_vre[it];
    uint32_t m = vhash_inv(g.out_h[pos]);  // the scan has just read this line
    uint32_t q = upper_bound_u64_interp(g.inn_key, vrs, vre, nbr_key(m, t));
    if (q > vrs) {
      uint64_t kk = g.inn_key[q - 1];  // the last m -> v edge at or before t, if any
      const int32_t tb = (int32_t)(uint32_t)kk;
      // the pair's first s -> m edge in the window; then the gather leg:
      // after it (ordered) or anywhere in the window (unordered).  The
      // short-circuit order keeps the time loads off the false positives.
      if ((uint32_t)(kk >> 32) == m && g.out_prv[pos] < lo && (mp.sg_unordered ? tb >= lo : tb > g.out_t[pos]))
        atomicAdd(&L.pr_cnt[a], 1u);
    }
  }
}

// Queue the Bloom-positive entries of one 64-entry step (lane l holds
// position pos0 + l) and verify a full batch of 64 when the queue holds at
// least that many.  Steps without a candidate cost one scalar test.
__device__ __forceinline__ void sg_push(const MineParams &mp, SgLds &L, uint32_t &cq, bool cand, uint32_t a,
                                        uint32_t pos) {
  uint64_t bc = __builtin_amdgcn_ballot_w64(cand);
  if (bc == 0) return;
  if (cand) {
    uint32_t slot = cq + __popcll(bc & lanemask_lt());
    L.cq_pair[slot] = (uint8_t)a;
    L.cq_pos[slot] = pos;
  }
  cq += __popcll(bc);
  if (cq >= AMLM_WAVE) {
    sg_verify(mp, L, cq, AMLM_WAVE);
    cq -= AMLM_WAVE;
  }
}

// Phase-ordered joins of a batch of pairs: one lane per pair, each scanning
// its slice serially (the filter of the segment rejects most entries).
// Phase-ordered join of the batch's pairs.  The (pair, out-window entry)
// items are flattened over the lanes in 64-lane steps, pairs in slot order
// and each pair's entries in time order: a lane tests its entry (the
// sender's first edge to an intermediate m != u, a filter hit, m's latest
// gather leg g_m up to t after it), and the step's hits, in lane order, are
// folded by each pair's own lane in that order into its k - 1 latest g_m,
// as the serial scan of sg_phase_pair does.  A pair is decided at the first
// interval where the condition holds; its later entries are skipped.
__device__ void sg_join_phase(const MineParams &mp, SgLds &L, uint32_t np, uint32_t words, uint32_t k) {
  const GraphView &g = mp.g;
  const uint32_t lane = lane_id();
  const uint64_t lt = lanemask_lt();
  const uint32_t need = k - 1;  // k >= 2 here (k < 2 needs no join)
  // this lane's pair: f_u (the sender's first edge to u in the window) and
  // the k - 1 latest gather times of its intervals so far
  int32_t f_u = 0;
  int32_t top[kPhaseKMax - 1];
#pragma unroll
  for (uint32_t i = 0; i < kPhaseKMax - 1; i++) top[i] = AMLM_INT_MIN;
  uint32_t my_n = 0;
  if (lane < np) {
    my_n = L.pr_n[lane];  // before the offsets take its place
    if (my_n) {
      const uint32_t it = L.pr_item[lane], s = g.out_src[L.pr_b[lane]], u = L.i_u[it];
      const int32_t lo = L.i_lo[it], t = L.i_t[it];
      const uint32_t urs = g.in_ptr[u], ure = g.in_ptr[u + 1];
      const uint64_t ku = nbr_key(s, lo < 0 ? 0 : lo);
      const uint32_t qu = ku ? upper_bound_u64_interp(g.inn_key, urs, ure, ku - 1) : urs;
      f_u = t;
      if (qu < ure && (uint32_t)(g.inn_key[qu] >> 32) == s) f_u = (int32_t)(uint32_t)g.inn_key[qu];
    }
  }
  const uint32_t incl = wave_incl_scan(my_n);
  const uint32_t T = rfl((uint32_t)__shfl(incl, AMLM_WAVE - 1, AMLM_WAVE));
  L.pr_off[lane] = incl - my_n;
  __syncthreads();
  for (uint32_t f0 = 0; f0 < T; f0 += AMLM_WAVE) {
    const uint32_t f = f0 + lane;
    bool hit = false;
    uint32_t a = 0;
    int32_t fm = 0, gm = 0;
    if (f < T) {
      a = owner_of(L.pr_off, np, f);
      if (L.pr_cnt[a] < need) {  // the pair is not decided yet
        const uint32_t pos = L.pr_b[a] + (f - L.pr_off[a]);
        const uint32_t it = L.pr_item[a], u = L.i_u[it];
        const int32_t lo = L.i_lo[it], t = L.i_t[it];
        const uint32_t m = g.out_nbr[pos];
        if (m != u && g.out_prv[pos] < lo && bloom_test(L.bloom, words, g.out_h[pos] ^ L.i_vk[it])) {
          const uint32_t vrs = L.i_vrs[it], vre = L.i_vre[it];
          const uint32_t q = upper_bound_u64_interp(g.inn_key, vrs, vre, nbr_key(m, t));
          if (q > vrs) {
            const uint64_t kk = g.inn_key[q - 1];
            gm = (int32_t)(uint32_t)kk;
            fm = g.out_t[pos];
            hit = (uint32_t)(kk >> 32) == m && gm >= lo && fm < gm;
          }
        }
      }
    }
    const uint64_t hm = __ballot(hit);
    if (!hm) continue;
    const uint32_t nh = (uint32_t)__popcll(hm);
    if (hit) {
      const uint32_t slot = (uint32_t)__popcll(hm & lt);
      L.cq_pos[slot] = (uint32_t)fm;
      L.cq_pos[AMLM_WAVE + slot] = (uint32_t)gm;
      L.cq_pair[slot] = (uint8_t)a;
    }
    __syncthreads();
    if (lane < np && L.pr_cnt[lane] < need) {
      for (uint32_t j = 0; j < nh; j++) {
        if (L.cq_pair[j] != lane) continue;
        int32_t x = (int32_t)L.cq_pos[AMLM_WAVE + j];
        const int32_t fj = (int32_t)L.cq_pos[j];
        // insert g into the descending list of the k - 1 largest
#pragma unroll
        for (uint32_t i = 0; i < kPhaseKMax - 1; i++) {
          if (i < need && x > top[i]) {
            const int32_t y = top[i];
            top[i] = x;
            x = y;
          }
        }
        int32_t kth = top[0];
#pragma unroll
        for (uint32_t i = 1; i < kPhaseKMax - 1; i++)
          if (i == need - 1) kth = top[i];
        if (kth > max(fj, f_u)) {
          L.pr_cnt[lane] = need;
          break;
        }
      }
    }
    __syncthreads();
  }
}

// Reverse join of the pairs in `rev` (degree-ordered intersection, Section
// 6: the smaller side is iterated).  Pair `slot` holds the sender in pr_b and
// the length of its anchor's gather window [r0, r1) (v's in-edges in
// [t - delta, t]) in pr_n.  Lanes are flattened over (pair, gather entry);
// an entry is the intermediate m's last edge into v at or before t (its
// next same-pair time is past t), so each distinct m is tried once, and m
// counts when the sender's first edge to m inside the window, found by a
// search in m's neighbour-sorted in-row, comes before that edge (ordered) or
// before t (unordered).  A pair stops once k - 1 intermediates besides u
// have qualified.
__device__ void sg_join_rev(const MineParams &mp, SgLds &L, uint32_t np, uint64_t rev, uint32_t need,
                            uint32_t nr) {
  const GraphView &g = mp.g;
  const uint32_t lane = lane_id();
  const uint32_t incl = wave_incl_scan(nr);
  const uint32_t T = rfl((uint32_t)__shfl(incl, AMLM_WAVE - 1, AMLM_WAVE));
  L.pr_off[lane] = incl - nr;
  for (uint32_t f0 = 0; f0 < T; f0 += AMLM_WAVE) {
    const uint32_t f = f0 + lane;
    if (f < T) {
      const uint32_t a = owner_of(L.pr_off, np, f);
      if (L.pr_cnt[a] < need) {
        const uint32_t it = L.pr_item[a];
        const uint32_t j = L.i_r0[it] + (f - L.pr_off[a]);
        const uint32_t m = g.in_nbr[j];
        const int32_t t = L.i_t[it];
        if (m != L.i_u[it] && g.in_nxt[j] > t) {
          const uint32_t s = L.pr_b[a];
          const int32_t lo = L.i_lo[it] < 0 ? 0 : L.i_lo[it];
          const uint64_t key = nbr_key(s, lo);
          const uint32_t ms = g.in_ptr[m], me = g.in_ptr[m + 1];
          // first (s, time >= lo) key of m's row: after every key <= key - 1
          const uint32_t qa = key ? upper_bound_u64_interp(g.inn_key, ms, me, key - 1) : ms;
          if (qa < me) {
            const uint64_t kk = g.inn_key[qa];
            const int32_t ta = (int32_t)(uint32_t)kk;
            if ((uint32_t)(kk >> 32) == s && ta < (mp.sg_unordered ? t : g.in_t[j])) atomicAdd(&L.pr_cnt[a], 1u);
          }
        }
      }
    }
    // every pair done: stop early
    if (__ballot(lane < np && ((rev >> lane) & 1ull) && L.pr_cnt[lane] < need) == 0) break;
  }
}

// Join one batch of np (anchor, sender) pairs: pair `slot` (= lane) holds
// its slice [pr_b, pr_b + pr_n) of the sender's out-row.  Long slices are
// scanned one pair at a time by the whole wave with the pair's fields in
// scalar registers; short ones are flattened over the lanes.
__device__ void sg_join(const MineParams &mp, SgLds &L, uint32_t np, uint64_t rev, uint32_t words, uint32_t k) {
  const GraphView &g = mp.g;
  const uint32_t lane = lane_id();
  const uint32_t need = k - 1;  // intermediates needed besides u
  uint32_t cq = 0;
  constexpr int U = kJoinUnroll;  // independent 256-byte loads in flight per wave
  const bool my_rev = (rev >> lane) & 1ull;
  // the slice lengths, before the offsets take their place
  const uint32_t pn = lane < np ? L.pr_n[lane] : 0u;
  const uint32_t my_n = my_rev ? 0u : pn;
  uint64_t longs = __ballot(my_n >= kLongPair);
  while (longs) {
    uint32_t a = __ffsll((long long)longs) - 1;
    longs &= longs - 1;
    const uint32_t b = rfl(L.pr_b[a]), n = rfl((uint32_t)__shfl(my_n, a, AMLM_WAVE));
    const uint32_t it = rfl((uint32_t)L.pr_item[a]);
    const uint32_t hu = rfl(L.i_hu[it]), vk = rfl(L.i_vk[it]);  // u itself is never a candidate
    for (uint32_t f0 = 0; f0 < n; f0 += U * AMLM_WAVE) {
      if (rfl(L.pr_cnt[a]) >= need) break;
      const uint32_t *src = g.out_h + b + f0 + lane;
      uint32_t h[U];
      auto step = [&]() {
#pragma unroll
        for (int r = 0; r < U; r++) {
          bool cand = (h[r] != hu) & bloom_test(L.bloom, words, h[r] ^ vk);
          sg_push(mp, L, cq, cand, a, b + f0 + r * AMLM_WAVE + lane);
        }
      };
      if (f0 + U * AMLM_WAVE <= n) {
#pragma unroll
        for (int r = 0; r < U; r++) h[r] = src[r * AMLM_WAVE];
        step();
      } else {
#pragma unroll
        for (int r = 0; r < U; r++) h[r] = f0 + r * AMLM_WAVE + lane < n ? src[r * AMLM_WAVE] : hu;
        step();
      }
      if (need <= kEagerNeed && cq > 0) {
        // few intermediates needed: confirm now, so the scan can stop
        sg_verify(mp, L, cq, cq);
        cq = 0;
      }
    }
  }
  // short pairs, flattened
  const uint32_t ns = my_n < kLongPair ? my_n : 0u;
  const uint32_t incl = wave_incl_scan(ns);
  const uint32_t T = rfl((uint32_t)__shfl(incl, AMLM_WAVE - 1, AMLM_WAVE));
  L.pr_off[lane] = incl - ns;
  for (uint32_t f0 = 0; f0 < T; f0 += AMLM_WAVE) {
    uint32_t f = f0 + lane;
    bool cand = false;
    uint32_t a = 0, pos = 0;
    if (f < T) {
      a = owner_of(L.pr_off, np, f);
      pos = L.pr_b[a] + (f - L.pr_off[a]);
      if (L.pr_cnt[a] < need) {
        uint32_t h = g.out_h[pos];
        const uint32_t it = L.pr_item[a];
        cand = h != L.i_hu[it] && bloom_test(L.bloom, words, h ^ L.i_vk[it]);
      }
    }
    sg_push(mp, L, cq, cand, a, pos);
    if (kEagerShort && need <= kEagerNeed && cq > 0) {
      sg_verify(mp, L, cq, cq);
      cq = 0;
    }
  }
  while (cq > 0) {
    uint32_t take = min(cq, (uint32_t)AMLM_WAVE);
    sg_verify(mp, L, cq, take);
    cq -= take;
  }
  if (rev) sg_join_rev(mp, L, np, rev, need, my_rev ? pn : 0u);
}

// Anchors [s0, s1) of the chunk: a group of nseg segments whose first
// anchors are grp_seg[0 .. nseg).  A segment is a run of anchors into one v
// inside one time bucket; its gather window, v's in-edges from its first
// anchor's window start to its last anchor's time, covers each anchor's.  One
// filter holds the pairs (v, m) of every segment window of the group, so the
// senders, pairs and joins of the whole group are flattened over the lanes
// together (a chunk of anchors into many light vertices is one pass, not one
// per vertex).
__device__ void sg_group(const MineParams &mp, SgLds &L, uint32_t s0, uint32_t s1, uint32_t nseg, uint32_t k) {
  const GraphView &g = mp.g;
  const uint32_t lane = lane_id();
  const uint64_t lt = lanemask_lt();
  const uint32_t nit = s1 - s0;
  const bool need_join = mp.col_sg >= 0 && k >= 2 &&
                         __ballot(lane >= s0 && lane < s1 && L.i_join[min(lane, kSgChunkMax - 1)] != 0) != 0;
  uint32_t words = 0;
  if (need_join) {
    // segment j holds anchors [grp_seg[j], grp_seg[j + 1]) (the last ends at
    // s1); the anchors are time-sorted inside it
    uint32_t len = 0;
    if (lane < nseg) {
      const uint32_t a0 = L.grp_seg[lane], a1 = lane + 1 < nseg ? L.grp_seg[lane + 1] : s1;
      len = L.i_r1[a1 - 1] - L.i_r0[a0];
    }
    const uint32_t incl = wave_incl_scan(len);
    const uint32_t nin = rfl((uint32_t)__shfl(incl, AMLM_WAVE - 1, AMLM_WAVE));
    if (lane < kSgChunkMax) L.seg_off[lane] = incl - len;
    int lg = 9;
    while (lg < kBloomLog2Max && (1u << lg) < nin * kBloomBitsPerEntry) lg++;
    words = min((1u << lg) >> 5, kBloomWordsMax);
    for (uint32_t q = lane; q < words; q += AMLM_WAVE) L.bloom[q] = 0;
    if (nseg == 1) {
      // one window (a hub's row, typically): strided loads, four in flight
      const uint32_t r0 = rfl(L.i_r0[s0]), r1 = r0 + nin, vk = rfl(L.i_vk[s0]);
      for (uint32_t q0 = r0; q0 < r1; q0 += 4 * AMLM_WAVE) {
        uint32_t mm[4];
#pragma unroll
        for (int r = 0; r < 4; r++) {
          uint32_t q = q0 + r * AMLM_WAVE + lane;
          mm[r] = q < r1 ? g.in_h[q] : 0u;
        }
#pragma unroll
        for (int r = 0; r < 4; r++) {
          if (q0 + r * AMLM_WAVE + lane < r1) bloom_insert(L.bloom, words, mm[r] ^ vk);
        }
      }
    } else {
      // the segment windows flattened over the lanes (at most kGroupCap entries)
      for (uint32_t f0 = 0; f0 < nin; f0 += 4 * AMLM_WAVE) {
        uint32_t mm[4];
#pragma unroll
        for (int r = 0; r < 4; r++) {
          const uint32_t f = f0 + r * AMLM_WAVE + lane;
          mm[r] = 0;
          if (f < nin) {
            const uint32_t j = owner_of(L.seg_off, nseg, f);
            const uint32_t a0 = L.grp_seg[j];
            mm[r] = L.i_vk[a0];
            mm[r] ^= g.in_h[L.i_r0[a0] + (f - L.seg_off[j])];
          }
        }
#pragma unroll
        for (int r = 0; r < 4; r++) {
          if (f0 + r * AMLM_WAVE + lane < nin) bloom_insert(L.bloom, words, mm[r]);
        }
      }
    }
    if (mp.work && lane < nit) {
      // each segment's gather entries, shared evenly by its anchors
      const uint32_t x = s0 + lane;
      uint32_t j = 0;
      for (uint32_t i = 1; i < nseg; i++) j = L.grp_seg[i] <= x ? i : j;
      const uint32_t a0 = L.grp_seg[j], a1 = j + 1 < nseg ? L.grp_seg[j + 1] : s1;
      const uint32_t share = kBytesGatherEntry * (L.i_r1[a1 - 1] - L.i_r0[a0]);
      L.i_work[x] += share / (a1 - a0) + (x == a0 ? share % (a1 - a0) : 0);
    }
  }
  // senders: flatten the anchors' windows [p0, p1) over the lanes
  uint32_t w = lane < nit ? L.i_wlen[s0 + lane] : 0u;
  uint32_t incl = wave_incl_scan(w);
  uint32_t W = rfl((uint32_t)__shfl(incl, AMLM_WAVE - 1, AMLM_WAVE));
  if (lane < kSgChunkMax) L.seg_off[lane] = incl - w;
  for (uint32_t f0 = 0; f0 < W; f0 += AMLM_WAVE) {
    uint32_t f = f0 + lane;
    bool is_s = false;
    uint32_t it = 0, nb = 0, j = 0;
    if (f < W) {
      uint32_t a = owner_of(L.seg_off, nit, f);
      it = s0 + a;
      j = L.i_p0[it] + (f - L.seg_off[a]);
      nb = g.in_nbr[j];
      if (vkey(nb) != L.i_vk[it]) {  // nb != v (vkey is a bijection)
        is_s = g.in_nxt[j] >= L.i_t[it];  // last sender edge before t: one per distinct s
        if (is_s) atomicAdd(&L.i_ns[it], 1u);
      }
      if (mp.work) atomicAdd(&L.i_work[it], kBytesSenderEntry);
    }
    if (!need_join) continue;
    const bool pair = is_s && L.i_join[it] != 0;
    uint64_t bs = __ballot(pair);
    if (!bs) continue;
    // this lane's pair: slice of s's out-row inside [lo, t)
    uint32_t b = 0, n = 0;
    bool rv = false;
    if (pair) {
      // s's out-window [lo, t) contains the s -> u edge: search outwards from it
      const uint32_t rs = g.out_ptr[nb], re = g.out_ptr[nb + 1];
      const uint4 m = g.out_tm[nb];
      b = tix_lower_bound(g.out_t, g.out_tix, m, rs, re, L.i_lo[it]);
      n = tix_lower_bound(g.out_t, g.out_tix, m, rs, re, L.i_t[it]) - b;
      // the smaller side: v's gather window when it is much shorter than
      // the sender's out-window (a gather entry costs a search, a scanned
      // out-entry one load and a filter test)
      const uint32_t r = L.i_r1[it] - L.i_r0[it];
      rv = !mp.sg_phase && (uint64_t)r * kRevRatio < n;
      if (rv) {
        b = nb;
        n = r;
      }
      if (mp.work) atomicAdd(&L.i_work[it], rv ? kBytesRevEntry * n : kBytesJoinEntry * n);
    }
    uint32_t np = __popcll(bs);
    if (pair) {
      uint32_t slot = __popcll(bs & lt);
      L.pr_item[slot] = (uint8_t)it;
      L.pr_rev[slot] = rv ? 1 : 0;
      L.pr_b[slot] = b;
      L.pr_n[slot] = n;
      L.pr_cnt[slot] = 0;
    }
    // reverse pairs by slot
    const uint64_t rev = __ballot(lane < np && L.pr_rev[lane] != 0);
    if (mp.sg_phase)
      sg_join_phase(mp, L, np, words, k);
    else
      sg_join(mp, L, np, rev, words, k);
    if (lane < np && L.pr_cnt[lane] >= k - 1) atomicAdd(&L.i_sg[L.pr_item[lane]], 1u);
  }
}

// ------------------------------------------------------------------ work units
// A unit of k_sg work is a block of up to `block` consecutive list items, or
// one slice of the sender window of a heavy anchor.  An anchor whose join
// runs over a long sender window is cut into slices, each a unit of its own,
// so that no unit dominates the kernel (on the 32M-edge graph the heaviest
// 8-anchor chunk held 3.8 MB of join reads, milliseconds of one wave).
// Slices add their partial SG_k and sender counts with atomics; k_split_gs
// turns an anchor's accumulated sender count into GS_k afterwards.
// unit = (first item, count) for a block; (item, kUnitHeavy | slices << 16 | slice)
constexpr uint32_t kUnitHeavy = 0x80000000u;

__device__ __forceinline__ uint32_t join_window(const MineParams &mp, const uint8_t *flags_sg, const uint4 *sg_win,
                                                uint32_t q) {
  // sender-window length of a scatter-gather anchor that runs a join, else 0
  if (mp.col_sg < 0 || (flags_sg[q] & kFlagSgNoJoin) || k_of(mp, mp.g.in_dst[q]) < 2) return 0;
  const uint4 pw = sg_win[q];
  return pw.y - pw.x;
}

// Size of item i for the split rule: the predicted scatter-gather bytes when
// the cost model runs (pred != NULL), else the sender-window length; 0 for
// items without a join.
__device__ __forceinline__ unsigned long long split_size(const MineParams &mp, const uint32_t *items,
                                                         const uint8_t *flags_sg, const uint4 *sg_win,
                                                         const float *pred, uint32_t i, uint32_t *w) {
  *w = join_window(mp, flags_sg, sg_win, items[i]);
  if (*w < 2) return 0;
  if (!pred) return *w;
  return (unsigned long long)fminf(expm1f(fminf(fmaxf(pred[i], 0.f), 40.f)), 2147483648.f);
}

// Predicted log1p(bytes) of the list items without the network: the
// sender-window length times a constant (length schedule), or the caller's
// per-edge costs (given schedule).
__global__ __launch_bounds__(256) void k_pred_rule(MineParams mp, const uint32_t *items, const uint32_t *n_items_p,
                                                   const uint8_t *flags_sg, const uint4 *sg_win, uint32_t sched,
                                                   float len_coef, const float *given, float *pred) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= *n_items_p) return;
  const uint32_t q = items[i];
  if (sched == kSchedGiven) {
    pred[i] = given[mp.g.in_eid[q]];
  } else {
    const uint32_t w = join_window(mp, flags_sg, sg_win, q);
    pred[i] = log1pf(len_coef * (float)w);
  }
}

__global__ __launch_bounds__(256) void k_split_weight(MineParams mp, const uint32_t *items, const uint32_t *n_items_p,
                                                      const uint8_t *flags_sg, const uint4 *sg_win,
                                                      const float *pred, uint32_t min_size, unsigned long long *W) {
  __shared__ unsigned long long ws[256 / AMLM_WAVE];
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (blockIdx.x * blockDim.x >= *n_items_p) return;  // the grid covers Ev items, the list fewer
  unsigned long long w = 0;
  if (i < *n_items_p) {
    uint32_t x;
    const unsigned long long z = split_size(mp, items, flags_sg, sg_win, pred, i, &x);
    if (z > min_size) w = z;
  }
  for (int o = 32; o > 0; o >>= 1) w += __shfl_xor(w, o, AMLM_WAVE);
  if (lane_id() == 0) ws[threadIdx.x / AMLM_WAVE] = w;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long t = 0;
    for (int q = 0; q < 256 / AMLM_WAVE; q++) t += ws[q];
    if (t) atomicAdd(W, t);
  }
}

// Slices of item i (0 for a light item): its size over the slice size, which
// is at least min_size and at least 16 W / Ev (W: the summed size of the
// items above min_size), so the slices of all anchors stay within Ev / 8.
__device__ __forceinline__ uint32_t item_slices(const MineParams &mp, const uint32_t *items, const uint8_t *flags_sg,
                                                const uint4 *sg_win, const float *pred, uint32_t min_size,
                                                unsigned long long W, uint32_t i) {
  uint32_t w;
  const unsigned long long z = split_size(mp, items, flags_sg, sg_win, pred, i, &w);
  const unsigned long long ev = mp.g.Ev ? mp.g.Ev : 1;
  const unsigned long long se = max((unsigned long long)min_size, (16ull * W + ev - 1) / ev);
  if (z <= se) return 0;
  return (uint32_t)min((unsigned long long)min(kSplitMax, w), (z + se - 1) / se);
}

__global__ __launch_bounds__(256) void k_unit_count(MineParams mp, const uint32_t *items, const uint32_t *n_items_p,
                                                    const uint8_t *flags_sg, const uint4 *sg_win, const float *pred,
                                                    uint32_t min_size, const unsigned long long *W_p, uint32_t block,
                                                    uint32_t n_max, uint32_t *nsub, uint32_t *cnt) {
  __shared__ uint32_t sl[256];
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t n = *n_items_p;
  if (blockIdx.x * blockDim.x >= n) return;  // the grid covers Ev items, the list fewer
  const unsigned long long W = *W_p;
  uint32_t ns = 0;
  if (i < n) {
    ns = item_slices(mp, items, flags_sg, sg_win, pred, min_size, W, i);
    if (ns == 1) ns = 0;
    nsub[i] = ns;
  }
  sl[threadIdx.x] = ns;
  __syncthreads();
  if (i >= n || i >= n_max) return;  // the scan of the counts stops at n
  bool start = false;
  if (!ns) {
    // the previous item's slices: from this block, or recomputed at its edge
    uint32_t prev = 0;
    if (i > 0) prev = threadIdx.x > 0 ? sl[threadIdx.x - 1]
                                      : item_slices(mp, items, flags_sg, sg_win, pred, min_size, W, i - 1);
    start = i % block == 0 || prev > 1;
  }
  cnt[i] = ns ? ns : (start ? 1u : 0u);
}

__global__ void k_unit_fill(MineParams mp, const uint32_t *items, const uint32_t *n_items_p, const uint32_t *nsub,
                            const uint32_t *cnt, const uint32_t *off, uint32_t block, uint2 *units) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t n = *n_items_p;
  if (i >= n || cnt[i] == 0) return;
  const uint32_t ns = nsub[i], o = off[i];
  if (ns) {
    for (uint32_t s = 0; s < ns; s++) units[o + s] = make_uint2(i, kUnitHeavy | (ns << 16) | s);
    // the slices accumulate into the outputs
    const uint32_t eid = mp.g.in_eid[items[i]];
    if (mp.col_sg >= 0) mp.counts[(uint64_t)mp.col_sg * mp.stride + eid] = 0;
    if (mp.col_gs >= 0) mp.counts[(uint64_t)mp.col_gs * mp.stride + eid] = 0;
  } else {
    uint32_t len = 1;
    while (len < block && i + len < n && (i + len) % block != 0 && nsub[i + len] == 0) len++;
    units[o] = make_uint2(i, len);
  }
}

// GS_k of the split anchors from their accumulated sender counts, and the
// ceiling on both of their accumulated columns.
__global__ void k_split_gs(MineParams mp, const uint32_t *items, const uint32_t *n_items_p, const uint32_t *nsub,
                           const uint8_t *flags_sg) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= *n_items_p || nsub[i] == 0) return;
  const uint32_t q = items[i], eid = mp.g.in_eid[q];
  if (mp.col_gs >= 0) {
    uint32_t *c = mp.counts + (uint64_t)mp.col_gs * mp.stride + eid;
    const uint32_t ns = *c;
    const bool d_ok = (flags_sg[q] & kFlagGsDest) != 0;  // split anchors have k >= 2
    *c = ns >= k_of(mp, mp.g.in_dst[q]) && d_ok ? min(ns, mp.ceil) : 0u;
  }
  if (mp.col_sg >= 0) {
    uint32_t *c = mp.counts + (uint64_t)mp.col_sg * mp.stride + eid;
    *c = min(*c, mp.ceil);
  }
}

// Units: with `units` NULL (static schedule) unit c is the block of items
// [c * block, (c + 1) * block) and n_count_p points at the item count; else
// units[c] and n_count_p points at the unit count.
__global__ __launch_bounds__(AMLM_WAVE) AMLM_SG_OCCUPANCY void k_sg(MineParams mp, const uint32_t *items,
                                                                    const uint2 *units, const uint32_t *n_count_p,
                                                                    uint32_t block, uint32_t *ctr,
                                                                    const uint4 *sg_win, const uint8_t *flags_sg) {
  __shared__ SgLds L;
  const GraphView &g = mp.g;
  const uint32_t lane = lane_id();
  const uint32_t n_count = *n_count_p;
  const uint32_t n_units = units ? n_count : (n_count + block - 1) / block;
  // the next unit is claimed while this one is mined, so the counter's
  // round trip overlaps the work (kPrefetchClaim)
  uint32_t next = 0;
  if (kPrefetchClaim && lane == 0) next = atomicAdd(ctr, 1u);
  for (;;) {
    uint32_t c = 0;
    if (kPrefetchClaim) {
      c = rfl((uint32_t)__shfl(next, 0, AMLM_WAVE));
      if (c >= n_units) break;
      if (lane == 0) next = atomicAdd(ctr, 1u);
    } else {
      if (lane == 0) c = atomicAdd(ctr, 1u);
      c = rfl((uint32_t)__shfl(c, 0, AMLM_WAVE));
      if (c >= n_units) break;
    }
    const uint2 un = units ? units[c] : make_uint2(c * block, min(block, n_count - c * block));
    const bool heavy = (un.y & kUnitHeavy) != 0;
    const uint32_t nr = heavy ? 1u : un.y;
    uint32_t v = 0xffffffffu, r0v = 0, r1v = 0, kv = 0, eid = 0;
    int64_t dl = 1;
    if (lane < nr) {
      uint32_t q = items[un.x + lane];
      eid = g.in_eid[q];
      int32_t t = g.in_t[q];
      uint4 pw = sg_win[q];
      uint32_t first_slice = 1;
      if (heavy) {  // slice s of ns: an even share of the sender window
        const uint32_t ns = (un.y >> 16) & 0x7fffu, sl = un.y & 0xffffu, w = pw.y - pw.x;
        const uint32_t a = (uint32_t)((uint64_t)w * sl / ns), b = (uint32_t)((uint64_t)w * (sl + 1) / ns);
        pw.y = pw.x + b;
        pw.x += a;
        first_slice = sl == 0;
      }
      v = g.in_dst[q];
      const uint32_t u = g.in_nbr[q];
      L.i_u[lane] = u;
      L.i_hu[lane] = vhash(u);
      L.i_vk[lane] = vkey(v);
      L.i_vrs[lane] = g.in_ptr[v];
      L.i_vre[lane] = g.in_ptr[v + 1];
      L.i_t[lane] = t;
      dl = delta_of(mp, v);
      L.i_lo[lane] = window_lo(t, dl);
      kv = k_of(mp, v);
      const uint8_t fl = flags_sg[q];
      L.i_join[lane] = (fl & kFlagSgNoJoin) ? 0 : 1;
      L.i_gsd[lane] = (fl & kFlagGsDest) ? 1 : 0;
      L.i_p0[lane] = pw.x;
      L.i_wlen[lane] = pw.y - pw.x;
      r0v = pw.z;
      r1v = pw.w;
      L.i_r0[lane] = pw.z;
      L.i_r1[lane] = pw.w;
      L.i_ns[lane] = 0;
      L.i_sg[lane] = 0;
      L.i_work[lane] = first_slice ? kBytesAnchorSg : 0u;
    }
    // segments: runs of anchors into the same v inside one time bucket of
    // width 2 delta share one filter; narrower buckets (delta / 4 .. delta)
    // rebuilt it more often than its shorter gather window saved
    const int32_t seg_span = (int32_t)max((int64_t)1, min(2 * dl, (int64_t)0x40000000));
    int32_t tb = lane < nr ? L.i_t[lane] / seg_span : 0;
    uint32_t vprev = __shfl_up(v, 1, AMLM_WAVE);
    int32_t tbprev = __shfl_up(tb, 1, AMLM_WAVE);
    const uint64_t heads = __ballot(lane < nr && (lane == 0 || v != vprev || tb != tbprev));
    // each segment's gather window (at its head lane): from its first
    // anchor's r0 to the r1 of the lane before the next head
    const uint64_t later = heads & ~((2ull << lane) - 1);
    const uint32_t send = later ? (uint32_t)(__ffsll((long long)later) - 1) : nr;
    const uint32_t r1_end = (uint32_t)__shfl(r1v, (int)(send > 0 ? send - 1 : 0), AMLM_WAVE);
    const uint32_t segw = r1_end - r0v;
    // groups: consecutive segments of one k whose windows total at most
    // kGroupCap entries (a longer window is a group of its own)
    uint64_t gheads = 0, hs = heads;
    uint32_t gk = 0;
    uint64_t gsum = 0;
    while (hs) {
      const uint32_t h0 = __ffsll((long long)hs) - 1;
      hs &= hs - 1;
      const uint32_t sw = rfl((uint32_t)__shfl(segw, h0, AMLM_WAVE));
      const uint32_t kk = rfl((uint32_t)__shfl(kv, h0, AMLM_WAVE));
      if (gheads == 0 || gsum + sw > kGroupCap || kk != gk) {
        gheads |= 1ull << h0;
        gsum = 0;
      }
      gsum += sw;
      gk = kk;
    }
    while (gheads) {
      const uint32_t g0 = __ffsll((long long)gheads) - 1;
      gheads &= gheads - 1;
      const uint32_t g1 = gheads ? (uint32_t)(__ffsll((long long)gheads) - 1) : nr;
      // the group's segment heads, in order
      const uint64_t sh = heads & ((1ull << g1) - 1) & ~((1ull << g0) - 1);  // g1 <= nr <= 16
      if ((sh >> lane) & 1ull) L.grp_seg[__popcll(sh & lanemask_lt())] = (uint8_t)lane;
      // groups are cut where k changes: the group's k is its first anchor's
      sg_group(mp, L, g0, g1, (uint32_t)__popcll(sh), rfl((uint32_t)__shfl(kv, g0, AMLM_WAVE)));
    }
    // gather-scatter and the outputs, one lane per anchor
    uint32_t sg = 0, gs = 0, work = 0;
    if (lane < nr) {
      const uint32_t k = kv, ns = L.i_ns[lane];
      sg = k == 1 ? ns : L.i_sg[lane];
      work = L.i_work[lane];
      // k == 1: v follows tau, so D is never empty
      if (mp.col_gs >= 0 && ns >= k && ns > 0 && (k == 1 || L.i_gsd[lane])) gs = ns;
    }
    if (lane < nr) {
      if (heavy) {
        // a slice: partial SG_k, and its senders towards the GS_k of k_split_gs
        // (plain adds: the sums are at most the number of accounts; the
        // ceiling is applied by k_split_gs)
        if (mp.col_sg >= 0 && sg) atomicAdd(mp.counts + (uint64_t)mp.col_sg * mp.stride + eid, sg);
        const uint32_t ns = L.i_ns[lane];
        if (mp.col_gs >= 0 && ns) atomicAdd(mp.counts + (uint64_t)mp.col_gs * mp.stride + eid, ns);
      } else {
        if (mp.col_sg >= 0) mp.counts[(uint64_t)mp.col_sg * mp.stride + eid] = min(sg, mp.ceil);
        if (mp.col_gs >= 0) mp.counts[(uint64_t)mp.col_gs * mp.stride + eid] = min(gs, mp.ceil);
      }
      if (mp.work) atomicAdd(&mp.work[kWorkSgImpl * mp.stride + eid], (unsigned long long)work);
    }
  }
}

// ------------------------------------------------------------------ k_cyc
// Depth-first search over frames of up to 64 partial paths.  Frame i holds
// paths of i edges (v -> ... -> head); each frame keeps its nodes' time
// slices flattened over the lanes and a cursor.  One step consumes 64
// entries of the top frame; the surviving children (ballot-compacted, at most
// 64) form the next frame, which is searched before the parent continues.
// LDS use is bounded by L - 1 frames whatever the size of the search tree.
struct CycFrame {
  uint8_t par[AMLM_WAVE];    // slot of the parent in the frame below
  uint8_t root[AMLM_WAVE];   // root (anchor) slot
  uint32_t eid[AMLM_WAVE];   // edge from the parent to this node
  uint32_t vert[AMLM_WAVE];  // head vertex
  // time of the last edge (first hop: lo - 1) until cyc_prepare reads it,
  // then the first entry of the node's slice (one array, less LDS)
  union {
    int32_t tau[AMLM_WAVE];
    uint32_t xb[AMLM_WAVE];
  };
  uint32_t xoff[AMLM_WAVE];  // exclusive prefix of slice sizes
  uint32_t n, T, cur;
};

// Frame i holds paths of i edges, so cycles of up to L edges need frames
// 0 .. L - 2: the kernel is built for L <= 6 (5 frames) and L <= 8 (7), and
// the smaller LDS footprint of the first runs more waves per CU.
template <int kFrames>
struct CycLds {
  uint32_t r_eid[AMLM_WAVE], r_u[AMLM_WAVE], r_L[AMLM_WAVE];
  int32_t r_t[AMLM_WAVE], r_lo[AMLM_WAVE];
  CycFrame fr[kFrames];
};

// +inc on column `len` for the anchor and every path edge of node (i, slot)
template <class S_t>
__device__ __forceinline__ void cyc_credit_path(const MineParams &mp, const S_t &S, uint32_t i, uint32_t slot,
                                                uint32_t len, uint32_t inc) {
  uint32_t *col = mp.counts + (uint64_t)(mp.col_cyc + (int)len - 2) * mp.stride;
  credit(col + S.r_eid[S.fr[i].root[slot]], inc, mp.ceil);
  for (uint32_t j = i; j >= 1; j--) {
    credit(col + S.fr[j].eid[slot], inc, mp.ceil);
    slot = S.fr[j].par[slot];
  }
}

template <class S_t>
__device__ __forceinline__ bool cyc_on_path(const S_t &S, uint32_t i, uint32_t slot, uint32_t w) {
  for (uint32_t j = i;; j--) {
    if (S.fr[j].vert[slot] == w) return true;
    if (j == 0) return false;
    slot = S.fr[j].par[slot];
  }
}

// Slice bounds of every node of frame i, or, at the last depth, the closing
// edges counted by binary search and credited at once.
template <class S_t>
__device__ void cyc_prepare(const MineParams &mp, S_t &S, uint32_t i) {
  const GraphView &g = mp.g;
  const uint32_t lane = lane_id();
  CycFrame &F = S.fr[i];
  const uint32_t n = rfl(F.n);
  uint32_t nsz = 0, xb = 0;
  if (lane < n) {
    uint32_t r = F.root[lane];
    uint32_t u = S.r_u[r];
    int32_t t = S.r_t[r];
    uint32_t h = F.vert[lane];
    int32_t tau = F.tau[lane];
    const uint32_t Lr = S.r_L[r];
    if (i + 2 == Lr) {
      uint32_t urs = g.in_ptr[u], ure = g.in_ptr[u + 1];
      int32_t tl = tau + 1 < 0 ? 0 : tau + 1;
      uint32_t qa = lower_bound_u64(g.inn_key, urs, ure, nbr_key(h, tl));
      uint32_t qb = lower_bound_u64(g.inn_key, qa, ure, nbr_key(h, t));
      // any order: closing edges at time t too, those before the anchor by id
      uint32_t qc = qb;
      if (mp.cyc_any)
        while (qc < ure && g.inn_key[qc] == nbr_key(h, t) && g.inn_eid[qc] < S.r_eid[r]) qc++;
      uint32_t *col = mp.counts + (uint64_t)(mp.col_cyc + (int)Lr - 2) * mp.stride;
      uint32_t ncl = qb - qa;
      if (mp.cyc_any) {
        ncl = 0;
        for (uint32_t q = qb; q < ure && g.inn_key[q] == nbr_key(h, t); q++) ncl += g.inn_eid[q] < S.r_eid[r];
        ncl += qb - qa;
      }
      if (ncl) {
        cyc_credit_path(mp, S, i, lane, Lr, ncl);
        for (uint32_t q = qa; q < qb; q++) credit(col + g.inn_eid[q], 1u, mp.ceil);
        if (mp.cyc_any)
          for (uint32_t q = qb; q < ure && g.inn_key[q] == nbr_key(h, t); q++)
            if (g.inn_eid[q] < S.r_eid[r]) credit(col + g.inn_eid[q], 1u, mp.ceil);
      }
      (void)qc;
      if (mp.work) {
        // one closing search when the head has an out-edge in its slice, and
        // the credits of the cycles found
        const uint32_t rs = g.out_ptr[h], re = g.out_ptr[h + 1];
        const uint32_t x0 = upper_bound_i32(g.out_t, rs, re, tau);
        unsigned long long w = (unsigned long long)kAlgCycleEdge * Lr * ncl;
        if (x0 < re && (mp.cyc_any ? g.out_t[x0] <= t : g.out_t[x0] < t)) w += kAlgElem * ceil_log2_u32(ure - urs);
        if (w) atomicAdd(&mp.work[kWorkCyc * mp.stride + S.r_eid[r]], w);
      }
    } else {
      uint32_t rs = g.out_ptr[h], re = g.out_ptr[h + 1];
      xb = upper_bound_i32(g.out_t, rs, re, tau);
      nsz = (mp.cyc_any ? upper_bound_i32(g.out_t, xb, re, t) : lower_bound_i32(g.out_t, xb, re, t)) - xb;
      if (mp.work && nsz) atomicAdd(&mp.work[kWorkCyc * mp.stride + S.r_eid[r]], (unsigned long long)kAlgCycElem * nsz);
    }
  }
  uint32_t incl = wave_incl_scan(nsz);
  F.xb[lane] = xb;
  F.xoff[lane] = incl - nsz;
  uint32_t T = (uint32_t)__shfl(incl, AMLM_WAVE - 1, AMLM_WAVE);
  if (lane == 0) {
    F.T = T;
    F.cur = 0;
  }
}

template <int kFrames>
__global__ __launch_bounds__(kCycThreads) void k_cyc(MineParams mp, const uint32_t *roots, const uint32_t *n_in_p,
                                                     uint32_t *ctr) {
  __shared__ CycLds<kFrames> lds[kCycThreads / AMLM_WAVE];
  CycLds<kFrames> &S = lds[threadIdx.x / AMLM_WAVE];
  const GraphView &g = mp.g;
  const uint32_t lane = lane_id();
  const uint64_t lt = lanemask_lt();
  const uint32_t n_in = *n_in_p;
  for (;;) {
    uint32_t base = 0;
    if (lane == 0) base = atomicAdd(ctr, AMLM_WAVE);
    base = rfl((uint32_t)__shfl(base, 0, AMLM_WAVE));
    if (base >= n_in) break;
    uint32_t nr = min((uint32_t)AMLM_WAVE, n_in - base);
    if (lane < nr) {
      uint32_t eid = roots[base + lane];  // edge id of the anchor
      uint32_t v = g.dst[eid];
      int32_t t = g.t[eid];
      uint32_t u = g.src[eid];
      S.r_eid[lane] = eid;
      S.r_u[lane] = u;
      S.r_t[lane] = t;
      S.r_L[lane] = L_of(mp, u);
      CycFrame &F0 = S.fr[0];
      F0.par[lane] = (uint8_t)lane;
      F0.root[lane] = (uint8_t)lane;
      F0.eid[lane] = 0xffffffffu;
      F0.vert[lane] = v;
      S.r_lo[lane] = window_lo(t, delta_of(mp, u));
      F0.tau[lane] = S.r_lo[lane] - 1;  // first hop at time >= lo
    }
    if (lane == 0) S.fr[0].n = nr;
    cyc_prepare(mp, S, 0);
    int sp = 0;
    while (sp >= 0) {
      CycFrame &F = S.fr[sp];
      const uint32_t T = rfl(F.T), cur = rfl(F.cur);
      if (cur >= T) {
        sp--;
        continue;
      }
      const uint32_t n = rfl(F.n);
      uint32_t f = cur + lane;
      bool child = false;
      uint32_t a = 0, w = 0, ceid = 0;
      int32_t ctau = 0;
      if (f < T) {
        uint32_t b = n - 1;
        while (a < b) {
          uint32_t mid = (a + b + 1) >> 1;
          if (F.xoff[mid] <= f) a = mid; else b = mid - 1;
        }
        uint32_t pos = F.xb[a] + (f - F.xoff[a]);
        w = g.out_nbr[pos];
        // any order: only edges before the anchor by (time, edge id), so each
        // cycle is found once, from its greatest edge
        const bool after_anchor = mp.cyc_any && g.out_t[pos] == S.r_t[F.root[a]] &&
                                  g.out_eid[pos] >= S.r_eid[F.root[a]];
        if (after_anchor) {
        } else if (w == S.r_u[F.root[a]]) {
          // closing hop: a cycle of sp + 2 edges
          cyc_credit_path(mp, S, sp, a, sp + 2, 1u);
          credit(mp.counts + (uint64_t)(mp.col_cyc + sp) * mp.stride + g.out_eid[pos], 1u, mp.ceil);
          if (mp.work) atomicAdd(&mp.work[kWorkCyc * mp.stride + S.r_eid[F.root[a]]],
                                 (unsigned long long)kAlgCycleEdge * (sp + 2));
        } else if ((uint32_t)sp + 3 <= S.r_L[F.root[a]] && !cyc_on_path(S, sp, a, w)) {
          child = true;
          ceid = g.out_eid[pos];
          ctau = g.out_t[pos];
        }
      }
      if (lane == 0) F.cur = cur + AMLM_WAVE;
      uint64_t bc = __ballot(child);
      if (bc) {
        CycFrame &G = S.fr[sp + 1];
        if (child) {
          uint32_t slot = __popcll(bc & lt);
          G.par[slot] = (uint8_t)a;
          G.root[slot] = F.root[a];
          G.eid[slot] = ceid;
          G.vert[slot] = w;
          // in order: the next hop leaves after this edge; any order: anywhere in the window
          G.tau[slot] = mp.cyc_any ? S.r_lo[F.root[a]] - 1 : ctau;
        }
        if (lane == 0) G.n = __popcll(bc);
        cyc_prepare(mp, S, sp + 1);
        sp++;
      }
    }
  }
}

// Order-preserving compaction of the indices i with flags[i] != 0 (block
// counts, exclusive scan, scatter).
__global__ void k_flag_count(const uint8_t *flags, uint32_t n, uint32_t *cnt) {
  __shared__ uint32_t ws[kFlagThreads / AMLM_WAVE];
  uint32_t tid = threadIdx.x, w = tid / AMLM_WAVE;
  uint32_t base = blockIdx.x * kFlagTile + tid * kFlagItems;
  uint32_t a = 0;
  for (uint32_t j = 0; j < kFlagItems; j++) a += base + j < n && flags[base + j] != 0;
  for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o, AMLM_WAVE);
  if (lane_id() == 0) ws[w] = a;
  __syncthreads();
  if (tid == 0) {
    uint32_t sa = 0;
    for (int q = 0; q < kFlagThreads / AMLM_WAVE; q++) sa += ws[q];
    cnt[blockIdx.x] = sa;
  }
}

__global__ void k_flag_scatter(const uint8_t *flags, uint32_t n, const uint32_t *off, uint32_t *list) {
  __shared__ uint32_t ws[kFlagThreads / AMLM_WAVE];
  uint32_t tid = threadIdx.x, w = tid / AMLM_WAVE;
  uint32_t base = blockIdx.x * kFlagTile + tid * kFlagItems;
  bool fa[kFlagItems];
  uint32_t a = 0;
  for (uint32_t j = 0; j < kFlagItems; j++) {
    fa[j] = base + j < n && flags[base + j] != 0;
    a += fa[j];
  }
  uint32_t ia = wave_incl_scan(a);
  if (lane_id() == AMLM_WAVE - 1) ws[w] = ia;
  __syncthreads();
  uint32_t pa = off[blockIdx.x] + ia - a;
  for (uint32_t q = 0; q < w; q++) pa += ws[q];
  for (uint32_t j = 0; j < kFlagItems; j++)
    if (fa[j]) list[pa++] = base + j;
}

}  // namespace

// ====================================================================== host

static hipError_t mine_stages(const MineParams &mp, MineScratch &ms, const MineLaunch &cfg, hipStream_t s,
                              StageTimer *tm) {
  hipError_t e;
#define CK(x)                       \
  do {                              \
    e = (x);                        \
    if (e != hipSuccess) return e;  \
  } while (0)
  const uint32_t Ev = mp.g.Ev, E = mp.g.E;
  // work-stealing counters and list sizes
  CK(launch_fill_u32(ms.ctr, 0, kCtrWords, s));
  if (mp.work && E) {
    // accounting run: every edge row's own bytes
    const uint32_t ncols = (mp.col_fo >= 0) + (mp.col_fi >= 0) + (mp.col_sg >= 0) + (mp.col_gs >= 0) +
                           (mp.col_cyc >= 0 ? mp.L - 1 : 0) + (mp.col_do >= 0) + (mp.col_di >= 0);
    hipLaunchKernelGGL(k_alg_io, dim3((E + 255) / 256), dim3(256), 0, s, mp, ncols);
    CK(hipGetLastError());
  }
  if (Ev == 0) return hipSuccess;
  CK(tm->begin(kStAnchor, s));
  CK(launch_fill_u32((uint32_t *)ms.flags, 0, (Ev + 3) / 4 + (E + 3) / 4, s));
  uint8_t *flags_sg = ms.flags, *flags_cy = ms.flags + 4 * ((Ev + 3) / 4);
  // the sliced schedules (the cost model's, the length rule's, the given
  // costs'): heavy anchors cut into slices by their estimated work
  const bool learned = cfg.sched != kSchedStatic && mp.col_sg >= 0 && mp.k >= 2;
  const bool use_mlp = learned && cfg.sched == kSchedLearned;
  uint32_t *feat = use_mlp ? ms.feat : (uint32_t *)nullptr;
  const bool want_sg = mp.col_sg >= 0 || mp.col_gs >= 0;
  const bool want_cyc = mp.col_cyc >= 0;
  uint32_t *n_sg = ms.ctr + kCtrNSg, *n_cy = ms.ctr + kCtrNCy;
  // the cycle roots' list, then the cycle search: on the second stream if
  // given, joined before k_sg
  auto cyc_list = [&]() -> hipError_t {
    hipError_t e;
    uint32_t nb = (E + kFlagTile - 1) / kFlagTile;
    hipLaunchKernelGGL(k_flag_count, dim3(nb), dim3(kFlagThreads), 0, s, flags_cy, E, ms.bcnt_cy);
    CK(hipGetLastError());
    CK(scan_exclusive_u32(ms.bcnt_cy, ms.boff_cy, nb, n_cy, ms.scan_tmp, s));
    hipLaunchKernelGGL(k_flag_scatter, dim3(nb), dim3(kFlagThreads), 0, s, flags_cy, E, ms.boff_cy, ms.list_cy);
    return hipGetLastError();
  };
  auto cyc_search = [&]() -> hipError_t {
    hipError_t e;
    hipStream_t cs = s;
    if (cfg.aux) {
      CK(hipEventRecord(cfg.ev_fork, s));
      CK(hipStreamWaitEvent(cfg.aux, cfg.ev_fork, 0));
      cs = cfg.aux;
    }
    CK(tm->begin(kStCyc, cs));
    if (mp.L <= kCycSmallL)
      hipLaunchKernelGGL(k_cyc<kCycSmallL - 1>, dim3(cfg.cyc_blocks_small), dim3(kCycThreads), 0, cs, mp, ms.list_cy,
                         n_cy, ms.ctr + kCtrCycWork);
    else
      hipLaunchKernelGGL(k_cyc<kMaxDepth + 1>, dim3(cfg.cyc_blocks), dim3(kCycThreads), 0, cs, mp, ms.list_cy, n_cy,
                         ms.ctr + kCtrCycWork);
    CK(hipGetLastError());
    CK(tm->end(kStCyc, cs));
    if (cfg.aux) CK(hipEventRecord(cfg.ev_join, cs));
    return hipSuccess;
  };
  const bool cyc_early = kCycEarly && want_cyc && cfg.aux;
  if (cyc_early) {
    hipLaunchKernelGGL(k_cyc_roots, dim3((Ev + 255) / 256), dim3(256), 0, s, mp, flags_cy);
    CK(hipGetLastError());
    CK(cyc_list());
    CK(cyc_search());
  }
  hipLaunchKernelGGL(k_anchor_out, dim3((Ev + 255) / 256), dim3(256), 0, s, mp, flags_sg, ms.sg_win, feat);
  CK(hipGetLastError());
  hipLaunchKernelGGL(k_anchor_in, dim3((Ev + 255) / 256), dim3(256), 0, s, mp, flags_sg,
                     cyc_early ? (uint8_t *)nullptr : flags_cy, ms.sg_win, feat);
  CK(hipGetLastError());
  CK(tm->end(kStAnchor, s));
  if (mp.work && (mp.col_sg >= 0 || mp.col_gs >= 0)) {
    // accounting run: the method's scatter-gather bytes of every anchor
    hipLaunchKernelGGL(k_alg_sg, dim3(std::min<uint32_t>((Ev + 3) / 4, 65536)), dim3(256), 0, s, mp);
    CK(hipGetLastError());
  }
  if (!want_sg && !want_cyc) return hipSuccess;
  CK(tm->begin(kStLists, s));
  if (want_sg) {
    uint32_t nb = (Ev + kFlagTile - 1) / kFlagTile;
    hipLaunchKernelGGL(k_flag_count, dim3(nb), dim3(kFlagThreads), 0, s, flags_sg, Ev, ms.bcnt_sg);
    CK(hipGetLastError());
    CK(scan_exclusive_u32(ms.bcnt_sg, ms.boff_sg, nb, n_sg, ms.scan_tmp, s));
    hipLaunchKernelGGL(k_flag_scatter, dim3(nb), dim3(kFlagThreads), 0, s, flags_sg, Ev, ms.boff_sg, ms.list_sg);
    CK(hipGetLastError());
  }
  if (want_cyc && !cyc_early) CK(cyc_list());
  CK(tm->end(kStLists, s));
  // independent of the scatter-gather stage: beside the cost model and the
  // work units, and joined before k_sg, which keeps the chip to itself
  if (want_cyc && !cyc_early) CK(cyc_search());
  if (want_sg) {
    // learned schedule: the cost model predicts each item's work, which sets
    // how finely the heavy anchors are sliced
    const float *pred = nullptr;
    if (learned) {
      CK(tm->begin(kStModel, s));
      if (use_mlp) {
        CK(mlp_infer(global_model(), ms.feat, ms.list_sg, 0, n_sg, cfg.delta_hours, (float)mp.L, ms.pred, s,
                     mp.vgraph ? mp.g.in_dst : nullptr, mp.vgraph, mp.sub));
      } else {
        hipLaunchKernelGGL(k_pred_rule, dim3((Ev + 255) / 256), dim3(256), 0, s, mp, ms.list_sg, n_sg,
                           (const uint8_t *)flags_sg, (const uint4 *)ms.sg_win, cfg.sched, cfg.len_coef, cfg.given,
                           ms.pred);
        CK(hipGetLastError());
      }
      pred = ms.pred;
      CK(tm->end(kStModel, s));
    }
    const uint32_t block = std::min(std::max(learned ? cfg.learned_chunk : cfg.sg_chunk, kMinBlock), kSgChunkMax);
    const uint32_t nb = (Ev + 255) / 256;
    if (learned) {
      // work units: blocks of light items and slices of the anchors whose
      // predicted work exceeds the split size, in list order
      CK(tm->begin(kStUnits, s));
      uint32_t *n_units = ms.ctr + kCtrNUnits;
      unsigned long long *W = (unsigned long long *)(ms.ctr + kCtrSplitW);
      hipLaunchKernelGGL(k_split_weight, dim3(nb), dim3(256), 0, s, mp, ms.list_sg, n_sg, flags_sg,
                         (const uint4 *)ms.sg_win, pred, cfg.split_bytes, W);
      CK(hipGetLastError());
      hipLaunchKernelGGL(k_unit_count, dim3(nb), dim3(256), 0, s, mp, ms.list_sg, n_sg, flags_sg,
                         (const uint4 *)ms.sg_win, pred, cfg.split_bytes, (const unsigned long long *)W, block, Ev,
                         ms.nsub, ms.ucnt);
      CK(hipGetLastError());
      CK(scan_exclusive_u32(ms.ucnt, ms.uoff, Ev, n_units, ms.scan_tmp, s, n_sg));
      hipLaunchKernelGGL(k_unit_fill, dim3(nb), dim3(256), 0, s, mp, ms.list_sg, n_sg, ms.nsub, ms.ucnt, ms.uoff,
                         block, ms.units);
      CK(hipGetLastError());
      CK(tm->end(kStUnits, s));
      if (cfg.aux && want_cyc) CK(hipStreamWaitEvent(s, cfg.ev_join, 0));
      CK(tm->begin(kStSg, s));
      hipLaunchKernelGGL(k_sg, dim3(cfg.sg_blocks), dim3(kSgThreads), 0, s, mp, ms.list_sg, (const uint2 *)ms.units,
                         (const uint32_t *)n_units, block, ms.ctr + kCtrSgWork, (const uint4 *)ms.sg_win,
                         (const uint8_t *)flags_sg);
      CK(hipGetLastError());
      {
        hipLaunchKernelGGL(k_split_gs, dim3(nb), dim3(256), 0, s, mp, ms.list_sg, n_sg, ms.nsub,
                           (const uint8_t *)flags_sg);
        CK(hipGetLastError());
      }
    } else {
      // static schedule: fixed blocks of the list
      if (cfg.aux && want_cyc) CK(hipStreamWaitEvent(s, cfg.ev_join, 0));
      CK(tm->begin(kStSg, s));
      hipLaunchKernelGGL(k_sg, dim3(cfg.sg_blocks), dim3(kSgThreads), 0, s, mp, ms.list_sg, (const uint2 *)nullptr,
                         (const uint32_t *)n_sg, block, ms.ctr + kCtrSgWork, (const uint4 *)ms.sg_win,
                         (const uint8_t *)flags_sg);
      CK(hipGetLastError());
    }
    CK(tm->end(kStSg, s));
  }
  if (cfg.aux && want_cyc && !want_sg) CK(hipStreamWaitEvent(s, cfg.ev_join, 0));
#undef CK
  return hipSuccess;
}

hipError_t mine_launch(const MineParams &mp, MineScratch &ms, const MineLaunch &cfg, hipStream_t s,
                       StageTimer *tm) {
  StageTimer none;
  if (!tm) tm = &none;
  // the whole mining, first kernel to last, on the mining stream (the
  // auxiliary stream is joined back before the end)
  hipError_t e = tm->begin(kStMine, s);
  if (e == hipSuccess) e = mine_stages(mp, ms, cfg, s, tm);
  if (e == hipSuccess) e = tm->end(kStMine, s);
  return e;
}

const void *k_sg_ptr() { return (const void *)k_sg; }
const void *k_cyc_ptr(bool small) {
  return small ? (const void *)k_cyc<kCycSmallL - 1> : (const void *)k_cyc<kMaxDepth + 1>;
}
