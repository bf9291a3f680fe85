// Instance columns: participation (AMLM_PART: for every edge, the number of
// scatter-gather and gather-scatter instances it belongs to; Section 8,
// Table 2: a transaction's features count the pattern instances it takes
// part in) and the scatter-gather size bins (AMLM_SG_SIZES: an anchor's
// instances with exactly k, k + 1, k + 2 and at least k + 3 intermediates;
// Section 5's streaming passage counts scatter-gathers of different sizes).
// An instance is an (anchor, sender) pair that SG_k or GS_k counts; an edge
// belongs to it when it is an edge of some realisation of it (one edge per
// leg, the order and window conditions met).
//
// A wave takes 64 anchors (one per lane) from an atomic counter and
// flattens their work over the lanes in three levels, with LDS tables: the
// anchors' sender windows in u's in-row, then for each (anchor, sender) pair
// the shorter of s's out-window [t - delta, t) (found through the out-row
// time index) and v's in-window, whose entries are tested by one search
// each: in v's (source, time)-sorted in-row for the intermediate's latest
// gather leg g_m, or in the intermediate's sorted in-row for a leg from s.
// Per-pair counts in LDS give |M_e(s)| (u included), hence the instance and
// its size bin.  The pass re-derives what it needs from the graph store (it
// does not read the SG / GS columns, which may be saturated).  Credits:
//  * scatter-gather: 1 to the anchor, to s's legs into u (a key range of
//    u's sorted in-row), to every scatter leg earlier than g_m and, from m's
//    first scatter leg f_m, to the gather legs in (f_m, t] (a key range of
//    v's sorted in-row), the instances' out-window entries flattened over
//    the lanes like the counts;
//  * gather-scatter (|S(e)| from the last-edge-of-its-pair test, tau from
//    the first sender entry, k distinct first legs of u in (tau, t] counted
//    by ballots): u's out-row slice (tau, t] gets |S(e)| each, the sender
//    entries 1 each, as range adds into difference arrays summed afterwards
//    (direct atomics on small graphs and narrow anchor ranges).
// Credits saturate at the graph's ceiling like every other count.
#include <algorithm>

#include "api_internal.h"
#include "costmodel.h"

namespace {

constexpr uint32_t kPartAnchors = AMLM_WAVE;  // anchors per claim: one per lane
constexpr uint32_t kPartWaves = 28;           // waves per CU in the grid (7 per SIMD: the register limit)
constexpr uint32_t kCtrPart = 40;             // claim counter word in the mining scratch
constexpr uint32_t kNoPos = 0xffffffffu;
constexpr uint32_t kDiffMinEdges = 4096;
constexpr uint32_t kFiltLog2 = 9, kFiltWords = 1u << kFiltLog2;  // 2 KB filter
constexpr int kFiltShift = 32 - (int)kFiltLog2;      // graphs with fewer valid edges credit gather-scatter directly

__device__ __forceinline__ int32_t part_window_lo(int32_t t, int64_t delta) {
  const int64_t lo = (int64_t)t - delta;
  return lo < -1 ? -1 : (int32_t)lo;
}

__device__ __forceinline__ uint32_t first_lane(uint64_t m) { return (uint32_t)__builtin_ctzll(m); }

// last index j in [0, n) with pref[j] <= f (pref[0] = 0 <= f)
__device__ __forceinline__ uint32_t slot_of(const uint32_t *pref, uint32_t n, uint32_t f) {
  uint32_t lo = 0, hi = n;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (pref[mid] <= f) lo = mid; else hi = mid;
  }
  return lo;
}

struct InstCols {
  int ps, pg, sz;  // SG_PART, GS_PART, first size bin (-1 when absent)
};

// one wave's tables: the chunk's anchors (one per lane) and the (anchor,
// sender) pairs of the current step
struct PartLds {
  uint32_t a_u[AMLM_WAVE], a_v[AMLM_WAVE], a_p0[AMLM_WAVE], a_pref[AMLM_WAVE];
  uint32_t a_vrs[AMLM_WAVE], a_vre[AMLM_WAVE], a_vq0[AMLM_WAVE], a_vlen[AMLM_WAVE];
  int32_t a_t[AMLM_WAVE], a_lo[AMLM_WAVE];
  uint32_t a_k[AMLM_WAVE];  // the anchor's threshold (its sub-graph's in a batched store)
  uint32_t a_inst[AMLM_WAVE], a_bin[4][AMLM_WAVE], a_ns[AMLM_WAVE], a_tau[AMLM_WAVE];
  uint32_t s_r0[AMLM_WAVE], s_pref[AMLM_WAVE], s_cnt[AMLM_WAVE], s_a[AMLM_WAVE], s_s[AMLM_WAVE];
  uint32_t filt[kFiltWords];  // v's in-neighbours, when the chunk's anchors share v
};

// Blocked Bloom filter over vertex hashes (vhash): the top bits pick a word,
// four 5-bit fields of the low bits pick its bits.
__device__ __forceinline__ uint32_t filt_bits(uint32_t h) {
  return (1u << (h & 31)) | (1u << ((h >> 5) & 31)) | (1u << ((h >> 10) & 31)) | (1u << ((h >> 15) & 31));
}

// One out-window entry x (an edge s -> m) of scatter-gather instance
// (anchor a of the chunk, sender s): x is credited when m != u has a gather
// leg into v after it in the window (any, unordered); s's first leg to m
// also credits m's gather legs after it (all in the window, unordered).
__device__ void credit_sg_entry(const MineParams &mp, const PartLds &L, uint32_t a, uint32_t x, uint32_t *col,
                                bool unordered) {
  const GraphView &g = mp.g;
  const uint32_t u = L.a_u[a], vrs = L.a_vrs[a], vre = L.a_vre[a];
  const int32_t t = L.a_t[a], lo = L.a_lo[a];
  const uint32_t m = g.out_nbr[x];
  if (m == u) return;
  const uint32_t qk = upper_bound_u64_interp(g.inn_key, vrs, vre, nbr_key(m, t));
  if (qk == vrs) return;
  const uint64_t key = g.inn_key[qk - 1];
  const int32_t gm = (int32_t)(uint32_t)key;
  if ((uint32_t)(key >> 32) != m || gm < lo) return;  // m has no gather leg in the window
  const int32_t ta = g.out_t[x];
  if (unordered || ta < gm) credit(col + g.out_eid[x], 1u, mp.ceil);
  if (g.out_prv[x] < lo) {  // s's first leg to m: the gather legs after it
    const uint32_t b0 = unordered ? lower_bound_u64(g.inn_key, vrs, qk, nbr_key(m, lo < 0 ? 0 : lo))
                                  : upper_bound_u64_interp(g.inn_key, vrs, qk, nbr_key(m, ta));
    for (uint32_t y = b0; y < qk; y++) credit(col + g.inn_eid[y], 1u, mp.ceil);
  }
}

// The same edges found from the gather side: entry x of v's in-window (an
// edge m -> v) stands for intermediate m when it is m's latest gather leg up
// to t; m belongs to the instance when m's sorted in-row holds a leg from s
// in [lo, g_m) ([lo, t) unordered).  Those legs (a key range of m's in-row)
// and m's gather legs after the first of them (all in the window,
// unordered; a key range of v's in-row) are credited.
__device__ void credit_sg_gather_entry(const MineParams &mp, const PartLds &L, uint32_t a, uint32_t s, uint32_t x,
                                       uint32_t *col, bool unordered) {
  const GraphView &g = mp.g;
  const uint32_t u = L.a_u[a], vrs = L.a_vrs[a], vre = L.a_vre[a];
  const int32_t t = L.a_t[a], lo = L.a_lo[a];
  const int32_t klo = lo < 0 ? 0 : lo;
  const uint32_t m = g.in_nbr[x];
  if (m == u || g.in_nxt[x] <= t) return;
  const int32_t gm = g.in_t[x];
  const uint32_t mrs = g.in_ptr[m], mre = g.in_ptr[m + 1];
  const uint32_t y0 = lower_bound_u64(g.inn_key, mrs, mre, nbr_key(s, klo));
  const uint32_t y1 = lower_bound_u64(g.inn_key, y0, mre, nbr_key(s, unordered ? t : gm));
  if (y0 == y1) return;  // no leg from s: m is not an intermediate of s
  for (uint32_t y = y0; y < y1; y++) credit(col + g.inn_eid[y], 1u, mp.ceil);
  const int32_t fm = (int32_t)(uint32_t)g.inn_key[y0];
  const uint32_t qk = upper_bound_u64_interp(g.inn_key, vrs, vre, nbr_key(m, t));
  const uint32_t b0 = unordered ? lower_bound_u64(g.inn_key, vrs, qk, nbr_key(m, klo))
                                : upper_bound_u64_interp(g.inn_key, vrs, qk, nbr_key(m, fm));
  for (uint32_t b = b0; b < qk; b++) credit(col + g.inn_eid[b], 1u, mp.ceil);
}

// items: every CSC position (ranged = 0), or the edge ids of the anchor
// range [anchor_lo, anchor_lo + n_items) (ranged = 1, self-loops skipped).
// Each anchor takes its (sub-)graph's window and threshold.
__global__ __launch_bounds__(64) void k_part(MineParams mp, InstCols cols, uint32_t n_items, uint32_t ranged,
                                             uint32_t *claim, unsigned long long *diff_r,
                                             unsigned long long *diff_c) {
  const GraphView &g = mp.g;
  __shared__ PartLds L;
  const uint32_t lane = lane_id();
  const bool unordered = mp.sg_unordered != 0;
  uint32_t *const col_ps = cols.ps >= 0 ? mp.counts + (uint64_t)cols.ps * mp.stride : nullptr;
  uint32_t *const col_pg = cols.pg >= 0 ? mp.counts + (uint64_t)cols.pg * mp.stride : nullptr;
  uint32_t *const col_sz = cols.sz >= 0 ? mp.counts + (uint64_t)cols.sz * mp.stride : nullptr;
  const bool want_sg = col_ps || col_sz;
  for (;;) {
    uint32_t i0 = 0;
    if (lane == 0) i0 = atomicAdd(claim, kPartAnchors);
    i0 = __shfl(i0, 0, AMLM_WAVE);
    if (i0 >= n_items) return;

    // 1. one anchor per lane: its senders' window [p0, p1) in u's in-row
    const uint32_t i = i0 + lane;
    bool act = i < n_items;
    uint32_t q = i;
    if (act && ranged) {
      const uint32_t e = mp.anchor_lo + i;
      act = g.src[e] != g.dst[e];
      q = act ? g.pos_in[e] : 0u;
    }
    uint32_t eid = 0, u = 0, v = 0, p0 = 0, p1 = 0, vrs = 0, vre = 0, vq0 = 0, vq1 = 0, k = 1;
    int32_t t = 0, lo = 0;
    if (act) {
      eid = g.in_eid[q];
      act = eid >= mp.anchor_lo && eid < mp.anchor_hi;
    }
    if (act) {
      u = g.in_nbr[q];
      v = g.in_dst[q];
      t = g.in_t[q];
      lo = part_window_lo(t, delta_of(mp, u));
      k = k_of(mp, u);
      const uint32_t cs = g.in_ptr[u], ce = g.in_ptr[u + 1];
      p1 = lower_bound_i32(g.in_t, cs, ce, t);
      p0 = lower_bound_i32(g.in_t, cs, p1, lo);
      vrs = g.in_ptr[v];
      vre = g.in_ptr[v + 1];
      if (want_sg && p1 > p0) {  // v's in-window [lo, t] around the anchor's own entry q
        vq0 = lower_bound_i32(g.in_t, vrs, q, lo);
        vq1 = upper_bound_i32(g.in_t, q + 1, vre, t);
      }
    }
    const uint32_t alen = p1 - p0;
    const uint32_t aincl = wave_incl_scan(alen);
    const uint32_t atotal = __shfl(aincl, AMLM_WAVE - 1, AMLM_WAVE);
    L.a_u[lane] = u;
    L.a_v[lane] = v;
    L.a_t[lane] = t;
    L.a_lo[lane] = lo;
    L.a_k[lane] = k;
    L.a_p0[lane] = p0;
    L.a_pref[lane] = aincl - alen;
    L.a_vrs[lane] = vrs;
    L.a_vre[lane] = vre;
    L.a_vq0[lane] = vq0;
    L.a_vlen[lane] = vq1 - vq0;
    L.a_inst[lane] = 0u;
    for (int b = 0; b < 4; b++) L.a_bin[b][lane] = 0u;
    L.a_ns[lane] = 0u;
    L.a_tau[lane] = kNoPos;
    // a chunk inside one v's in-row (a hub's, typically): a filter of v's
    // in-neighbours over the union of the anchors' windows rejects most
    // forward join entries before their search (no false negatives: every
    // anchor's window lies inside the union)
    const uint64_t amask = __ballot(act);
    bool use_filt = false;
    if (want_sg && amask) {
      const uint32_t v0 = __shfl(v, (int)first_lane(amask), AMLM_WAVE);
      use_filt = !__ballot(act && v != v0);
      if (use_filt) {
        int32_t wlo = act ? lo : AMLM_INT_MAX, whi = act ? t : AMLM_INT_MIN;
        for (int o = AMLM_WAVE / 2; o > 0; o >>= 1) {
          wlo = min(wlo, __shfl_xor(wlo, o, AMLM_WAVE));
          whi = max(whi, __shfl_xor(whi, o, AMLM_WAVE));
        }
        const uint32_t frs = g.in_ptr[v0], fre = g.in_ptr[v0 + 1];
        const uint32_t f0 = lower_bound_i32(g.in_t, frs, fre, wlo), f1 = upper_bound_i32(g.in_t, f0, fre, whi);
        for (uint32_t w = lane; w < kFiltWords; w += AMLM_WAVE) L.filt[w] = 0u;
        __syncthreads();
        for (uint32_t q = f0 + lane; q < f1; q += AMLM_WAVE) {
          const uint32_t h = g.in_h[q];
          atomicOr(&L.filt[h >> kFiltShift], filt_bits(h));
        }
      }
    }
    __syncthreads();

    // 2. every (anchor, sender-window entry) item over the lanes: distinct
    //    senders (the last edge of their pair before t), |S(e)| and tau
    for (uint32_t f0 = 0; f0 < atotal; f0 += AMLM_WAVE) {
      const uint32_t f = f0 + lane;
      bool snd = false;
      uint32_t a = 0, s = 0, r0 = 0, r1 = 0;
      if (f < atotal) {
        a = slot_of(L.a_pref, AMLM_WAVE, f);
        const uint32_t p = L.a_p0[a] + (f - L.a_pref[a]);
        const uint32_t sn = g.in_nbr[p];
        if (sn != L.a_v[a]) {
          if (col_pg) atomicMin(&L.a_tau[a], p);
          if (g.in_nxt[p] >= L.a_t[a]) {
            snd = true;
            s = sn;
            if (col_pg) atomicAdd(&L.a_ns[a], 1u);
          }
        }
      }
      if (!want_sg) continue;
      if (snd) {  // s's out-window [lo, t) through the out-row time index
        const uint32_t rs = g.out_ptr[s], re = g.out_ptr[s + 1];
        const uint4 tm = g.out_tm[s];
        r0 = tix_lower_bound(g.out_t, g.out_tix, tm, rs, re, L.a_lo[a]);
        r1 = tix_lower_bound(g.out_t, g.out_tix, tm, rs, re, L.a_t[a]);
      }
      const uint64_t smask = __ballot(snd);
      if (!smask) continue;
      // degree-ordered join: the shorter of s's out-window and v's in-window
      const uint32_t rv = snd ? L.a_vlen[a] : 0u;
      const bool rev = rv < r1 - r0;
      const uint32_t len = rev ? rv : r1 - r0;
      const uint32_t incl = wave_incl_scan(len);
      const uint32_t total = __shfl(incl, AMLM_WAVE - 1, AMLM_WAVE);
      const uint32_t slot = (uint32_t)__popcll(smask & lanemask_lt());
      const uint32_t nsnd = (uint32_t)__popcll(smask);
      if (snd) {
        L.s_r0[slot] = rev ? L.a_vq0[a] : r0;
        L.s_pref[slot] = incl - len;
        L.s_cnt[slot] = 0u;
        L.s_a[slot] = a | (rev ? 0x80000000u : 0u);
        L.s_s[slot] = s;
      }
      __syncthreads();
      // 3. every (pair, join entry) item.  Forward (an entry of s's
      //    out-window): s's first leg to an intermediate m != u counts when m
      //    has a gather leg into v in the window, later than the scatter leg
      //    unless unordered.  Reversed (an entry of v's in-window): m's latest
      //    gather leg g_m up to t counts when m's sorted in-row holds a leg
      //    from s in [lo, g_m) ([lo, t) unordered).
      for (uint32_t h0 = 0; h0 < total; h0 += AMLM_WAVE) {
        const uint32_t h = h0 + lane;
        if (h >= total) continue;
        const uint32_t j = slot_of(L.s_pref, nsnd, h);
        const uint32_t x = L.s_r0[j] + (h - L.s_pref[j]);
        const uint32_t pa = L.s_a[j] & 0x7fffffffu;
        // a pair's count matters up to k - 1 (the instance), or k + 2 (the
        // size bins): entries after that are skipped
        if (L.s_cnt[j] >= (col_sz ? L.a_k[pa] + 2 : L.a_k[pa] - 1)) continue;
        const int32_t plo = L.a_lo[pa];
        if (L.s_a[j] >> 31) {
          const uint32_t m = g.in_nbr[x];
          const int32_t pt = L.a_t[pa];
          if (m == L.a_u[pa] || g.in_nxt[x] <= pt) continue;
          const uint32_t ms = L.s_s[j], mrs = g.in_ptr[m], mre = g.in_ptr[m + 1];
          const uint32_t y = lower_bound_u64(g.inn_key, mrs, mre, nbr_key(ms, plo < 0 ? 0 : plo));
          if (y < mre && g.inn_key[y] < nbr_key(ms, unordered ? pt : g.in_t[x])) atomicAdd(&L.s_cnt[j], 1u);
          continue;
        }
        const uint32_t m = g.out_nbr[x];
        if (m == L.a_u[pa] || g.out_prv[x] >= plo) continue;
        if (use_filt) {
          const uint32_t h = g.out_h[x], fb = filt_bits(h);
          if ((L.filt[h >> kFiltShift] & fb) != fb) continue;  // no edge m -> v in the chunk's windows
        }
        const uint32_t pvrs = L.a_vrs[pa], pvre = L.a_vre[pa];
        const uint32_t qk = upper_bound_u64_interp(g.inn_key, pvrs, pvre, nbr_key(m, L.a_t[pa]));
        if (qk == pvrs) continue;
        const uint64_t key = g.inn_key[qk - 1];
        const int32_t gm = (int32_t)(uint32_t)key;
        if ((uint32_t)(key >> 32) == m && gm >= plo && (unordered || gm > g.out_t[x])) atomicAdd(&L.s_cnt[j], 1u);
      }
      __syncthreads();
      // |M_e(s)| = 1 (u) + the intermediates counted (at least the cap once
      // it is reached): the instance and its bin
      const uint32_t size = snd ? 1u + L.s_cnt[slot] : 0u, ka = snd ? L.a_k[a] : 1u;
      const bool inst = snd && size >= ka;
      if (inst) {
        atomicAdd(&L.a_inst[a], 1u);
        atomicAdd(&L.a_bin[size - ka < 3 ? size - ka : 3u][a], 1u);
      }
      const uint64_t imask = col_ps ? __ballot(inst) : 0ull;
      __syncthreads();  // the pair slots are rewritten below and by the next step
      if (!imask) continue;
      // 3b. the instances' edges.  Each instance's lane credits s's legs
      //     into u in [lo, t) (a key range of u's sorted in-row); the
      //     instances' out-window entries are flattened over the lanes
      // (the shorter of s's out-window and v's in-window, as for the counts)
      const uint32_t ilen = inst ? (rev ? rv : r1 - r0) : 0u;
      const uint32_t iincl = wave_incl_scan(ilen);
      const uint32_t itotal = __shfl(iincl, AMLM_WAVE - 1, AMLM_WAVE);
      const uint32_t ni = (uint32_t)__popcll(imask);
      if (inst) {
        const uint32_t islot = (uint32_t)__popcll(imask & lanemask_lt());
        L.s_r0[islot] = rev ? L.a_vq0[a] : r0;
        L.s_pref[islot] = iincl - ilen;
        L.s_a[islot] = a | (rev ? 0x80000000u : 0u);
        L.s_s[islot] = s;
        const uint32_t ua = L.a_u[a];
        const int32_t la = L.a_lo[a];
        const uint32_t cs = g.in_ptr[ua], ce = g.in_ptr[ua + 1];
        const uint32_t a0 = lower_bound_u64(g.inn_key, cs, ce, nbr_key(s, la < 0 ? 0 : la));
        const uint32_t a1 = lower_bound_u64(g.inn_key, a0, ce, nbr_key(s, L.a_t[a]));
        for (uint32_t x = a0; x < a1; x++) credit(col_ps + g.inn_eid[x], 1u, mp.ceil);
      }
      __syncthreads();
      for (uint32_t h0 = 0; h0 < itotal; h0 += AMLM_WAVE) {
        const uint32_t h = h0 + lane;
        if (h >= itotal) continue;
        const uint32_t j = slot_of(L.s_pref, ni, h);
        const uint32_t x = L.s_r0[j] + (h - L.s_pref[j]), pa = L.s_a[j] & 0x7fffffffu;
        if (L.s_a[j] >> 31) {
          credit_sg_gather_entry(mp, L, pa, L.s_s[j], x, col_ps, unordered);
        } else {
          if (use_filt) {  // m without an edge to v in the windows credits nothing
            const uint32_t hx = g.out_h[x], fb = filt_bits(hx);
            if ((L.filt[hx >> kFiltShift] & fb) != fb) continue;
          }
          credit_sg_entry(mp, L, pa, x, col_ps, unordered);
        }
      }
      __syncthreads();  // the pair slots are rewritten by the next step
    }
    __syncthreads();

    // 4. gather-scatter: |S(e)| >= k and k distinct destinations of u in
    //    (tau, t]; its edges are u's out-edges there (|S(e)| instances each)
    //    and the sender entries
    if (col_pg) {
      bool cand = false;
      uint32_t ns = 0, d0 = 0, d1 = 0;
      int32_t tau = 0;
      if (act && L.a_tau[lane] != kNoPos && L.a_ns[lane] >= k) {
        cand = true;
        ns = L.a_ns[lane];
        tau = g.in_t[L.a_tau[lane]];
        const uint32_t rs = g.out_ptr[u], re = g.out_ptr[u + 1];
        d0 = upper_bound_i32(g.out_t, rs, re, tau);
        d1 = upper_bound_i32(g.out_t, d0, re, t);
      }
      uint64_t cmask = __ballot(cand);
      while (cmask) {
        const uint32_t j = first_lane(cmask);
        cmask &= cmask - 1;
        const uint32_t kj = __shfl(k, (int)j, AMLM_WAVE), nj = __shfl(ns, (int)j, AMLM_WAVE);
        const int32_t tj = __shfl(tau, (int)j, AMLM_WAVE);
        const uint32_t dj0 = __shfl(d0, (int)j, AMLM_WAVE), dj1 = __shfl(d1, (int)j, AMLM_WAVE);
        // k distinct destinations: first edges of their pairs in (tau, t], by ballots
        uint32_t nd = 0;
        for (uint32_t b = dj0; b < dj1 && nd < kj; b += AMLM_WAVE) {
          const uint32_t p = b + lane;
          nd += (uint32_t)__popcll(__ballot(p < dj1 && g.out_prv[p] <= tj));
        }
        if (nd < kj) continue;
        const uint32_t vj = __shfl(v, (int)j, AMLM_WAVE);
        const uint32_t pj0 = __shfl(p0, (int)j, AMLM_WAVE), pj1 = __shfl(p1, (int)j, AMLM_WAVE);
        if (diff_r) {
          // range adds: u's out-row slice [d0, d1) by |S(e)|, the sender
          // entries [p0, p1) by 1, less the entries from v (summed later)
          if (lane == 0) {
            atomicAdd(&diff_r[dj0], (unsigned long long)nj);
            atomicAdd(&diff_r[dj1], 0ull - nj);
            atomicAdd(&diff_c[pj0], 1ull);
            atomicAdd(&diff_c[pj1], ~0ull);
          }
          for (uint32_t p = pj0 + lane; p < pj1; p += AMLM_WAVE)
            if (g.in_nbr[p] == vj) {
              atomicAdd(&diff_c[p], ~0ull);
              atomicAdd(&diff_c[p + 1], 1ull);
            }
        } else {
          for (uint32_t p = dj0 + lane; p < dj1; p += AMLM_WAVE) credit(col_pg + g.out_eid[p], nj, mp.ceil);
          for (uint32_t p = pj0 + lane; p < pj1; p += AMLM_WAVE)
            if (g.in_nbr[p] != vj) credit(col_pg + g.in_eid[p], 1u, mp.ceil);
        }
      }
    }

    // 5. the anchor's own counts
    if (act) {
      if (col_ps && L.a_inst[lane]) credit(col_ps + eid, L.a_inst[lane], mp.ceil);
      for (int b = 0; b < 4 && col_sz; b++)
        if (L.a_bin[b][lane]) credit(col_sz + (uint64_t)b * mp.stride + eid, L.a_bin[b][lane], mp.ceil);
    }
    __syncthreads();  // the tables are rewritten by the next chunk
  }
}

// Range adds of the gather-scatter credits, summed: positions are split in
// tiles of kDiffTile; the tiles' sums, their exclusive scan, then each
// position's running sum credited to its edge (values are sums of
// non-negative counts modulo 2^64, so the wrapped negative markers cancel).
constexpr uint32_t kDiffThreads = 256, kDiffItems = 8, kDiffTile = kDiffThreads * kDiffItems;

__global__ __launch_bounds__(kDiffThreads) void k_diff_tile_sums(const unsigned long long *diff, uint32_t n,
                                                                 unsigned long long *sums) {
  __shared__ unsigned long long ws[kDiffThreads / AMLM_WAVE];
  const uint32_t base = blockIdx.x * kDiffTile;
  unsigned long long x = 0;
  for (uint32_t i = threadIdx.x; i < kDiffTile; i += kDiffThreads)
    if (base + i < n) x += diff[base + i];
  for (int o = AMLM_WAVE / 2; o > 0; o >>= 1) x += __shfl_xor(x, o, AMLM_WAVE);
  if (lane_id() == 0) ws[threadIdx.x / AMLM_WAVE] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long t = 0;
    for (uint32_t w = 0; w < kDiffThreads / AMLM_WAVE; w++) t += ws[w];
    sums[blockIdx.x] = t;
  }
}

__device__ __forceinline__ unsigned long long wave_incl_scan_u64(unsigned long long x) {
  const uint32_t lane = lane_id();
#pragma unroll
  for (int d = 1; d < AMLM_WAVE; d <<= 1) {
    const unsigned long long y = __shfl_up(x, d, AMLM_WAVE);
    if (lane >= (uint32_t)d) x += y;
  }
  return x;
}

// exclusive scan of the nt tile sums, in place (one block)
__global__ __launch_bounds__(1024) void k_diff_scan_sums(unsigned long long *sums, uint32_t nt) {
  __shared__ unsigned long long ws[1024 / AMLM_WAVE];
  __shared__ unsigned long long carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (uint32_t b = 0; b < nt; b += 1024) {
    const uint32_t i = b + threadIdx.x;
    const unsigned long long x = i < nt ? sums[i] : 0ull;
    const unsigned long long y = wave_incl_scan_u64(x);
    if (lane_id() == AMLM_WAVE - 1) ws[threadIdx.x / AMLM_WAVE] = y;
    __syncthreads();
    unsigned long long before = carry;
    for (uint32_t w = 0; w < threadIdx.x / AMLM_WAVE; w++) before += ws[w];
    if (i < nt) sums[i] = before + y - x;
    __syncthreads();
    if (threadIdx.x == 1023) carry = before + y;
    __syncthreads();
  }
}

// position p's running sum, credited to edge eid[p]
__global__ __launch_bounds__(kDiffThreads) void k_diff_apply(const unsigned long long *diff, uint32_t n,
                                                             const unsigned long long *offs, const uint32_t *eid,
                                                             uint32_t *col, uint32_t ceil) {
  __shared__ unsigned long long ws[kDiffThreads / AMLM_WAVE];
  const uint32_t base = blockIdx.x * kDiffTile + threadIdx.x * kDiffItems;
  unsigned long long v[kDiffItems];
  unsigned long long run = 0;
#pragma unroll
  for (uint32_t j = 0; j < kDiffItems; j++) {
    run += base + j < n ? diff[base + j] : 0ull;
    v[j] = run;
  }
  const unsigned long long incl = wave_incl_scan_u64(run);
  if (lane_id() == AMLM_WAVE - 1) ws[threadIdx.x / AMLM_WAVE] = incl;
  __syncthreads();
  unsigned long long before = offs[blockIdx.x] + incl - run;
  for (uint32_t w = 0; w < threadIdx.x / AMLM_WAVE; w++) before += ws[w];
#pragma unroll
  for (uint32_t j = 0; j < kDiffItems; j++) {
    const unsigned long long x = before + v[j];
    if (base + j < n && x) credit(col + eid[base + j], x < 0xffffffffull ? (uint32_t)x : 0xffffffffu, ceil);
  }
}

// the instance columns' output bytes of each anchor in range
__global__ __launch_bounds__(256) void k_part_io(MineParams mp, uint32_t ncols_part) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= mp.g.E || i < mp.anchor_lo || i >= mp.anchor_hi) return;
  mp.work[kWorkIo * mp.stride + i] += (unsigned long long)kAlgCount * ncols_part;
}

}  // namespace

void part_columns(const amlm_params *p, int *c_ps, int *c_pg, int *c_sz) {
  *c_ps = *c_pg = *c_sz = -1;
  int c = (int)amlm_num_columns(p);
  if (p->patterns & AMLM_SG_SIZES) *c_sz = c -= 4;
  if (!(p->patterns & AMLM_PART)) return;
  if (p->patterns & AMLM_GS) *c_pg = --c;
  if (p->patterns & AMLM_SG) *c_ps = --c;
}

hipError_t part_launch(const MineParams &mp, const amlm_params *p, MineScratch &ms, hipStream_t s) {
  InstCols cols;
  part_columns(p, &cols.ps, &cols.pg, &cols.sz);
  if (cols.ps < 0 && cols.pg < 0 && cols.sz < 0) return hipSuccess;
  const uint32_t npart = (cols.ps >= 0) + (cols.pg >= 0) + (cols.sz >= 0 ? 4 : 0);
  if (mp.work && mp.g.E) {
    hipLaunchKernelGGL(k_part_io, dim3((mp.g.E + 255) / 256), dim3(256), 0, s, mp, npart);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (mp.g.Ev == 0) return hipSuccess;
  // a narrow anchor range (the server's batches) is walked by edge id
  const uint32_t hi = (uint32_t)std::min<uint64_t>(mp.anchor_hi, mp.g.E);
  const uint32_t lo = std::min(mp.anchor_lo, hi);
  const bool ranged = hi - lo < mp.g.Ev;
  const uint32_t n_items = ranged ? hi - lo : mp.g.Ev;
  if (n_items == 0) return hipSuccess;
  uint32_t *claim = ms.ctr + kCtrPart;
  hipError_t e = launch_fill_u32(claim, 0, 1, s);
  if (e != hipSuccess) return e;
  // gather-scatter credits as range adds into two difference arrays (CSR
  // and CSC positions), in the cost model's feature buffer, which the
  // mining no longer needs: Ev + 1 entries each, then the tile sums; small
  // graphs and narrow anchor ranges (stream batches) credit directly
  const uint32_t Ev = mp.g.Ev, nt = (Ev + kDiffTile - 1) / kDiffTile;
  unsigned long long *diff_r = nullptr, *diff_c = nullptr, *sums_r = nullptr, *sums_c = nullptr;
  const uint64_t need = 2ull * (Ev + 1) + 2ull * nt;  // 64-bit words
  if (cols.pg >= 0 && !ranged && Ev >= kDiffMinEdges && need * 2 <= (uint64_t)kMlpRaw * ms.cap_ev) {
    diff_r = (unsigned long long *)ms.feat;
    diff_c = diff_r + Ev + 1;
    sums_r = diff_c + Ev + 1;
    sums_c = sums_r + nt;
    e = launch_fill_u32(ms.feat, 0, 4ull * (Ev + 1), s);
    if (e != hipSuccess) return e;
  }
  const uint32_t blocks = std::min<uint32_t>((uint32_t)device_info().num_cu * kPartWaves,
                                             (n_items + kPartAnchors - 1) / kPartAnchors);
  hipLaunchKernelGGL(k_part, dim3(blocks), dim3(64), 0, s, mp, cols, n_items, ranged ? 1u : 0u, claim, diff_r,
                     diff_c);
  e = hipGetLastError();
  if (e != hipSuccess || !diff_r) return e;
  uint32_t *col_pg = mp.counts + (uint64_t)cols.pg * mp.stride;
  for (int side = 0; side < 2; side++) {
    unsigned long long *d = side ? diff_c : diff_r, *sm = side ? sums_c : sums_r;
    const uint32_t *eids = side ? mp.g.in_eid : mp.g.out_eid;
    hipLaunchKernelGGL(k_diff_tile_sums, dim3(nt), dim3(kDiffThreads), 0, s, d, Ev, sm);
    hipLaunchKernelGGL(k_diff_scan_sums, dim3(1), dim3(1024), 0, s, sm, nt);
    hipLaunchKernelGGL(k_diff_apply, dim3(nt), dim3(kDiffThreads), 0, s, d, Ev, (const unsigned long long *)sm, eids,
                       col_pg, mp.ceil);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}
