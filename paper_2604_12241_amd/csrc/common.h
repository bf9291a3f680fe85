// Device-side helpers and the graph store layout shared by the build and the
// mining kernels.  gfx950 (CDNA4): 64-lane wavefronts, 64-bit ballot masks.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define AMLM_WAVE 64
#define AMLM_INT_MAX 0x7fffffff
#define AMLM_INT_MIN (-0x7fffffff - 1)


// Graph store in HBM.  All positions and edge ids fit in 32 bits.
//  * anchors: valid (non-self-loop) edge ids in (time, id) order
//  * CSR (out): rows by source, each row sorted by (time, id); per entry the
//    destination, the time, the edge id and the time of the previous edge of
//    the same (source, destination) pair (AMLM_INT_MIN if none), and
//    vhash(destination) (the scatter-gather join's filter key); a time index
//    per row
//  * CSC (in): rows by destination, sorted by (time, id); per entry the
//    source, time, edge id and the time of the next edge of the same pair
//    (AMLM_INT_MAX if none)
//  * CSC-N: the CSC rows re-sorted by (source, time); 64-bit keys
//    (source << 32 | time) for binary search, and the edge ids
struct GraphView {
  uint32_t V;
  uint32_t E;   // all edges, including self-loops
  uint32_t Ev;  // non-self-loop edges
  const uint32_t *src, *dst;
  const int32_t *t;  // time relative to the minimum timestamp
  const uint32_t *anc;
  const uint32_t *pos_out, *pos_in;  // edge id -> CSR / CSC position
  const uint32_t *out_ptr, *out_nbr, *out_eid, *out_src;  // out_src: row (source) of each entry
  const uint32_t *out_h;  // vhash(out_nbr[p])
  // time index of the out-rows (see tix_lower_bound): per vertex (offset,
  // buckets, first time, bucket shift), and the bucket starts
  const uint4 *out_tm;
  const uint32_t *out_tix;
  const int32_t *out_t, *out_prv;
  const uint32_t *in_ptr, *in_nbr, *in_eid, *in_dst;  // in_dst: row (destination) of each entry
  const uint32_t *in_h;  // vhash(in_nbr[q])
  const int32_t *in_t, *in_nxt;
  const uint64_t *inn_key;
  const uint32_t *inn_eid;
};

// MurmurHash3's 32-bit finaliser (fmix32): a bijection on 32-bit words with
// full avalanche, so two vertices share a hash only if they are equal.
constexpr uint32_t kFmixC1 = 0x85EBCA6Bu, kFmixC2 = 0xC2B2AE35u;
constexpr uint32_t inverse_mod_2_32(uint32_t c) {  // c odd; Newton steps double the correct bits
  uint32_t x = c;
  for (int i = 0; i < 5; i++) x *= 2u - c * x;
  return x;
}
__host__ __device__ __forceinline__ uint32_t vhash(uint32_t x) {
  x ^= x >> 16;
  x *= kFmixC1;
  x ^= x >> 13;
  x *= kFmixC2;
  x ^= x >> 16;
  return x;
}
__host__ __device__ __forceinline__ uint32_t vhash_inv(uint32_t x) {
  x ^= x >> 16;
  x *= inverse_mod_2_32(kFmixC2);
  x ^= (x >> 13) ^ (x >> 26);
  x *= inverse_mod_2_32(kFmixC1);
  x ^= x >> 16;
  return x;
}

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }
__device__ __forceinline__ uint64_t lanemask_lt() { return (1ull << __lane_id()) - 1ull; }

// first index in [b, e) with a[i] >= x
__device__ __forceinline__ uint32_t lower_bound_i32(const int32_t *a, uint32_t b, uint32_t e, int32_t x) {
  while (b < e) {
    uint32_t m = b + ((e - b) >> 1);
    if (a[m] < x) b = m + 1; else e = m;
  }
  return b;
}
// first index in [b, e) with a[i] > x
__device__ __forceinline__ uint32_t upper_bound_i32(const int32_t *a, uint32_t b, uint32_t e, int32_t x) {
  while (b < e) {
    uint32_t m = b + ((e - b) >> 1);
    if (a[m] <= x) b = m + 1; else e = m;
  }
  return b;
}
// first index in [b, e) with a[i] >= x
__device__ __forceinline__ uint32_t lower_bound_u64(const uint64_t *a, uint32_t b, uint32_t e, uint64_t x) {
  while (b < e) {
    uint32_t m = b + ((e - b) >> 1);
    if (a[m] < x) b = m + 1; else e = m;
  }
  return b;
}

// Galloping searches from a known position.  gallop_lower_left: first index
// in [b, p] with a[i] >= x, given a[p] >= x.  gallop_lower_right: first index
// in [p, e) with a[i] >= x (e if none), given that every a[i] before p is < x.
__device__ __forceinline__ uint32_t gallop_lower_left(const int32_t *a, uint32_t b, uint32_t p, int32_t x) {
  uint32_t hi = p, step = 1;
  while (hi > b) {
    uint32_t probe = hi - b > step ? hi - step : b;
    if (a[probe] < x) return lower_bound_i32(a, probe + 1, hi, x);
    hi = probe;
    step <<= 1;
  }
  return b;
}
__device__ __forceinline__ uint32_t gallop_lower_right(const int32_t *a, uint32_t p, uint32_t e, int32_t x) {
  uint32_t lo = p, step = 1;
  while (lo < e) {
    uint32_t probe = e - lo > step ? lo + step - 1 : e - 1;
    if (a[probe] >= x) return lower_bound_i32(a, lo, probe, x);
    lo = probe + 1;
    step <<= 1;
  }
  return e;
}

// Row time index.  A row longer than kTixMinRow entries is cut into nb
// buckets of 2^w time units starting at its first time t0, with w the
// smallest shift that leaves at most ceil(len / kTixPerBucket) buckets;
// tix[off + i] is the first position whose time is >= t0 + (i << w), and
// tix[off + nb] is the row end.  m = (off, nb, t0, w); nb = 0 for short rows.
constexpr uint32_t kTixMinRow = 32, kTixPerBucket = 16;

// first position in the row [rs, re) with time >= x
__device__ __forceinline__ uint32_t tix_lower_bound(const int32_t *t, const uint32_t *tix, uint4 m, uint32_t rs,
                                                    uint32_t re, int32_t x) {
  if (m.y == 0) return lower_bound_i32(t, rs, re, x);
  const int32_t t0 = (int32_t)m.z;
  if (x <= t0) return rs;
  const uint32_t i = (uint32_t)(x - t0) >> m.w;
  if (i >= m.y) return re;
  return lower_bound_i32(t, tix[m.x + i], tix[m.x + i + 1], x);
}

// First index in [b, e) with a[i] > key, for sorted 64-bit keys.
// Interpolation steps (on the key values) alternate with bisection steps, so
// the search takes at most about twice the steps of a binary search and a
// few steps when the keys are spread evenly; the last <= 8 entries are
// compared with independent loads.
__device__ __forceinline__ uint32_t upper_bound_u64_interp(const uint64_t *a, uint32_t b, uint32_t e, uint64_t key) {
  if (b >= e) return b;
  uint32_t lo = b, hi = e;  // answer in [lo, hi]
  uint64_t klo = a[b], khi = a[e - 1];
  if (key < klo) return b;
  if (key >= khi) return e;
  // here a[lo] <= key < a[hi - 1]; klo = a[lo], khi = a[hi - 1]
  bool interp = true;
  while (hi - lo > 8) {
    uint32_t mid;
    if (interp && khi > klo) {
      double frac = (double)(key - klo) / (double)(khi - klo);
      mid = lo + (uint32_t)(frac * (double)(hi - 1 - lo));
      if (mid <= lo) mid = lo + 1;
      if (mid >= hi - 1) mid = hi - 2;
    } else {
      mid = lo + ((hi - lo) >> 1);
    }
    interp = !interp;
    uint64_t km = a[mid];
    if (km <= key) {
      lo = mid;
      klo = km;
    } else {
      hi = mid + 1;
      khi = km;
    }
  }
  // answer = first i in (lo, hi) with a[i] > key (a[hi - 1] > key holds)
  uint32_t ans = hi - 1;
#pragma unroll
  for (int j = 8; j >= 1; j--) {
    uint32_t i = lo + (uint32_t)j;
    if (i < hi - 1 && a[i] > key) ans = i;
  }
  return ans;
}

// first index in [p, e) with a[i] > x, given that every a[i] before p is <= x
__device__ __forceinline__ uint32_t gallop_upper_right(const int32_t *a, uint32_t p, uint32_t e, int32_t x) {
  return gallop_lower_right(a, p, e, x + 1);  // integer times: > x is >= x + 1 (x < INT_MAX)
}

__device__ __forceinline__ uint64_t nbr_key(uint32_t nbr, int32_t t) {
  return ((uint64_t)nbr << 32) | (uint32_t)t;
}

// Wave-wide inclusive scan of a 32-bit value (64 lanes).
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x) {
  uint32_t lane = lane_id();
#pragma unroll
  for (int d = 1; d < AMLM_WAVE; d <<= 1) {
    uint32_t y = __shfl_up(x, d, AMLM_WAVE);
    if (lane >= (uint32_t)d) x += y;
  }
  return x;
}

// Saturating credit: adds inc to *p, which ends at ceil if the sum of all
// credits to it passes ceil (or 2^32 - 1).  A thread whose add wraps raises
// the word to 2^32 - 1 and one whose add lands above ceil lowers it to ceil;
// every add that finds the word at or above ceil (or wraps it) does the same
// afterwards, so the last operation on a saturated word leaves ceil in it,
// whatever the interleaving, while sums that stay within ceil are untouched.
__device__ __forceinline__ void credit(uint32_t *p, uint32_t inc, uint32_t ceil) {
  const uint32_t old = atomicAdd(p, inc);
  const uint32_t sum = old + inc;
  if (sum < old) atomicMax(p, 0xffffffffu);
  if ((sum < old || sum > ceil) && ceil != 0xffffffffu) atomicMin(p, ceil);
}
