// Mining kernels.
//
//  k_anchor  one lane per anchor (time order): window bounds by binary search
//            (Find_Starting_Edge, Algorithm 1), FAN_OUT / FAN_IN, the size of
//            the sender set S(e) when its window slice is short, and the
//            classification of the anchor into the scatter-gather and cycle
//            work lists.
//  k_sg      one wave per scatter-gather anchor (Section 5 scatter-gather
//            decomposition, Section 6 compiled example): the wave scans the
//            anchor's sender window, stages v's in-window in an LDS Bloom
//            filter, then scans every sender's out-window, lanes flattened
//            over (sender, entry) pairs; filter hits are confirmed by binary
//            search in the neighbour-sorted in-index.  Also gather-scatter.
//  k_cyc     bounded time-respecting cycle search (Section 5 cycle
//            decomposition; Section 6 4-cycle example: expansion, then the
//            closing intersection by binary search over sorted neighbour
//            lists).  A wave takes 64 anchors and searches depth first over
//            frames of up to 64 partial paths; each frame's time slices are
//            flattened over the lanes and the surviving paths are compacted
//            into the next frame with ballot + popcount.
#include "mine.h"

namespace {

__device__ __forceinline__ int32_t window_lo(int32_t t, int64_t delta) {
  int64_t lo = (int64_t)t - delta;
  return lo < -1 ? -1 : (int32_t)lo;
}

__device__ __forceinline__ uint32_t rfl(uint32_t x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ int32_t rfl(int32_t x) { return (int32_t)__builtin_amdgcn_readfirstlane((uint32_t)x); }

// ------------------------------------------------------------------ k_anchor
__global__ __launch_bounds__(256) void k_anchor(MineParams mp, uint8_t *flags) {
  const GraphView &g = mp.g;
  uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= g.Ev) return;
  uint32_t eid = g.anc[p];
  uint32_t u = g.src[eid], v = g.dst[eid];
  int32_t t = g.t[eid];
  int32_t lo = window_lo(t, mp.delta);
  uint8_t f = 0;
  if (mp.col_fo >= 0) {
    uint32_t rs = g.out_ptr[u], re = g.out_ptr[u + 1], pu = g.pos_out[eid];
    uint32_t hi = upper_bound_i32(g.out_t, pu + 1, re, t);
    uint32_t lb = lower_bound_i32(g.out_t, rs, pu, lo);
    mp.counts[(uint64_t)mp.col_fo * mp.stride + eid] = hi - lb;
  }
  if (mp.col_fi >= 0) {
    uint32_t rs = g.in_ptr[v], re = g.in_ptr[v + 1], pv = g.pos_in[eid];
    uint32_t hi = upper_bound_i32(g.in_t, pv + 1, re, t);
    uint32_t lb = lower_bound_i32(g.in_t, rs, pv, lo);
    mp.counts[(uint64_t)mp.col_fi * mp.stride + eid] = hi - lb;
  }
  if (mp.col_sg >= 0 || mp.col_gs >= 0) {
    uint32_t cs = g.in_ptr[u], ce = g.in_ptr[u + 1];
    uint32_t p0 = lower_bound_i32(g.in_t, cs, ce, lo);
    uint32_t p1 = lower_bound_i32(g.in_t, p0, ce, t);
    if (p1 > p0) {
      if (p1 - p0 <= kAnchorScanCap) {
        uint32_t ns = 0;
        for (uint32_t j = p0; j < p1; j++) ns += (g.in_nbr[j] != v) & (g.in_nxt[j] >= t);
        if (ns > 0) {
          if (mp.k == 1) {
            // every sender has u as its first intermediate and v is always a
            // scatter destination after the first gather: SG_1 = GS_1 = |S|
            if (mp.col_sg >= 0) mp.counts[(uint64_t)mp.col_sg * mp.stride + eid] = ns;
            if (mp.col_gs >= 0) mp.counts[(uint64_t)mp.col_gs * mp.stride + eid] = ns;
          } else {
            f |= kFlagSG;
          }
        }
      } else {
        f |= kFlagSG;
      }
    }
  }
  if (mp.col_cyc >= 0) {
    uint32_t vs = g.out_ptr[v], ve = g.out_ptr[v + 1];
    uint32_t q0 = lower_bound_i32(g.out_t, vs, ve, lo);
    if (q0 < ve && g.out_t[q0] < t) f |= kFlagCYC;
  }
  flags[p] = f;
}

// ------------------------------------------------------------------ k_sg
__device__ __forceinline__ uint32_t bloom_h1(uint32_t m) { return m * 0x9E3779B1u; }
__device__ __forceinline__ uint32_t bloom_h2(uint32_t m) {
  uint32_t x = m ^ (m >> 15);
  x *= 0x85EBCA6Bu;
  x ^= x >> 13;
  return x * 0xC2B2AE35u;
}

struct SgLds {
  uint32_t bloom[kBloomWordsMax];
  uint32_t sb[AMLM_WAVE], soff[AMLM_WAVE], scnt[AMLM_WAVE], sid[AMLM_WAVE];
};

__device__ void sg_item(const MineParams &mp, uint32_t p, SgLds &L) {
  const GraphView &g = mp.g;
  const uint32_t lane = lane_id();
  const uint64_t lt = lanemask_lt();
  const uint32_t k = mp.k;
  uint32_t eid = rfl(g.anc[p]);
  uint32_t u = rfl(g.src[eid]), v = rfl(g.dst[eid]);
  int32_t t = rfl(g.t[eid]);
  int32_t lo = window_lo(t, mp.delta);
  uint32_t cs = rfl(g.in_ptr[u]), ce = rfl(g.in_ptr[u + 1]);
  uint32_t p0 = rfl(lower_bound_i32(g.in_t, cs, ce, lo));
  uint32_t p1 = rfl(lower_bound_i32(g.in_t, p0, ce, t));
  const bool need_join = mp.col_sg >= 0 && k >= 2;
  int bloom_shift = -1;
  uint32_t vrs = rfl(g.in_ptr[v]), vre = rfl(g.in_ptr[v + 1]);
  uint32_t nS = 0, sg = 0, work = 0;
  int32_t tau = AMLM_INT_MAX;
  for (uint32_t c = p0; c < p1; c += AMLM_WAVE) {
    uint32_t j = c + lane;
    bool valid = j < p1;
    uint32_t nb = valid ? g.in_nbr[j] : v;
    bool not_v = valid && nb != v;
    int32_t nx = not_v ? g.in_nxt[j] : 0;
    int32_t tj = not_v ? g.in_t[j] : AMLM_INT_MAX;
    uint64_t bnv = __ballot(not_v);
    if (tau == AMLM_INT_MAX && bnv) tau = __shfl(tj, __ffsll((long long)bnv) - 1, AMLM_WAVE);
    bool is_s = not_v && nx >= t;
    uint64_t bs = __ballot(is_s);
    uint32_t ns = __popcll(bs);
    nS += ns;
    work += kBytesSenderEntry * min((uint32_t)AMLM_WAVE, p1 - c);
    if (!need_join || ns == 0) continue;
    if (bloom_shift < 0) {
      // stage the gather side: every in-neighbour of v inside [lo, t]
      uint32_t r0 = rfl(lower_bound_i32(g.in_t, vrs, vre, lo));
      uint32_t r1 = rfl(upper_bound_i32(g.in_t, r0, vre, t));
      uint32_t nin = r1 - r0;
      uint32_t want = nin * kBloomBitsPerEntry;
      int lg = 9;
      while (lg < kBloomLog2Max && (1u << lg) < want) lg++;
      uint32_t words = (1u << lg) >> 5;
      for (uint32_t q = lane; q < words; q += AMLM_WAVE) L.bloom[q] = 0;
      bloom_shift = 32 - lg;
      for (uint32_t q = r0 + lane; q < r1; q += AMLM_WAVE) {
        uint32_t m = g.in_nbr[q];
        uint32_t h1 = bloom_h1(m) >> bloom_shift, h2 = bloom_h2(m) >> bloom_shift;
        atomicOr(&L.bloom[h1 >> 5], 1u << (h1 & 31));
        atomicOr(&L.bloom[h2 >> 5], 1u << (h2 & 31));
      }
      work += kBytesGatherEntry * nin;
    }
    if (is_s) L.sid[__popcll(bs & lt)] = nb;
    uint32_t sbv = 0, n_i = 0;
    if (lane < ns) {
      uint32_t s = L.sid[lane];
      uint32_t rs = g.out_ptr[s], re = g.out_ptr[s + 1];
      sbv = lower_bound_i32(g.out_t, rs, re, lo);
      n_i = lower_bound_i32(g.out_t, sbv, re, t) - sbv;
    }
    uint32_t incl = wave_incl_scan(n_i);
    uint32_t T = rfl((uint32_t)__shfl(incl, AMLM_WAVE - 1, AMLM_WAVE));
    if (lane < ns) {
      L.sb[lane] = sbv;
      L.soff[lane] = incl - n_i;
      L.scnt[lane] = 1;  // u is an intermediate of every sender
    }
    work += kBytesJoinEntry * T;
    const uint64_t act = ns == AMLM_WAVE ? ~0ull : ((1ull << ns) - 1ull);
    for (uint32_t f0 = 0; f0 < T; f0 += AMLM_WAVE) {
      uint32_t f = f0 + lane;
      if (f < T) {
        uint32_t a = 0, b = ns - 1;
        while (a < b) {
          uint32_t mid = (a + b + 1) >> 1;
          if (L.soff[mid] <= f) a = mid; else b = mid - 1;
        }
        if (L.scnt[a] < k) {
          uint32_t pos = L.sb[a] + (f - L.soff[a]);
          uint32_t m = g.out_nbr[pos];
          if (m != u) {
            uint32_t h1 = bloom_h1(m) >> bloom_shift, h2 = bloom_h2(m) >> bloom_shift;
            bool maybe = ((L.bloom[h1 >> 5] >> (h1 & 31)) & (L.bloom[h2 >> 5] >> (h2 & 31)) & 1u) != 0;
            if (maybe && g.out_prv[pos] < lo) {  // first (s, m) edge inside the window
              int32_t at = g.out_t[pos];
              uint32_t q = lower_bound_u64(g.inn_key, vrs, vre, nbr_key(m, t) + 1ull);
              if (q > vrs) {
                uint64_t kk = g.inn_key[q - 1];
                if ((uint32_t)(kk >> 32) == m && (int32_t)(uint32_t)kk > at) atomicAdd(&L.scnt[a], 1u);
              }
            }
          }
        }
      }
      uint64_t done = __ballot(lane < ns && L.scnt[lane] >= k);
      if (done == act) break;
    }
    sg += __popcll(__ballot(lane < ns && L.scnt[lane] >= k));
  }
  if (k == 1) sg = nS;
  uint32_t gs = 0;
  if (mp.col_gs >= 0 && nS >= k && nS > 0) {
    if (k == 1) {
      gs = nS;
    } else {
      uint32_t rs = rfl(g.out_ptr[u]), re = rfl(g.out_ptr[u + 1]);
      uint32_t d0 = rfl(upper_bound_i32(g.out_t, rs, re, tau));
      uint32_t d1 = rfl(upper_bound_i32(g.out_t, d0, re, t));
      uint32_t nd = 0;
      for (uint32_t c = d0; c < d1; c += AMLM_WAVE) {
        uint32_t j = c + lane;
        bool first = j < d1 && g.out_prv[j] <= tau;  // first (u, d) edge after tau
        nd += __popcll(__ballot(first));
        work += kBytesScatterEntry * min((uint32_t)AMLM_WAVE, d1 - c);
        if (nd >= k) break;
      }
      gs = nd >= k ? nS : 0;
    }
  }
  if (lane == 0) {
    if (mp.col_sg >= 0) mp.counts[(uint64_t)mp.col_sg * mp.stride + eid] = sg;
    if (mp.col_gs >= 0) mp.counts[(uint64_t)mp.col_gs * mp.stride + eid] = gs;
    if (mp.work) atomicAdd(&mp.work[eid], work + kBytesAnchorSg);
  }
}

__global__ __launch_bounds__(kSgThreads) void k_sg(MineParams mp, const uint32_t *items, const uint32_t *n_items_p,
                                                   uint32_t *ctr, uint32_t chunk) {
  __shared__ SgLds lds[kSgThreads / AMLM_WAVE];
  SgLds &L = lds[threadIdx.x / AMLM_WAVE];
  const uint32_t n_items = *n_items_p;
  for (;;) {
    uint32_t base = 0;
    if (lane_id() == 0) base = atomicAdd(ctr, chunk);
    base = rfl((uint32_t)__shfl(base, 0, AMLM_WAVE));
    if (base >= n_items) break;
    uint32_t end = min(base + chunk, n_items);
    for (uint32_t i = base; i < end; i++) sg_item(mp, items[i], L);
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
  uint32_t par[AMLM_WAVE];   // slot of the parent in the frame below
  uint32_t root[AMLM_WAVE];  // root (anchor) slot
  uint32_t eid[AMLM_WAVE];   // edge from the parent to this node
  uint32_t vert[AMLM_WAVE];  // head vertex
  int32_t tau[AMLM_WAVE];    // time of the last edge (first hop: lo - 1)
  uint32_t xb[AMLM_WAVE];    // first slice entry
  uint32_t xoff[AMLM_WAVE];  // exclusive prefix of slice sizes
  uint32_t n, T, cur;
};

struct CycLds {
  uint32_t r_eid[AMLM_WAVE], r_u[AMLM_WAVE];
  int32_t r_t[AMLM_WAVE];
  CycFrame fr[kMaxDepth + 1];
};

// +inc on column `len` for the anchor and every path edge of node (i, slot)
__device__ __forceinline__ void cyc_credit_path(const MineParams &mp, const CycLds &S, uint32_t i, uint32_t slot,
                                                uint32_t len, uint32_t inc) {
  uint32_t *col = mp.counts + (uint64_t)(mp.col_cyc + (int)len - 2) * mp.stride;
  credit(col + S.r_eid[S.fr[i].root[slot]], inc, mp.err);
  for (uint32_t j = i; j >= 1; j--) {
    credit(col + S.fr[j].eid[slot], inc, mp.err);
    slot = S.fr[j].par[slot];
  }
}

__device__ __forceinline__ bool cyc_on_path(const CycLds &S, uint32_t i, uint32_t slot, uint32_t w) {
  for (uint32_t j = i;; j--) {
    if (S.fr[j].vert[slot] == w) return true;
    if (j == 0) return false;
    slot = S.fr[j].par[slot];
  }
}

// Slice bounds of every node of frame i, or, at the last depth, the closing
// edges counted by binary search and credited at once.
__device__ void cyc_prepare(const MineParams &mp, CycLds &S, uint32_t i) {
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
    if (i + 2 == mp.L) {
      uint32_t urs = g.in_ptr[u], ure = g.in_ptr[u + 1];
      int32_t tl = tau + 1 < 0 ? 0 : tau + 1;
      uint32_t qa = lower_bound_u64(g.inn_key, urs, ure, nbr_key(h, tl));
      uint32_t qb = lower_bound_u64(g.inn_key, qa, ure, nbr_key(h, t));
      if (qb > qa) {
        cyc_credit_path(mp, S, i, lane, mp.L, qb - qa);
        uint32_t *col = mp.counts + (uint64_t)(mp.col_cyc + (int)mp.L - 2) * mp.stride;
        for (uint32_t q = qa; q < qb; q++) credit(col + g.inn_eid[q], 1u, mp.err);
      }
      if (mp.work) atomicAdd(&mp.work[mp.stride + S.r_eid[r]], kBytesClosureSearch);
    } else {
      uint32_t rs = g.out_ptr[h], re = g.out_ptr[h + 1];
      xb = upper_bound_i32(g.out_t, rs, re, tau);
      nsz = lower_bound_i32(g.out_t, xb, re, t) - xb;
      if (mp.work) atomicAdd(&mp.work[mp.stride + S.r_eid[r]], kBytesPathNode + kBytesPathEntry * nsz);
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

__global__ __launch_bounds__(kCycThreads) void k_cyc(MineParams mp, const uint32_t *roots, const uint32_t *n_in_p,
                                                     uint32_t *ctr) {
  __shared__ CycLds lds[kCycThreads / AMLM_WAVE];
  CycLds &S = lds[threadIdx.x / AMLM_WAVE];
  const GraphView &g = mp.g;
  const uint32_t lane = lane_id();
  const uint64_t lt = lanemask_lt();
  const uint32_t Lmax = mp.L;
  const uint32_t n_in = *n_in_p;
  for (;;) {
    uint32_t base = 0;
    if (lane == 0) base = atomicAdd(ctr, AMLM_WAVE);
    base = rfl((uint32_t)__shfl(base, 0, AMLM_WAVE));
    if (base >= n_in) break;
    uint32_t nr = min((uint32_t)AMLM_WAVE, n_in - base);
    if (lane < nr) {
      uint32_t eid = g.anc[roots[base + lane]];
      uint32_t v = g.dst[eid];
      int32_t t = g.t[eid];
      S.r_eid[lane] = eid;
      S.r_u[lane] = g.src[eid];
      S.r_t[lane] = t;
      CycFrame &F0 = S.fr[0];
      F0.par[lane] = lane;
      F0.root[lane] = lane;
      F0.eid[lane] = 0xffffffffu;
      F0.vert[lane] = v;
      F0.tau[lane] = window_lo(t, mp.delta) - 1;  // first hop at time >= lo
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
        if (w == S.r_u[F.root[a]]) {
          // closing hop: a cycle of sp + 2 edges
          cyc_credit_path(mp, S, sp, a, sp + 2, 1u);
          credit(mp.counts + (uint64_t)(mp.col_cyc + sp) * mp.stride + g.out_eid[pos], 1u, mp.err);
        } else if ((uint32_t)sp + 3 <= Lmax && !cyc_on_path(S, sp, a, w)) {
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
          G.par[slot] = a;
          G.root[slot] = F.root[a];
          G.eid[slot] = ceid;
          G.vert[slot] = w;
          G.tau[slot] = ctau;
        }
        if (lane == 0) G.n = __popcll(bc);
        cyc_prepare(mp, S, sp + 1);
        sp++;
      }
    }
  }
}

__global__ void k_flag_count(const uint8_t *flags, uint32_t n, uint32_t *c_sg, uint32_t *c_cy) {
  __shared__ uint32_t ws[2][kFlagThreads / AMLM_WAVE];
  uint32_t tid = threadIdx.x, w = tid / AMLM_WAVE;
  uint32_t base = blockIdx.x * kFlagTile + tid * kFlagItems;
  uint32_t a = 0, b = 0;
  for (uint32_t j = 0; j < kFlagItems; j++) {
    uint32_t idx = base + j;
    uint8_t f = idx < n ? flags[idx] : 0;
    a += (f & kFlagSG) != 0;
    b += (f & kFlagCYC) != 0;
  }
  for (int o = 32; o > 0; o >>= 1) {
    a += __shfl_xor(a, o, AMLM_WAVE);
    b += __shfl_xor(b, o, AMLM_WAVE);
  }
  if (lane_id() == 0) {
    ws[0][w] = a;
    ws[1][w] = b;
  }
  __syncthreads();
  if (tid == 0) {
    uint32_t sa = 0, sb = 0;
    for (int q = 0; q < kFlagThreads / AMLM_WAVE; q++) {
      sa += ws[0][q];
      sb += ws[1][q];
    }
    c_sg[blockIdx.x] = sa;
    c_cy[blockIdx.x] = sb;
  }
}

// order-preserving scatter of flagged anchor positions
__global__ void k_flag_scatter(const uint8_t *flags, uint32_t n, const uint32_t *o_sg, const uint32_t *o_cy,
                               uint32_t *l_sg, uint32_t *l_cy) {
  __shared__ uint32_t ws[2][kFlagThreads / AMLM_WAVE];
  uint32_t tid = threadIdx.x, w = tid / AMLM_WAVE;
  uint32_t base = blockIdx.x * kFlagTile + tid * kFlagItems;
  uint8_t f[kFlagItems];
  uint32_t a = 0, b = 0;
  for (uint32_t j = 0; j < kFlagItems; j++) {
    uint32_t idx = base + j;
    f[j] = idx < n ? flags[idx] : 0;
    a += (f[j] & kFlagSG) != 0;
    b += (f[j] & kFlagCYC) != 0;
  }
  uint32_t ia = wave_incl_scan(a), ib = wave_incl_scan(b);
  if (lane_id() == AMLM_WAVE - 1) {
    ws[0][w] = ia;
    ws[1][w] = ib;
  }
  __syncthreads();
  uint32_t pa = o_sg[blockIdx.x] + ia - a, pb = o_cy[blockIdx.x] + ib - b;
  for (uint32_t q = 0; q < w; q++) {
    pa += ws[0][q];
    pb += ws[1][q];
  }
  for (uint32_t j = 0; j < kFlagItems; j++) {
    if (f[j] & kFlagSG) l_sg[pa++] = base + j;
    if (f[j] & kFlagCYC) l_cy[pb++] = base + j;
  }
}

}  // namespace

// ====================================================================== host

hipError_t mine_launch(const MineParams &mp, MineScratch &ms, const MineLaunch &cfg, hipStream_t s,
                       StageTimer *tm) {
  StageTimer none;
  if (!tm) tm = &none;
  hipError_t e;
#define CK(x)                       \
  do {                              \
    e = (x);                        \
    if (e != hipSuccess) return e;  \
  } while (0)
  const uint32_t Ev = mp.g.Ev;
  // work-stealing counters and list sizes
  CK(launch_fill_u32(ms.ctr, 0, kCtrWords, s));
  if (Ev == 0) return hipSuccess;
  CK(tm->begin(kStAnchor, s));
  hipLaunchKernelGGL(k_anchor, dim3((Ev + 255) / 256), dim3(256), 0, s, mp, ms.flags);
  CK(hipGetLastError());
  CK(tm->end(kStAnchor, s));
  const bool want_sg = mp.col_sg >= 0 || mp.col_gs >= 0;
  const bool want_cyc = mp.col_cyc >= 0;
  if (!want_sg && !want_cyc) return hipSuccess;
  uint32_t nb = (Ev + kFlagTile - 1) / kFlagTile;
  CK(tm->begin(kStLists, s));
  hipLaunchKernelGGL(k_flag_count, dim3(nb), dim3(kFlagThreads), 0, s, ms.flags, Ev, ms.bcnt_sg, ms.bcnt_cy);
  CK(hipGetLastError());
  uint32_t *n_sg = ms.ctr + kCtrNSg, *n_cy = ms.ctr + kCtrNCy;
  CK(scan_exclusive_u32(ms.bcnt_sg, ms.boff_sg, nb, n_sg, ms.scan_tmp, s));
  CK(scan_exclusive_u32(ms.bcnt_cy, ms.boff_cy, nb, n_cy, ms.scan_tmp, s));
  hipLaunchKernelGGL(k_flag_scatter, dim3(nb), dim3(kFlagThreads), 0, s, ms.flags, Ev, ms.boff_sg, ms.boff_cy,
                     ms.list_sg, ms.list_cy);
  CK(hipGetLastError());
  CK(tm->end(kStLists, s));
  if (want_sg) {
    CK(tm->begin(kStSg, s));
    hipLaunchKernelGGL(k_sg, dim3(cfg.sg_blocks), dim3(kSgThreads), 0, s, mp, ms.list_sg, n_sg,
                       ms.ctr + kCtrSgWork, cfg.sg_chunk);
    CK(hipGetLastError());
    CK(tm->end(kStSg, s));
  }
  if (want_cyc) {
    CK(tm->begin(kStCyc, s));
    hipLaunchKernelGGL(k_cyc, dim3(cfg.cyc_blocks), dim3(kCycThreads), 0, s, mp, ms.list_cy, n_cy,
                       ms.ctr + kCtrCycWork);
    CK(hipGetLastError());
    CK(tm->end(kStCyc, s));
  }
#undef CK
  return hipSuccess;
}

const void *k_sg_ptr() { return (const void *)k_sg; }
const void *k_cyc_ptr() { return (const void *)k_cyc; }
