// Graph store construction on the GPU: validation, relative times, an LSD
// radix sort of our own, and the time-sorted CSR / CSC plus the
// neighbour-sorted in-index with same-pair time links.
#include "internal.h"

namespace {

constexpr int kThreads = 256;
constexpr int kItems = 16;
constexpr uint32_t kTile = kThreads * kItems;  // 4096 elements per block
constexpr int64_t kInt64Max = 0x7fffffffffffffffll;

__global__ void k_fill_u32(uint32_t *p, uint32_t v, uint64_t n) {
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = v;
}

// stats[0] = min ts (biased to unsigned order), [1] = max ts (biased),
// [2] = ids >= V, [3] = self-loops, [4] = i with ts[i] > ts[i+1].
// Each block writes its five partial results; k_validate_final folds them.
__global__ __launch_bounds__(256) void k_validate(const uint32_t *src, const uint32_t *dst, const int64_t *ts,
                                                  uint64_t E, uint32_t V, unsigned long long *part) {
  const unsigned long long bias = 0x8000000000000000ull;
  unsigned long long mn = ~0ull, mx = 0ull, bad = 0, loops = 0, unsorted = 0;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  constexpr int U = 4;  // independent loads in flight per thread
  for (uint64_t i0 = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i0 < E; i0 += U * stride) {
    int64_t tv[U], tn[U];
    uint32_t sv[U], dv[U];
#pragma unroll
    for (int r = 0; r < U; r++) {
      uint64_t i = i0 + r * stride;
      bool in = i < E;
      tv[r] = in ? ts[i] : 0;
      tn[r] = in && i + 1 < E ? ts[i + 1] : kInt64Max;
      sv[r] = in ? src[i] : 0u;
      dv[r] = in ? dst[i] : 1u;
    }
#pragma unroll
    for (int r = 0; r < U; r++) {
      if (i0 + r * stride >= E) continue;
      unsigned long long b = (unsigned long long)tv[r] ^ bias;
      mn = b < mn ? b : mn;
      mx = b > mx ? b : mx;
      bad += (sv[r] >= V) | (dv[r] >= V);
      loops += (sv[r] == dv[r]);
      unsorted += tv[r] > tn[r];
    }
  }
  for (int o = 32; o > 0; o >>= 1) {
    unsigned long long a = __shfl_xor(mn, o, AMLM_WAVE);
    mn = a < mn ? a : mn;
    a = __shfl_xor(mx, o, AMLM_WAVE);
    mx = a > mx ? a : mx;
    bad += __shfl_xor(bad, o, AMLM_WAVE);
    loops += __shfl_xor(loops, o, AMLM_WAVE);
    unsorted += __shfl_xor(unsorted, o, AMLM_WAVE);
  }
  __shared__ unsigned long long ws[4][5];
  const uint32_t w = threadIdx.x / AMLM_WAVE;
  if (lane_id() == 0) {
    ws[w][0] = mn;
    ws[w][1] = mx;
    ws[w][2] = bad;
    ws[w][3] = loops;
    ws[w][4] = unsorted;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (uint32_t q = 1; q < blockDim.x / AMLM_WAVE; q++) {
      mn = ws[q][0] < mn ? ws[q][0] : mn;
      mx = ws[q][1] > mx ? ws[q][1] : mx;
      bad += ws[q][2];
      loops += ws[q][3];
      unsorted += ws[q][4];
    }
    unsigned long long *o = part + 5ull * blockIdx.x;
    o[0] = mn;
    o[1] = mx;
    o[2] = bad;
    o[3] = loops;
    o[4] = unsorted;
  }
}

// Folds the per-block results; blocks that saw no element report the
// neutral values, so the fold starts from them too.
__global__ void k_validate_final(const unsigned long long *part, uint32_t nblocks, unsigned long long *stats) {
  unsigned long long mn = ~0ull, mx = 0ull, bad = 0, loops = 0, unsorted = 0;
  for (uint32_t b = lane_id(); b < nblocks; b += AMLM_WAVE) {
    const unsigned long long *o = part + 5ull * b;
    mn = o[0] < mn ? o[0] : mn;
    mx = o[1] > mx ? o[1] : mx;
    bad += o[2];
    loops += o[3];
    unsorted += o[4];
  }
  for (int o = 32; o > 0; o >>= 1) {
    unsigned long long a = __shfl_xor(mn, o, AMLM_WAVE);
    mn = a < mn ? a : mn;
    a = __shfl_xor(mx, o, AMLM_WAVE);
    mx = a > mx ? a : mx;
    bad += __shfl_xor(bad, o, AMLM_WAVE);
    loops += __shfl_xor(loops, o, AMLM_WAVE);
    unsorted += __shfl_xor(unsorted, o, AMLM_WAVE);
  }
  if (lane_id() == 0) {
    stats[0] = mn;
    stats[1] = mx;
    stats[2] = bad;
    stats[3] = loops;
    stats[4] = unsorted;
  }
}

// relative times, edge copies, and the first sort key:
// key = self_loop << t_bits | t_rel, value = edge id
__global__ void k_reltime(const int64_t *ts, int64_t tmin, const uint32_t *src, const uint32_t *dst, uint32_t E,
                          int t_bits, int32_t *t, uint32_t *key, uint32_t *val, int with_time_key, uint2 *ep_dt,
                          uint2 *ep_st) {
  uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= E) return;
  int32_t tr = (int32_t)(ts[i] - tmin);
  uint32_t s = src[i], d = dst[i];
  t[i] = tr;
  // (other endpoint, time) per edge id: one line per random read in the row
  // fills, from an array small enough to stay in the last-level cache
  ep_dt[i] = make_uint2(d, (uint32_t)tr);
  ep_st[i] = make_uint2(s, (uint32_t)tr);
  uint32_t loop = s == d;
  key[i] = with_time_key ? ((loop << t_bits) | (uint32_t)tr) : loop;
  val[i] = i;
}

// ---------------------------------------------------------------- scan
constexpr uint32_t kScanBlock = 2048;  // elements per block (256 threads x 8)

__global__ void k_scan_block(const uint32_t *in, uint32_t *out, uint32_t n, uint32_t *block_sums,
                             const uint32_t *n_dev) {
  __shared__ uint32_t wsum[kThreads / AMLM_WAVE];
  if (n_dev) n = min(n, *n_dev);
  uint32_t tid = threadIdx.x, w = tid / AMLM_WAVE;
  uint32_t base = blockIdx.x * kScanBlock + tid * 8;
  uint32_t v[8], s = 0;
#pragma unroll
  for (int j = 0; j < 8; j++) {
    uint32_t idx = base + j;
    v[j] = idx < n ? in[idx] : 0;
    s += v[j];
  }
  uint32_t incl = wave_incl_scan(s);
  if (lane_id() == AMLM_WAVE - 1) wsum[w] = incl;
  __syncthreads();
  uint32_t woff = 0;
  for (uint32_t q = 0; q < w; q++) woff += wsum[q];
  uint32_t run = woff + incl - s;
#pragma unroll
  for (int j = 0; j < 8; j++) {
    uint32_t idx = base + j;
    if (idx < n) out[idx] = run;
    run += v[j];
  }
  if (tid == kThreads - 1 && block_sums) block_sums[blockIdx.x] = woff + incl;
}

__global__ void k_scan_add(uint32_t *out, uint32_t n, const uint32_t *block_offsets, const uint32_t *n_dev) {
  if (n_dev) n = min(n, *n_dev);
  uint32_t b = blockIdx.x;
  if (b * kScanBlock >= n) return;
  uint32_t add = block_offsets[b];
  uint32_t base = b * kScanBlock;
  for (uint32_t j = threadIdx.x; j < kScanBlock; j += blockDim.x) {
    uint32_t idx = base + j;
    if (idx < n) out[idx] += add;
  }
}

__global__ void k_scan_total(const uint32_t *in, const uint32_t *out, uint32_t n, uint32_t *total,
                             const uint32_t *n_dev) {
  if (n_dev) n = min(n, *n_dev);
  if (threadIdx.x == 0) *total = n ? out[n - 1] + in[n - 1] : 0;
}

// ---------------------------------------------------------------- radix sort
__global__ __launch_bounds__(kThreads) void k_rs_hist(const uint32_t *keys, uint32_t n, int shift,
                                                      uint32_t *hist, uint32_t nblocks) {
  __shared__ uint32_t h[kThreads / AMLM_WAVE][256];
  uint32_t tid = threadIdx.x, w = tid / AMLM_WAVE;
  for (int q = 0; q < kThreads / AMLM_WAVE; q++) h[q][tid] = 0;
  __syncthreads();
  uint32_t base = blockIdx.x * kTile;
#pragma unroll 4
  for (int j = 0; j < kItems; j++) {
    uint32_t idx = base + j * kThreads + tid;
    if (idx < n) atomicAdd(&h[w][(keys[idx] >> shift) & 255u], 1u);
  }
  __syncthreads();
  uint32_t s = 0;
  for (int q = 0; q < kThreads / AMLM_WAVE; q++) s += h[q][tid];
  hist[tid * nblocks + blockIdx.x] = s;
}

// Stable scatter.  Ranks follow the (iteration, wave, lane) order, which is
// the input order inside the tile; the tile is first sorted by digit in LDS
// and then written out bucket by bucket, so that consecutive threads store
// to consecutive addresses of one bucket.
__global__ __launch_bounds__(kThreads) void k_rs_scatter(const uint32_t *kin, const uint32_t *vin, uint32_t *kout,
                                                         uint32_t *vout, uint32_t n, int shift,
                                                         const uint32_t *offs, uint32_t nblocks) {
  constexpr int NW = kThreads / AMLM_WAVE;
  __shared__ uint32_t sk[kTile], sv[kTile];
  __shared__ uint32_t run[256], start[256], gbase[256];
  __shared__ uint32_t wc[NW][256];
  __shared__ uint32_t wsum[NW];
  const uint32_t tid = threadIdx.x, w = tid / AMLM_WAVE, lane = lane_id();
  const uint32_t base = blockIdx.x * kTile;
  const uint32_t tn = min(kTile, n - base);
  // the whole tile is loaded up front, so the loads overlap
  uint32_t kr[kItems], vr[kItems];
#pragma unroll
  for (int j = 0; j < kItems; j++) {
    uint32_t idx = j * kThreads + tid;
    kr[j] = idx < tn ? kin[base + idx] : 0u;
    vr[j] = idx < tn ? vin[base + idx] : 0u;
  }
  // tile histogram, then its exclusive scan: the tile-local start of each bucket
  for (int q = 0; q < NW; q++) wc[q][tid] = 0;
  __syncthreads();
#pragma unroll
  for (int j = 0; j < kItems; j++) {
    uint32_t idx = j * kThreads + tid;
    if (idx < tn) atomicAdd(&wc[w][(kr[j] >> shift) & 255u], 1u);
  }
  __syncthreads();
  uint32_t cnt = 0;
  for (int q = 0; q < NW; q++) {
    cnt += wc[q][tid];
    wc[q][tid] = 0;
  }
  const uint32_t incl = wave_incl_scan(cnt);
  if (lane == AMLM_WAVE - 1) wsum[w] = incl;
  __syncthreads();
  uint32_t before = 0;
  for (uint32_t q = 0; q < w; q++) before += wsum[q];
  start[tid] = before + incl - cnt;
  run[tid] = before + incl - cnt;
  gbase[tid] = offs[tid * nblocks + blockIdx.x];
  __syncthreads();
  const uint64_t lt = lanemask_lt();
#pragma unroll
  for (int j = 0; j < kItems; j++) {
    uint32_t idx = j * kThreads + tid;
    bool valid = idx < tn;
    uint32_t key = kr[j];
    uint32_t val = vr[j];
    uint32_t d = (key >> shift) & 255u;
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; b++) {
      uint32_t bit = (d >> b) & 1u;
      uint64_t bb = __ballot(bit);
      peers &= bit ? bb : ~bb;
    }
    uint32_t rank = __popcll(peers & lt);
    if (valid && rank == 0) wc[w][d] = __popcll(peers);
    __syncthreads();
    if (valid) {
      uint32_t pos = run[d] + rank;
      for (uint32_t q = 0; q < w; q++) pos += wc[q][d];
      sk[pos] = key;
      sv[pos] = val;
    }
    __syncthreads();
    uint32_t tot = 0;
    for (int q = 0; q < NW; q++) {
      tot += wc[q][tid];
      wc[q][tid] = 0;
    }
    run[tid] += tot;
    __syncthreads();
  }
  for (uint32_t i = tid; i < tn; i += kThreads) {
    uint32_t key = sk[i];
    uint32_t d = (key >> shift) & 255u;
    uint32_t pos = gbase[d] + (i - start[d]);
    kout[pos] = key;
    vout[pos] = sv[i];
  }
}

// ---------------------------------------------------------------- CSR pieces
__global__ void k_gather_key(const uint32_t *keysrc, const uint32_t *ids, uint32_t *key, uint32_t *val, uint32_t n) {
  uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint32_t e = ids[i];
  key[i] = keysrc[e];
  val[i] = e;
}

// row pointers from sorted row keys: ptr[x] = first position with key >= x
__global__ void k_row_ptr(const uint32_t *keys, uint32_t n, uint32_t V, uint32_t *ptr) {
  uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p > n) return;
  int64_t kp = p < n ? (int64_t)keys[p] : (int64_t)V;
  int64_t kprev = p > 0 ? (int64_t)keys[p - 1] : -1;
  for (int64_t x = kprev + 1; x <= kp; x++) ptr[x] = p;
}

// Row fill after a sort: entry p takes edge eids[p], whose other endpoint
// and time come packed from ep.
__global__ void k_fill_rows(const uint32_t *eids, uint32_t *eids_out, const uint2 *ep, uint32_t n,
                            uint32_t *nbr, int32_t *tt, uint32_t *pos, const uint32_t *rowkey, uint32_t *row,
                            uint32_t *hnbr) {
  uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  uint32_t e = eids[p];
  uint2 x = ep[e];
  uint32_t o = x.x;
  eids_out[p] = e;
  nbr[p] = o;
  if (hnbr) hnbr[p] = vhash(o);
  tt[p] = (int32_t)x.y;
  pos[e] = p;
  row[p] = rowkey[p];
}

// Row time index (layout next to tix_lower_bound): bucket counts per row ...
__global__ void k_tix_count(const uint32_t *ptr, const int32_t *t, uint32_t V, uint4 *meta, uint32_t *cnt) {
  uint32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= V) return;
  const uint32_t rs = ptr[v], re = ptr[v + 1], len = re - rs;
  uint4 m = make_uint4(0u, 0u, 0u, 0u);
  if (len > kTixMinRow) {
    const int32_t t0 = t[rs], t1 = t[re - 1];
    const uint32_t span = (uint32_t)(t1 - t0), maxnb = (len + kTixPerBucket - 1) / kTixPerBucket;
    uint32_t w = 0;
    while ((span >> w) + 1 > maxnb) w++;
    m = make_uint4(0u, (span >> w) + 1, (uint32_t)t0, w);
  }
  meta[v] = m;
  cnt[v] = m.y ? m.y + 1 : 0u;
}
// ... their offsets ...
__global__ void k_tix_offsets(const uint32_t *off, uint32_t V, uint4 *meta) {
  uint32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v < V) meta[v].x = off[v];
}
// ... and the bucket starts: entry p writes the buckets that begin after its
// predecessor's time and at or before its own (the row's last entry also
// writes the ones after it, up to the end sentinel).
__global__ void k_tix_fill(const uint32_t *ptr, const int32_t *t, const uint32_t *row, uint32_t n, const uint4 *meta,
                           uint32_t *tix) {
  uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const uint32_t v = row[p];
  const uint4 m = meta[v];
  if (m.y == 0) return;
  const uint32_t rs = ptr[v], re = ptr[v + 1];
  const int32_t t0 = (int32_t)m.z;
  const int32_t bp = (int32_t)((uint32_t)(t[p] - t0) >> m.w);
  const int32_t bq = p == rs ? -1 : (int32_t)((uint32_t)(t[p - 1] - t0) >> m.w);
  for (int32_t i = bq + 1; i <= bp; i++) tix[m.x + i] = p;
  if (p == re - 1)
    for (uint32_t i = (uint32_t)bp + 1; i <= m.y; i++) tix[m.x + i] = re;
}

__global__ void k_inn_keys(const uint32_t *eids, uint32_t *eids_out, const uint2 *ep, uint32_t n, uint64_t *key) {
  uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  uint32_t e = eids[q];
  uint2 x = ep[e];
  eids_out[q] = e;
  key[q] = nbr_key(x.x, (int32_t)x.y);
}

// same-pair time links from the (dst, src, time)-sorted index
__global__ void k_links(const uint32_t *dkeys, const uint64_t *inn_key, const uint32_t *inn_eid, uint32_t n,
                        const uint32_t *pos_in, const uint32_t *pos_out, int32_t *in_nxt, int32_t *out_prv) {
  uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  uint32_t d = dkeys[q];
  uint64_t k = inn_key[q];
  uint32_t s = (uint32_t)(k >> 32);
  int32_t nxt = AMLM_INT_MAX, prv = AMLM_INT_MIN;
  if (q + 1 < n && dkeys[q + 1] == d && (uint32_t)(inn_key[q + 1] >> 32) == s) nxt = (int32_t)(uint32_t)inn_key[q + 1];
  if (q > 0 && dkeys[q - 1] == d && (uint32_t)(inn_key[q - 1] >> 32) == s) prv = (int32_t)(uint32_t)inn_key[q - 1];
  uint32_t e = inn_eid[q];
  in_nxt[pos_in[e]] = nxt;
  out_prv[pos_out[e]] = prv;
}

inline uint32_t nblk(uint64_t n, uint32_t per) { return (uint32_t)((n + per - 1) / per); }

}  // namespace

// ====================================================================== host

int bits_for(uint64_t max_value) {
  int b = 0;
  while (b < 64 && (max_value >> b) != 0) b++;
  return b;
}

hipError_t launch_fill_u32(uint32_t *p, uint32_t value, uint64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  uint32_t blocks = (uint32_t)std::min<uint64_t>((n + 255) / 256, 16384);
  hipLaunchKernelGGL(k_fill_u32, dim3(blocks), dim3(256), 0, s, p, value, n);
  return hipGetLastError();
}

size_t scan_tmp_words(uint64_t n) {
  size_t w = 0;
  while (n > kScanBlock) {
    n = (n + kScanBlock - 1) / kScanBlock;
    w += 2 * n + 64;
  }
  return w + 64;
}

// (blocks past a device-side count write zero block sums, so the scan of
// the block sums is a plain one)
static hipError_t scan_rec(const uint32_t *in, uint32_t *out, uint32_t n, uint32_t *tmp, hipStream_t s,
                           const uint32_t *n_dev) {
  if (n == 0) return hipSuccess;
  uint32_t nb = nblk(n, kScanBlock);
  if (nb == 1) {
    hipLaunchKernelGGL(k_scan_block, dim3(1), dim3(kThreads), 0, s, in, out, n, (uint32_t *)nullptr, n_dev);
    return hipGetLastError();
  }
  uint32_t *sums = tmp, *sums_scan = tmp + nb, *rest = tmp + 2 * nb + 64;
  hipLaunchKernelGGL(k_scan_block, dim3(nb), dim3(kThreads), 0, s, in, out, n, sums, n_dev);
  hipError_t e = scan_rec(sums, sums_scan, nb, rest, s, nullptr);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_scan_add, dim3(nb), dim3(kThreads), 0, s, out, n, sums_scan, n_dev);
  return hipGetLastError();
}

hipError_t scan_exclusive_u32(const uint32_t *in, uint32_t *out, uint32_t n, uint32_t *total, uint32_t *tmp,
                              hipStream_t s, const uint32_t *n_dev) {
  hipError_t e = scan_rec(in, out, n, tmp, s, n_dev);
  if (e != hipSuccess) return e;
  if (total) {
    hipLaunchKernelGGL(k_scan_total, dim3(1), dim3(64), 0, s, in, out, n, total, n_dev);
    e = hipGetLastError();
  }
  return e;
}

size_t radix_hist_words(uint64_t n) { return (size_t)256 * nblk(n ? n : 1, kTile) + 64; }

hipError_t radix_sort_pairs(uint32_t *ka, uint32_t *va, uint32_t *kb, uint32_t *vb, uint32_t n, int bits,
                            uint32_t *hist, uint32_t *hist2, uint32_t *scan_tmp, hipStream_t s,
                            uint32_t **kout, uint32_t **vout) {
  uint32_t *kin = ka, *vin = va, *ko = kb, *vo = vb;
  if (n > 1) {
    uint32_t nb = nblk(n, kTile);
    for (int shift = 0; shift < bits; shift += 8) {
      hipLaunchKernelGGL(k_rs_hist, dim3(nb), dim3(kThreads), 0, s, kin, n, shift, hist, nb);
      hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
      e = scan_exclusive_u32(hist, hist2, 256 * nb, nullptr, scan_tmp, s);
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL(k_rs_scatter, dim3(nb), dim3(kThreads), 0, s, kin, vin, ko, vo, n, shift, hist2, nb);
      e = hipGetLastError();
      if (e != hipSuccess) return e;
      std::swap(kin, ko);
      std::swap(vin, vo);
    }
  }
  *kout = kin;
  *vout = vin;
  return hipSuccess;
}

hipError_t validate_edges(const uint32_t *src, const uint32_t *dst, const int64_t *ts, uint64_t E, uint32_t V,
                          uint64_t *stats_dev, ValidateResult *res, hipStream_t s) {
  unsigned long long *st = (unsigned long long *)stats_dev;
  const uint32_t blocks = E ? (uint32_t)std::min<uint64_t>((E + 1023) / 1024, kValidateBlocks) : 1u;
  hipLaunchKernelGGL(k_validate, dim3(blocks), dim3(256), 0, s, src, dst, ts, E, V, st + 8);
  hipLaunchKernelGGL(k_validate_final, dim3(1), dim3(AMLM_WAVE), 0, s, (const unsigned long long *)(st + 8), blocks,
                     st);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  unsigned long long h[5];
  e = hipMemcpyAsync(h, st, sizeof(h), hipMemcpyDeviceToHost, s);
  if (e != hipSuccess) return e;
  e = hipStreamSynchronize(s);
  if (e != hipSuccess) return e;
  const unsigned long long bias = 0x8000000000000000ull;
  res->tmin = E ? (int64_t)(h[0] ^ bias) : 0;
  res->tmax = E ? (int64_t)(h[1] ^ bias) : 0;
  res->bad_ids = h[2];
  res->self_loops = h[3];
  res->unsorted = h[4];
  return hipSuccess;
}

// Time index of the rows (ptr, t); row[p] is the row of entry p.
static hipError_t build_tix(const uint32_t *ptr, const int32_t *t, const uint32_t *row, uint32_t V, uint32_t n,
                            uint4 *meta, uint32_t *tix, uint32_t *cnt, uint32_t *off, uint32_t *scan_tmp,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_tix_count, dim3(nblk(V, 256)), dim3(256), 0, s, ptr, t, V, meta, cnt);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = scan_exclusive_u32(cnt, off, V, nullptr, scan_tmp, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_tix_offsets, dim3(nblk(V, 256)), dim3(256), 0, s, off, V, meta);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_tix_fill, dim3(nblk(n, 256)), dim3(256), 0, s, ptr, t, row, n, (const uint4 *)meta, tix);
  return hipGetLastError();
}

hipError_t build_graph(const GraphArrays &a, const int64_t *ts, int64_t tmin, uint32_t E, uint32_t Ev, uint32_t V,
                       int t_bits, bool time_sorted, uint64_t n_self, BuildBuffers &bb, hipStream_t s) {
  hipError_t e;
#define CK(x)                       \
  do {                              \
    e = (x);                        \
    if (e != hipSuccess) return e;  \
  } while (0)
  const int vbits = bits_for(V ? V - 1 : 0);
  uint2 *ep_dt = (uint2 *)bb.ep, *ep_st = (uint2 *)bb.ep + E;
  // 1. relative times and the anchor order (valid edges by (time, id))
  if (E) {
    int with_time = time_sorted ? 0 : 1;
    hipLaunchKernelGGL(k_reltime, dim3(nblk(E, 256)), dim3(256), 0, s, ts, tmin, a.src, a.dst, E, t_bits, a.t,
                       bb.ka, bb.va, with_time, ep_dt, ep_st);
    CK(hipGetLastError());
    int sort_bits = time_sorted ? (n_self ? 1 : 0) : t_bits + 1;
    uint32_t *ks, *vs;
    CK(radix_sort_pairs(bb.ka, bb.va, bb.kb, bb.vb, E, sort_bits, bb.hist, bb.hist2, bb.scan_tmp, s, &ks, &vs));
    CK(hipMemcpyAsync(a.anc, vs, sizeof(uint32_t) * Ev, hipMemcpyDeviceToDevice, s));
  }
  // 2. CSR: stable sort of the anchor order by source
  CK(launch_fill_u32(a.out_ptr, 0, (uint64_t)V + 1, s));
  CK(launch_fill_u32(a.in_ptr, 0, (uint64_t)V + 1, s));
  if (Ev) {
    uint32_t *ks, *vs;
    hipLaunchKernelGGL(k_gather_key, dim3(nblk(Ev, 256)), dim3(256), 0, s, a.src, a.anc, bb.ka, bb.va, Ev);
    CK(hipGetLastError());
    CK(radix_sort_pairs(bb.ka, bb.va, bb.kb, bb.vb, Ev, vbits, bb.hist, bb.hist2, bb.scan_tmp, s, &ks, &vs));
    hipLaunchKernelGGL(k_row_ptr, dim3(nblk((uint64_t)Ev + 1, 256)), dim3(256), 0, s, ks, Ev, V, a.out_ptr);
    CK(hipGetLastError());
    hipLaunchKernelGGL(k_fill_rows, dim3(nblk(Ev, 256)), dim3(256), 0, s, (const uint32_t *)vs, a.out_eid,
                       (const uint2 *)ep_dt, Ev, a.out_nbr, a.out_t, a.pos_out, (const uint32_t *)ks, a.out_src,
                       a.out_h);
    CK(hipGetLastError());
    CK(build_tix(a.out_ptr, a.out_t, a.out_src, V, Ev, a.out_tm, a.out_tix, a.tix_cnt, a.tix_off, bb.scan_tmp, s));
    // 3. CSC: stable sort of the anchor order by destination
    hipLaunchKernelGGL(k_gather_key, dim3(nblk(Ev, 256)), dim3(256), 0, s, a.dst, a.anc, bb.ka, bb.va, Ev);
    CK(hipGetLastError());
    CK(radix_sort_pairs(bb.ka, bb.va, bb.kb, bb.vb, Ev, vbits, bb.hist, bb.hist2, bb.scan_tmp, s, &ks, &vs));
    hipLaunchKernelGGL(k_row_ptr, dim3(nblk((uint64_t)Ev + 1, 256)), dim3(256), 0, s, ks, Ev, V, a.in_ptr);
    CK(hipGetLastError());
    hipLaunchKernelGGL(k_fill_rows, dim3(nblk(Ev, 256)), dim3(256), 0, s, (const uint32_t *)vs, a.in_eid,
                       (const uint2 *)ep_st, Ev, a.in_nbr, a.in_t, a.pos_in, (const uint32_t *)ks, a.in_dst,
                       a.in_h);
    CK(hipGetLastError());
    // 4. CSC-N: stable sort of the CSR order (source, time, id) by destination
    //    (the destination of CSR entry p is out_nbr[p])
    CK(hipMemcpyAsync(bb.ka, a.out_nbr, sizeof(uint32_t) * Ev, hipMemcpyDeviceToDevice, s));
    CK(hipMemcpyAsync(bb.va, a.out_eid, sizeof(uint32_t) * Ev, hipMemcpyDeviceToDevice, s));
    CK(radix_sort_pairs(bb.ka, bb.va, bb.kb, bb.vb, Ev, vbits, bb.hist, bb.hist2, bb.scan_tmp, s, &ks, &vs));
    hipLaunchKernelGGL(k_inn_keys, dim3(nblk(Ev, 256)), dim3(256), 0, s, (const uint32_t *)vs, a.inn_eid,
                       (const uint2 *)ep_st, Ev, a.inn_key);
    CK(hipGetLastError());
    // 5. same-pair links (ks still holds the destination of every CSC-N entry)
    hipLaunchKernelGGL(k_links, dim3(nblk(Ev, 256)), dim3(256), 0, s, ks, a.inn_key, a.inn_eid, Ev, a.pos_in,
                       a.pos_out, a.in_nxt, a.out_prv);
    CK(hipGetLastError());
  }
#undef CK
  return hipSuccess;
}

// ---------------------------------------------------------------- copy probe
namespace {
// Plain streaming copy (16-byte vector loads and stores, grid-stride): the
// achievable-bandwidth probe and the byte-count calibration for the
// hardware traffic counters.
__global__ __launch_bounds__(256) void k_copy(const uint4 *__restrict__ src, uint4 *__restrict__ dst, uint64_t n16) {
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (; i < n16; i += stride) dst[i] = src[i];
}
}  // namespace

extern "C" amlm_status amlm_copy(void *dst, const void *src, uint64_t bytes, void *hip_stream) {
  if (bytes % 16 || ((uintptr_t)dst | (uintptr_t)src) % 16) {
    set_error("amlm_copy needs 16-byte aligned pointers and sizes");
    return AMLM_E_INVALID;
  }
  uint64_t n16 = bytes / 16;
  if (!n16) return AMLM_OK;
  uint32_t blocks = (uint32_t)std::min<uint64_t>((n16 + 255) / 256, 256 * 64);
  hipLaunchKernelGGL(k_copy, dim3(blocks), dim3(256), 0, (hipStream_t)hip_stream, (const uint4 *)src, (uint4 *)dst,
                     n16);
  HIP_TRY(hipGetLastError());
  return AMLM_OK;
}
