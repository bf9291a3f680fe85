// Streaming server: continuous batching of transaction batches over a
// resident graph.  Each incoming edge's columns come from the instances that
// end at it, and cycles it closes credit older edges (streaming integration,
// Section 5; incremental, localized updates instead of a full recompute).
//
// Sliding-window store.  Every search of the mining is bounded above by its
// anchor's time (windows [t - delta, t], paths and legs no later than t), and
// batches arrive strictly later than everything before them.  So a batch's
// results depend only on the edges inside [t_first - delta, t_last] of the
// batch, and edges of LATER batches in the same store change nothing.  The
// server therefore keeps one window store: the edges no older than delta
// before the oldest batch still to be mined, in time order.  A committer
// thread appends all queued batches at once (group commit), drops the edges
// that fell out of the window, and rebuilds the store's graph (ping-pong
// versions, so batches of the previous version keep mining meanwhile).
// Each batch is then mined on its own slot stream with its own edges as the
// only anchors; slots run concurrently on the same store version, each with
// its own mining scratch.  Memory is bounded by the window, not by the
// stream's length.
//
// Admission: a committed batch starts when a slot is free and the HBM budget
// allows its counts buffer.
#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstring>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <numeric>
#include <thread>
#include <vector>

#include "api_internal.h"

namespace {

// time-ordered copy of the resident graph's valid edges [p0, Ev) (anchor
// order) into the first store version, with their global edge ids
__global__ void k_store_from_graph(GraphView g, int64_t t_base, uint32_t p0, int64_t *ts, uint32_t *src,
                                   uint32_t *dst, uint32_t *geid) {
  uint32_t p = p0 + blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= g.Ev) return;
  uint32_t e = g.anc[p];
  ts[p - p0] = t_base + g.t[e];
  src[p - p0] = g.src[e];
  dst[p - p0] = g.dst[e];
  geid[p - p0] = e;
}

// first anchor-order position whose edge time is >= thr (one thread)
__global__ void k_first_at_or_after(GraphView g, int32_t thr, uint32_t *out) {
  uint32_t b = 0, e = g.Ev;
  while (b < e) {
    uint32_t m = b + ((e - b) >> 1);
    if (g.t[g.anc[m]] < thr) b = m + 1; else e = m;
  }
  *out = b;
}

// nonzero credits of context edges [0, n_ctx) in columns [col_cyc, col_cyc +
// ncyc) (cycles, participation) -> (global id, column, value)
__global__ void k_collect_deltas(const uint32_t *counts, uint64_t stride, uint32_t col_cyc, uint32_t ncyc,
                                 uint32_t n_ctx, const uint32_t *geid, uint32_t *cnt, uint32_t cap, uint32_t *o_eid,
                                 uint32_t *o_col, uint32_t *o_val) {
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (uint64_t)ncyc * n_ctx) return;
  uint32_t c = (uint32_t)(i / n_ctx), pos = (uint32_t)(i - (uint64_t)c * n_ctx);
  uint32_t v = counts[(uint64_t)(col_cyc + c) * stride + pos];
  if (v == 0) return;
  uint32_t slot = atomicAdd(cnt, 1u);
  if (slot < cap) {
    o_eid[slot] = geid[pos];
    o_col[slot] = col_cyc + c;
    o_val[slot] = v;
  }
}

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

// finished tickets whose timing records are kept after their results were
// taken (older records are dropped)
constexpr size_t kKeepTimes = 1u << 16;
// a group commit appends at most about this many edges
constexpr uint64_t kCommitEdges = 2ull << 20;

}  // namespace

struct ServerJob {
  uint64_t ticket = 0;
  uint64_t geid0 = 0, n = 0;
  int64_t tmin = 0;
  // the batch in time order (host, until committed) and the submitted order
  std::vector<uint32_t> src, dst, geid;
  std::vector<int64_t> ts;
  std::vector<uint32_t> order;            // time-order index -> index in submitted order
  int ver = -1;                           // store version it is mined on
  uint64_t lo = 0, hi = 0;                // its edges in that version
  uint64_t est_bytes = 0;
  double t_submit = 0, t_admit = 0, t_done = 0;
  std::vector<uint32_t> counts;           // [ncols][n], submitted order
  std::vector<uint64_t> d_eid;
  std::vector<uint32_t> d_col, d_val;
  amlm_status status = AMLM_OK;
  std::string err;
  bool committed = false, admitted = false, done = false, taken = false;
};

// One version of the window store: its edges in time order (device staging,
// global ids, host times) and the graph built from them.
struct StoreVer {
  amlm_graph *g = nullptr;
  uint32_t *src = nullptr, *dst = nullptr, *geid = nullptr;
  int64_t *ts = nullptr;
  uint64_t cap = 0, n = 0;
  std::vector<int64_t> host_ts;
  int refs = 0;  // jobs in flight on this version
};

struct ServerSlot {
  std::thread th;
  hipStream_t stream = nullptr;
  MineScratch ms{};
  uint64_t ms_cap = 0;
  std::vector<void *> allocs;  // the scratch's buffers
  uint32_t *counts = nullptr;
  uint64_t counts_cap = 0;
  uint32_t *dbuf = nullptr;    // [count, eid[cap], col[cap], val[cap]]
  uint64_t dcap = 0;
};

constexpr int kVersions = 3;

struct amlm_server {
  int device = 0;
  amlm_params p{};
  uint32_t ncols = 0, col_cyc = 0, ncyc = 0;
  uint32_t V = 0;
  uint64_t budget = 0, in_use = 0;
  StoreVer ver[kVersions];
  int cur = 0;                  // version holding every committed edge
  int64_t t_last = INT64_MIN;   // latest timestamp accepted
  uint64_t next_geid = 0, next_ticket = 1;
  uint64_t commits = 0, max_store = 0, batches_done = 0;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<ServerJob *> pending;   // submitted, not yet in a store version
  std::deque<ServerJob *> ready;     // committed, waiting for a slot and budget
  std::map<uint64_t, ServerJob *> jobs;
  std::deque<uint64_t> taken;        // tickets whose results were taken, oldest first
  bool stop = false;
  hipStream_t commit_stream = nullptr;
  std::thread committer;
  std::vector<ServerSlot> slots;
  uint32_t max_queue = 0;
};

static uint64_t estimate_bytes(uint64_t n_store, uint32_t ncols) {
  // counts of the store (every column) and the delta buffer
  return n_store * 4ull * ncols + (n_store / 4 + (1u << 16)) * 12ull + (1ull << 20);
}

static amlm_status grow(void **p, uint64_t *cap, uint64_t need, size_t elem) {
  if (*cap >= need) return AMLM_OK;
  if (*p) (void)hipFree(*p);
  // spare room: every window is a little larger than the last while the
  // stream is young, and a free synchronises the device
  uint64_t n = std::max<uint64_t>(need + need / 4, *cap * 2);
  if (hipMalloc(p, n * elem) != hipSuccess) {
    (void)hipGetLastError();
    *p = nullptr;
    *cap = 0;
    set_error("server: device allocation failed");
    return AMLM_E_NOMEM;
  }
  *cap = n;
  return AMLM_OK;
}

static amlm_status store_reserve(StoreVer &v, uint64_t need) {
  if (v.cap >= need) return AMLM_OK;
  uint64_t c = std::max<uint64_t>(need + need / 4, 1u << 16);
  for (void **p : {(void **)&v.src, (void **)&v.dst, (void **)&v.geid, (void **)&v.ts}) {
    if (*p) (void)hipFree(*p);
    *p = nullptr;
  }
  v.cap = 0;
  if (hipMalloc(&v.src, 4 * c) != hipSuccess || hipMalloc(&v.dst, 4 * c) != hipSuccess ||
      hipMalloc(&v.geid, 4 * c) != hipSuccess || hipMalloc(&v.ts, 8 * c) != hipSuccess) {
    (void)hipGetLastError();
    set_error("server: store allocation failed");
    return AMLM_E_NOMEM;
  }
  v.cap = c;
  return AMLM_OK;
}

static amlm_status store_build(amlm_server *S, StoreVer &v, hipStream_t s) {
  if (!v.g) return amlm_graph_create(v.src, v.dst, v.ts, nullptr, v.n, S->V, 1, s, &v.g);
  return amlm_graph_rebuild(v.g, v.src, v.dst, v.ts, v.n, S->V, 1, s);
}

// Group commit of `batch` into version f: the edges of the current version
// that are still inside the first batch's window, then every batch in order.
static amlm_status commit_group(amlm_server *S, int f, const std::vector<ServerJob *> &batch) {
  hipStream_t s = S->commit_stream;
  StoreVer &cur = S->ver[S->cur], &nx = S->ver[f];
  const int64_t w_start = batch.front()->tmin - S->p.delta;
  const uint64_t c0 = std::lower_bound(cur.host_ts.begin(), cur.host_ts.end(), w_start) - cur.host_ts.begin();
  const uint64_t keep = cur.n - c0;
  uint64_t n_new = 0;
  for (ServerJob *j : batch) n_new += j->n;
  amlm_status st = store_reserve(nx, keep + n_new);
  if (st != AMLM_OK) return st;
  auto dev_fail = [&](const char *what) {
    (void)hipGetLastError();
    set_error(std::string("server: ") + what);
    return AMLM_E_DEVICE;
  };
  if (keep) {
    if (hipMemcpyAsync(nx.src, cur.src + c0, 4 * keep, hipMemcpyDeviceToDevice, s) != hipSuccess ||
        hipMemcpyAsync(nx.dst, cur.dst + c0, 4 * keep, hipMemcpyDeviceToDevice, s) != hipSuccess ||
        hipMemcpyAsync(nx.geid, cur.geid + c0, 4 * keep, hipMemcpyDeviceToDevice, s) != hipSuccess ||
        hipMemcpyAsync(nx.ts, cur.ts + c0, 8 * keep, hipMemcpyDeviceToDevice, s) != hipSuccess)
      return dev_fail("store copy failed");
  }
  nx.host_ts.assign(cur.host_ts.begin() + c0, cur.host_ts.end());
  uint64_t o = keep;
  for (ServerJob *j : batch) {
    j->lo = o;
    j->hi = o + j->n;
    if (j->n) {
      if (hipMemcpyAsync(nx.src + o, j->src.data(), 4 * j->n, hipMemcpyHostToDevice, s) != hipSuccess ||
          hipMemcpyAsync(nx.dst + o, j->dst.data(), 4 * j->n, hipMemcpyHostToDevice, s) != hipSuccess ||
          hipMemcpyAsync(nx.geid + o, j->geid.data(), 4 * j->n, hipMemcpyHostToDevice, s) != hipSuccess ||
          hipMemcpyAsync(nx.ts + o, j->ts.data(), 8 * j->n, hipMemcpyHostToDevice, s) != hipSuccess)
        return dev_fail("ingest copy failed");
      nx.host_ts.insert(nx.host_ts.end(), j->ts.begin(), j->ts.end());
    }
    o += j->n;
  }
  nx.n = o;
  // the host copies are read by the (synchronous) build below
  st = store_build(S, nx, s);
  if (st != AMLM_OK) return st;
  for (ServerJob *j : batch) {
    std::vector<uint32_t>().swap(j->src);
    std::vector<uint32_t>().swap(j->dst);
    std::vector<uint32_t>().swap(j->geid);
    std::vector<int64_t>().swap(j->ts);
  }
  return AMLM_OK;
}

static void committer(amlm_server *S) {
  (void)hipSetDevice(S->device);
  for (;;) {
    std::vector<ServerJob *> batch;
    int f = -1;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      S->cv.wait(lk, [&] {
        if (S->stop) return true;
        if (S->pending.empty()) return false;
        for (int i = 1; i < kVersions; i++) {
          int c = (S->cur + i) % kVersions;
          if (S->ver[c].refs == 0) return true;
        }
        return false;
      });
      if (S->stop) return;
      for (int i = 1; i < kVersions && f < 0; i++) {
        int c = (S->cur + i) % kVersions;
        if (S->ver[c].refs == 0) f = c;
      }
      uint64_t acc = 0;
      while (!S->pending.empty() && (batch.empty() || acc + S->pending.front()->n <= kCommitEdges)) {
        acc += S->pending.front()->n;
        batch.push_back(S->pending.front());
        S->pending.pop_front();
      }
    }
    amlm_status st = commit_group(S, f, batch);
    std::string err = st == AMLM_OK ? std::string() : std::string(amlm_last_error());
    {
      std::lock_guard<std::mutex> lk(S->mu);
      if (st == AMLM_OK) {
        S->cur = f;
        S->commits++;
        S->max_store = std::max(S->max_store, S->ver[f].n);
        const uint64_t nst = S->ver[f].n;
        for (ServerJob *j : batch) {
          j->ver = f;
          j->committed = true;
          j->est_bytes = estimate_bytes(nst, S->ncols);
          S->ver[f].refs++;
          S->ready.push_back(j);
        }
      } else {
        // the store keeps its previous version; these batches fail
        for (ServerJob *j : batch) {
          j->status = st;
          j->err = err;
          j->committed = j->admitted = j->done = true;
          j->t_admit = j->t_done = now_s();
        }
      }
    }
    S->cv.notify_all();
  }
}

// Mining scratch of a slot, sized for stores of up to `need` edges.
static amlm_status slot_scratch(ServerSlot &sl, uint64_t need) {
  if (sl.ms_cap >= need && sl.ms.flags) return AMLM_OK;
  for (void *p : sl.allocs) (void)hipFree(p);
  sl.allocs.clear();
  sl.ms = MineScratch();
  sl.ms_cap = 0;
  const uint64_t cap = need + need / 4 + 1024;
  amlm_status st = alloc_scratch(sl.ms, cap, [&](void **p, size_t bytes) -> amlm_status {
    if (hipMalloc(p, bytes ? bytes : 256) != hipSuccess) {
      (void)hipGetLastError();
      *p = nullptr;
      set_error("server: scratch allocation failed");
      return AMLM_E_NOMEM;
    }
    sl.allocs.push_back(*p);
    return AMLM_OK;
  });
  if (st == AMLM_OK) sl.ms_cap = cap;
  return st;
}

static void run_job(amlm_server *S, ServerSlot &sl, ServerJob *job) {
  hipStream_t s = sl.stream;
  auto fail = [&](amlm_status st) {
    job->status = st;
    job->err = amlm_last_error();
  };
  StoreVer &V = S->ver[job->ver];
  const uint64_t n_st = V.n, lo = job->lo, hi = job->hi;
  amlm_status st;
  if ((st = slot_scratch(sl, n_st)) != AMLM_OK) return fail(st);
  if ((st = grow((void **)&sl.counts, &sl.counts_cap, (uint64_t)S->ncols * std::max<uint64_t>(n_st, 1), 4)) != AMLM_OK)
    return fail(st);
  if ((st = mine_with_scratch(V.g, &S->p, sl.counts, sl.ms, s, (uint32_t)lo, (uint32_t)hi)) != AMLM_OK)
    return fail(st);
  // the batch's own rows, time order
  std::vector<uint32_t> rows((size_t)S->ncols * job->n);
  if (job->n) {
    if (hipMemcpy2DAsync(rows.data(), 4 * job->n, sl.counts + lo, 4 * n_st, 4 * job->n, S->ncols,
                         hipMemcpyDeviceToHost, s) != hipSuccess) {
      set_error("server: copy of the batch rows failed");
      return fail(AMLM_E_DEVICE);
    }
  }
  // cycle and participation credits to older edges (store positions [0, lo))
  uint32_t nd = 0;
  if (S->ncyc && lo) {
    uint64_t cap = std::max<uint64_t>(1u << 16, lo / 4);
    for (int attempt = 0; attempt < 2; attempt++) {
      if (sl.dcap < cap) {
        if (sl.dbuf) (void)hipFree(sl.dbuf);
        sl.dbuf = nullptr;
        sl.dcap = 0;
        uint64_t c = cap + cap / 2;
        if (hipMalloc(&sl.dbuf, 4 * (1 + 3 * c)) != hipSuccess) {
          (void)hipGetLastError();
          set_error("server: device allocation failed");
          return fail(AMLM_E_NOMEM);
        }
        sl.dcap = c;
      }
      if (launch_fill_u32(sl.dbuf, 0, 1, s) != hipSuccess) return fail(AMLM_E_DEVICE);
      uint64_t tot = (uint64_t)S->ncyc * lo;
      hipLaunchKernelGGL(k_collect_deltas, dim3((uint32_t)((tot + 255) / 256)), dim3(256), 0, s, sl.counts, n_st,
                         S->col_cyc, S->ncyc, (uint32_t)lo, V.geid, sl.dbuf, (uint32_t)sl.dcap, sl.dbuf + 1,
                         sl.dbuf + 1 + sl.dcap, sl.dbuf + 1 + 2 * sl.dcap);
      if (hipGetLastError() != hipSuccess) return fail(AMLM_E_DEVICE);
      if (hipMemcpyAsync(&nd, sl.dbuf, 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
          hipStreamSynchronize(s) != hipSuccess)
        return fail(AMLM_E_DEVICE);
      if (nd <= sl.dcap) break;
      cap = (uint64_t)nd + 1024;  // more deltas than room: grow and collect again
    }
  }
  std::vector<uint32_t> de(nd), dc(nd), dv(nd);
  if (nd) {
    if (hipMemcpyAsync(de.data(), sl.dbuf + 1, 4ull * nd, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(dc.data(), sl.dbuf + 1 + sl.dcap, 4ull * nd, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(dv.data(), sl.dbuf + 1 + 2 * sl.dcap, 4ull * nd, hipMemcpyDeviceToHost, s) != hipSuccess)
      return fail(AMLM_E_DEVICE);
  }
  if (hipStreamSynchronize(s) != hipSuccess) {
    set_error("server: mining stream failed");
    return fail(AMLM_E_DEVICE);
  }
  // back to the submitted order
  job->counts.assign((size_t)S->ncols * job->n, 0);
  for (uint32_t c = 0; c < S->ncols; c++)
    for (uint64_t r = 0; r < job->n; r++) job->counts[(size_t)c * job->n + job->order[r]] = rows[(size_t)c * job->n + r];
  std::vector<uint32_t>().swap(job->order);
  // deltas sorted by (edge id, column): the collection order is not fixed
  std::vector<uint32_t> idx(nd);
  std::iota(idx.begin(), idx.end(), 0u);
  std::sort(idx.begin(), idx.end(), [&](uint32_t a, uint32_t b) {
    return de[a] != de[b] ? de[a] < de[b] : dc[a] < dc[b];
  });
  job->d_eid.resize(nd);
  job->d_col.resize(nd);
  job->d_val.resize(nd);
  for (uint32_t i = 0; i < nd; i++) {
    job->d_eid[i] = de[idx[i]];
    job->d_col[i] = dc[idx[i]];
    job->d_val[i] = dv[idx[i]];
  }
}

static void worker(amlm_server *S, uint32_t k) {
  (void)hipSetDevice(S->device);
  ServerSlot &sl = S->slots[k];
  for (;;) {
    ServerJob *job = nullptr;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      S->cv.wait(lk, [&] {
        if (S->stop) return true;
        if (S->ready.empty()) return false;
        ServerJob *j = S->ready.front();
        return S->budget == 0 || S->in_use == 0 || S->in_use + j->est_bytes <= S->budget;
      });
      if (S->stop) return;
      job = S->ready.front();
      S->ready.pop_front();
      S->in_use += job->est_bytes;
      job->admitted = true;
      job->t_admit = now_s();
    }
    S->cv.notify_all();
    run_job(S, sl, job);
    {
      std::lock_guard<std::mutex> lk(S->mu);
      S->in_use -= job->est_bytes;
      S->ver[job->ver].refs--;
      S->batches_done++;
      job->t_done = now_s();
      job->done = true;
    }
    S->cv.notify_all();
  }
}

// A server without its first store version or threads (freed by
// amlm_server_destroy).
static amlm_status server_init(const amlm_params *p, uint64_t hbm_budget_bytes, uint32_t max_slots, uint32_t V,
                               amlm_server **out) {
  amlm_status st = check_params(p);
  if (st != AMLM_OK) return st;
  amlm_server *S = new amlm_server();
  (void)hipGetDevice(&S->device);
  S->p = *p;
  S->ncols = amlm_num_columns(p);
  S->V = V;
  S->budget = hbm_budget_bytes;
  uint32_t c = 0;
  if (p->patterns & AMLM_FAN_OUT) c++;
  if (p->patterns & AMLM_FAN_IN) c++;
  if (p->patterns & AMLM_SG) c++;
  if (p->patterns & AMLM_GS) c++;
  // columns that credit older edges: the cycles and the participation
  // columns (every column from the first cycle column on is collected; the
  // distinct-counterparty and size columns among them are the anchors' own,
  // zero there)
  S->col_cyc = c;
  S->ncyc = (p->patterns & (AMLM_CYCLES | AMLM_PART)) ? S->ncols - c : 0;
  max_slots = std::max(1u, std::min(max_slots, 16u));
  S->max_queue = 64 * max_slots;
  S->slots.resize(max_slots);
  if (hipStreamCreateWithFlags(&S->commit_stream, hipStreamNonBlocking) != hipSuccess) {
    (void)hipGetLastError();
    set_error("server: stream creation failed");
    amlm_server_destroy(S);
    return AMLM_E_DEVICE;
  }
  for (uint32_t k = 0; k < max_slots; k++) {
    if (hipStreamCreateWithFlags(&S->slots[k].stream, hipStreamNonBlocking) != hipSuccess) {
      (void)hipGetLastError();
      set_error("server: stream creation failed");
      amlm_server_destroy(S);
      return AMLM_E_DEVICE;
    }
  }
  *out = S;
  return AMLM_OK;
}

// Build the first store version from its staged edges and start the threads.
static amlm_status server_start(amlm_server *S) {
  StoreVer &v0 = S->ver[0];
  amlm_status st = store_build(S, v0, S->commit_stream);
  if (st != AMLM_OK) return st;
  S->cur = 0;
  S->max_store = v0.n;
  S->committer = std::thread(committer, S);
  for (uint32_t k = 0; k < S->slots.size(); k++) S->slots[k].th = std::thread(worker, S, k);
  return AMLM_OK;
}

extern "C" amlm_status amlm_server_create(amlm_graph *resident, const amlm_params *p, uint64_t hbm_budget_bytes,
                                          uint32_t max_slots, amlm_server **out) {
  if (!resident || !out) {
    set_error("null argument");
    return AMLM_E_INVALID;
  }
  *out = nullptr;
  if (resident->batch.n) {
    set_error("a batched store cannot be served");
    return AMLM_E_INVALID;
  }
  amlm_status st = sticky_check(resident);
  if (st != AMLM_OK) return st;
  amlm_server *S = nullptr;
  if ((st = server_init(p, hbm_budget_bytes, max_slots, resident->V, &S)) != AMLM_OK) return st;
  auto bail = [&](amlm_status code, const char *msg) {
    (void)hipGetLastError();
    if (msg) set_error(msg);
    amlm_server_destroy(S);
    return code;
  };
  // the first store version: the resident edges no older than delta before
  // its latest edge (the first batch is later still)
  const uint64_t Ev = resident->Ev;
  if (resident->E) S->t_last = resident->t_base + (int64_t)resident->t_span;
  uint32_t p0 = 0;
  if (Ev) {
    const int64_t thr = (int64_t)resident->t_span - p->delta;
    uint32_t *d_p0 = nullptr;
    if (hipMalloc(&d_p0, 4) != hipSuccess) return bail(AMLM_E_NOMEM, "server: device allocation failed");
    hipLaunchKernelGGL(k_first_at_or_after, dim3(1), dim3(1), 0, S->commit_stream, graph_view(resident),
                       (int32_t)std::max<int64_t>(thr, INT32_MIN), d_p0);
    bool ok = hipGetLastError() == hipSuccess &&
              hipMemcpyAsync(&p0, d_p0, 4, hipMemcpyDeviceToHost, S->commit_stream) == hipSuccess &&
              hipStreamSynchronize(S->commit_stream) == hipSuccess;
    (void)hipFree(d_p0);
    if (!ok) return bail(AMLM_E_DEVICE, "server: reading the resident graph failed");
  }
  StoreVer &v0 = S->ver[0];
  const uint64_t n0 = Ev - p0;
  if ((st = store_reserve(v0, n0)) != AMLM_OK) return bail(st, nullptr);
  v0.n = n0;
  if (n0) {
    hipLaunchKernelGGL(k_store_from_graph, dim3((uint32_t)((n0 + 255) / 256)), dim3(256), 0, S->commit_stream,
                       graph_view(resident), resident->t_base, p0, v0.ts, v0.src, v0.dst, v0.geid);
    v0.host_ts.resize(n0);
    if (hipGetLastError() != hipSuccess ||
        hipMemcpyAsync(v0.host_ts.data(), v0.ts, 8 * n0, hipMemcpyDeviceToHost, S->commit_stream) != hipSuccess ||
        hipStreamSynchronize(S->commit_stream) != hipSuccess)
      return bail(AMLM_E_DEVICE, "server: copying the resident graph failed");
  }
  S->next_geid = resident->E;
  if ((st = server_start(S)) != AMLM_OK) return bail(st, nullptr);
  *out = S;
  return AMLM_OK;
}

// Snapshot file: magic, the parameters, n_vertices, the latest timestamp, the
// next edge id, the window store's edge count, then its src, dst, ts and
// global edge ids in time order.
static const char kSnapMagic[8] = {'A', 'M', 'L', 'M', 'S', 'N', 'P', '1'};

extern "C" amlm_status amlm_server_snapshot(amlm_server *S, const char *path) {
  if (!S || !path) {
    set_error("null argument");
    return AMLM_E_INVALID;
  }
  std::vector<uint32_t> src, dst, geid;
  std::vector<int64_t> ts;
  int64_t t_last;
  uint64_t next_geid, n;
  amlm_params p;
  {
    std::unique_lock<std::mutex> lk(S->mu);
    // every submitted batch in the store (mining may still go on: it only
    // reads the version)
    S->cv.wait(lk, [&] { return S->pending.empty() || S->stop; });
    StoreVer &v = S->ver[S->cur];
    n = v.n;
    src.resize(n);
    dst.resize(n);
    geid.resize(n);
    ts.resize(n);
    if (n && (hipMemcpyAsync(src.data(), v.src, 4 * n, hipMemcpyDeviceToHost, S->commit_stream) != hipSuccess ||
              hipMemcpyAsync(dst.data(), v.dst, 4 * n, hipMemcpyDeviceToHost, S->commit_stream) != hipSuccess ||
              hipMemcpyAsync(geid.data(), v.geid, 4 * n, hipMemcpyDeviceToHost, S->commit_stream) != hipSuccess ||
              hipMemcpyAsync(ts.data(), v.ts, 8 * n, hipMemcpyDeviceToHost, S->commit_stream) != hipSuccess ||
              hipStreamSynchronize(S->commit_stream) != hipSuccess)) {
      (void)hipGetLastError();
      set_error("server: snapshot copy failed");
      return AMLM_E_DEVICE;
    }
    t_last = S->t_last;
    next_geid = S->next_geid;
    p = S->p;
  }
  FILE *f = fopen(path, "wb");
  if (!f) {
    set_error(std::string("cannot open ") + path);
    return AMLM_E_INVALID;
  }
  bool ok = fwrite(kSnapMagic, 1, 8, f) == 8 && fwrite(&p, sizeof(p), 1, f) == 1 && fwrite(&S->V, 4, 1, f) == 1 &&
            fwrite(&t_last, 8, 1, f) == 1 && fwrite(&next_geid, 8, 1, f) == 1 && fwrite(&n, 8, 1, f) == 1 &&
            fwrite(src.data(), 4, n, f) == n && fwrite(dst.data(), 4, n, f) == n && fwrite(ts.data(), 8, n, f) == n &&
            fwrite(geid.data(), 4, n, f) == n;
  ok = (fclose(f) == 0) && ok;
  if (!ok) {
    set_error("server: short write of the snapshot");
    return AMLM_E_INVALID;
  }
  return AMLM_OK;
}

extern "C" amlm_status amlm_server_resume(const char *path, uint64_t hbm_budget_bytes, uint32_t max_slots,
                                          amlm_server **out) {
  if (!path || !out) {
    set_error("null argument");
    return AMLM_E_INVALID;
  }
  *out = nullptr;
  FILE *f = fopen(path, "rb");
  if (!f) {
    set_error(std::string("cannot open ") + path);
    return AMLM_E_INVALID;
  }
  char magic[8];
  amlm_params p;
  uint32_t V = 0;
  int64_t t_last = 0;
  uint64_t next_geid = 0, n = 0;
  bool ok = fread(magic, 1, 8, f) == 8 && memcmp(magic, kSnapMagic, 8) == 0 && fread(&p, sizeof(p), 1, f) == 1 &&
            fread(&V, 4, 1, f) == 1 && fread(&t_last, 8, 1, f) == 1 && fread(&next_geid, 8, 1, f) == 1 &&
            fread(&n, 8, 1, f) == 1 && n < 0xffffffffull;
  std::vector<uint32_t> src, dst, geid;
  std::vector<int64_t> ts;
  if (ok) {
    src.resize(n);
    dst.resize(n);
    geid.resize(n);
    ts.resize(n);
    ok = fread(src.data(), 4, n, f) == n && fread(dst.data(), 4, n, f) == n && fread(ts.data(), 8, n, f) == n &&
         fread(geid.data(), 4, n, f) == n;
  }
  fclose(f);
  if (!ok) {
    set_error("not a server snapshot, or a truncated one");
    return AMLM_E_INVALID;
  }
  for (uint64_t i = 0; i < n; i++)
    if (src[i] >= V || dst[i] >= V || (i && ts[i] < ts[i - 1])) {
      set_error("corrupt server snapshot");
      return AMLM_E_INVALID;
    }
  amlm_server *S = nullptr;
  amlm_status st = server_init(&p, hbm_budget_bytes, max_slots, V, &S);
  if (st != AMLM_OK) return st;
  StoreVer &v0 = S->ver[0];
  if ((st = store_reserve(v0, n)) != AMLM_OK) {
    amlm_server_destroy(S);
    return st;
  }
  v0.n = n;
  v0.host_ts = ts;
  hipStream_t s = S->commit_stream;
  if (n && (hipMemcpyAsync(v0.src, src.data(), 4 * n, hipMemcpyHostToDevice, s) != hipSuccess ||
            hipMemcpyAsync(v0.dst, dst.data(), 4 * n, hipMemcpyHostToDevice, s) != hipSuccess ||
            hipMemcpyAsync(v0.geid, geid.data(), 4 * n, hipMemcpyHostToDevice, s) != hipSuccess ||
            hipMemcpyAsync(v0.ts, ts.data(), 8 * n, hipMemcpyHostToDevice, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)) {
    (void)hipGetLastError();
    set_error("server: restoring the snapshot failed");
    amlm_server_destroy(S);
    return AMLM_E_DEVICE;
  }
  S->t_last = t_last;
  S->next_geid = next_geid;
  if ((st = server_start(S)) != AMLM_OK) {
    amlm_server_destroy(S);
    return st;
  }
  *out = S;
  return AMLM_OK;
}

extern "C" amlm_status amlm_server_submit(amlm_server *S, const uint32_t *src, const uint32_t *dst, const int64_t *ts,
                                          uint64_t n, int wait, uint64_t *ticket) {
  if (!S || !ticket || (n && (!src || !dst || !ts))) {
    set_error("null argument");
    return AMLM_E_INVALID;
  }
  // ordered by time inside the batch (stable); the submitted order is kept
  // for the results
  ServerJob *job = new ServerJob();
  job->order.resize(n);
  std::iota(job->order.begin(), job->order.end(), 0u);
  if (!std::is_sorted(ts, ts + n))
    std::stable_sort(job->order.begin(), job->order.end(), [&](uint32_t a, uint32_t b) { return ts[a] < ts[b]; });
  job->src.resize(n);
  job->dst.resize(n);
  job->ts.resize(n);
  job->geid.resize(n);
  for (uint64_t i = 0; i < n; i++) {
    uint32_t j = job->order[i];
    if (src[j] >= S->V || dst[j] >= S->V) {
      delete job;
      set_error("stream edge endpoint >= n_vertices");
      return AMLM_E_INVALID;
    }
    job->src[i] = src[j];
    job->dst[i] = dst[j];
    job->ts[i] = ts[j];
  }
  std::unique_lock<std::mutex> lk(S->mu);
  if (n && job->ts[0] <= S->t_last) {
    delete job;
    set_error("a stream batch must be strictly later than every earlier edge");
    return AMLM_E_ORDER;
  }
  if (n && job->ts[n - 1] - job->ts[0] >= 0x7fffffffll - S->p.delta) {
    delete job;
    set_error("a stream batch spans too long a time for 32-bit relative times");
    return AMLM_E_RANGE;
  }
  auto backlog = [&] { return S->pending.size() + S->ready.size(); };
  if (!wait && backlog() >= S->max_queue) {
    delete job;
    set_error("server queue is full");
    return AMLM_E_BUSY;
  }
  if (wait) S->cv.wait(lk, [&] { return backlog() < S->max_queue || S->stop; });
  job->ticket = S->next_ticket++;
  job->n = n;
  job->geid0 = S->next_geid;
  job->tmin = n ? job->ts[0] : S->t_last;
  job->t_submit = now_s();
  for (uint64_t i = 0; i < n; i++) job->geid[i] = (uint32_t)(job->geid0 + job->order[i]);
  if (n) {
    S->t_last = job->ts[n - 1];
    S->next_geid += n;
  }
  S->jobs[job->ticket] = job;
  S->pending.push_back(job);
  *ticket = job->ticket;
  S->cv.notify_all();
  return AMLM_OK;
}

// Drop the timing records of the oldest taken tickets beyond kKeepTimes.
static void trim_taken(amlm_server *S) {
  while (S->taken.size() > kKeepTimes) {
    auto it = S->jobs.find(S->taken.front());
    if (it != S->jobs.end()) {
      delete it->second;
      S->jobs.erase(it);
    }
    S->taken.pop_front();
  }
}

extern "C" amlm_status amlm_server_wait(amlm_server *S, uint64_t ticket, uint32_t *new_counts_host,
                                        uint64_t *n_deltas, uint64_t *delta_eid, uint32_t *delta_col,
                                        uint32_t *delta_val, uint64_t cap) {
  if (!S) {
    set_error("null server");
    return AMLM_E_INVALID;
  }
  std::unique_lock<std::mutex> lk(S->mu);
  auto it = S->jobs.find(ticket);
  if (it == S->jobs.end() || it->second->taken) {
    set_error("unknown ticket, or its results were already taken");
    return AMLM_E_INVALID;
  }
  ServerJob *job = it->second;
  S->cv.wait(lk, [&] { return job->done; });
  job->taken = true;
  S->taken.push_back(ticket);
  if (job->status != AMLM_OK) {
    amlm_status st = job->status;
    set_error(job->err);
    trim_taken(S);
    return st;
  }
  if (new_counts_host && !job->counts.empty())
    memcpy(new_counts_host, job->counts.data(), 4 * job->counts.size());
  uint64_t nd = job->d_eid.size();
  if (n_deltas) *n_deltas = nd;
  uint64_t m = std::min(nd, cap);
  for (uint64_t i = 0; i < m; i++) {
    if (delta_eid) delta_eid[i] = job->d_eid[i];
    if (delta_col) delta_col[i] = job->d_col[i];
    if (delta_val) delta_val[i] = job->d_val[i];
  }
  // keep the timing record, drop the payload
  std::vector<uint32_t>().swap(job->counts);
  std::vector<uint64_t>().swap(job->d_eid);
  std::vector<uint32_t>().swap(job->d_col);
  std::vector<uint32_t>().swap(job->d_val);
  trim_taken(S);
  return AMLM_OK;
}

extern "C" amlm_status amlm_server_ticket_times(amlm_server *S, uint64_t ticket, double *t_submit, double *t_admit,
                                                double *t_done) {
  if (!S) {
    set_error("null server");
    return AMLM_E_INVALID;
  }
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->jobs.find(ticket);
  if (it == S->jobs.end()) {
    set_error("unknown ticket (or its timing record was dropped)");
    return AMLM_E_INVALID;
  }
  ServerJob *job = it->second;
  if (t_submit) *t_submit = job->t_submit;
  if (t_admit) *t_admit = job->t_admit;
  if (t_done) *t_done = job->t_done;
  return AMLM_OK;
}

extern "C" amlm_status amlm_server_stats(amlm_server *S, uint64_t *window_edges, uint64_t *max_window_edges,
                                         uint64_t *commits, uint64_t *batches_done) {
  if (!S) {
    set_error("null server");
    return AMLM_E_INVALID;
  }
  std::lock_guard<std::mutex> lk(S->mu);
  if (window_edges) *window_edges = S->ver[S->cur].n;
  if (max_window_edges) *max_window_edges = S->max_store;
  if (commits) *commits = S->commits;
  if (batches_done) *batches_done = S->batches_done;
  return AMLM_OK;
}

extern "C" void amlm_server_destroy(amlm_server *S) {
  if (!S) return;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
  }
  S->cv.notify_all();
  if (S->committer.joinable()) S->committer.join();
  for (ServerSlot &sl : S->slots)
    if (sl.th.joinable()) sl.th.join();
  (void)hipDeviceSynchronize();
  for (ServerSlot &sl : S->slots) {
    for (void *p : sl.allocs) (void)hipFree(p);
    if (sl.counts) (void)hipFree(sl.counts);
    if (sl.dbuf) (void)hipFree(sl.dbuf);
    if (sl.stream) (void)hipStreamDestroy(sl.stream);
  }
  for (StoreVer &v : S->ver) {
    if (v.g) amlm_graph_destroy(v.g);
    for (void *p : {(void *)v.src, (void *)v.dst, (void *)v.geid, (void *)v.ts})
      if (p) (void)hipFree(p);
  }
  for (auto &kv : S->jobs) delete kv.second;
  if (S->commit_stream) (void)hipStreamDestroy(S->commit_stream);
  delete S;
}
