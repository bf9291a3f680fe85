// Streaming server: continuous batching of transaction batches over a
// resident graph.  Each incoming edge's columns come from the instances that
// end at it, and cycles it closes credit older edges (streaming integration,
// Section 5; incremental, localized updates instead of a full recompute).
//
// History: every resident and submitted edge, time-sorted, in device memory.
// A batch is mined on its own window graph = the history suffix within delta
// of the batch plus the batch itself, with only the batch's edges as anchors.
// Admission: a batch starts when a slot is free and the HBM budget allows;
// slots run concurrently, each on its own HIP stream.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <numeric>
#include <thread>
#include <vector>

#include "api_internal.h"

namespace {

// time-ordered copy of a resident graph's valid edges into the history
__global__ void k_hist_from_graph(GraphView g, int64_t t_base, int64_t *ts, uint32_t *src, uint32_t *dst,
                                  uint32_t *geid) {
  uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= g.Ev) return;
  uint32_t e = g.anc[p];
  ts[p] = t_base + g.t[e];
  src[p] = g.src[e];
  dst[p] = g.dst[e];
  geid[p] = e;
}

// nonzero cycle credits of context edges -> (global edge id, column, value)
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

}  // namespace

struct ServerJob {
  uint64_t ticket = 0;
  uint64_t hist_begin = 0, hist_end = 0;  // the batch's edges in the history
  uint64_t geid0 = 0, n = 0;
  int64_t tmin = 0;
  std::vector<uint32_t> order;            // history offset -> index in submitted order
  uint64_t est_bytes = 0;
  double t_submit = 0, t_admit = 0, t_done = 0;
  std::vector<uint32_t> counts;           // [ncols][n], submitted order
  std::vector<uint64_t> d_eid;
  std::vector<uint32_t> d_col, d_val;
  amlm_status status = AMLM_OK;
  std::string err;
  bool admitted = false, done = false;
};

struct ServerSlot {
  std::thread th;
  hipStream_t stream = nullptr;
  amlm_graph *g = nullptr;
  uint32_t *counts = nullptr;
  uint64_t counts_cap = 0;
  uint32_t *dbuf = nullptr;  // [count, eid[cap], col[cap], val[cap]]
  uint64_t dcap = 0;
};

struct amlm_server {
  int device = 0;
  amlm_params p{};
  uint32_t ncols = 0, col_cyc = 0, ncyc = 0;
  uint32_t V = 0;
  uint64_t budget = 0, in_use = 0;
  // history
  int64_t *h_ts = nullptr;
  uint32_t *h_src = nullptr, *h_dst = nullptr, *h_geid = nullptr;
  uint64_t h_len = 0, h_cap = 0;
  std::vector<int64_t> host_ts;
  int64_t t_last = INT64_MIN;
  uint64_t next_geid = 0, next_ticket = 1;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<ServerJob *> queue;
  std::map<uint64_t, ServerJob *> jobs;
  bool stop = false;
  hipStream_t ingest = nullptr;
  std::vector<ServerSlot> slots;
  uint32_t max_queue = 0;
};

static uint64_t estimate_bytes(uint64_t n_window, uint32_t ncols) {
  // graph store (~110 B per edge) + counts + mining scratch
  return n_window * (110 + 4ull * ncols + 40) + (1ull << 20);
}

static amlm_status grow(void **p, uint64_t *cap, uint64_t need, size_t elem) {
  if (*cap >= need) return AMLM_OK;
  if (*p) (void)hipFree(*p);
  uint64_t n = std::max<uint64_t>(need, *cap * 2);
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

static void run_job(amlm_server *S, ServerSlot &sl, ServerJob *job) {
  hipStream_t s = sl.stream;
  auto fail = [&](amlm_status st) {
    job->status = st;
    job->err = amlm_last_error();
  };
  // context: history entries within delta of the batch's first edge
  uint64_t c0;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    int64_t lo = job->tmin - S->p.delta;
    c0 = std::lower_bound(S->host_ts.begin(), S->host_ts.begin() + job->hist_begin, lo) - S->host_ts.begin();
  }
  const uint64_t n_ctx = job->hist_begin - c0, n_win = job->hist_end - c0;
  amlm_status st;
  if (!sl.g) {
    st = amlm_graph_create(S->h_src + c0, S->h_dst + c0, S->h_ts + c0, nullptr, n_win, S->V, 1, s, &sl.g);
  } else {
    st = amlm_graph_rebuild(sl.g, S->h_src + c0, S->h_dst + c0, S->h_ts + c0, n_win, S->V, 1, s);
  }
  if (st != AMLM_OK) return fail(st);
  if ((st = grow((void **)&sl.counts, &sl.counts_cap, (uint64_t)S->ncols * n_win, 4)) != AMLM_OK) return fail(st);
  if ((st = mine_common(sl.g, &S->p, sl.counts, nullptr, s, (uint32_t)n_ctx)) != AMLM_OK) return fail(st);
  // the batch's own rows, history order
  std::vector<uint32_t> rows((size_t)S->ncols * job->n);
  if (job->n) {
    if (hipMemcpy2DAsync(rows.data(), 4 * job->n, sl.counts + n_ctx, 4 * n_win, 4 * job->n, S->ncols,
                         hipMemcpyDeviceToHost, s) != hipSuccess) {
      set_error("server: copy of the batch rows failed");
      return fail(AMLM_E_DEVICE);
    }
  }
  // cycle credits to older edges
  uint32_t nd = 0;
  if (S->ncyc && n_ctx) {
    uint64_t cap = std::max<uint64_t>(1u << 16, n_ctx / 4);
    if (sl.dcap < cap) {
      // regrown with room to spare: freeing synchronises the device
      cap += cap / 2;
      if (sl.dbuf) (void)hipFree(sl.dbuf);
      sl.dbuf = nullptr;
      sl.dcap = 0;
      if (hipMalloc(&sl.dbuf, 4 * (1 + 3 * cap)) != hipSuccess) {
        (void)hipGetLastError();
        set_error("server: device allocation failed");
        return fail(AMLM_E_NOMEM);
      }
      sl.dcap = cap;
    }
    for (int attempt = 0; attempt < 2; attempt++) {
      if (launch_fill_u32(sl.dbuf, 0, 1, s) != hipSuccess) return fail(AMLM_E_DEVICE);
      uint64_t tot = (uint64_t)S->ncyc * n_ctx;
      hipLaunchKernelGGL(k_collect_deltas, dim3((uint32_t)((tot + 255) / 256)), dim3(256), 0, s, sl.counts, n_win,
                         S->col_cyc, S->ncyc, (uint32_t)n_ctx, S->h_geid + c0, sl.dbuf, (uint32_t)sl.dcap,
                         sl.dbuf + 1, sl.dbuf + 1 + sl.dcap, sl.dbuf + 1 + 2 * sl.dcap);
      if (hipGetLastError() != hipSuccess) return fail(AMLM_E_DEVICE);
      if (hipMemcpyAsync(&nd, sl.dbuf, 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
          hipStreamSynchronize(s) != hipSuccess)
        return fail(AMLM_E_DEVICE);
      if (nd <= sl.dcap) break;
      // more deltas than room: grow and collect again
      (void)hipFree(sl.dbuf);
      sl.dbuf = nullptr;
      sl.dcap = 0;
      uint64_t cap2 = (uint64_t)nd + 1024;
      if (hipMalloc(&sl.dbuf, 4 * (1 + 3 * cap2)) != hipSuccess) {
        (void)hipGetLastError();
        set_error("server: device allocation failed");
        return fail(AMLM_E_NOMEM);
      }
      sl.dcap = cap2;
    }
  }
  std::vector<uint32_t> de(nd), dc(nd), dv(nd);
  if (nd) {
    if (hipMemcpyAsync(de.data(), sl.dbuf + 1, 4ull * nd, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(dc.data(), sl.dbuf + 1 + sl.dcap, 4ull * nd, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(dv.data(), sl.dbuf + 1 + 2 * sl.dcap, 4ull * nd, hipMemcpyDeviceToHost, s) != hipSuccess)
      return fail(AMLM_E_DEVICE);
  }
  if (hipStreamSynchronize(s) != hipSuccess) return fail(AMLM_E_DEVICE);
  if ((st = amlm_graph_sync(sl.g, s)) != AMLM_OK) return fail(st);
  // back to the submitted order
  job->counts.assign((size_t)S->ncols * job->n, 0);
  for (uint32_t c = 0; c < S->ncols; c++)
    for (uint64_t r = 0; r < job->n; r++) job->counts[(size_t)c * job->n + job->order[r]] = rows[(size_t)c * job->n + r];
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
        if (S->queue.empty()) return false;
        ServerJob *j = S->queue.front();
        return S->budget == 0 || S->in_use == 0 || S->in_use + j->est_bytes <= S->budget;
      });
      if (S->stop && S->queue.empty()) return;
      job = S->queue.front();
      S->queue.pop_front();
      S->in_use += job->est_bytes;
      job->admitted = true;
      job->t_admit = now_s();
    }
    S->cv.notify_all();
    run_job(S, sl, job);
    {
      std::lock_guard<std::mutex> lk(S->mu);
      S->in_use -= job->est_bytes;
      job->t_done = now_s();
      job->done = true;
    }
    S->cv.notify_all();
  }
}

extern "C" amlm_status amlm_server_create(amlm_graph *resident, const amlm_params *p, uint64_t hbm_budget_bytes,
                                          uint32_t max_slots, amlm_server **out) {
  if (!resident || !out) {
    set_error("null argument");
    return AMLM_E_INVALID;
  }
  *out = nullptr;
  amlm_status st = check_params(p);
  if (st != AMLM_OK) return st;
  if (resident->batch.n) {
    set_error("a batched store cannot be served");
    return AMLM_E_INVALID;
  }
  amlm_server *S = new amlm_server();
  (void)hipGetDevice(&S->device);
  S->p = *p;
  S->ncols = amlm_num_columns(p);
  S->V = resident->V;
  S->budget = hbm_budget_bytes;
  uint32_t c = 0;
  if (p->patterns & AMLM_FAN_OUT) c++;
  if (p->patterns & AMLM_FAN_IN) c++;
  if (p->patterns & AMLM_SG) c++;
  if (p->patterns & AMLM_GS) c++;
  S->col_cyc = c;
  S->ncyc = (p->patterns & AMLM_CYCLES) ? p->max_cycle_len - 1 : 0;
  max_slots = std::max(1u, std::min(max_slots, 16u));
  S->max_queue = 64 * max_slots;
  const uint64_t Ev = resident->Ev;
  S->h_cap = std::max<uint64_t>(Ev + (16ull << 20), 1ull << 20);
  if (S->h_cap >= 0xffffffffull) S->h_cap = 0xfffffffeull;
  bool ok = hipMalloc(&S->h_ts, 8 * S->h_cap) == hipSuccess && hipMalloc(&S->h_src, 4 * S->h_cap) == hipSuccess &&
            hipMalloc(&S->h_dst, 4 * S->h_cap) == hipSuccess && hipMalloc(&S->h_geid, 4 * S->h_cap) == hipSuccess &&
            hipStreamCreateWithFlags(&S->ingest, hipStreamNonBlocking) == hipSuccess;
  if (!ok) {
    (void)hipGetLastError();
    set_error("server: device allocation failed");
    amlm_server_destroy(S);
    return AMLM_E_NOMEM;
  }
  if (Ev) {
    hipLaunchKernelGGL(k_hist_from_graph, dim3((uint32_t)((Ev + 255) / 256)), dim3(256), 0, S->ingest,
                       graph_view(resident), resident->t_base, S->h_ts, S->h_src, S->h_dst, S->h_geid);
    S->host_ts.resize(Ev);
    if (hipGetLastError() != hipSuccess ||
        hipMemcpyAsync(S->host_ts.data(), S->h_ts, 8 * Ev, hipMemcpyDeviceToHost, S->ingest) != hipSuccess ||
        hipStreamSynchronize(S->ingest) != hipSuccess) {
      set_error("server: copying the resident graph failed");
      amlm_server_destroy(S);
      return AMLM_E_DEVICE;
    }
    S->t_last = S->host_ts.back();
  }
  S->h_len = Ev;
  S->next_geid = resident->E;
  S->slots.resize(max_slots);
  for (uint32_t k = 0; k < max_slots; k++) {
    if (hipStreamCreateWithFlags(&S->slots[k].stream, hipStreamNonBlocking) != hipSuccess) {
      set_error("server: stream creation failed");
      amlm_server_destroy(S);
      return AMLM_E_DEVICE;
    }
  }
  for (uint32_t k = 0; k < max_slots; k++) S->slots[k].th = std::thread(worker, S, k);
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
  std::vector<uint32_t> ord(n);
  std::iota(ord.begin(), ord.end(), 0u);
  std::stable_sort(ord.begin(), ord.end(), [&](uint32_t a, uint32_t b) { return ts[a] < ts[b]; });
  std::vector<uint32_t> s2(n), d2(n), g2(n);
  std::vector<int64_t> t2(n);
  for (uint64_t i = 0; i < n; i++) {
    uint32_t j = ord[i];
    if (src[j] >= S->V || dst[j] >= S->V) {
      set_error("stream edge endpoint >= n_vertices");
      return AMLM_E_INVALID;
    }
    s2[i] = src[j];
    d2[i] = dst[j];
    t2[i] = ts[j];
  }
  std::unique_lock<std::mutex> lk(S->mu);
  if (n && t2[0] <= S->t_last) {
    set_error("a stream batch must be strictly later than every earlier edge");
    return AMLM_E_ORDER;
  }
  if (!wait && S->queue.size() >= S->max_queue) {
    set_error("server queue is full");
    return AMLM_E_BUSY;
  }
  if (S->h_len + n > S->h_cap) {
    set_error("server history capacity exceeded");
    return AMLM_E_NOMEM;
  }
  ServerJob *job = new ServerJob();
  job->ticket = S->next_ticket++;
  job->n = n;
  job->geid0 = S->next_geid;
  job->hist_begin = S->h_len;
  job->hist_end = S->h_len + n;
  job->tmin = n ? t2[0] : S->t_last;
  job->order = ord;
  job->t_submit = now_s();
  for (uint64_t i = 0; i < n; i++) g2[i] = (uint32_t)(job->geid0 + ord[i]);
  if (n) {
    uint64_t h = S->h_len;
    bool ok = hipMemcpyAsync(S->h_src + h, s2.data(), 4 * n, hipMemcpyHostToDevice, S->ingest) == hipSuccess &&
              hipMemcpyAsync(S->h_dst + h, d2.data(), 4 * n, hipMemcpyHostToDevice, S->ingest) == hipSuccess &&
              hipMemcpyAsync(S->h_ts + h, t2.data(), 8 * n, hipMemcpyHostToDevice, S->ingest) == hipSuccess &&
              hipMemcpyAsync(S->h_geid + h, g2.data(), 4 * n, hipMemcpyHostToDevice, S->ingest) == hipSuccess &&
              hipStreamSynchronize(S->ingest) == hipSuccess;
    if (!ok) {
      delete job;
      set_error("server: ingest copy failed");
      return AMLM_E_DEVICE;
    }
    S->host_ts.insert(S->host_ts.end(), t2.begin(), t2.end());
    S->h_len += n;
    S->t_last = t2[n - 1];
    S->next_geid += n;
  }
  int64_t lo = job->tmin - S->p.delta;
  uint64_t c0 = std::lower_bound(S->host_ts.begin(), S->host_ts.begin() + job->hist_begin, lo) - S->host_ts.begin();
  job->est_bytes = estimate_bytes(job->hist_end - c0, S->ncols);
  S->jobs[job->ticket] = job;
  S->queue.push_back(job);
  *ticket = job->ticket;
  S->cv.notify_all();
  if (wait) S->cv.wait(lk, [&] { return job->admitted || S->stop; });
  return AMLM_OK;
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
  if (it == S->jobs.end()) {
    set_error("unknown ticket");
    return AMLM_E_INVALID;
  }
  ServerJob *job = it->second;
  S->cv.wait(lk, [&] { return job->done; });
  if (job->status != AMLM_OK) {
    amlm_status st = job->status;
    set_error(job->err);
    S->jobs.erase(it);
    delete job;
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
  job->counts.clear();
  job->counts.shrink_to_fit();
  job->d_eid.clear();
  job->d_col.clear();
  job->d_val.clear();
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
    set_error("unknown ticket");
    return AMLM_E_INVALID;
  }
  ServerJob *job = it->second;
  if (t_submit) *t_submit = job->t_submit;
  if (t_admit) *t_admit = job->t_admit;
  if (t_done) *t_done = job->t_done;
  return AMLM_OK;
}

extern "C" void amlm_server_destroy(amlm_server *S) {
  if (!S) return;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
  }
  S->cv.notify_all();
  for (ServerSlot &sl : S->slots)
    if (sl.th.joinable()) sl.th.join();
  for (ServerSlot &sl : S->slots) {
    if (sl.g) amlm_graph_destroy(sl.g);
    if (sl.counts) (void)hipFree(sl.counts);
    if (sl.dbuf) (void)hipFree(sl.dbuf);
    if (sl.stream) (void)hipStreamDestroy(sl.stream);
  }
  for (auto &kv : S->jobs) delete kv.second;
  if (S->h_ts) (void)hipFree(S->h_ts);
  if (S->h_src) (void)hipFree(S->h_src);
  if (S->h_dst) (void)hipFree(S->h_dst);
  if (S->h_geid) (void)hipFree(S->h_geid);
  if (S->ingest) (void)hipStreamDestroy(S->ingest);
  delete S;
}
