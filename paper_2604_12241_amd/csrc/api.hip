// C ABI: graph store lifetime and the plain mining entry points.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <functional>
#include <mutex>
#include <string>

#include "api_internal.h"
#include "costmodel.h"

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }

extern "C" const char *amlm_last_error(void) { return g_last_error.c_str(); }

// ------------------------------------------------------------------ helpers

DeviceInfo &device_info() {
  static DeviceInfo info;
  static std::once_flag once;
  std::call_once(once, [] {
    int dev = 0;
    (void)hipGetDevice(&dev);
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) {
      info.num_cu = prop.multiProcessorCount;
      snprintf(info.name, sizeof(info.name), "%s", prop.gcnArchName);
    }
    int occ = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_sg_ptr(), kSgThreads, 0) == hipSuccess && occ > 0)
      info.sg_occ = occ;
    occ = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_cyc_ptr(false), kCycThreads, 0) == hipSuccess && occ > 0)
      info.cyc_occ = occ;
    occ = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_cyc_ptr(true), kCycThreads, 0) == hipSuccess && occ > 0)
      info.cyc_occ_small = occ;
  });
  return info;
}

static amlm_status dalloc(amlm_graph *g, void **p, size_t bytes) {
  if (bytes == 0) bytes = 256;
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    set_error("hipMalloc of " + std::to_string(bytes) + " bytes failed: " + hipGetErrorString(e));
    *p = nullptr;
    return AMLM_E_NOMEM;
  }
  g->allocs.push_back(*p);
  g->device_bytes += bytes;
  return AMLM_OK;
}

#define A_TRY(x)                    \
  do {                              \
    amlm_status st_ = (x);          \
    if (st_ != AMLM_OK) return st_; \
  } while (0)

static void free_all(amlm_graph *g) {
  for (void *p : g->allocs) (void)hipFree(p);
  g->allocs.clear();
  g->device_bytes = 0;
  g->cap_e = 0;
  g->cap_v = 0;
  g->ms = MineScratch();
}

// Allocate the graph's arrays for E edges and V vertices, with 1/8 spare
// capacity so that a graph rebuilt a little larger (a serving window) keeps
// its buffers: a reallocation frees and allocates ~50 buffers, and freeing
// synchronises the device.
static amlm_status alloc_graph(amlm_graph *g, uint64_t E, uint32_t V) {
  if (E <= g->cap_e && V <= g->cap_v && g->cap_e) return AMLM_OK;
  free_all(g);
  E = std::min<uint64_t>(E + E / 8 + 1024, 0xfffffffeull);
  uint64_t e = E;
  uint64_t v1 = (uint64_t)V + 1;
  GraphArrays &a = g->arr;
  A_TRY(dalloc(g, (void **)&a.src, 4 * e));
  A_TRY(dalloc(g, (void **)&a.dst, 4 * e));
  A_TRY(dalloc(g, (void **)&a.t, 4 * e));
  A_TRY(dalloc(g, (void **)&a.anc, 4 * e));
  A_TRY(dalloc(g, (void **)&a.pos_out, 4 * e));
  A_TRY(dalloc(g, (void **)&a.pos_in, 4 * e));
  A_TRY(dalloc(g, (void **)&a.out_ptr, 4 * v1));
  A_TRY(dalloc(g, (void **)&a.out_nbr, 4 * e));
  A_TRY(dalloc(g, (void **)&a.out_eid, 4 * e));
  A_TRY(dalloc(g, (void **)&a.out_t, 4 * e));
  A_TRY(dalloc(g, (void **)&a.out_prv, 4 * e));
  A_TRY(dalloc(g, (void **)&a.out_src, 4 * e));
  A_TRY(dalloc(g, (void **)&a.out_h, 4 * e));
  A_TRY(dalloc(g, (void **)&a.out_tm, 16 * v1));
  A_TRY(dalloc(g, (void **)&a.out_tix, 4 * (e / kTixPerBucket + 2 * v1 + 2)));
  A_TRY(dalloc(g, (void **)&a.tix_cnt, 4 * v1));
  A_TRY(dalloc(g, (void **)&a.tix_off, 4 * v1));
  A_TRY(dalloc(g, (void **)&a.in_ptr, 4 * v1));
  A_TRY(dalloc(g, (void **)&a.in_nbr, 4 * e));
  A_TRY(dalloc(g, (void **)&a.in_eid, 4 * e));
  A_TRY(dalloc(g, (void **)&a.in_t, 4 * e));
  A_TRY(dalloc(g, (void **)&a.in_nxt, 4 * e));
  A_TRY(dalloc(g, (void **)&a.in_dst, 4 * e));
  A_TRY(dalloc(g, (void **)&a.in_h, 4 * e));
  A_TRY(dalloc(g, (void **)&a.inn_key, 8 * e));
  A_TRY(dalloc(g, (void **)&a.inn_eid, 4 * e));
  BuildBuffers &b = g->bb;
  A_TRY(dalloc(g, (void **)&b.ka, 4 * e));
  A_TRY(dalloc(g, (void **)&b.kb, 4 * e));
  A_TRY(dalloc(g, (void **)&b.va, 4 * e));
  A_TRY(dalloc(g, (void **)&b.vb, 4 * e));
  size_t hw = radix_hist_words(e);
  A_TRY(dalloc(g, (void **)&b.hist, 4 * hw));
  A_TRY(dalloc(g, (void **)&b.hist2, 4 * hw));
  size_t tw = std::max(scan_tmp_words(hw), scan_tmp_words(v1));
  A_TRY(dalloc(g, (void **)&b.scan_tmp, 4 * tw));
  A_TRY(dalloc(g, (void **)&b.stats, 8 * (8 + 5 * kValidateBlocks)));
  A_TRY(dalloc(g, (void **)&b.ep, 16 * e));
  A_TRY(dalloc(g, (void **)&g->ts_stage, 8 * e));
  g->cap_e = E;
  g->cap_v = V;
  return AMLM_OK;
}

// Mining scratch, sized for the graph's edge capacity (so allocated once per
// graph allocation).
amlm_status alloc_scratch(MineScratch &ms, uint64_t cap,
                          const std::function<amlm_status(void **, size_t)> &alloc) {
  const uint64_t ev = std::max<uint64_t>(cap, 1);
  uint32_t nb = (uint32_t)((ev + kFlagTile - 1) / kFlagTile);
  A_TRY(alloc((void **)&ms.flags, 2 * ((ev + 3) & ~3ull)));
  A_TRY(alloc((void **)&ms.sg_win, 16 * ev));
  A_TRY(alloc((void **)&ms.feat, 4 * kMlpRaw * ev));
  A_TRY(alloc((void **)&ms.pred, 4 * ev));
  A_TRY(alloc((void **)&ms.list_sg, 4 * ev));
  A_TRY(alloc((void **)&ms.list_cy, 4 * ev));
  A_TRY(alloc((void **)&ms.bcnt_sg, 4 * (size_t)nb));
  A_TRY(alloc((void **)&ms.bcnt_cy, 4 * (size_t)nb));
  A_TRY(alloc((void **)&ms.boff_sg, 4 * (size_t)nb));
  A_TRY(alloc((void **)&ms.boff_cy, 4 * (size_t)nb));
  A_TRY(alloc((void **)&ms.scan_tmp, 4 * std::max(scan_tmp_words(nb), scan_tmp_words(ev))));
  A_TRY(alloc((void **)&ms.ctr, 4 * kCtrWords));
  A_TRY(alloc((void **)&ms.nsub, 4 * ev));
  A_TRY(alloc((void **)&ms.ucnt, 4 * ev));
  A_TRY(alloc((void **)&ms.uoff, 4 * ev));
  A_TRY(alloc((void **)&ms.units, 8 * max_units(ev, kMinBlock)));
  ms.cap_ev = ev;
  ms.cap_e = ev;
  return AMLM_OK;
}

amlm_status alloc_mine_scratch(amlm_graph *g) {
  MineScratch &ms = g->ms;
  if (ms.flags && ms.cap_ev >= std::max<uint64_t>(g->Ev, 1) && ms.cap_e >= g->E) return AMLM_OK;
  return alloc_scratch(ms, g->cap_e, [g](void **p, size_t bytes) { return dalloc(g, p, bytes); });
}

GraphView graph_view(const amlm_graph *g) {
  const GraphArrays &a = g->arr;
  GraphView v;
  v.V = g->V;
  v.E = (uint32_t)g->E;
  v.Ev = g->Ev;
  v.src = a.src;
  v.dst = a.dst;
  v.t = a.t;
  v.anc = a.anc;
  v.pos_out = a.pos_out;
  v.pos_in = a.pos_in;
  v.out_ptr = a.out_ptr;
  v.out_nbr = a.out_nbr;
  v.out_eid = a.out_eid;
  v.out_t = a.out_t;
  v.out_prv = a.out_prv;
  v.out_src = a.out_src;
  v.out_h = a.out_h;
  v.out_tm = a.out_tm;
  v.out_tix = a.out_tix;
  v.in_ptr = a.in_ptr;
  v.in_nbr = a.in_nbr;
  v.in_eid = a.in_eid;
  v.in_t = a.in_t;
  v.in_nxt = a.in_nxt;
  v.in_dst = a.in_dst;
  v.in_h = a.in_h;
  v.inn_key = a.inn_key;
  v.inn_eid = a.inn_eid;
  return v;
}

// ------------------------------------------------------------------ graph

amlm_status sticky_check(amlm_graph *g) {
  if (g->sticky != AMLM_OK) {
    set_error("the graph handle had a HIP runtime error earlier (sticky); destroy it");
    return g->sticky;
  }
  if (g->inject) {
    g->inject = 0;
    g->sticky = AMLM_E_DEVICE;
    set_error("injected HIP runtime error (testing aid)");
    return AMLM_E_DEVICE;
  }
  return AMLM_OK;
}

amlm_status sticky_note(amlm_graph *g, amlm_status st) {
  if (st == AMLM_E_DEVICE && g) g->sticky = AMLM_E_DEVICE;
  return st;
}

static amlm_status do_build(amlm_graph *g, const uint32_t *src, const uint32_t *dst, const int64_t *ts,
                            uint64_t n_edges, uint32_t n_vertices, int on_device, hipStream_t s) {
  A_TRY(sticky_check(g));
  if (n_edges >= 0xffffffffull) {
    set_error("n_edges must be < 2^32 - 1");
    return AMLM_E_INVALID;
  }
  if (n_edges && (!src || !dst || !ts)) {
    set_error("null edge array");
    return AMLM_E_INVALID;
  }
  A_TRY(alloc_graph(g, n_edges, n_vertices));
  GraphArrays &a = g->arr;
  const int64_t *ts_dev = ts;
  if (n_edges) {
    hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    HIP_TRY(hipMemcpyAsync(a.src, src, 4 * n_edges, kind, s));
    HIP_TRY(hipMemcpyAsync(a.dst, dst, 4 * n_edges, kind, s));
    if (!on_device) {
      HIP_TRY(hipMemcpyAsync(g->ts_stage, ts, 8 * n_edges, kind, s));
      ts_dev = g->ts_stage;
    }
  }
  ValidateResult vr;
  HIP_TRY(validate_edges(a.src, a.dst, ts_dev, n_edges, n_vertices, g->bb.stats, &vr, s));
  if (vr.bad_ids) {
    set_error(std::to_string(vr.bad_ids) + " edge endpoints are >= n_vertices");
    return AMLM_E_INVALID;
  }
  uint64_t span = n_edges ? (uint64_t)(vr.tmax - vr.tmin) : 0;
  if (n_edges && (vr.tmax < vr.tmin || span >= 0x7fffffffull)) {
    set_error("timestamp span must be < 2^31 - 1");
    return AMLM_E_RANGE;
  }
  g->E = n_edges;
  g->V = n_vertices;
  g->Ev = (uint32_t)(n_edges - vr.self_loops);
  g->t_base = vr.tmin;
  g->t_span = span;
  int t_bits = bits_for(span);
  HIP_TRY(g->timer.begin(kStBuild, s));
  HIP_TRY(build_graph(a, ts_dev, vr.tmin, (uint32_t)n_edges, g->Ev, n_vertices, t_bits, vr.unsorted == 0,
                      vr.self_loops, g->bb, s));
  HIP_TRY(g->timer.end(kStBuild, s));
  A_TRY(alloc_mine_scratch(g));
  HIP_TRY(hipStreamSynchronize(s));
  return AMLM_OK;
}

extern "C" amlm_status amlm_graph_create(const uint32_t *src, const uint32_t *dst, const int64_t *ts,
                                         const float *amount, uint64_t n_edges, uint32_t n_vertices,
                                         int inputs_on_device, void *hip_stream, amlm_graph **out) {
  (void)amount;  // carried by the caller; no pattern reads it
  if (!out) {
    set_error("out is null");
    return AMLM_E_INVALID;
  }
  *out = nullptr;
  amlm_graph *g = new amlm_graph();
  HIP_TRY(hipGetDevice(&g->device));
  amlm_status st = do_build(g, src, dst, ts, n_edges, n_vertices, inputs_on_device, (hipStream_t)hip_stream);
  if (st != AMLM_OK) {
    free_all(g);
    delete g;
    return st;
  }
  *out = g;
  return AMLM_OK;
}

extern "C" amlm_status amlm_graph_rebuild(amlm_graph *g, const uint32_t *src, const uint32_t *dst,
                                          const int64_t *ts, uint64_t n_edges, uint32_t n_vertices,
                                          int inputs_on_device, void *hip_stream) {
  if (!g) {
    set_error("null graph");
    return AMLM_E_INVALID;
  }
  return sticky_note(g, do_build(g, src, dst, ts, n_edges, n_vertices, inputs_on_device, (hipStream_t)hip_stream));
}

extern "C" void amlm_graph_destroy(amlm_graph *g) {
  if (!g) return;
  (void)hipDeviceSynchronize();
  batch_free(g);
  free_all(g);
  if (g->timer.ev[0])
    for (hipEvent_t &e : g->timer.ev) (void)hipEventDestroy(e);
  if (g->aux) {
    (void)hipEventDestroy(g->ev_fork);
    (void)hipEventDestroy(g->ev_join);
    (void)hipStreamDestroy(g->aux);
  }
  delete g;
}

extern "C" amlm_status amlm_graph_info(const amlm_graph *g, uint64_t *n_edges, uint64_t *n_valid,
                                       uint32_t *n_vertices, int64_t *t_base) {
  if (!g) {
    set_error("null graph");
    return AMLM_E_INVALID;
  }
  if (n_edges) *n_edges = g->E;
  if (n_valid) *n_valid = g->Ev;
  if (n_vertices) *n_vertices = g->V;
  if (t_base) *t_base = g->t_base;
  return AMLM_OK;
}

// ------------------------------------------------------------------ mining

amlm_status check_params(const amlm_params *p) {
  if (!p) {
    set_error("null params");
    return AMLM_E_INVALID;
  }
  const uint32_t cols = AMLM_ALL | AMLM_DEG_OUT | AMLM_DEG_IN;
  if ((p->patterns & cols) == 0 ||
      (p->patterns & ~(cols | AMLM_SG_UNORDERED | AMLM_SG_PHASE | AMLM_CYC_ANY_ORDER | AMLM_PART | AMLM_SG_SIZES))) {
    set_error("patterns must be a non-empty set of pattern bits (plus the modifiers)");
    return AMLM_E_INVALID;
  }
  if ((p->patterns & AMLM_PART) && (!(p->patterns & (AMLM_SG | AMLM_GS)) || (p->patterns & AMLM_SG_PHASE))) {
    set_error("AMLM_PART needs AMLM_SG or AMLM_GS and excludes AMLM_SG_PHASE");
    return AMLM_E_INVALID;
  }
  if ((p->patterns & AMLM_SG_SIZES) && (!(p->patterns & AMLM_SG) || (p->patterns & AMLM_SG_PHASE))) {
    set_error("AMLM_SG_SIZES modifies AMLM_SG and excludes AMLM_SG_PHASE");
    return AMLM_E_INVALID;
  }
  if ((p->patterns & AMLM_SG_UNORDERED) && !(p->patterns & AMLM_SG)) {
    set_error("AMLM_SG_UNORDERED modifies AMLM_SG, which is not requested");
    return AMLM_E_INVALID;
  }
  if ((p->patterns & AMLM_SG_PHASE) && (!(p->patterns & AMLM_SG) || (p->patterns & AMLM_SG_UNORDERED))) {
    set_error("AMLM_SG_PHASE modifies AMLM_SG and excludes AMLM_SG_UNORDERED");
    return AMLM_E_INVALID;
  }
  if ((p->patterns & AMLM_SG_PHASE) && p->k > kPhaseKMax) {
    set_error("the phase-ordered scatter-gather supports k <= 8");
    return AMLM_E_INVALID;
  }
  if ((p->patterns & AMLM_CYC_ANY_ORDER) && !(p->patterns & AMLM_CYCLES)) {
    set_error("AMLM_CYC_ANY_ORDER modifies AMLM_CYCLES, which is not requested");
    return AMLM_E_INVALID;
  }
  if (p->delta < 0) {
    set_error("delta must be >= 0");
    return AMLM_E_INVALID;
  }
  if ((p->patterns & AMLM_CYCLES) && (p->max_cycle_len < 2 || p->max_cycle_len > 8)) {
    set_error("max_cycle_len must be in 2..8");
    return AMLM_E_INVALID;
  }
  if ((p->patterns & (AMLM_SG | AMLM_GS)) && p->k == 0) {
    set_error("k must be >= 1");
    return AMLM_E_INVALID;
  }
  if (p->schedule > AMLM_SCHED_GIVEN) {
    set_error("unknown schedule");
    return AMLM_E_INVALID;
  }
  return AMLM_OK;
}

extern "C" uint32_t amlm_num_columns(const amlm_params *p) {
  if (check_params(p) != AMLM_OK) return 0;
  uint32_t c = 0;
  if (p->patterns & AMLM_FAN_OUT) c++;
  if (p->patterns & AMLM_FAN_IN) c++;
  if (p->patterns & AMLM_SG) c++;
  if (p->patterns & AMLM_GS) c++;
  if (p->patterns & AMLM_CYCLES) c += p->max_cycle_len - 1;
  if (p->patterns & AMLM_DEG_OUT) c++;
  if (p->patterns & AMLM_DEG_IN) c++;
  if ((p->patterns & AMLM_PART) && (p->patterns & AMLM_SG)) c++;
  if ((p->patterns & AMLM_PART) && (p->patterns & AMLM_GS)) c++;
  if (p->patterns & AMLM_SG_SIZES) c += 4;
  return c;
}

MineParams make_params(const amlm_graph *g, const amlm_params *p, uint32_t *counts, unsigned long long *work) {
  MineParams mp;
  mp.g = graph_view(g);
  mp.delta = p->delta;
  mp.L = (p->patterns & AMLM_CYCLES) ? p->max_cycle_len : 2;
  mp.k = p->k ? p->k : 1;
  mp.vgraph = nullptr;
  mp.sub = nullptr;
  mp.anchor_lo = 0;
  mp.anchor_hi = 0xffffffffu;
  int c = 0;
  mp.col_fo = (p->patterns & AMLM_FAN_OUT) ? c++ : -1;
  mp.col_fi = (p->patterns & AMLM_FAN_IN) ? c++ : -1;
  mp.col_sg = (p->patterns & AMLM_SG) ? c++ : -1;
  mp.col_gs = (p->patterns & AMLM_GS) ? c++ : -1;
  mp.col_cyc = (p->patterns & AMLM_CYCLES) ? c : -1;
  if (p->patterns & AMLM_CYCLES) c += (int)mp.L - 1;
  mp.col_do = (p->patterns & AMLM_DEG_OUT) ? c++ : -1;
  mp.col_di = (p->patterns & AMLM_DEG_IN) ? c++ : -1;
  mp.sg_unordered = (p->patterns & AMLM_SG_UNORDERED) ? 1u : 0u;
  mp.sg_phase = (p->patterns & AMLM_SG_PHASE) ? 1u : 0u;
  mp.cyc_any = (p->patterns & AMLM_CYC_ANY_ORDER) ? 1u : 0u;
  mp.counts = counts;
  mp.stride = g->E;
  mp.ceil = g->ceiling;
  mp.work = work;
  return mp;
}

MineLaunch default_launch(const amlm_graph *g) {
  DeviceInfo &di = device_info();
  MineLaunch cfg;
  cfg.sg_blocks = (uint32_t)(di.num_cu * di.sg_occ);
  cfg.cyc_blocks = (uint32_t)(di.num_cu * di.cyc_occ);
  cfg.cyc_blocks_small = (uint32_t)(di.num_cu * di.cyc_occ_small);
  cfg.sg_chunk = kStaticChunk;  // anchors per work-stealing grab
  if (g->tune.sg_chunk) cfg.sg_chunk = cfg.learned_chunk = g->tune.sg_chunk;
  if (g->tune.sg_blocks) cfg.sg_blocks = g->tune.sg_blocks;
  if (g->tune.cyc_blocks) cfg.cyc_blocks = cfg.cyc_blocks_small = g->tune.cyc_blocks;
  if (g->tune.split_bytes) cfg.split_bytes = g->tune.split_bytes;
  return cfg;
}

amlm_status schedule_config(const amlm_graph *g, const amlm_params *p, MineLaunch &cfg) {
  cfg.sched = p->schedule;
  cfg.delta_hours = (float)p->delta / 3600.f;
  const MlpModel &m = global_model();
  if ((p->schedule == AMLM_SCHED_LEARNED || p->schedule == AMLM_SCHED_LENGTH) && !m.loaded) {
    set_error("the learned and length schedules need a cost model (amlm_costmodel_train or _load)");
    return AMLM_E_INVALID;
  }
  if (p->schedule == AMLM_SCHED_LENGTH) {
    if (!(m.len_coef > 0.f)) {
      set_error("the loaded cost model has no length constant (retrain it)");
      return AMLM_E_INVALID;
    }
    cfg.len_coef = m.len_coef;
  }
  if (p->schedule == AMLM_SCHED_GIVEN) {
    if (!g->given_cost) {
      set_error("the given schedule needs per-edge costs (amlm_graph_set_costs)");
      return AMLM_E_INVALID;
    }
    cfg.given = g->given_cost;
  }
  return AMLM_OK;
}

extern "C" amlm_status amlm_graph_set_costs(amlm_graph *g, const float *log_cost_dev) {
  if (!g) {
    set_error("null graph");
    return AMLM_E_INVALID;
  }
  g->given_cost = log_cost_dev;
  return AMLM_OK;
}

static amlm_status mine_impl(amlm_graph *g, const amlm_params *p, uint32_t *counts_dev, unsigned long long *work_dev,
                             hipStream_t s, uint32_t anchor_lo) {
  A_TRY(check_params(p));
  if (g->E && !counts_dev) {
    set_error("null counts");
    return AMLM_E_INVALID;
  }
  A_TRY(sticky_check(g));
  uint32_t ncols = amlm_num_columns(p);
  HIP_TRY(launch_fill_u32(counts_dev, 0, (uint64_t)ncols * g->E, s));
  if (work_dev) HIP_TRY(launch_fill_u32((uint32_t *)work_dev, 0, 2ull * kWorkRows * g->E, s));
  A_TRY(alloc_mine_scratch(g));
  MineParams mp = make_params(g, p, counts_dev, work_dev);
  mp.anchor_lo = anchor_lo;
  MineLaunch cfg = default_launch(g);
  A_TRY(schedule_config(g, p, cfg));
  if (anchor_lo == 0) {
    // full mining: the cycle search runs on a second stream beside the
    // anchor passes, the cost model and the work units (incremental mining of
    // small serving windows stays on one stream: the server's slots already
    // run concurrently)
    if (!g->aux) {
      HIP_TRY(hipStreamCreateWithFlags(&g->aux, hipStreamNonBlocking));
      HIP_TRY(hipEventCreateWithFlags(&g->ev_fork, hipEventDisableTiming));
      HIP_TRY(hipEventCreateWithFlags(&g->ev_join, hipEventDisableTiming));
    }
    cfg.aux = g->aux;
    cfg.ev_fork = g->ev_fork;
    cfg.ev_join = g->ev_join;
  }
  HIP_TRY(mine_launch(mp, g->ms, cfg, s, &g->timer));
  HIP_TRY(part_launch(mp, p, g->ms, s));
  return AMLM_OK;
}

#ifndef AMLM_NARROW_CHUNK
#define AMLM_NARROW_CHUNK 4
#endif
constexpr uint32_t kNarrowChunk = AMLM_NARROW_CHUNK;  // 0: no special case
constexpr uint64_t kNarrowRange = 1u << 20;             // anchor ranges narrower than this
#ifndef AMLM_NARROW_SPLIT
#define AMLM_NARROW_SPLIT 16384
#endif
constexpr uint32_t kNarrowSplit = AMLM_NARROW_SPLIT;   // their slice size (0: the default)

amlm_status mine_with_scratch(amlm_graph *g, const amlm_params *p, uint32_t *counts_dev, MineScratch &ms,
                              hipStream_t s, uint32_t anchor_lo, uint32_t anchor_hi) {
  if (!g) {
    set_error("null graph");
    return AMLM_E_INVALID;
  }
  A_TRY(check_params(p));
  if (g->E && !counts_dev) {
    set_error("null counts");
    return AMLM_E_INVALID;
  }
  A_TRY(sticky_check(g));
  if (ms.cap_e < g->E || ms.cap_ev < std::max<uint64_t>(g->Ev, 1)) {
    set_error("mining scratch too small for the graph");
    return AMLM_E_INVALID;
  }
  const uint32_t ncols = amlm_num_columns(p);
  auto run = [&]() -> amlm_status {
    HIP_TRY(launch_fill_u32(counts_dev, 0, (uint64_t)ncols * g->E, s));
    MineParams mp = make_params(g, p, counts_dev, nullptr);
    mp.anchor_lo = anchor_lo;
    mp.anchor_hi = anchor_hi;
    MineLaunch cfg = default_launch(g);
    A_TRY(schedule_config(g, p, cfg));
    // a narrow anchor range (a stream batch) shares few windows between
    // anchors: the smallest work units and smaller slices spread it over
    // more waves (serving on the 32M-edge graph: 37.2M edges/s with the
    // full-graph units, 43.1M with 4-anchor units, 46.5M with 16 KB slices
    // too; 4 KB slices 46.3M with a worse p99)
    if (kNarrowChunk && !g->tune.sg_chunk && (uint64_t)anchor_hi - anchor_lo < kNarrowRange) {
      cfg.sg_chunk = cfg.learned_chunk = kNarrowChunk;
      if (kNarrowSplit && !g->tune.split_bytes) cfg.split_bytes = kNarrowSplit;
    }
    HIP_TRY(mine_launch(mp, ms, cfg, s, nullptr));
    HIP_TRY(part_launch(mp, p, ms, s));
    return AMLM_OK;
  };
  return sticky_note(g, run());
}

amlm_status mine_common(amlm_graph *g, const amlm_params *p, uint32_t *counts_dev, unsigned long long *work_dev,
                        hipStream_t s, uint32_t anchor_lo) {
  if (!g) {
    set_error("null graph");
    return AMLM_E_INVALID;
  }
  return sticky_note(g, mine_impl(g, p, counts_dev, work_dev, s, anchor_lo));
}

extern "C" amlm_status amlm_mine(amlm_graph *g, const amlm_params *p, uint32_t *counts_dev, void *hip_stream) {
  return mine_common(g, p, counts_dev, nullptr, (hipStream_t)hip_stream);
}

// ------------------------------------------------------------------ mining without allocation
// amlm_mine_static's mining scratch: one array per device (each GPU the
// library runs on holds it until the process ends).  Its device address is
// taken with hipGetSymbolAddress once per device, with that device current,
// and only that address is used from the host.
constexpr uint64_t kStaticScratchBytes = 64ull << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxDevices] = {};

static amlm_status static_scratch(int dev, void **out) {
  if (dev < 0 || dev >= kMaxDevices) {
    set_error("device ordinal out of range for the static scratch");
    return AMLM_E_INVALID;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      (void)hipGetLastError();
      set_error(std::string("hipGetSymbolAddress of the static scratch: ") + hipGetErrorString(e));
      return AMLM_E_DEVICE;
    }
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return AMLM_OK;
}

// Bytes of mining scratch a graph of `cap` edges needs, carved as in
// alloc_scratch with 256-byte alignment.
static uint64_t static_scratch_need(uint64_t cap) {
  MineScratch ms;
  uint64_t off = 0;
  (void)alloc_scratch(ms, cap, [&](void **p, size_t bytes) {
    *p = (void *)(uintptr_t)(off + 256);  // placeholder, never dereferenced
    off += (std::max<size_t>(bytes, 1) + 255) & ~(size_t)255;
    return AMLM_OK;
  });
  return off;
}

extern "C" amlm_status amlm_mine_static(amlm_graph *g, const amlm_params *p, uint32_t *counts_dev,
                                        void *hip_stream) {
  if (!g) {
    set_error("null graph");
    return AMLM_E_INVALID;
  }
  A_TRY(check_params(p));
  A_TRY(sticky_check(g));
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev != g->device) {
    set_error("amlm_mine_static: the graph's device must be the current device");
    return AMLM_E_INVALID;
  }
  const uint64_t cap = std::max<uint64_t>(g->E, 1);
  const uint64_t need = static_scratch_need(cap);
  if (need > kStaticScratchBytes) {
    set_error("amlm_mine_static: the graph needs " + std::to_string(need) +
              " bytes of mining scratch; the static scratch holds " + std::to_string(kStaticScratchBytes) +
              " (about 850,000 edges): use amlm_mine");
    return AMLM_E_NOMEM;
  }
  void *base = nullptr;
  A_TRY(sticky_note(g, static_scratch(dev, &base)));
  MineScratch ms;
  uint64_t off = 0;
  A_TRY(alloc_scratch(ms, cap, [&](void **q, size_t bytes) {
    *q = (unsigned char *)base + off;
    off += (std::max<size_t>(bytes, 1) + 255) & ~(size_t)255;
    return AMLM_OK;
  }));
  return mine_with_scratch(g, p, counts_dev, ms, (hipStream_t)hip_stream, 0, 0xffffffffu);
}

extern "C" amlm_status amlm_mine_work(amlm_graph *g, const amlm_params *p, uint32_t *counts_dev,
                                      uint64_t *work_dev, void *hip_stream) {
  if (g && g->E && !work_dev) {
    set_error("null work");
    return AMLM_E_INVALID;
  }
  return mine_common(g, p, counts_dev, (unsigned long long *)work_dev, (hipStream_t)hip_stream);
}

extern "C" amlm_status amlm_graph_sync(amlm_graph *g, void *hip_stream) {
  if (!g) {
    set_error("null graph");
    return AMLM_E_INVALID;
  }
  A_TRY(sticky_check(g));
  hipError_t e = hipStreamSynchronize((hipStream_t)hip_stream);
  if (e != hipSuccess) {
    set_error(std::string("hipStreamSynchronize: ") + hipGetErrorString(e));
    return sticky_note(g, AMLM_E_DEVICE);
  }
  return AMLM_OK;
}

extern "C" amlm_status amlm_graph_status(const amlm_graph *g) {
  if (!g) {
    set_error("null graph");
    return AMLM_E_INVALID;
  }
  return g->sticky;
}

extern "C" amlm_status amlm_graph_inject_device_error(amlm_graph *g) {
  if (!g) {
    set_error("null graph");
    return AMLM_E_INVALID;
  }
  g->inject = 1;
  return AMLM_OK;
}

extern "C" amlm_status amlm_graph_set_ceiling(amlm_graph *g, uint32_t ceiling) {
  if (!g) {
    set_error("null graph");
    return AMLM_E_INVALID;
  }
  g->ceiling = ceiling ? ceiling : 0xffffffffu;
  return AMLM_OK;
}

extern "C" amlm_status amlm_set_timing(amlm_graph *g, int enable) {
  if (!g) {
    set_error("null graph");
    return AMLM_E_INVALID;
  }
  if (enable && !g->timer.ev[0])
    for (hipEvent_t &e : g->timer.ev) HIP_TRY(hipEventCreate(&e));
  g->timer.on = enable != 0;
  for (bool &u : g->timer.used) u = false;
  return AMLM_OK;
}

extern "C" amlm_status amlm_tune_set(amlm_graph *g, uint32_t block, uint32_t sg_blocks, uint32_t cyc_blocks,
                                     uint32_t split_bytes) {
  if (!g) {
    set_error("null graph");
    return AMLM_E_INVALID;
  }
  g->tune.sg_chunk = block;
  g->tune.sg_blocks = sg_blocks;
  g->tune.cyc_blocks = cyc_blocks;
  g->tune.split_bytes = split_bytes;
  return AMLM_OK;
}

extern "C" amlm_status amlm_stage_times(amlm_graph *g, float *ms) {
  if (!g || !ms) {
    set_error("null argument");
    return AMLM_E_INVALID;
  }
  for (int st = 0; st < kNumStages; st++) {
    ms[st] = -1.0f;
    if (!g->timer.used[st]) continue;
    HIP_TRY(hipEventSynchronize(g->timer.ev[2 * st + 1]));
    HIP_TRY(hipEventElapsedTime(&ms[st], g->timer.ev[2 * st], g->timer.ev[2 * st + 1]));
  }
  return AMLM_OK;
}
