// Host-side graph handle and helpers shared by the C ABI translation units.
#pragma once

#include <cstring>
#include <functional>
#include <string>
#include <vector>

#include "mine.h"

struct DeviceInfo {
  int num_cu = 256;
  int sg_occ = 4;
  int cyc_occ = 3, cyc_occ_small = 3;
  char name[64] = "gfx950";
};
DeviceInfo &device_info();

struct TuneParams {
  uint32_t sg_chunk = 0, sg_blocks = 0, cyc_blocks = 0, split_bytes = 0;  // 0 = default
};

// Batched store state (batch.hip): sub-graph layout, device parameter
// tables and the captured launch sequence.
struct BatchState {
  uint32_t n = 0;                      // number of sub-graphs (0: ordinary graph)
  std::vector<uint64_t> eoff;          // edge offsets [n + 1]
  std::vector<uint32_t> voff;          // vertex offsets [n + 1]
  uint64_t *d_eoff = nullptr;
  uint32_t *d_voff = nullptr, *vgraph = nullptr, *d_ncols = nullptr;
  SubParams *d_sub = nullptr;
  uint32_t **d_outs = nullptr;
  uint32_t *comb = nullptr;            // combined counts [ncols][E]
  uint32_t comb_cols = 0;
  hipGraphExec_t exec = nullptr;
  hipStream_t cap_stream = nullptr;
  std::string sig;
  uint32_t captures = 0;
  std::vector<void *> allocs;
};
void batch_free(amlm_graph *g);

struct amlm_graph {
  int device = 0;
  uint64_t E = 0;
  uint32_t V = 0, Ev = 0;
  int64_t t_base = 0;
  uint64_t t_span = 0;
  uint64_t cap_e = 0;
  uint32_t cap_v = 0;
  GraphArrays arr{};
  BuildBuffers bb{};
  int64_t *ts_stage = nullptr;
  MineScratch ms{};
  TuneParams tune{};
  StageTimer timer{};
  hipStream_t aux = nullptr;  // second mining stream (cycle kernel), created on first use
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  BatchState batch{};
  uint32_t ceiling = 0xffffffffu;  // counts saturate here
  const float *given_cost = nullptr;  // AMLM_SCHED_GIVEN: caller's log1p(bytes) per edge id
  // AMLM_E_DEVICE once a HIP runtime call failed inside a call on this
  // handle; every later call except destroy / info / status returns it
  amlm_status sticky = AMLM_OK;
  uint32_t inject = 0;             // testing aid: fail the next mining or build call
  std::vector<void *> allocs;
  uint64_t device_bytes = 0;
};

amlm_status check_params(const amlm_params *p);
GraphView graph_view(const amlm_graph *g);
MineParams make_params(const amlm_graph *g, const amlm_params *p, uint32_t *counts, unsigned long long *work);
MineLaunch default_launch(const amlm_graph *g);
// The scatter-gather schedule of p on g (cost model, length constant or
// given costs as needed): AMLM_E_INVALID when what it needs is missing.
amlm_status schedule_config(const amlm_graph *g, const amlm_params *p, MineLaunch &cfg);
amlm_status alloc_mine_scratch(amlm_graph *g);
// Mining scratch for graphs of up to cap edges, each buffer from `alloc`.
amlm_status alloc_scratch(MineScratch &ms, uint64_t cap, const std::function<amlm_status(void **, size_t)> &alloc);
// Mining of the anchors with ids in [anchor_lo, anchor_hi) with the caller's
// scratch (sized for g by alloc_scratch) on stream s only: several calls may
// run concurrently on one graph, each with its own scratch and counts.
amlm_status mine_with_scratch(amlm_graph *g, const amlm_params *p, uint32_t *counts_dev, MineScratch &ms,
                              hipStream_t s, uint32_t anchor_lo, uint32_t anchor_hi);
// Mining with the edges of id >= anchor_lo as the only anchors (0 = all).
amlm_status mine_common(amlm_graph *g, const amlm_params *p, uint32_t *counts_dev, unsigned long long *work_dev,
                        hipStream_t s, uint32_t anchor_lo = 0);
// Instance columns (AMLM_PART, AMLM_SG_SIZES; part.hip): their column
// indices in p's layout (-1 when absent; c_sz is the first of four), and the
// pass that fills them for the anchors of mp's range (after mine_launch on
// the same stream; the columns must start at zero).
void part_columns(const amlm_params *p, int *c_ps, int *c_pg, int *c_sz);
hipError_t part_launch(const MineParams &mp, const amlm_params *p, MineScratch &ms, hipStream_t s);
// Sticky device errors: returns g's sticky status if set; otherwise, if a
// fault was injected for this call, records it and returns AMLM_E_DEVICE.
amlm_status sticky_check(amlm_graph *g);
// Records AMLM_E_DEVICE as g's sticky status; returns st unchanged.
amlm_status sticky_note(amlm_graph *g, amlm_status st);
