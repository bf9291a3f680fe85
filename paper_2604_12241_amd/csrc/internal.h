// Host-side declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/amlm.h"
#include "common.h"

// ---------------------------------------------------------------- errors
void set_error(const std::string &msg);
#define HIP_TRY(expr)                                                            \
  do {                                                                           \
    hipError_t e_ = (expr);                                                      \
    if (e_ != hipSuccess) {                                                      \
      set_error(std::string(#expr) + ": " + hipGetErrorString(e_));             \
      return AMLM_E_DEVICE;                                                      \
    }                                                                            \
  } while (0)

// ---------------------------------------------------------------- build
struct BuildBuffers {
  uint32_t *ka = nullptr, *kb = nullptr, *va = nullptr, *vb = nullptr;
  uint32_t *hist = nullptr, *hist2 = nullptr, *scan_tmp = nullptr;
  uint64_t *stats = nullptr;  // [8] validation results, then 5 per validation block
  uint4 *ep = nullptr;        // per edge id: (destination, time) pairs, then (source, time) pairs
  size_t cap_n = 0, cap_hist = 0, cap_tmp = 0;
};

// Exclusive scan of n u32 values; out may alias nothing.  total (device,
// optional) receives the sum.  tmp must hold scan_tmp_words(n) words.  With
// n_dev (device, optional) only the first min(*n_dev, n) values are scanned
// (a count known on the device only; n bounds the launch).
size_t scan_tmp_words(uint64_t n);
hipError_t scan_exclusive_u32(const uint32_t *in, uint32_t *out, uint32_t n, uint32_t *total, uint32_t *tmp,
                              hipStream_t s, const uint32_t *n_dev = nullptr);

// Stable LSD radix sort of (key, value) pairs by the low `bits` bits of the
// key.  Input in (ka, va); result pointers returned through *kout, *vout
// (either the a or the b buffers).
hipError_t radix_sort_pairs(uint32_t *ka, uint32_t *va, uint32_t *kb, uint32_t *vb, uint32_t n, int bits,
                            uint32_t *hist, uint32_t *hist2, uint32_t *scan_tmp, hipStream_t s,
                            uint32_t **kout, uint32_t **vout);
size_t radix_hist_words(uint64_t n);

hipError_t launch_fill_u32(uint32_t *p, uint32_t value, uint64_t n, hipStream_t s);

// Graph build pipeline.  Device inputs src/dst/ts (E edges).  Fills the
// graph arrays described by `gv` (non-const aliases passed in `w`).
struct GraphArrays {
  uint32_t *src, *dst;
  int32_t *t;
  uint32_t *anc, *pos_out, *pos_in;
  uint32_t *out_ptr, *out_nbr, *out_eid, *out_src, *out_h;
  int32_t *out_t, *out_prv;
  uint4 *out_tm;        // [V]: out-row time index headers
  uint32_t *out_tix;    // bucket starts, at most Ev / 16 + 2 V + 2 entries
  uint32_t *tix_cnt, *tix_off;  // [V + 1] build scratch
  uint32_t *in_ptr, *in_nbr, *in_eid, *in_dst, *in_h;
  int32_t *in_t, *in_nxt;
  uint64_t *inn_key;
  uint32_t *inn_eid;
};

constexpr uint32_t kValidateBlocks = 2048;  // most blocks of the validation pass

struct ValidateResult {
  int64_t tmin, tmax;
  uint64_t bad_ids, self_loops, unsorted;
};

hipError_t validate_edges(const uint32_t *src, const uint32_t *dst, const int64_t *ts, uint64_t E, uint32_t V,
                          uint64_t *stats_dev, ValidateResult *res, hipStream_t s);
hipError_t build_graph(const GraphArrays &a, const int64_t *ts, int64_t tmin, uint32_t E, uint32_t Ev, uint32_t V,
                       int t_bits, bool time_sorted, uint64_t n_self, BuildBuffers &bb, hipStream_t s);

int bits_for(uint64_t max_value);  // number of bits to represent [0, max_value]
