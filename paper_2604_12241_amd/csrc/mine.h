// Mining launch interface shared by the C ABI, batching and serving code.
#pragma once

#include "internal.h"

constexpr uint8_t kFlagSG = 1, kFlagCYC = 2;
// scatter-gather anchor whose v has no in-neighbour other than u inside the
// anchor's window: no intermediate besides u exists, so SG_k is 0 for k >= 2
// and the anchor needs no join (only its senders, for GS_k)
constexpr uint8_t kFlagSgNoJoin = 4;
// scatter-gather anchor (k >= 2) whose u has at least k distinct scatter
// destinations in (tau, t], tau the earliest sender time: decided by the CSR
// pass, where u's out-row is at hand
constexpr uint8_t kFlagGsDest = 8;
// senders-window slices up to this length are classified by the anchor lane
constexpr uint32_t kAnchorScanCap = 16;

constexpr int kSgThreads = 64;   // one wave per block
#ifndef AMLM_PREFETCH_CLAIM
#define AMLM_PREFETCH_CLAIM 0
#endif
constexpr bool kPrefetchClaim = AMLM_PREFETCH_CLAIM != 0;
// occupancy target for k_sg (waves per SIMD): six keep it within 80 VGPRs
// without spills, and its LDS allows about as many
#ifndef AMLM_SG_WAVES_PER_EU
#define AMLM_SG_WAVES_PER_EU 6
#endif
#if AMLM_SG_WAVES_PER_EU > 0
#define AMLM_SG_OCCUPANCY __attribute__((amdgpu_waves_per_eu(AMLM_SG_WAVES_PER_EU, AMLM_SG_WAVES_PER_EU)))
#else
#define AMLM_SG_OCCUPANCY
#endif
#ifndef AMLM_BLOOM_LOG2_MAX
#define AMLM_BLOOM_LOG2_MAX 15
#endif
#ifndef AMLM_BLOOM_BITS_PER_ENTRY
#define AMLM_BLOOM_BITS_PER_ENTRY 128
#endif
#ifndef AMLM_BLOOM_K
#define AMLM_BLOOM_K 4
#endif
#ifndef AMLM_SG_CHUNK_MAX
#define AMLM_SG_CHUNK_MAX 16
#endif
#ifndef AMLM_JOIN_UNROLL
#define AMLM_JOIN_UNROLL 8
#endif
constexpr int kBloomLog2Max = AMLM_BLOOM_LOG2_MAX;      // 32 Kbit (4 KB) filter: occupancy beats a lower false-positive rate
#ifndef AMLM_BLOOM_WORDS_MAX
#define AMLM_BLOOM_WORDS_MAX 960
#endif
// the largest filter, in 32-bit words: 960 (3840 bytes) rather than 1024
// keeps a k_sg wave's LDS within 6400 bytes, 24 waves per CU
constexpr uint32_t kBloomWordsMax = AMLM_BLOOM_WORDS_MAX < (1u << kBloomLog2Max) / 32 ? AMLM_BLOOM_WORDS_MAX
                                                                                       : (1u << kBloomLog2Max) / 32;
// filter bits per gathered entry, up to the maximum size: 128 gives short
// segments a sparse filter (fewer false positives to verify); 32 and 64 were
// slower, 256 and more no faster
constexpr uint32_t kBloomBitsPerEntry = AMLM_BLOOM_BITS_PER_ENTRY;
constexpr int kBloomK = AMLM_BLOOM_K;                   // bits set per key, all in one 32-bit word
#ifndef AMLM_GROUP_CAP
#define AMLM_GROUP_CAP 256
#endif
// segments of a k_sg chunk (runs of anchors into one vertex) share one filter
// and one flattened pass while their gather windows total at most this many
// entries (256: each keeps kBloomBitsPerEntry bits of the largest filter)
constexpr uint32_t kGroupCap = AMLM_GROUP_CAP;
constexpr int kJoinUnroll = AMLM_JOIN_UNROLL;
constexpr uint32_t kSgChunkMax = AMLM_SG_CHUNK_MAX;     // anchors per k_sg chunk (<= 64)
// default anchors per work unit: the static schedule's blocks of the list
// (8: its units of one hub then spread over more waves; 16 measured slower,
// k_sg 10.4 -> 11.5 ms) and the learned schedule's light blocks, whose heavy
// anchors are already sliced (16: k_sg 7.9 -> 7.5 ms on the 32M-edge graph)
constexpr uint32_t kStaticChunk = 8, kLearnedChunk = 16;
constexpr uint32_t kLongPair = 64;                      // slices scanned by the whole wave
#ifndef AMLM_REV_RATIO
#define AMLM_REV_RATIO 32
#endif
// a pair's join iterates the gather side when the sender's out-window is
// more than this many times longer
constexpr uint32_t kRevRatio = AMLM_REV_RATIO;
#ifndef AMLM_EAGER_NEED
#define AMLM_EAGER_NEED 0
#endif
// pairs that need at most this many intermediates besides u confirm their
// filter hits after every scan step (early exit), the others in batches of
// 64; 0 (batches only) was measured fastest: a check after every step puts
// a dependent search on each step's critical path (k_sg 11.0 -> 19.8 ms
// static on the 32M-edge graph)
constexpr uint32_t kEagerNeed = AMLM_EAGER_NEED;
#ifndef AMLM_EAGER_SHORT
#define AMLM_EAGER_SHORT 1
#endif
// eager checks also in the flattened short-pair loop (else long pairs only)
constexpr bool kEagerShort = AMLM_EAGER_SHORT != 0;

// phase-ordered scatter-gather keeps the k - 1 latest gather times of a
// sender's intervals in registers: k is at most this
constexpr uint32_t kPhaseKMax = 8;

#ifndef AMLM_CYC_EARLY
#define AMLM_CYC_EARLY 1
#endif
// 1: when a second stream is given, the cycle roots are found by a pass of
// their own and the cycle search starts on that stream before the anchor
// passes (static schedule: mining 15.27 -> 14.68 ms on the 32M-edge graph,
// the search no longer alone on the critical path; learned schedule
// unchanged, 12.17 ms: the anchor passes beside the search take as long as
// the search takes beside the cost model and the work units)
constexpr bool kCycEarly = AMLM_CYC_EARLY != 0;
constexpr int kCycThreads = 64;  // one wave per block: ~13 KB of LDS each
constexpr uint32_t kMaxDepth = 6;    // L <= 8: at most 6 path edges before the closing hop
constexpr uint32_t kCycSmallL = 6;   // cycle kernel built with fewer frames for L <= 6

constexpr uint32_t kFlagThreads = 256, kFlagItems = 16, kFlagTile = kFlagThreads * kFlagItems;

// device counter words
constexpr uint32_t kCtrSgWork = 0;
constexpr uint32_t kCtrCycWork = 1;
constexpr uint32_t kCtrNSg = 32, kCtrNCy = 33;
constexpr uint32_t kCtrSplitW = 34;   // 64-bit: sender-window entries of the splittable anchors
constexpr uint32_t kCtrNUnits = 36;   // scatter-gather work units
constexpr uint32_t kCtrWords = 64;

// Per-sub-graph parameters of a batched store (see batch.hip).
struct SubParams {
  int64_t delta;
  uint32_t L, k;
};

struct MineParams {
  GraphView g;
  int64_t delta;
  uint32_t L, k;          // L: the largest cycle length over all sub-graphs
  const uint32_t *vgraph; // batched store: sub-graph of each vertex (else NULL)
  const SubParams *sub;   // batched store: parameters per sub-graph
  uint32_t anchor_lo, anchor_hi;  // only edges with ids in [anchor_lo, anchor_hi) are anchors
  int col_fo, col_fi, col_sg, col_gs, col_cyc;  // -1 when not requested
  int col_do, col_di;    // distinct counterparties (after the cycle columns), -1 when not requested
  uint32_t sg_unordered;  // 1: an intermediate's two legs in either order
  uint32_t sg_phase;      // 1: every scatter leg before every gather leg (k <= kPhaseKMax)
  uint32_t cyc_any;       // 1: a cycle's edges in any order inside the window
  uint32_t *counts;
  uint64_t stride;   // row stride of counts (= number of edges)
  uint32_t ceil;     // every count saturates at this value (2^32 - 1 by default)
  // optional per-edge byte counters, rows of `stride` entries: kWorkIo,
  // kWorkSg, kWorkCyc the method's algorithmic bytes of each anchor (the
  // canonical procedure: see k_alg_sg and k_cyc), kWorkSgImpl the bytes the
  // scatter-gather kernel itself reads for it (the cost model's label)
  unsigned long long *work;
};
enum { kWorkIo = 0, kWorkSg = 1, kWorkCyc = 2, kWorkSgImpl = 3, kWorkRows = 4 };

struct MineScratch {
  uint8_t *flags = nullptr;   // [0, Ev): scatter-gather flag per CSC position;
                              // then the cycle-root flag per edge id [0, E)
  uint4 *sg_win = nullptr;    // per CSC position: senders window [p0, p1) in u's
                              // in-row and v's in-window [r0, r1)
  uint32_t *feat = nullptr;   // per CSC position: raw cost-model features [8]
  float *pred = nullptr;      // per list item: predicted log-work
  uint32_t *list_sg = nullptr, *list_cy = nullptr;
  uint32_t *bcnt_sg = nullptr, *bcnt_cy = nullptr, *boff_sg = nullptr, *boff_cy = nullptr;
  uint32_t *scan_tmp = nullptr;
  uint32_t *ctr = nullptr;
  // scatter-gather work units (see k_unit_fill): per list item its slice
  // count and unit count, their offsets, and the units
  uint32_t *nsub = nullptr, *ucnt = nullptr, *uoff = nullptr;
  uint2 *units = nullptr;
  uint64_t cap_ev = 0, cap_e = 0;
};

// Units: light blocks of at least kMinBlock items (smaller requests are
// raised), heavy slices bounded by the split rule; max_units() bounds both.
constexpr uint32_t kMinBlock = 4;
constexpr uint32_t kSplitMax = 64;   // an anchor is cut into at most this many slices
inline uint64_t max_units(uint64_t ev, uint32_t block) { return ev / block + ev / 16 + ev / 8 + 64; }
#ifndef AMLM_SPLIT_BYTES
#define AMLM_SPLIT_BYTES 32768
#endif
// learned schedule: predicted bytes per slice (32 KB: learned k_sg 6.83 ms
// at 64 KB, 6.59 at 32, 6.67 at 24 and 48, 6.98 at 16 on the 32M-edge graph)
constexpr uint32_t kSplitBytes = AMLM_SPLIT_BYTES;

// scatter-gather schedules: fixed blocks of the list (static), or heavy
// anchors cut into slices by an estimate of their work: the cost model
// (learned), the sender-window length times a constant fitted with the
// model (length), or per-edge costs given by the caller (given)
enum { kSchedStatic = 0, kSchedLearned = 1, kSchedLength = 2, kSchedGiven = 3 };

struct MineLaunch {
  uint32_t sg_blocks, sg_chunk, cyc_blocks, cyc_blocks_small;  // cycle grids for L > 6 and L <= 6
  uint32_t sched = kSchedStatic;
  float len_coef = 0.f;          // length schedule: bytes per sender-window entry
  const float *given = nullptr;  // given schedule: log1p(bytes) per edge id
  uint32_t learned_chunk = kLearnedChunk;  // anchors per chunk in the sliced schedules
  uint32_t split_bytes = kSplitBytes;    // learned schedule: predicted bytes per slice
  // optional second stream: the cycle kernel runs there, concurrently with
  // the cost model and work units (fork and join through the two events)
  hipStream_t aux = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  float delta_hours = 24.f;
};


// Optional HIP-event timing of the stages (recorded on the mining stream).
enum { kStBuild = 0, kStAnchor = 1, kStLists = 2, kStSg = 3, kStCyc = 4, kStModel = 5, kStUnits = 6, kStMine = 7, kNumStages = 8 };
struct StageTimer {
  bool on = false;
  hipEvent_t ev[2 * kNumStages] = {};
  bool used[kNumStages] = {};
  hipError_t begin(int st, hipStream_t s) { return on ? hipEventRecord(ev[2 * st], s) : hipSuccess; }
  hipError_t end(int st, hipStream_t s) {
    if (!on) return hipSuccess;
    used[st] = true;
    return hipEventRecord(ev[2 * st + 1], s);
  }
};

hipError_t mine_launch(const MineParams &mp, MineScratch &ms, const MineLaunch &cfg, hipStream_t s,
                       StageTimer *tm = nullptr);

// kernel handles for occupancy queries
const void *k_sg_ptr();
const void *k_cyc_ptr(bool small);  // small: the build for L <= kCycSmallL

// Bytes the scatter-gather kernel reads per unit of its own work, at the
// width of the fields it loads (its work counter, kWorkSgImpl: the cost
// model's training label):
constexpr uint32_t kBytesAnchorSg = 16;      // anchor (edge id, u, v, t)
constexpr uint32_t kBytesSenderEntry = 12;   // in-window of u: neighbour, next-same-pair time, time
constexpr uint32_t kBytesGatherEntry = 4;    // in-window of v: neighbour id
constexpr uint32_t kBytesJoinEntry = 4;      // out-window of a sender: neighbour id
constexpr uint32_t kBytesScatterEntry = 4;   // out-window of u after tau: previous-same-pair time
constexpr uint32_t kBytesRevEntry = 20;      // gather entry of the reverse join: neighbour, next time,
                                             // time, and the key found by the search
// The method's algorithmic bytes (kWorkIo .. kWorkCyc): an element of a
// scanned slice is a neighbour id and a time, 8 bytes, 12 in the cycle scan
// (plus the edge id it credits); an edge row is read as (src, dst, ts) and
// written as one count per column.
constexpr uint32_t kAlgEdgeRow = 12, kAlgCount = 4, kAlgElem = 8, kAlgCycElem = 12, kAlgCycleEdge = 8;

// Window, cycle length and threshold of the (sub-)graph that vertex x belongs to.
__device__ __forceinline__ int64_t delta_of(const MineParams &mp, uint32_t x) {
  return mp.vgraph ? mp.sub[mp.vgraph[x]].delta : mp.delta;
}
__device__ __forceinline__ uint32_t L_of(const MineParams &mp, uint32_t x) {
  return mp.vgraph ? mp.sub[mp.vgraph[x]].L : mp.L;
}
__device__ __forceinline__ uint32_t k_of(const MineParams &mp, uint32_t x) {
  return mp.vgraph ? mp.sub[mp.vgraph[x]].k : mp.k;
}
