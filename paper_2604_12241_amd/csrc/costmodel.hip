// Learned cost model: MLP forward / backward / Adam kernels, training loop,
// inference for the scheduler, and save / load.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <random>
#include <vector>

#include "api_internal.h"
#include "costmodel.h"

uint16_t f32_to_bf16(float f) {
  uint32_t u;
  memcpy(&u, &f, 4);
  uint32_t lsb = (u >> 16) & 1u;
  u += 0x7fffu + lsb;  // round to nearest, ties to even
  return (uint16_t)(u >> 16);
}
float bf16_to_f32(uint16_t h) {
  uint32_t u = (uint32_t)h << 16;
  float f;
  memcpy(&f, &u, 4);
  return f;
}

MlpModel &global_model() {
  static MlpModel m;
  return m;
}

namespace {

__device__ __forceinline__ float dbf16(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ uint16_t d_f32_to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// network input from the raw counts (log1p, then standardisation)
__device__ __forceinline__ void mlp_input(const uint32_t *r, float dh, float L, const float *norm, float *x) {
#pragma unroll
  for (int i = 0; i < kMlpRaw; i++) x[i] = log1pf((float)r[i]);
  x[8] = log1pf((float)r[2] * (float)r[1]);
  x[9] = log1pf((float)r[2] * (float)r[3]);
  x[10] = log1pf(dh);
  x[11] = log1pf(L);
#pragma unroll
  for (int i = 0; i < kMlpF; i++) x[i] = (x[i] - norm[i]) * norm[kMlpF + i];
}

// Forward pass of one sample with the weights in LDS (FP32 copies of the
// BF16 values).  Returns the output; h1 is left in registers by the caller.
__device__ __forceinline__ float mlp_forward(const float *W, const float *x, float *h1) {
#pragma unroll
  for (int j = 0; j < kMlpH; j++) {
    float a = W[kOffB1 + j];
#pragma unroll
    for (int f = 0; f < kMlpF; f++) a = fmaf(W[kOffW1 + j * kMlpF + f], x[f], a);
    h1[j] = a > 0.f ? a : 0.f;
  }
  float y = W[kOffB3];
  for (int j = 0; j < kMlpH; j++) {
    float a = W[kOffB2 + j];
#pragma unroll
    for (int i = 0; i < kMlpH; i++) a = fmaf(W[kOffW2 + j * kMlpH + i], h1[i], a);
    y = fmaf(W[kOffW3 + j], a > 0.f ? a : 0.f, y);
  }
  return y;
}

// ---- MFMA inference: 16 anchors per v_mfma_f32_16x16x32_bf16 tile ----
// Operand layout of gfx950's 16x16x32 BF16 MFMA (64 lanes, l = lane):
//   A (16 x 32, M x K): lane l holds row l % 16, k = 8 (l / 16) + 0..7
//   B (32 x 16, K x N): lane l holds col l % 16, k = 8 (l / 16) + 0..7
//   C (16 x 16):        lane l holds col l % 16, rows 4 (l / 16) + 0..3
// The three layers are dense products [16 x K] x [K x 64] (K = 32 with the
// 12 inputs zero-padded, then 64 as two K-steps, then 64 x 16 with w3 in
// column 0); every weight operand stays in registers, and the activations
// go through a 16 x 64 BF16 tile in LDS to move from the C layout to the A
// layout.
typedef short shortx8_t __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float floatx4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ short bf16_bits(float f) { return (short)d_f32_to_bf16(f); }

__device__ __forceinline__ floatx4_t mfma_bf16(const shortx8_t &a, const shortx8_t &b, floatx4_t c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8_t, a), __builtin_bit_cast(bf16x8_t, b), c,
                                                 0, 0, 0);
}

constexpr int kTileRows = 16;
constexpr int kActPad = kMlpH + 8;  // bf16 per LDS row (pad against bank conflicts)
constexpr int kKStep = 32;          // K of one MFMA
constexpr int kKSteps = kMlpH / kKStep;

template <bool kFromRaw>
__global__ __launch_bounds__(256) void k_mlp_mfma(const uint16_t *w16, const float *norm, const uint32_t *feat,
                                                  const uint32_t *idx, const float *X, const uint32_t *n_p,
                                                  uint32_t n_host, float dh, float L, float *pred,
                                                  const uint32_t *in_dst, const uint32_t *vgraph,
                                                  const SubParams *sub) {
  __shared__ short act[256 / AMLM_WAVE][kTileRows][kActPad];
  const uint32_t lane = lane_id(), w = threadIdx.x / AMLM_WAVE;
  const uint32_t col = lane % 16, kq = (lane / 16) * 8, rq = (lane / 16) * 4;
  // weights as B operands, in registers
  shortx8_t B1[4], B2[kKSteps][4], B3[kKSteps];
  float bias1[4], bias2[4];
#pragma unroll
  for (int nt = 0; nt < 4; nt++) {
    uint32_t n = nt * 16 + col;
#pragma unroll
    for (int i = 0; i < 8; i++) {
      uint32_t k = kq + i;
      B1[nt][i] = k < kMlpF ? (short)w16[kOffW1 + n * kMlpF + k] : (short)0;
    }
    bias1[nt] = dbf16(w16[kOffB1 + n]);
    bias2[nt] = dbf16(w16[kOffB2 + n]);
#pragma unroll
    for (int kt = 0; kt < kKSteps; kt++)
#pragma unroll
      for (int i = 0; i < 8; i++) B2[kt][nt][i] = (short)w16[kOffW2 + n * kMlpH + kt * kKStep + kq + i];
  }
#pragma unroll
  for (int kt = 0; kt < kKSteps; kt++)
#pragma unroll
    for (int i = 0; i < 8; i++) B3[kt][i] = col == 0 ? (short)w16[kOffW3 + kt * kKStep + kq + i] : (short)0;
  const float b3 = dbf16(w16[kOffB3]);
  float nrm[2 * kMlpF];
#pragma unroll
  for (int i = 0; i < 2 * kMlpF; i++) nrm[i] = kFromRaw ? norm[i] : 0.f;
  const uint32_t n = n_p ? *n_p : n_host;
  const uint32_t n_tiles = (n + kTileRows - 1) / kTileRows;
  const uint32_t wave_id = blockIdx.x * (256 / AMLM_WAVE) + w, n_waves = gridDim.x * (256 / AMLM_WAVE);
  for (uint32_t tile = wave_id; tile < n_tiles; tile += n_waves) {
    const uint32_t row = lane % 16;
    const uint32_t item = tile * kTileRows + row;
    const bool valid = item < n;
    // A operand of layer 1: this lane's eight inputs of its row (k >= 12: 0)
    float x[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if (valid && kq < (uint32_t)kMlpF) {
      if (kFromRaw) {
        uint32_t r[kMlpRaw];
        uint64_t rr = idx ? idx[item] : item;
#pragma unroll
        for (int q = 0; q < kMlpRaw; q++) r[q] = feat[rr * kMlpRaw + q];
        float xf[kMlpF];
        float dh_i = dh, L_i = L;
        if (vgraph) {  // batched store: the item's own sub-graph
          const SubParams sp = sub[vgraph[in_dst[rr]]];
          dh_i = (float)sp.delta / 3600.f;
          L_i = (float)sp.L;
        }
        mlp_input(r, dh_i, L_i, nrm, xf);
#pragma unroll
        for (int i = 0; i < 8; i++) x[i] = kq + i < kMlpF ? xf[kq + i] : 0.f;
      } else {
#pragma unroll
        for (int i = 0; i < 8; i++) x[i] = kq + i < kMlpF ? X[(uint64_t)item * kMlpF + kq + i] : 0.f;
      }
    }
    shortx8_t a1;
#pragma unroll
    for (int i = 0; i < 8; i++) a1[i] = bf16_bits(x[i]);
    // layer 1 -> act (bf16, relu)
#pragma unroll
    for (int nt = 0; nt < 4; nt++) {
      floatx4_t c = {0.f, 0.f, 0.f, 0.f};
      c = mfma_bf16(a1, B1[nt], c);
#pragma unroll
      for (int i = 0; i < 4; i++) {
        float h = c[i] + bias1[nt];
        act[w][rq + i][nt * 16 + col] = bf16_bits(h > 0.f ? h : 0.f);
      }
    }
    __builtin_amdgcn_s_waitcnt(0);
    __builtin_amdgcn_wave_barrier();
    // layer 2
    shortx8_t a2[kKSteps];
#pragma unroll
    for (int kt = 0; kt < kKSteps; kt++)
#pragma unroll
      for (int i = 0; i < 8; i++) a2[kt][i] = act[w][row][kt * kKStep + kq + i];
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int nt = 0; nt < 4; nt++) {
      floatx4_t c = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int kt = 0; kt < kKSteps; kt++) c = mfma_bf16(a2[kt], B2[kt][nt], c);
#pragma unroll
      for (int i = 0; i < 4; i++) {
        float h = c[i] + bias2[nt];
        act[w][rq + i][nt * 16 + col] = bf16_bits(h > 0.f ? h : 0.f);
      }
    }
    __builtin_amdgcn_s_waitcnt(0);
    __builtin_amdgcn_wave_barrier();
    // layer 3 (w3 in column 0)
    shortx8_t a3[kKSteps];
#pragma unroll
    for (int kt = 0; kt < kKSteps; kt++)
#pragma unroll
      for (int i = 0; i < 8; i++) a3[kt][i] = act[w][row][kt * kKStep + kq + i];
    __builtin_amdgcn_wave_barrier();
    floatx4_t c = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kt = 0; kt < kKSteps; kt++) c = mfma_bf16(a3[kt], B3[kt], c);
    if (col == 0) {
#pragma unroll
      for (int i = 0; i < 4; i++) {
        uint32_t it = tile * kTileRows + rq + i;
        if (it < n) pred[it] = c[i] + b3;
      }
    }
  }
}

// Forward pass on standardised inputs X[n][12].
__global__ __launch_bounds__(256) void k_mlp_fwd_x(const uint16_t *w16, const float *X, uint32_t n, float *y) {
  __shared__ float W[kMlpParams];
  for (int p = threadIdx.x; p < kMlpParams; p += blockDim.x) W[p] = dbf16(w16[p]);
  __syncthreads();
  uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float x[kMlpF], h1[kMlpH];
#pragma unroll
  for (int f = 0; f < kMlpF; f++) x[f] = X[(uint64_t)i * kMlpF + f];
  y[i] = mlp_forward(W, x, h1);
}

// Raw inputs -> standardised FP32 inputs (training samples).
__global__ void k_mlp_inputs(const uint32_t *feat, uint32_t n, float dh, float L, const float *norm, float *X) {
  uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint32_t r[kMlpRaw];
#pragma unroll
  for (int q = 0; q < kMlpRaw; q++) r[q] = feat[(uint64_t)i * kMlpRaw + q];
  float x[kMlpF];
  mlp_input(r, dh, L, norm, x);
#pragma unroll
  for (int f = 0; f < kMlpF; f++) X[(uint64_t)i * kMlpF + f] = x[f];
}

// Forward + backward of 64 samples (one per lane) of a minibatch, with the
// per-parameter sums over the 64 samples taken in a fixed order; writes this
// block's partial gradient of  sum_s scale * (y_s - t_s)^2 / 2 * 2 ... i.e.
// scale * (y_s - t_s) * dy_s/dtheta summed over s.
constexpr int kPad = kMlpH + 1;
__global__ __launch_bounds__(64) void k_mlp_grad(const uint16_t *w16, const float *X, const float *Y, uint32_t n,
                                                 const uint32_t *order, uint32_t base, uint32_t count, float scale,
                                                 float *partial, float *loss_partial) {
  __shared__ float W[kMlpParams];
  __shared__ float H1[AMLM_WAVE][kPad];   // h1, later dL/dh1
  __shared__ float H2[AMLM_WAVE][kPad];   // h2, later dL/dh2
  __shared__ float Xs[AMLM_WAVE][kMlpF + 1];
  __shared__ float Dy[AMLM_WAVE];
  const uint32_t s = threadIdx.x;
  for (int p = s; p < kMlpParams; p += AMLM_WAVE) W[p] = dbf16(w16[p]);
  const uint32_t slot = blockIdx.x * AMLM_WAVE + s;
  const bool valid = slot < count;
  uint32_t idx = 0;
  if (valid) idx = order ? order[base + slot] : base + slot;
  __syncthreads();
  float x[kMlpF];
#pragma unroll
  for (int f = 0; f < kMlpF; f++) {
    x[f] = valid ? X[(uint64_t)idx * kMlpF + f] : 0.f;
    Xs[s][f] = x[f];
  }
  float h1[kMlpH];
#pragma unroll
  for (int j = 0; j < kMlpH; j++) {
    float a = W[kOffB1 + j];
#pragma unroll
    for (int f = 0; f < kMlpF; f++) a = fmaf(W[kOffW1 + j * kMlpF + f], x[f], a);
    h1[j] = a > 0.f ? a : 0.f;
    H1[s][j] = h1[j];
  }
  float y = W[kOffB3];
  for (int j = 0; j < kMlpH; j++) {
    float a = W[kOffB2 + j];
#pragma unroll
    for (int i = 0; i < kMlpH; i++) a = fmaf(W[kOffW2 + j * kMlpH + i], h1[i], a);
    float h2 = a > 0.f ? a : 0.f;
    H2[s][j] = h2;
    y = fmaf(W[kOffW3 + j], h2, y);
  }
  float err = valid ? (y - Y[idx]) : 0.f;
  Dy[s] = scale * err;  // dL/dy for L = scale/2 * sum (y - t)^2
  __syncthreads();
  float *out = partial + (uint64_t)blockIdx.x * kMlpParams;
  // layer 3
  {
    float g = 0.f;
    for (int q = 0; q < AMLM_WAVE; q++) g = fmaf(Dy[q], H2[q][s], g);
    out[kOffW3 + s] = g;
    if (s == 0) {
      float gb = 0.f, l = 0.f;
      for (int q = 0; q < AMLM_WAVE; q++) gb += Dy[q];
      out[kOffB3] = gb;
      (void)l;
    }
  }
  __syncthreads();
  // dL/dh2 (masked by the ReLU), in place of h2
  {
    float d = Dy[s];
    for (int j = 0; j < kMlpH; j++) H2[s][j] = H2[s][j] > 0.f ? d * W[kOffW3 + j] : 0.f;
  }
  __syncthreads();
  // layer 2: row j = s of W2
  {
    float gb = 0.f;
    for (int q = 0; q < AMLM_WAVE; q++) gb += H2[q][s];
    out[kOffB2 + s] = gb;
    for (int i = 0; i < kMlpH; i++) {
      float g = 0.f;
      for (int q = 0; q < AMLM_WAVE; q++) g = fmaf(H2[q][s], H1[q][i], g);
      out[kOffW2 + s * kMlpH + i] = g;
    }
  }
  // dL/dh1 of this sample (masked), in registers
  float d1[kMlpH];
#pragma unroll
  for (int i = 0; i < kMlpH; i++) d1[i] = 0.f;
  for (int j = 0; j < kMlpH; j++) {
    float dj = H2[s][j];
#pragma unroll
    for (int i = 0; i < kMlpH; i++) d1[i] = fmaf(W[kOffW2 + j * kMlpH + i], dj, d1[i]);
  }
  __syncthreads();  // every lane has finished reading H1 for the W2 gradient
#pragma unroll
  for (int i = 0; i < kMlpH; i++) H1[s][i] = h1[i] > 0.f ? d1[i] : 0.f;
  __syncthreads();
  // layer 1: row j = s of W1
  {
    float gb = 0.f;
    for (int q = 0; q < AMLM_WAVE; q++) gb += H1[q][s];
    out[kOffB1 + s] = gb;
    for (int f = 0; f < kMlpF; f++) {
      float g = 0.f;
      for (int q = 0; q < AMLM_WAVE; q++) g = fmaf(H1[q][s], Xs[q][f], g);
      out[kOffW1 + s * kMlpF + f] = g;
    }
  }
  if (loss_partial) {
    // fixed-order sum of the squared errors of the block
    Dy[s] = err * err;
    __syncthreads();
    if (s == 0) {
      float l = 0.f;
      for (int q = 0; q < AMLM_WAVE; q++) l += Dy[q];
      loss_partial[blockIdx.x] = l;
    }
  }
}

__global__ void k_mlp_reduce(const float *partial, uint32_t nblk, float *grad) {
  uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= kMlpParams) return;
  float g = 0.f;
  for (uint32_t b = 0; b < nblk; b++) g += partial[(uint64_t)b * kMlpParams + p];
  grad[p] = g;
}

__global__ void k_adam(float *master, float *m, float *v, const float *grad, uint16_t *w16, float lr, float b1,
                       float b2, float eps, float c1, float c2) {
  uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= kMlpParams) return;
  float g = grad[p];
  float mm = b1 * m[p] + (1.f - b1) * g;
  float vv = b2 * v[p] + (1.f - b2) * g * g;
  m[p] = mm;
  v[p] = vv;
  float w = master[p] - lr * (mm / c1) / (sqrtf(vv / c2) + eps);
  master[p] = w;
  w16[p] = d_f32_to_bf16(w);
}

// raw features of every anchor (time order) + its scatter-gather label
// (work: the scatter-gather kernel's own bytes per edge id, kWorkSgImpl row)
__global__ void k_sample_features(GraphView g, int64_t delta, const unsigned long long *work, uint32_t *feat,
                                  float *label, uint32_t *keep) {
  uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= g.Ev) return;
  uint32_t eid = g.anc[p];
  uint32_t u = g.src[eid], v = g.dst[eid];
  int32_t t = g.t[eid];
  int64_t lo64 = (int64_t)t - delta;
  int32_t lo = lo64 < -1 ? -1 : (int32_t)lo64;
  uint32_t r[kMlpRaw];
  uint32_t ors = g.out_ptr[u], ore = g.out_ptr[u + 1], irs = g.in_ptr[v], ire = g.in_ptr[v + 1];
  uint32_t pu = g.pos_out[eid], pv = g.pos_in[eid];
  r[0] = upper_bound_i32(g.out_t, pu + 1, ore, t) - lower_bound_i32(g.out_t, ors, pu, lo);
  r[1] = upper_bound_i32(g.in_t, pv + 1, ire, t) - lower_bound_i32(g.in_t, irs, pv, lo);
  uint32_t cs = g.in_ptr[u], ce = g.in_ptr[u + 1];
  uint32_t p0 = lower_bound_i32(g.in_t, cs, ce, lo);
  r[2] = lower_bound_i32(g.in_t, p0, ce, t) - p0;
  uint32_t vs = g.out_ptr[v], ve = g.out_ptr[v + 1];
  uint32_t q0 = lower_bound_i32(g.out_t, vs, ve, lo);
  r[3] = lower_bound_i32(g.out_t, q0, ve, t) - q0;
  r[4] = ore - ors;
  r[5] = ce - cs;
  r[6] = ve - vs;
  r[7] = ire - irs;
#pragma unroll
  for (int q = 0; q < kMlpRaw; q++) feat[(uint64_t)p * kMlpRaw + q] = r[q];
  const unsigned long long w = work[eid];
  label[p] = log1pf((float)w);
  keep[p] = w > 0;
}

__global__ void k_gather_samples(const uint32_t *keep_list, uint32_t n, const uint32_t *feat_in, const float *lab_in,
                                 uint32_t *feat_out, float *lab_out, uint32_t out_base) {
  uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint32_t p = keep_list[i];
#pragma unroll
  for (int q = 0; q < kMlpRaw; q++) feat_out[(uint64_t)(out_base + i) * kMlpRaw + q] = feat_in[(uint64_t)p * kMlpRaw + q];
  lab_out[out_base + i] = lab_in[p];
}

__global__ void k_compact_keep(const uint32_t *keep, const uint32_t *off, uint32_t n, uint32_t *list) {
  uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  if (keep[p]) list[off[p]] = p;
}

// Per-block partial sums (fixed order) of log(bytes) - log(sender-window
// length) over samples with a non-empty sender window, and their count: the
// length rule's constant is exp(mean).
__global__ void k_len_moments(const uint32_t *feat, const float *label, uint32_t n, double *part) {
  __shared__ double acc[256][2];
  double s = 0.0, c = 0.0;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const uint32_t w = feat[(uint64_t)i * kMlpRaw + 2];
    const double by = expm1((double)label[i]);
    if (w < 2 || by <= 0.0) continue;  // anchors the split rule never cuts
    s += log(by) - log((double)w);
    c += 1.0;
  }
  acc[threadIdx.x][0] = s;
  acc[threadIdx.x][1] = c;
  __syncthreads();
  if (threadIdx.x < 2) {
    double t = 0.0;
    for (int q = 0; q < (int)blockDim.x; q++) t += acc[q][threadIdx.x];
    part[blockIdx.x * 2 + threadIdx.x] = t;
  }
}

// Per-block partial sums (fixed order) of the unstandardised inputs and their
// squares, for the normalisation statistics.
__global__ void k_input_moments(const uint32_t *feat, uint32_t n, float dh, float L, double *part) {
  __shared__ double acc[256][2 * kMlpF];
  const float zero[2 * kMlpF] = {};
  double s[2 * kMlpF];
  for (int f = 0; f < 2 * kMlpF; f++) s[f] = 0.0;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    uint32_t r[kMlpRaw];
    for (int q = 0; q < kMlpRaw; q++) r[q] = feat[(uint64_t)i * kMlpRaw + q];
    float x[kMlpF];
    float id[2 * kMlpF];
    for (int f = 0; f < kMlpF; f++) {
      id[f] = 0.f;
      id[kMlpF + f] = 1.f;
    }
    mlp_input(r, dh, L, id, x);
    for (int f = 0; f < kMlpF; f++) {
      s[f] += x[f];
      s[kMlpF + f] += (double)x[f] * x[f];
    }
  }
  (void)zero;
  for (int f = 0; f < 2 * kMlpF; f++) acc[threadIdx.x][f] = s[f];
  __syncthreads();
  if (threadIdx.x < 2 * kMlpF) {
    double t = 0.0;
    for (int q = 0; q < (int)blockDim.x; q++) t += acc[q][threadIdx.x];
    part[blockIdx.x * 2 * kMlpF + threadIdx.x] = t;
  }
}

}  // namespace

// ====================================================================== host

hipError_t model_upload(MlpModel &m) {
  hipError_t e;
  if (!m.d_w16) {
    if ((e = hipMalloc(&m.d_w16, 2 * kMlpParams)) != hipSuccess) return e;
    if ((e = hipMalloc(&m.d_norm, 4 * 2 * kMlpF)) != hipSuccess) return e;
  }
  std::vector<uint16_t> w(kMlpParams);
  for (int p = 0; p < kMlpParams; p++) w[p] = f32_to_bf16(m.master[p]);
  float nrm[2 * kMlpF];
  for (int f = 0; f < kMlpF; f++) {
    nrm[f] = m.mean[f];
    nrm[kMlpF + f] = m.inv_std[f];
  }
  if ((e = hipMemcpy(m.d_w16, w.data(), 2 * kMlpParams, hipMemcpyHostToDevice)) != hipSuccess) return e;
  return hipMemcpy(m.d_norm, nrm, sizeof(nrm), hipMemcpyHostToDevice);
}

#ifndef AMLM_MLP_INFER_BPC
#define AMLM_MLP_INFER_BPC 2
#endif
// inference blocks per CU: the kernel runs beside the cycle search, which
// needs the rest of the chip
constexpr uint32_t kMlpInferBlocksPerCu = AMLM_MLP_INFER_BPC;

hipError_t mlp_infer(const MlpModel &m, const uint32_t *feat, const uint32_t *idx, uint32_t n_host,
                     const uint32_t *n_dev, float delta_hours, float L, float *pred, hipStream_t s,
                     const uint32_t *in_dst, const uint32_t *vgraph, const SubParams *sub) {
  uint32_t blocks = kMlpInferBlocksPerCu * device_info().num_cu;
  hipLaunchKernelGGL(k_mlp_mfma<true>, dim3(blocks), dim3(256), 0, s, m.d_w16, m.d_norm, feat, idx,
                     (const float *)nullptr, n_dev, n_host, delta_hours, L, pred, in_dst, vgraph, sub);
  return hipGetLastError();
}

static void init_weights(float *w, uint64_t seed) {
  std::mt19937_64 rng(seed);
  auto uni = [&](float a) { return (float)((double)(rng() >> 11) * 0x1.0p-53 * 2.0 - 1.0) * a; };
  for (int i = 0; i < kMlpH * kMlpF; i++) w[kOffW1 + i] = uni(std::sqrt(6.f / kMlpF));
  for (int i = 0; i < kMlpH; i++) w[kOffB1 + i] = 0.f;
  for (int i = 0; i < kMlpH * kMlpH; i++) w[kOffW2 + i] = uni(std::sqrt(6.f / kMlpH));
  for (int i = 0; i < kMlpH; i++) w[kOffB2 + i] = 0.f;
  for (int i = 0; i < kMlpH; i++) w[kOffW3 + i] = uni(std::sqrt(3.f / kMlpH));
  w[kOffB3] = 0.f;
}

#define A_TRY(x)                    \
  do {                              \
    amlm_status st_ = (x);          \
    if (st_ != AMLM_OK) return st_; \
  } while (0)

struct DevBuf {
  std::vector<void *> ptrs;
  ~DevBuf() {
    for (void *p : ptrs) (void)hipFree(p);
  }
  template <class T>
  amlm_status get(T **p, size_t count) {
    if (hipMalloc((void **)p, sizeof(T) * (count ? count : 1)) != hipSuccess) {
      (void)hipGetLastError();
      set_error("cost model: device allocation failed");
      return AMLM_E_NOMEM;
    }
    ptrs.push_back(*p);
    return AMLM_OK;
  }
};

// Gradient of  (1/n) sum_s (y_s - t_s)^2 / 2  ... scaled so that it equals
// d/dtheta of  mean_s (y_s - t_s)^2  (scale = 2 / n), summed over blocks.
static amlm_status device_grad(const uint16_t *w16, const float *X, const float *Y, uint32_t n, const uint32_t *order,
                               uint32_t base, uint32_t count, float scale, float *partial, float *grad, float *lossp,
                               hipStream_t s) {
  uint32_t nblk = (count + AMLM_WAVE - 1) / AMLM_WAVE;
  hipLaunchKernelGGL(k_mlp_grad, dim3(nblk), dim3(AMLM_WAVE), 0, s, w16, X, Y, n, order, base, count, scale, partial,
                     lossp);
  HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_mlp_reduce, dim3((kMlpParams + 255) / 256), dim3(256), 0, s, partial, nblk, grad);
  HIP_TRY(hipGetLastError());
  return AMLM_OK;
}

extern "C" amlm_status amlm_mlp_grad(const float *w_host, const float *x_host, const float *y_host, uint32_t n,
                                     float *grad_host, float *loss_host) {
  if (!w_host || (n && (!x_host || !y_host)) || !grad_host) {
    set_error("null argument");
    return AMLM_E_INVALID;
  }
  DevBuf b;
  uint16_t *w16;
  float *X, *Y, *partial, *grad, *lossp;
  uint32_t nblk = std::max(1u, (n + AMLM_WAVE - 1) / AMLM_WAVE);
  A_TRY(b.get(&w16, kMlpParams));
  A_TRY(b.get(&X, (size_t)n * kMlpF));
  A_TRY(b.get(&Y, n));
  A_TRY(b.get(&partial, (size_t)nblk * kMlpParams));
  A_TRY(b.get(&grad, kMlpParams));
  A_TRY(b.get(&lossp, nblk));
  std::vector<uint16_t> w(kMlpParams);
  for (int p = 0; p < kMlpParams; p++) w[p] = f32_to_bf16(w_host[p]);
  HIP_TRY(hipMemcpy(w16, w.data(), 2 * kMlpParams, hipMemcpyHostToDevice));
  if (n) {
    HIP_TRY(hipMemcpy(X, x_host, 4ull * n * kMlpF, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(Y, y_host, 4ull * n, hipMemcpyHostToDevice));
  }
  A_TRY(device_grad(w16, X, Y, n, nullptr, 0, n, n ? 2.f / (float)n : 0.f, partial, grad, lossp, 0));
  HIP_TRY(hipMemcpy(grad_host, grad, 4 * kMlpParams, hipMemcpyDeviceToHost));
  if (loss_host) {
    std::vector<float> lp(nblk);
    HIP_TRY(hipMemcpy(lp.data(), lossp, 4ull * nblk, hipMemcpyDeviceToHost));
    double l = 0;
    for (float v : lp) l += v;
    *loss_host = n ? (float)(l / n) : 0.f;
  }
  return AMLM_OK;
}

extern "C" amlm_status amlm_mlp_forward(const float *w_host, const float *x_host, uint32_t n, float *y_host) {
  if (!w_host || (n && (!x_host || !y_host))) {
    set_error("null argument");
    return AMLM_E_INVALID;
  }
  if (n == 0) return AMLM_OK;
  DevBuf b;
  uint16_t *w16;
  float *X, *Y;
  A_TRY(b.get(&w16, kMlpParams));
  A_TRY(b.get(&X, (size_t)n * kMlpF));
  A_TRY(b.get(&Y, n));
  std::vector<uint16_t> w(kMlpParams);
  for (int p = 0; p < kMlpParams; p++) w[p] = f32_to_bf16(w_host[p]);
  HIP_TRY(hipMemcpy(w16, w.data(), 2 * kMlpParams, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(X, x_host, 4ull * n * kMlpF, hipMemcpyHostToDevice));
  hipLaunchKernelGGL(k_mlp_fwd_x, dim3((n + 255) / 256), dim3(256), 0, 0, w16, X, n, Y);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpy(y_host, Y, 4ull * n, hipMemcpyDeviceToHost));
  return AMLM_OK;
}

extern "C" amlm_status amlm_mlp_predict(const float *w_host, const float *x_host, uint32_t n, float *y_host) {
  if (!w_host || (n && (!x_host || !y_host))) {
    set_error("null argument");
    return AMLM_E_INVALID;
  }
  if (n == 0) return AMLM_OK;
  DevBuf b;
  uint16_t *w16;
  float *X, *Y;
  A_TRY(b.get(&w16, kMlpParams));
  A_TRY(b.get(&X, (size_t)n * kMlpF));
  A_TRY(b.get(&Y, n));
  std::vector<uint16_t> w(kMlpParams);
  for (int p = 0; p < kMlpParams; p++) w[p] = f32_to_bf16(w_host[p]);
  HIP_TRY(hipMemcpy(w16, w.data(), 2 * kMlpParams, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(X, x_host, 4ull * n * kMlpF, hipMemcpyHostToDevice));
  hipLaunchKernelGGL(k_mlp_mfma<false>, dim3(std::max(1u, std::min(1024u, (n + 63) / 64))), dim3(256), 0, 0, w16,
                     (const float *)nullptr, (const uint32_t *)nullptr, (const uint32_t *)nullptr, X,
                     (const uint32_t *)nullptr, n, 0.f, 0.f, Y, (const uint32_t *)nullptr,
                     (const uint32_t *)nullptr, (const SubParams *)nullptr);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpy(y_host, Y, 4ull * n, hipMemcpyDeviceToHost));
  return AMLM_OK;
}

extern "C" amlm_status amlm_costmodel_train(amlm_graph *const *gs, const amlm_params *ps, uint32_t n_graphs,
                                            uint32_t epochs, uint32_t batch, uint64_t seed, const char *out_path,
                                            void *hip_stream) {
  if (!gs || !ps || n_graphs == 0) {
    set_error("no training graphs");
    return AMLM_E_INVALID;
  }
  hipStream_t s = (hipStream_t)hip_stream;
  if (epochs == 0) epochs = 4;
  if (batch == 0) batch = 4096;
  batch = (batch + AMLM_WAVE - 1) / AMLM_WAVE * AMLM_WAVE;
  const float dh = (float)ps[0].delta / 3600.f;
  const float Lf = (float)((ps[0].patterns & AMLM_CYCLES) ? ps[0].max_cycle_len : 2);
  // 1. labels from the plain miner's work counters, features per anchor
  uint64_t total = 0;
  for (uint32_t i = 0; i < n_graphs; i++) total += gs[i]->Ev;
  DevBuf b;
  uint32_t *feat_all, *keep, *koff, *klist, *cnt_dev;
  float *lab_all;
  uint64_t cap = 0;
  for (uint32_t i = 0; i < n_graphs; i++) cap = std::max<uint64_t>(cap, gs[i]->E);
  uint32_t *fs, *ctmp;
  unsigned long long *wk;
  float *ls;
  A_TRY(b.get(&feat_all, total * kMlpRaw));
  A_TRY(b.get(&lab_all, total));
  A_TRY(b.get(&fs, cap * kMlpRaw));
  A_TRY(b.get(&ls, cap));
  A_TRY(b.get(&keep, cap));
  A_TRY(b.get(&koff, cap));
  A_TRY(b.get(&klist, cap));
  A_TRY(b.get(&cnt_dev, 4));
  A_TRY(b.get(&wk, kWorkRows * cap));
  uint32_t ncol_max = 16;
  A_TRY(b.get(&ctmp, cap * ncol_max));
  uint32_t *scan_tmp;
  A_TRY(b.get(&scan_tmp, scan_tmp_words(cap)));
  uint32_t n_samples = 0;
  for (uint32_t i = 0; i < n_graphs; i++) {
    amlm_graph *g = gs[i];
    A_TRY(mine_common(g, &ps[i], ctmp, wk, s));
    if (g->Ev == 0) continue;
    hipLaunchKernelGGL(k_sample_features, dim3((g->Ev + 255) / 256), dim3(256), 0, s, graph_view(g), ps[i].delta,
                       (const unsigned long long *)(wk + kWorkSgImpl * g->E), fs, ls, keep);
    HIP_TRY(hipGetLastError());
    HIP_TRY(scan_exclusive_u32(keep, koff, g->Ev, cnt_dev, scan_tmp, s));
    hipLaunchKernelGGL(k_compact_keep, dim3((g->Ev + 255) / 256), dim3(256), 0, s, keep, koff, g->Ev, klist);
    HIP_TRY(hipGetLastError());
    uint32_t nk = 0;
    HIP_TRY(hipMemcpyAsync(&nk, cnt_dev, 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (nk) {
      hipLaunchKernelGGL(k_gather_samples, dim3((nk + 255) / 256), dim3(256), 0, s, klist, nk, fs, ls, feat_all,
                         lab_all, n_samples);
      HIP_TRY(hipGetLastError());
    }
    n_samples += nk;
  }
  if (n_samples < AMLM_WAVE) {
    set_error("too few training samples");
    return AMLM_E_INVALID;
  }
  // 2. input standardisation from fixed-order partial sums
  MlpModel &m = global_model();
  const uint32_t mblk = 256;
  double *mpart;
  A_TRY(b.get(&mpart, (size_t)mblk * 2 * kMlpF));
  hipLaunchKernelGGL(k_input_moments, dim3(mblk), dim3(256), 0, s, feat_all, n_samples, dh, Lf, mpart);
  HIP_TRY(hipGetLastError());
  std::vector<double> mp((size_t)mblk * 2 * kMlpF);
  HIP_TRY(hipMemcpyAsync(mp.data(), mpart, 8 * mp.size(), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  for (int f = 0; f < kMlpF; f++) {
    double s1 = 0, s2 = 0;
    for (uint32_t q = 0; q < mblk; q++) {
      s1 += mp[q * 2 * kMlpF + f];
      s2 += mp[q * 2 * kMlpF + kMlpF + f];
    }
    double mean = s1 / n_samples, var = s2 / n_samples - mean * mean;
    m.mean[f] = (float)mean;
    m.inv_std[f] = var > 1e-12 ? (float)(1.0 / std::sqrt(var)) : 1.f;
  }
  {
    // the length rule on the same labels
    double *lpart;
    A_TRY(b.get(&lpart, (size_t)mblk * 2));
    hipLaunchKernelGGL(k_len_moments, dim3(mblk), dim3(256), 0, s, feat_all, lab_all, n_samples, lpart);
    HIP_TRY(hipGetLastError());
    std::vector<double> lp((size_t)mblk * 2);
    HIP_TRY(hipMemcpyAsync(lp.data(), lpart, 8 * lp.size(), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    double s1 = 0, c1 = 0;
    for (uint32_t q = 0; q < mblk; q++) {
      s1 += lp[2 * q];
      c1 += lp[2 * q + 1];
    }
    m.len_coef = c1 > 0 ? (float)std::exp(s1 / c1) : 0.f;
  }
  init_weights(m.master, seed);
  HIP_TRY(model_upload(m));
  float *X, *mom1, *mom2, *master, *grad, *partial;
  A_TRY(b.get(&X, (size_t)n_samples * kMlpF));
  hipLaunchKernelGGL(k_mlp_inputs, dim3((n_samples + 255) / 256), dim3(256), 0, s, feat_all, n_samples, dh, Lf,
                     m.d_norm, X);
  HIP_TRY(hipGetLastError());
  A_TRY(b.get(&mom1, kMlpParams));
  A_TRY(b.get(&mom2, kMlpParams));
  A_TRY(b.get(&master, kMlpParams));
  A_TRY(b.get(&grad, kMlpParams));
  A_TRY(b.get(&partial, (size_t)(batch / AMLM_WAVE) * kMlpParams));
  HIP_TRY(hipMemsetAsync(mom1, 0, 4 * kMlpParams, s));
  HIP_TRY(hipMemsetAsync(mom2, 0, 4 * kMlpParams, s));
  HIP_TRY(hipMemcpyAsync(master, m.master, 4 * kMlpParams, hipMemcpyHostToDevice, s));
  // 3. minibatch Adam over a seeded permutation per epoch
  uint32_t *order;
  A_TRY(b.get(&order, n_samples));
  std::vector<uint32_t> perm(n_samples);
  std::mt19937_64 rng(seed ^ 0x5eedull);
  const float lr = 2e-3f, b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  uint64_t step = 0;
  for (uint32_t ep = 0; ep < epochs; ep++) {
    for (uint32_t i = 0; i < n_samples; i++) perm[i] = i;
    for (uint32_t i = n_samples - 1; i > 0; i--) std::swap(perm[i], perm[rng() % (i + 1)]);
    HIP_TRY(hipMemcpyAsync(order, perm.data(), 4ull * n_samples, hipMemcpyHostToDevice, s));
    for (uint32_t base = 0; base + batch <= n_samples; base += batch) {
      A_TRY(device_grad(m.d_w16, X, lab_all, n_samples, order, base, batch, 2.f / (float)batch, partial, grad,
                        nullptr, s));
      step++;
      float c1 = 1.f - std::pow(b1, (float)step), c2 = 1.f - std::pow(b2, (float)step);
      hipLaunchKernelGGL(k_adam, dim3((kMlpParams + 255) / 256), dim3(256), 0, s, master, mom1, mom2, grad,
                         m.d_w16, lr, b1, b2, eps, c1, c2);
      HIP_TRY(hipGetLastError());
    }
    HIP_TRY(hipStreamSynchronize(s));
  }
  HIP_TRY(hipMemcpyAsync(m.master, master, 4 * kMlpParams, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  m.loaded = true;
  m.train_samples = n_samples;
  if (out_path) return amlm_costmodel_save(out_path);
  return AMLM_OK;
}

static const char kMagic[8] = {'A', 'M', 'L', 'M', 'M', 'L', 'P', '2'};
static const char kMagicV1[8] = {'A', 'M', 'L', 'M', 'M', 'L', 'P', '1'};  // without the length constant

extern "C" amlm_status amlm_costmodel_save(const char *path) {
  MlpModel &m = global_model();
  if (!m.loaded) {
    set_error("no cost model is loaded");
    return AMLM_E_INVALID;
  }
  FILE *f = fopen(path, "wb");
  if (!f) {
    set_error(std::string("cannot open ") + path);
    return AMLM_E_INVALID;
  }
  bool ok = fwrite(kMagic, 1, 8, f) == 8 && fwrite(m.mean, 4, kMlpF, f) == (size_t)kMlpF &&
            fwrite(m.inv_std, 4, kMlpF, f) == (size_t)kMlpF &&
            fwrite(m.master, 4, kMlpParams, f) == (size_t)kMlpParams && fwrite(&m.len_coef, 4, 1, f) == 1;
  fclose(f);
  if (!ok) {
    set_error("short write");
    return AMLM_E_INVALID;
  }
  return AMLM_OK;
}

extern "C" amlm_status amlm_costmodel_load(const char *path) {
  FILE *f = fopen(path, "rb");
  if (!f) {
    set_error(std::string("cannot open ") + path);
    return AMLM_E_INVALID;
  }
  char magic[8];
  MlpModel &m = global_model();
  MlpModel tmp;
  bool ok = fread(magic, 1, 8, f) == 8 && (memcmp(magic, kMagic, 8) == 0 || memcmp(magic, kMagicV1, 8) == 0);
  const bool v2 = ok && memcmp(magic, kMagic, 8) == 0;
  ok = ok && fread(tmp.mean, 4, kMlpF, f) == (size_t)kMlpF && fread(tmp.inv_std, 4, kMlpF, f) == (size_t)kMlpF &&
       fread(tmp.master, 4, kMlpParams, f) == (size_t)kMlpParams;
  tmp.len_coef = 0.f;
  if (ok && v2) ok = fread(&tmp.len_coef, 4, 1, f) == 1;
  fclose(f);
  if (!ok) {
    set_error("not a cost model file");
    return AMLM_E_INVALID;
  }
  memcpy(m.mean, tmp.mean, sizeof(m.mean));
  memcpy(m.inv_std, tmp.inv_std, sizeof(m.inv_std));
  memcpy(m.master, tmp.master, sizeof(m.master));
  m.len_coef = tmp.len_coef;
  HIP_TRY(model_upload(m));
  m.loaded = true;
  return AMLM_OK;
}

extern "C" amlm_status amlm_costmodel_get(float *weights, float *mean, float *inv_std) {
  MlpModel &m = global_model();
  if (!m.loaded) {
    set_error("no cost model is loaded");
    return AMLM_E_INVALID;
  }
  if (weights) memcpy(weights, m.master, sizeof(m.master));
  if (mean) memcpy(mean, m.mean, sizeof(m.mean));
  if (inv_std) memcpy(inv_std, m.inv_std, sizeof(m.inv_std));
  return AMLM_OK;
}

extern "C" amlm_status amlm_costmodel_eval(amlm_graph *g, const amlm_params *p, uint64_t cap, float *pred,
                                           float *label, uint32_t *window_len, uint64_t *n_out, void *hip_stream) {
  if (!g || !p || !n_out) {
    set_error("null argument");
    return AMLM_E_INVALID;
  }
  MlpModel &m = global_model();
  if (!m.loaded) {
    set_error("no cost model is loaded");
    return AMLM_E_INVALID;
  }
  hipStream_t s = (hipStream_t)hip_stream;
  *n_out = 0;
  if (g->Ev == 0) return AMLM_OK;
  DevBuf b;
  const uint64_t E = std::max<uint64_t>(g->E, 1);
  uint32_t *fs, *keep, *koff, *klist, *cnt_dev, *ctmp, *scan_tmp, *fk;
  float *ls, *lk, *yk;
  unsigned long long *wk;
  A_TRY(b.get(&fs, E * kMlpRaw));
  A_TRY(b.get(&ls, E));
  A_TRY(b.get(&keep, E));
  A_TRY(b.get(&koff, E));
  A_TRY(b.get(&klist, E));
  A_TRY(b.get(&cnt_dev, 4));
  A_TRY(b.get(&wk, kWorkRows * E));
  A_TRY(b.get(&ctmp, E * (uint64_t)std::max(1u, amlm_num_columns(p))));
  A_TRY(b.get(&scan_tmp, scan_tmp_words(E)));
  A_TRY(mine_common(g, p, ctmp, wk, s));
  hipLaunchKernelGGL(k_sample_features, dim3((g->Ev + 255) / 256), dim3(256), 0, s, graph_view(g), p->delta,
                     (const unsigned long long *)(wk + kWorkSgImpl * g->E), fs, ls, keep);
  HIP_TRY(hipGetLastError());
  HIP_TRY(scan_exclusive_u32(keep, koff, g->Ev, cnt_dev, scan_tmp, s));
  hipLaunchKernelGGL(k_compact_keep, dim3((g->Ev + 255) / 256), dim3(256), 0, s, keep, koff, g->Ev, klist);
  HIP_TRY(hipGetLastError());
  uint32_t nk = 0;
  HIP_TRY(hipMemcpyAsync(&nk, cnt_dev, 4, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  *n_out = nk;
  if (nk == 0) return AMLM_OK;
  A_TRY(b.get(&fk, (uint64_t)nk * kMlpRaw));
  A_TRY(b.get(&lk, nk));
  A_TRY(b.get(&yk, nk));
  hipLaunchKernelGGL(k_gather_samples, dim3((nk + 255) / 256), dim3(256), 0, s, klist, nk, fs, ls, fk, lk, 0u);
  HIP_TRY(hipGetLastError());
  const float dh = (float)p->delta / 3600.f;
  const float Lf = (float)((p->patterns & AMLM_CYCLES) ? p->max_cycle_len : 2);
  HIP_TRY(mlp_infer(m, fk, nullptr, nk, nullptr, dh, Lf, yk, s));
  const uint64_t k = std::min<uint64_t>(nk, cap);
  if (k) {
    if (pred) HIP_TRY(hipMemcpyAsync(pred, yk, 4 * k, hipMemcpyDeviceToHost, s));
    if (label) HIP_TRY(hipMemcpyAsync(label, lk, 4 * k, hipMemcpyDeviceToHost, s));
    if (window_len) HIP_TRY(hipMemcpy2DAsync(window_len, 4, fk + 2, 4 * kMlpRaw, 4, k, hipMemcpyDeviceToHost, s));
  }
  HIP_TRY(hipStreamSynchronize(s));
  return AMLM_OK;
}

extern "C" amlm_status amlm_costmodel_length_coef(float *coef) {
  MlpModel &m = global_model();
  if (!coef) {
    set_error("null argument");
    return AMLM_E_INVALID;
  }
  if (!m.loaded) {
    set_error("no cost model is loaded");
    return AMLM_E_INVALID;
  }
  *coef = m.len_coef;
  return AMLM_OK;
}
