// mlp.hip -- surrogate network 4-64-64-2 (SiLU) on gfx950 BF16 matrix cores.
//
// Maps standardized cluster/laser features to standardized (absorbed energy, mean charge).
// Number formats: FP32 master weights and Adam moments; BF16 copies of the weights, the
// inputs, both hidden activations and the back-propagated hidden-2 gradient feed the
// products; every product accumulates in FP32.  The 64x64 layer (forward, input-gradient and
// weight-gradient products) runs on v_mfma_f32_16x16x32_bf16; the 4-wide input layer and the
// 2-wide output layer are VALU dot products.
//
// MFMA 16x16x32 BF16 operand layout (checked on the device): lane l holds
//   A[l % 16][8 (l / 16) + i], B[8 (l / 16) + i][l % 16] for i = 0..7, and the result
//   D[4 (l / 16) + r][l % 16] for r = 0..3.
//
// Training runs as one workgroup that loops over the steps (every reduction has a fixed
// order, so training is bitwise reproducible); inference runs one wave per 16 rows.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>

#include "lc_internal.h"

namespace lc {
namespace {

constexpr int kIn = 4, kH = 64, kOut = 2;
constexpr int kMaxBatch = 256;
// master parameter offsets (floats)
constexpr int oW1 = 0, oB1 = oW1 + kH * kIn, oW2 = oB1 + kH, oB2 = oW2 + kH * kH, oW3 = oB2 + kH,
              oB3 = oW3 + kOut * kH, kParams = oB3 + kOut;  // 4610

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// State buffer layout (bytes, 256-aligned blocks):
//   params[4610] f32 | adam m[4610] | adam v[4610] | grad[4610] | scaler[16] f32 | meta (int)
//   scratch: z1, z2, dz2 [256][64] f32; h1, h2, dz2b [256][64] bf16 (as u16);
//            h1T, dz2bT [64][256] u16; xs [256][4] f32; ts [256][2] f32; dy [256][2] f32
struct MlpState {
  float* p;
  float* m;
  float* v;
  float* g;
  float* scaler;  // x_mu[4], x_sd[4], y_mu[2], y_sd[2]
  int32_t* meta;  // [0] Adam step count
  float* z1;
  float* z2;
  float* dz2;
  uint16_t* h1;
  uint16_t* h2;
  uint16_t* dz2b;
  uint16_t* h1T;
  uint16_t* dz2bT;
  float* xs;
  float* ts;
  float* dy;
};

size_t al256(size_t b) { return (b + 255) & ~(size_t)255; }

size_t carve(void* base, MlpState* s) {
  char* p = (char*)base;
  size_t o = 0;
  auto take = [&](size_t b) { char* r = p + o; o += al256(b); return r; };
  MlpState t;
  t.p = (float*)take(sizeof(float) * kParams);
  t.m = (float*)take(sizeof(float) * kParams);
  t.v = (float*)take(sizeof(float) * kParams);
  t.g = (float*)take(sizeof(float) * kParams);
  t.scaler = (float*)take(sizeof(float) * 16);
  t.meta = (int32_t*)take(sizeof(int32_t) * 16);
  t.z1 = (float*)take(sizeof(float) * kMaxBatch * kH);
  t.z2 = (float*)take(sizeof(float) * kMaxBatch * kH);
  t.dz2 = (float*)take(sizeof(float) * kMaxBatch * kH);
  t.h1 = (uint16_t*)take(2 * kMaxBatch * kH);
  t.h2 = (uint16_t*)take(2 * kMaxBatch * kH);
  t.dz2b = (uint16_t*)take(2 * kMaxBatch * kH);
  t.h1T = (uint16_t*)take(2 * kMaxBatch * kH);
  t.dz2bT = (uint16_t*)take(2 * kMaxBatch * kH);
  t.xs = (float*)take(sizeof(float) * kMaxBatch * kIn);
  t.ts = (float*)take(sizeof(float) * kMaxBatch * kOut);
  t.dy = (float*)take(sizeof(float) * kMaxBatch * kOut);
  if (s) *s = t;
  return o;
}

// FP32 -> BF16 with round-to-nearest-even (NaN stays NaN).
__device__ inline uint16_t bf16_bits(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ inline float bf16_float(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }
__device__ inline float round_bf16(float f) { return bf16_float(bf16_bits(f)); }

__device__ inline float sigmoidf_(float z) { return 1.0f / (1.0f + expf(-z)); }
__device__ inline float silu(float z) { return z * sigmoidf_(z); }
__device__ inline float dsilu(float z) {
  const float s = sigmoidf_(z);
  return s * (1.0f + z * (1.0f - s));
}

__device__ inline bf16x8 load8(const uint16_t* q) {
  bf16x8 v;
  uint16_t tmp[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) tmp[i] = q[i];
  memcpy(&v, tmp, sizeof(v));
  return v;
}

__device__ inline f32x4 mfma(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// Shared-memory copy of the BF16 weights used by the products.
struct WeightsLds {
  uint16_t w1[kH * kIn];
  uint16_t w2[kH * kH];    // [n][k] (row n of W2)
  uint16_t w2t[kH * kH];   // [k][n]
  uint16_t w3[kOut * kH];
  float b1[kH];
  float b2[kH];
  float b3[kOut];
};

__device__ void load_weights(const float* p, WeightsLds* w) {
  for (int i = threadIdx.x; i < kH * kIn; i += blockDim.x) w->w1[i] = bf16_bits(p[oW1 + i]);
  for (int i = threadIdx.x; i < kH * kH; i += blockDim.x) {
    const uint16_t b = bf16_bits(p[oW2 + i]);
    w->w2[i] = b;
    w->w2t[(i % kH) * kH + i / kH] = b;
  }
  for (int i = threadIdx.x; i < kOut * kH; i += blockDim.x) w->w3[i] = bf16_bits(p[oW3 + i]);
  for (int i = threadIdx.x; i < kH; i += blockDim.x) { w->b1[i] = p[oB1 + i]; w->b2[i] = p[oB2 + i]; }
  if (threadIdx.x < kOut) w->b3[threadIdx.x] = p[oB3 + threadIdx.x];
}

// ----------------------------------------------------------------------------- training
// One workgroup of 256 threads (4 waves).  Per step: minibatch rows idx[step*B .. +B).
__global__ __launch_bounds__(256) void k_mlp_train(MlpState s, const float* X, const float* Y, const int32_t* idx,
                                                   int64_t n, int B, int steps, float lr, float beta1, float beta2, float eps,
                                                   float* loss_out, int update) {
  __shared__ WeightsLds w;
  __shared__ float red[256];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  for (int step = 0; step < steps; ++step) {
    __syncthreads();
    load_weights(s.p, &w);
    // minibatch: standardized, BF16-rounded inputs; standardized targets
    for (int e = tid; e < B * kIn; e += 256) {
      const int r = e / kIn, k = e % kIn;
      int row = idx[(int64_t)step * B + r];
      if (row < 0 || row >= n) { s.meta[1] = 1; row = 0; }  // out-of-range row: flagged, row 0 used
      s.xs[e] = round_bf16((X[(int64_t)row * kIn + k] - s.scaler[k]) / s.scaler[4 + k]);
    }
    for (int e = tid; e < B * kOut; e += 256) {
      const int r = e / kOut, o = e % kOut;
      int row = idx[(int64_t)step * B + r];
      if (row < 0 || row >= n) row = 0;
      s.ts[e] = (Y[(int64_t)row * kOut + o] - s.scaler[8 + o]) / s.scaler[10 + o];
    }
    __syncthreads();
    // layer 1 (VALU): z1 = W1 x + b1
    for (int e = tid; e < B * kH; e += 256) {
      const int r = e / kH, j = e % kH;
      float z = w.b1[j];
#pragma unroll
      for (int k = 0; k < kIn; ++k) z = __builtin_fmaf(bf16_float(w.w1[j * kIn + k]), s.xs[r * kIn + k], z);
      s.z1[e] = z;
      const uint16_t h = bf16_bits(silu(z));
      s.h1[e] = h;
      s.h1T[j * kMaxBatch + r] = h;
    }
    __syncthreads();
    // layer 2 (MFMA): z2[r][n] = sum_k h1[r][k] W2[n][k] + b2[n]; tiles of 16 rows x 16 cols
    const int tiles2 = (B / 16) * (kH / 16);
    for (int t = wave; t < tiles2; t += 4) {
      const int tr = t / (kH / 16), tc = t % (kH / 16);
      f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int kk = 0; kk < kH; kk += 32) {
        const bf16x8 a = load8(&s.h1[(tr * 16 + lane % 16) * kH + kk + 8 * (lane / 16)]);
        const bf16x8 b = load8(&w.w2[(tc * 16 + lane % 16) * kH + kk + 8 * (lane / 16)]);
        acc = mfma(a, b, acc);
      }
      const int n = tc * 16 + lane % 16;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = tr * 16 + 4 * (lane / 16) + q;
        const float z = acc[q] + w.b2[n];
        s.z2[r * kH + n] = z;
        s.h2[r * kH + n] = bf16_bits(silu(z));
      }
    }
    __syncthreads();
    // layer 3 (VALU) and loss: y = W3 h2 + b3; dy = (y - t) / B
    {
      float l = 0.f;
      for (int e = tid; e < B * kOut; e += 256) {
        const int r = e / kOut, o = e % kOut;
        float y = w.b3[o];
        for (int j = 0; j < kH; ++j) y = __builtin_fmaf(bf16_float(w.w3[o * kH + j]), bf16_float(s.h2[r * kH + j]), y);
        const float d = y - s.ts[e];
        s.dy[e] = d / (float)B;
        l += d * d;
      }
      red[tid] = l;
    }
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if (tid < o) red[tid] += red[tid + o];
      __syncthreads();
    }
    if (tid == 0 && loss_out) loss_out[step] = red[0] / (2.0f * (float)B);
    // output layer gradients: dW3[o][j] = sum_r dy[r][o] h2[r][j]; db3[o] = sum_r dy[r][o]
    for (int e = tid; e < kOut * kH + kOut; e += 256) {
      if (e < kOut * kH) {
        const int o = e / kH, j = e % kH;
        float g = 0.f;
        for (int r = 0; r < B; ++r) g = __builtin_fmaf(s.dy[r * kOut + o], bf16_float(s.h2[r * kH + j]), g);
        s.g[oW3 + e] = g;
      } else {
        const int o = e - kOut * kH;
        float g = 0.f;
        for (int r = 0; r < B; ++r) g += s.dy[r * kOut + o];
        s.g[oB3 + o] = g;
      }
    }
    // hidden-2 gradient: dz2 = (W3^T dy) * silu'(z2)
    for (int e = tid; e < B * kH; e += 256) {
      const int r = e / kH, j = e % kH;
      float g = 0.f;
#pragma unroll
      for (int o = 0; o < kOut; ++o) g = __builtin_fmaf(bf16_float(w.w3[o * kH + j]), s.dy[r * kOut + o], g);
      const float d = g * dsilu(s.z2[e]);
      s.dz2[e] = d;
      const uint16_t b = bf16_bits(d);
      s.dz2b[e] = b;
      s.dz2bT[j * kMaxBatch + r] = b;
    }
    __syncthreads();
    // db2[n] = sum_r dz2[r][n]
    if (tid < kH) {
      float g = 0.f;
      for (int r = 0; r < B; ++r) g += s.dz2[r * kH + tid];
      s.g[oB2 + tid] = g;
    }
    // dW2[n][k] = sum_r dz2b[r][n] h1[r][k]  (MFMA, K = batch)
    for (int t = wave; t < (kH / 16) * (kH / 16); t += 4) {
      const int tm = t / (kH / 16), tn = t % (kH / 16);
      f32x4 acc = {0.f, 0.f, 0.f, 0.f};
      for (int kk = 0; kk < B; kk += 32) {
        const bf16x8 a = load8(&s.dz2bT[(tm * 16 + lane % 16) * kMaxBatch + kk + 8 * (lane / 16)]);
        const bf16x8 b = load8(&s.h1T[(tn * 16 + lane % 16) * kMaxBatch + kk + 8 * (lane / 16)]);
        acc = mfma(a, b, acc);
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int n = tm * 16 + 4 * (lane / 16) + q, k = tn * 16 + lane % 16;
        s.g[oW2 + n * kH + k] = acc[q];
      }
    }
    // hidden-1 gradient: g1[r][k] = sum_n dz2b[r][n] W2[n][k]  (MFMA); dz1 = g1 * silu'(z1)
    // (dz1 overwrites z1 after use)
    for (int t = wave; t < (B / 16) * (kH / 16); t += 4) {
      const int tr = t / (kH / 16), tc = t % (kH / 16);
      f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int kk = 0; kk < kH; kk += 32) {
        const bf16x8 a = load8(&s.dz2b[(tr * 16 + lane % 16) * kH + kk + 8 * (lane / 16)]);
        const bf16x8 b = load8(&w.w2t[(tc * 16 + lane % 16) * kH + kk + 8 * (lane / 16)]);
        acc = mfma(a, b, acc);
      }
      const int k = tc * 16 + lane % 16;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = tr * 16 + 4 * (lane / 16) + q;
        s.z1[r * kH + k] = acc[q] * dsilu(s.z1[r * kH + k]);
      }
    }
    __syncthreads();
    // dW1[j][k] = sum_r dz1[r][j] x[r][k]; db1[j] = sum_r dz1[r][j]
    for (int e = tid; e < kH * kIn + kH; e += 256) {
      if (e < kH * kIn) {
        const int j = e / kIn, k = e % kIn;
        float g = 0.f;
        for (int r = 0; r < B; ++r) g = __builtin_fmaf(s.z1[r * kH + j], s.xs[r * kIn + k], g);
        s.g[oW1 + e] = g;
      } else {
        const int j = e - kH * kIn;
        float g = 0.f;
        for (int r = 0; r < B; ++r) g += s.z1[r * kH + j];
        s.g[oB1 + j] = g;
      }
    }
    __syncthreads();
    if (update) {
      // Adam (Kingma & Ba) on the FP32 master weights
      const int t = s.meta[0] + 1;
      const float c1 = 1.0f - powf(beta1, (float)t), c2 = 1.0f - powf(beta2, (float)t);
      for (int i = tid; i < kParams; i += 256) {
        const float g = s.g[i];
        const float m = beta1 * s.m[i] + (1.0f - beta1) * g;
        const float v = beta2 * s.v[i] + (1.0f - beta2) * g * g;
        s.m[i] = m;
        s.v[i] = v;
        s.p[i] -= lr * (m / c1) / (sqrtf(v / c2) + eps);
      }
      __syncthreads();
      if (tid == 0) s.meta[0] = t;
    }
  }
}

// ----------------------------------------------------------------------------- scaler
// Feature and target means and standard deviations (population), FP64 sums in row order.
__global__ __launch_bounds__(64) void k_mlp_scaler(MlpState s, const float* X, const float* Y, int64_t n) {
  const int c = threadIdx.x;  // column: 0..3 features, 4..5 targets
  if (c >= kIn + kOut) return;
  const float* src = c < kIn ? X : Y;
  const int stride = c < kIn ? kIn : kOut;
  const int col = c < kIn ? c : c - kIn;
  double sum = 0.0;
  for (int64_t i = 0; i < n; ++i) sum += (double)src[i * stride + col];
  const double mu = sum / (double)n;
  double ss = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    const double d = (double)src[i * stride + col] - mu;
    ss += d * d;
  }
  double sd = sqrt(ss / (double)n);
  if (!(sd > 0.0)) sd = 1.0;
  if (c < kIn) { s.scaler[col] = (float)mu; s.scaler[4 + col] = (float)sd; }
  else { s.scaler[8 + col] = (float)mu; s.scaler[10 + col] = (float)sd; }
}

// ----------------------------------------------------------------------------- inference
// One wave per 16 rows: layer 1 on VALU, layer 2 on MFMA, layer 3 on VALU; outputs
// de-standardized.
__global__ __launch_bounds__(256) void k_mlp_infer(const float* p, const float* scaler, const float* X, float* Y,
                                                   int64_t n) {
  __shared__ WeightsLds w;
  __shared__ uint16_t h1[4][16 * kH];
  __shared__ uint16_t h2[4][16 * kH];
  load_weights(p, &w);
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t r0 = ((int64_t)blockIdx.x * 4 + wave) * 16;  // rows past n are computed but not stored
  for (int e = lane; e < 16 * kH; e += 64) {
    const int r = e / kH, j = e % kH;
    const int64_t row = r0 + r;
    float z = w.b1[j];
    if (row < n) {
#pragma unroll
      for (int k = 0; k < kIn; ++k) {
        const float x = round_bf16((X[row * kIn + k] - scaler[k]) / scaler[4 + k]);
        z = __builtin_fmaf(bf16_float(w.w1[j * kIn + k]), x, z);
      }
    }
    h1[wave][e] = bf16_bits(silu(z));
  }
  __syncthreads();
  for (int tc = 0; tc < kH / 16; ++tc) {
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kk = 0; kk < kH; kk += 32) {
      const bf16x8 a = load8(&h1[wave][(lane % 16) * kH + kk + 8 * (lane / 16)]);
      const bf16x8 b = load8(&w.w2[(tc * 16 + lane % 16) * kH + kk + 8 * (lane / 16)]);
      acc = mfma(a, b, acc);
    }
    const int col = tc * 16 + lane % 16;
#pragma unroll
    for (int q = 0; q < 4; ++q) h2[wave][(4 * (lane / 16) + q) * kH + col] = bf16_bits(silu(acc[q] + w.b2[col]));
  }
  __syncthreads();
  if (lane < 16 * kOut) {
    const int r = lane / kOut, o = lane % kOut;
    const int64_t row = r0 + r;
    float y = w.b3[o];
    for (int j = 0; j < kH; ++j) y = __builtin_fmaf(bf16_float(w.w3[o * kH + j]), bf16_float(h2[wave][r * kH + j]), y);
    if (row < n) Y[row * kOut + o] = y * scaler[10 + o] + scaler[8 + o];
  }
}

}  // namespace
}  // namespace lc

using namespace lc;

extern "C" {

size_t lc_mlp_state_bytes(void) { return carve(nullptr, nullptr); }

int lc_mlp_n_params(void) { return kParams; }

int lc_mlp_set_params(void* d_state, const float* host_params, void* stream) {
  if (!d_state || !host_params || ((uintptr_t)d_state & 255)) return LC_E_INVALID;
  MlpState s;
  carve(d_state, &s);
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = hipStreamSynchronize(st);
  if (e == hipSuccess) e = hipMemcpy(s.p, host_params, sizeof(float) * kParams, hipMemcpyHostToDevice);
  // zero Adam moments and step count, identity scaler
  static const float zeros[kParams] = {};
  if (e == hipSuccess) e = hipMemcpy(s.m, zeros, sizeof(float) * kParams, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(s.v, zeros, sizeof(float) * kParams, hipMemcpyHostToDevice);
  const float sc[16] = {0, 0, 0, 0, 1, 1, 1, 1, 0, 0, 1, 1, 0, 0, 0, 0};
  if (e == hipSuccess) e = hipMemcpy(s.scaler, sc, sizeof(sc), hipMemcpyHostToDevice);
  const int32_t meta[16] = {};
  if (e == hipSuccess) e = hipMemcpy(s.meta, meta, sizeof(meta), hipMemcpyHostToDevice);
  return e == hipSuccess ? LC_OK : LC_E_HIP;
}

int lc_mlp_get_params(const void* d_state, float* host_params, float* host_scaler, void* stream) {
  if (!d_state || ((uintptr_t)d_state & 255)) return LC_E_INVALID;
  MlpState s;
  carve((void*)d_state, &s);
  hipError_t e = hipStreamSynchronize((hipStream_t)stream);
  if (e == hipSuccess && host_params) e = hipMemcpy(host_params, s.p, sizeof(float) * kParams, hipMemcpyDeviceToHost);
  if (e == hipSuccess && host_scaler) e = hipMemcpy(host_scaler, s.scaler, sizeof(float) * 12, hipMemcpyDeviceToHost);
  return e == hipSuccess ? LC_OK : LC_E_HIP;
}

int lc_mlp_status(const void* d_state, void* stream) {
  if (!d_state || ((uintptr_t)d_state & 255)) return LC_E_INVALID;
  MlpState s;
  carve((void*)d_state, &s);
  int32_t meta[2] = {0, 0};
  hipError_t e = hipStreamSynchronize((hipStream_t)stream);
  if (e == hipSuccess) e = hipMemcpy(meta, s.meta, sizeof(meta), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return LC_E_HIP;
  return meta[1] ? LC_E_INVALID : LC_OK;
}

int lc_mlp_fit_scaler(void* d_state, const float* d_X, const float* d_Y, int64_t n, void* stream) {
  if (!d_state || !d_X || !d_Y || n < 1 || ((uintptr_t)d_state & 255)) return LC_E_INVALID;
  MlpState s;
  carve(d_state, &s);
  k_mlp_scaler<<<1, 64, 0, (hipStream_t)stream>>>(s, d_X, d_Y, n);
  return hipGetLastError() == hipSuccess ? LC_OK : LC_E_HIP;
}

int lc_mlp_train(void* d_state, const float* d_X, const float* d_Y, int64_t n, const int32_t* d_rows, int32_t batch,
                 int32_t steps, float lr, float* d_loss, void* stream) {
  if (!d_state || !d_X || !d_Y || !d_rows || n < 1 || steps < 0 || ((uintptr_t)d_state & 255)) return LC_E_INVALID;
  if (batch < 32 || batch > kMaxBatch || batch % 32 != 0 || !(lr > 0.0f)) return LC_E_INVALID;
  if (steps == 0) return LC_OK;
  MlpState s;
  carve(d_state, &s);
  k_mlp_train<<<1, 256, 0, (hipStream_t)stream>>>(s, d_X, d_Y, d_rows, n, batch, steps, lr, 0.9f, 0.999f, 1e-8f, d_loss, 1);
  return hipGetLastError() == hipSuccess ? LC_OK : LC_E_HIP;
}

int lc_mlp_grad(void* d_state, const float* d_X, const float* d_Y, int64_t n, const int32_t* d_rows, int32_t batch,
                float* d_grad, float* d_loss, void* stream) {
  if (!d_state || !d_X || !d_Y || !d_rows || !d_grad || n < 1 || ((uintptr_t)d_state & 255)) return LC_E_INVALID;
  if (batch < 32 || batch > kMaxBatch || batch % 32 != 0) return LC_E_INVALID;
  MlpState s;
  carve(d_state, &s);
  hipStream_t st = (hipStream_t)stream;
  k_mlp_train<<<1, 256, 0, st>>>(s, d_X, d_Y, d_rows, n, batch, 1, 1.0f, 0.9f, 0.999f, 1e-8f, d_loss, 0);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpyAsync(d_grad, s.g, sizeof(float) * kParams, hipMemcpyDeviceToDevice, st);
  return e == hipSuccess ? LC_OK : LC_E_HIP;
}

int lc_mlp_infer(const void* d_state, const float* d_X, float* d_Y, int64_t n, void* stream) {
  if (!d_state || n < 0 || ((uintptr_t)d_state & 255)) return LC_E_INVALID;
  if (n == 0) return LC_OK;
  if (!d_X || !d_Y) return LC_E_INVALID;
  MlpState s;
  carve((void*)d_state, &s);
  const int64_t blocks = (n + 63) / 64;
  if (blocks > 0x7fffffff) return LC_E_INVALID;
  k_mlp_infer<<<(int)blocks, 256, 0, (hipStream_t)stream>>>(s.p, s.scaler, d_X, d_Y, n);
  return hipGetLastError() == hipSuccess ? LC_OK : LC_E_HIP;
}

}  // extern "C"
