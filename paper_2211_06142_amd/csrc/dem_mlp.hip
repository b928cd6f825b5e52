// dem_mlp.hip -- the learned closure network on the matrix cores (an extension
// of the method; not in arXiv:2211.06142).
//
// Network 6 -> 64 -> 64 -> 64 -> 2, GELU (erf form) on the hidden layers,
// BF16 operands with FP32 accumulation on the matrix cores: gfx950's
// v_mfma_f32_16x16x32_bf16 for every contraction over 64 features and over the
// samples, v_mfma_f32_16x16x16_bf16 where the contraction has at most 16 terms
// (the 6 inputs of layer 1, the 2 outputs in the backward pass).  Flat
// parameter layout (FP32 master, BF16 copy at the same offsets):
//   W1 6x64 | b1 | W2 64x64 | b2 | W3 64x64 | b3 | W4 64x2 | b4,  W[k][m] row-major
//
// Transposed evaluation.  One wavefront takes 16 samples and computes
// Z^T = W^T H^T: the 16x16 output fragment of one MFMA holds features
// 4(lane/16)+i of sample lane%16.  The K = 32 MFMA pairs element j of lane group
// q of A with element j of lane group q of B; a contraction is a sum, so any
// assignment of the 32 features of a K tile to (q, j) serves if A and B share
// it.  Taking j < 4 from output tile 2t and j >= 4 from tile 2t + 1 (feature
// 32t + 4q + (j mod 4) + 16 (j div 4)) makes the B operand of the next layer
// the two output fragments side by side, so activations never leave the
// registers between layers (no LDS transposes, no lane exchange).  The backward pass runs the same way with W in place of
// W^T.  Weight gradients contract over the samples: a split-K MFMA product per
// chunk of samples, then a fixed-order sum over chunks, so every result is
// bitwise reproducible.
#include <algorithm>
#include <cmath>
#include <mutex>
#include <vector>

#include "dem_device.h"

namespace dem {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kW1 = 0, kB1 = 384, kW2 = 448, kB2 = 4544, kW3 = 4608, kB3 = 8704, kW4 = 8768, kB4 = 8896;
constexpr int kNParams = 8898;
constexpr int kChunk = 1024;   // samples per split-K chunk of the weight gradients

// float -> bfloat16 bits, round to nearest even (finite inputs)
__device__ inline short f2bf(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (short)(u >> 16);
}
__device__ inline float bf2f(short h) { return __uint_as_float(((uint32_t)(uint16_t)h) << 16); }

__device__ inline float gelu_f(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ inline float gelu_df(float z) {
  return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * expf(-0.5f * z * z) * 0.39894228040143268f;
}

__device__ inline f32x4 mfma16(bf16x4 a, bf16x4 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

typedef short bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
// D += A B over K = 32: lane l holds A[l % 16][8 (l / 16) + j] and B[8 (l / 16) + j][l % 16]
// (j = 0 .. 7) and receives D[4 (l / 16) + i][l % 16]
__device__ inline f32x4 mfma32(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8_t, a), __builtin_bit_cast(bf16x8_t, b), c,
                                                 0, 0, 0);
}
// two output fragments side by side: the B operand of a K = 32 tile
__device__ inline bf16x8 cat8(bf16x4 a, bf16x4 b) { return __builtin_shufflevector(a, b, 0, 1, 2, 3, 4, 5, 6, 7); }
// feature of element j of lane group q in K tile t (the assignment above)
__device__ inline int kperm(int t, int q, int j) { return 32 * t + 4 * q + (j & 3) + 16 * (j >> 2); }

// A fragment of W^T (rows = outputs m, columns = inputs k) for output tile mt
// and input tile kt of a K x M layer: lane holds W[16kt + 4q + i][16mt + r]
__device__ inline bf16x4 wt_frag(const short* wb, int off, int K, int M, int mt, int kt, int q, int r) {
  bf16x4 a;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    int k = 16 * kt + 4 * q + i, m = 16 * mt + r;
    a[i] = (k < K && m < M) ? wb[off + k * M + m] : (short)0;
  }
  return a;
}
// K = 32 fragment of W^T for output tile mt and K tile t: lane holds
// W[kperm(t, q, j)][16mt + r]
__device__ inline bf16x8 wt_frag32(const short* wb, int off, int K, int M, int mt, int t, int q, int r) {
  bf16x8 a;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    int k = kperm(t, q, j), m = 16 * mt + r;
    a[j] = (k < K && m < M) ? wb[off + k * M + m] : (short)0;
  }
  return a;
}
// K = 32 fragment of W (contraction over the outputs m) for input tile kt and
// K tile t: lane holds W[16kt + r][kperm(t, q, j)]
__device__ inline bf16x8 w_frag32(const short* wb, int off, int K, int M, int kt, int t, int q, int r) {
  bf16x8 a;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    int k = 16 * kt + r, m = kperm(t, q, j);
    a[j] = (k < K && m < M) ? wb[off + k * M + m] : (short)0;
  }
  return a;
}

// A fragment of W (rows = inputs k, columns = outputs m) for input tile kt and
// output tile mt: lane holds W[16kt + r][16mt + 4q + i]
__device__ inline bf16x4 w_frag(const short* wb, int off, int K, int M, int kt, int mt, int q, int r) {
  bf16x4 a;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    int k = 16 * kt + r, m = 16 * mt + 4 * q + i;
    a[i] = (k < K && m < M) ? wb[off + k * M + m] : (short)0;
  }
  return a;
}
__device__ inline f32x4 bias_frag(const float* pf, int off, int M, int mt, int q) {
  f32x4 b;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    int m = 16 * mt + 4 * q + i;
    b[i] = m < M ? pf[off + m] : 0.0f;
  }
  return b;
}

// training record of a batch (sample-major rows)
struct MlpTrainBuf {
  short* h0;     // B x 16 (input, padded)
  short* h[3];   // B x 64 activations of the hidden layers
  float* z[3];   // B x 64 pre-activations
  short* g[3];   // B x 64 loss gradients w.r.t. the hidden pre-activations
  float* g4;     // B x 2 loss gradient w.r.t. the output
  float* err;    // B: squared error of the sample
};

// The lane's fragments of every weight and bias (about 90 registers), loaded
// once per wavefront and kept across the tiles it evaluates.
struct WeightFrags {
  bf16x4 w1[4];
  bf16x8 w2[4][2], w3[4][2], w4[2];
  f32x4 b1[4], b2[4], b3[4], b4;
};
__device__ inline WeightFrags load_frags(const short* wb, const float* pf, int q, int r) {
  WeightFrags W;
#pragma unroll
  for (int mt = 0; mt < 4; ++mt) {
    W.w1[mt] = wt_frag(wb, kW1, 6, 64, mt, 0, q, r);
    W.b1[mt] = bias_frag(pf, kB1, 64, mt, q);
    W.b2[mt] = bias_frag(pf, kB2, 64, mt, q);
    W.b3[mt] = bias_frag(pf, kB3, 64, mt, q);
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      W.w2[mt][t] = wt_frag32(wb, kW2, 64, 64, mt, t, q, r);
      W.w3[mt][t] = wt_frag32(wb, kW3, 64, 64, mt, t, q, r);
    }
  }
#pragma unroll
  for (int t = 0; t < 2; ++t) W.w4[t] = wt_frag32(wb, kW4, 64, 2, 0, t, q, r);
  W.b4 = bias_frag(pf, kB4, 2, 0, q);
  return W;
}

// One tile of 16 samples (rows s0 .. s0+15; rows >= B are padding).  Returns
// the output fragment: lanes 0-15, items 0-1 hold y0, y1 of sample lane.
template <bool kTrain>
__device__ f32x4 forward_tile(const WeightFrags& W, bf16x4 a0, int q, int r, int64_t s0, int64_t B,
                              const MlpTrainBuf& tb) {
  const int64_t s = s0 + r;
  const bool valid = s < B;
  if (kTrain && valid && q < 4) {
    short* dst = tb.h0 + s * 16 + 4 * q;
#pragma unroll
    for (int i = 0; i < 4; ++i) dst[i] = a0[i];
  }
  bf16x4 h[4];
  // layer 1: 6 -> 64
#pragma unroll
  for (int mt = 0; mt < 4; ++mt) {
    f32x4 acc = mfma16(W.w1[mt], a0, W.b1[mt]);
#pragma unroll
    for (int i = 0; i < 4; ++i) h[mt][i] = f2bf(gelu_f(acc[i]));
    if (kTrain && valid) {
      *(f32x4*)(tb.z[0] + s * 64 + 16 * mt + 4 * q) = acc;
      *(bf16x4*)(tb.h[0] + s * 64 + 16 * mt + 4 * q) = h[mt];
    }
  }
  // layers 2 and 3: 64 -> 64
#pragma unroll
  for (int l = 1; l < 3; ++l) {
    bf16x4 hn[4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
      f32x4 acc = l == 1 ? W.b2[mt] : W.b3[mt];
#pragma unroll
      for (int t = 0; t < 2; ++t)
        acc = mfma32(l == 1 ? W.w2[mt][t] : W.w3[mt][t], cat8(h[2 * t], h[2 * t + 1]), acc);
#pragma unroll
      for (int i = 0; i < 4; ++i) hn[mt][i] = f2bf(gelu_f(acc[i]));
      if (kTrain && valid) {
        *(f32x4*)(tb.z[l] + s * 64 + 16 * mt + 4 * q) = acc;
        *(bf16x4*)(tb.h[l] + s * 64 + 16 * mt + 4 * q) = hn[mt];
      }
    }
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) h[mt] = hn[mt];
  }
  // layer 4: 64 -> 2 (one padded output tile)
  f32x4 y = W.b4;
#pragma unroll
  for (int t = 0; t < 2; ++t) y = mfma32(W.w4[t], cat8(h[2 * t], h[2 * t + 1]), y);
  return y;
}

// input fragment of layer 1 from FP32 normalised features (row stride ldx)
__device__ inline bf16x4 input_frag(const float* x, int64_t ldx, int64_t s, int64_t B, int q) {
  bf16x4 a;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    int k = 4 * q + i;
    a[i] = (s < B && k < 6) ? f2bf(x[s * ldx + k]) : (short)0;
  }
  return a;
}

__global__ __launch_bounds__(256) void k_mlp_forward(const short* wb, const float* pf, const float* x, int64_t B,
                                                     float* y) {
  const int lane = threadIdx.x & 63, q = lane >> 4, r = lane & 15;
  const int64_t nt = (B + 15) / 16;
  const int64_t w0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
  MlpTrainBuf none{};
  const WeightFrags W = load_frags(wb, pf, q, r);
  for (int64_t t = w0; t < nt; t += nw) {
    const int64_t s = t * 16 + r;
    f32x4 out = forward_tile<false>(W, input_frag(x, 6, s, B, q), q, r, t * 16, B, none);
    if (q == 0 && s < B) {
      y[2 * s] = out[0];
      y[2 * s + 1] = out[1];
    }
  }
}

// forward of a training batch: records activations, the output gradient of
// L = mean (y - t)^2 and the squared error per sample
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_mlp_forward_train(const short* wb, const float* pf, const float* x,
                                                           const float* tgt, int64_t B, MlpTrainBuf tb) {
  const int lane = threadIdx.x & 63, q = lane >> 4, r = lane & 15;
  const int64_t nt = (B + 15) / 16;
  const int64_t w0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
  const float scale = 2.0f / (2.0f * (float)B);
  const WeightFrags W = load_frags(wb, pf, q, r);
  for (int64_t t = w0; t < nt; t += nw) {
    const int64_t s = t * 16 + r;
    f32x4 out = forward_tile<true>(W, input_frag(x, 6, s, B, q), q, r, t * 16, B, tb);
    if (q == 0 && s < B) {
      float e0 = out[0] - tgt[2 * s], e1 = out[1] - tgt[2 * s + 1];
      tb.g4[2 * s] = scale * e0;
      tb.g4[2 * s + 1] = scale * e1;
      tb.err[s] = e0 * e0 + e1 * e1;
    }
  }
}

// backward through the hidden layers: G_l = (W_l G_{l+1}) * gelu'(Z_l)
__global__ __launch_bounds__(256) void k_mlp_backward(const short* wb, int64_t B, MlpTrainBuf tb) {
  const int lane = threadIdx.x & 63, q = lane >> 4, r = lane & 15;
  const int64_t nt = (B + 15) / 16;
  const int64_t w0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t t = w0; t < nt; t += nw) {
    const int64_t s = t * 16 + r;
    const bool valid = s < B;
    bf16x4 g4;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      int m = 4 * q + i;
      g4[i] = (valid && m < 2) ? f2bf(tb.g4[2 * s + m]) : (short)0;
    }
    // dH3 = W4 G4 (input tile kt = 0: the 2 outputs, padded)
    bf16x4 g[4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
      f32x4 acc = {0.f, 0.f, 0.f, 0.f};
      acc = mfma16(w_frag(wb, kW4, 64, 2, mt, 0, q, r), g4, acc);
      f32x4 z = valid ? *(const f32x4*)(tb.z[2] + s * 64 + 16 * mt + 4 * q) : f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int i = 0; i < 4; ++i) g[mt][i] = f2bf(acc[i] * gelu_df(z[i]));
      if (valid) *(bf16x4*)(tb.g[2] + s * 64 + 16 * mt + 4 * q) = g[mt];
    }
    // dH2 = W3 G3, dH1 = W2 G2
#pragma unroll
    for (int l = 1; l >= 0; --l) {
      const int offW = l == 1 ? kW3 : kW2;
      bf16x4 gn[4];
#pragma unroll
      for (int mt = 0; mt < 4; ++mt) {
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int t = 0; t < 2; ++t)
          acc = mfma32(w_frag32(wb, offW, 64, 64, mt, t, q, r), cat8(g[2 * t], g[2 * t + 1]), acc);
        f32x4 z = valid ? *(const f32x4*)(tb.z[l] + s * 64 + 16 * mt + 4 * q) : f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int i = 0; i < 4; ++i) gn[mt][i] = f2bf(acc[i] * gelu_df(z[i]));
        if (valid) *(bf16x4*)(tb.g[l] + s * 64 + 16 * mt + 4 * q) = gn[mt];
      }
#pragma unroll
      for (int mt = 0; mt < 4; ++mt) g[mt] = gn[mt];
    }
  }
}

// Weight and bias gradients of one chunk of samples for one layer:
// dW[k][m] = sum_s H[s][k] G[s][m] as MFMA products with the samples as the
// contraction, a bias gradient with an all-ones A operand.  The block stages
// 64-sample tiles of H and G in LDS with coalesced loads; each wavefront keeps
// the accumulators of its output tiles (at most 5) in registers.
constexpr int kSub = 64;   // samples per LDS tile

__global__ __launch_bounds__(256) void k_mlp_wgrad(int64_t B, MlpTrainBuf tb, float* part) {
  __shared__ short Hs[kSub][64];
  __shared__ short Gs[kSub][64];
  const int lane = threadIdx.x & 63, q = lane >> 4, r = lane & 15, wv = threadIdx.x >> 6;
  const int chunk = blockIdx.x >> 2, layer = blockIdx.x & 3;
  const int64_t c0 = (int64_t)chunk * kChunk;
  const int64_t c1 = c0 + kChunk < B ? c0 + kChunk : B;
  const int K = layer == 0 ? 6 : 64, M = layer == 3 ? 2 : 64;
  const int KT = layer == 0 ? 1 : 4, MT = layer == 3 ? 1 : 4;       // input and output tiles
  const int njobs = KT * MT + MT;                                   // weight tiles, then bias tiles
  const int ldh = layer == 0 ? 16 : 64;
  const short* H = layer == 0 ? tb.h0 : tb.h[layer - 1];
  f32x4 acc[5];
#pragma unroll
  for (int u = 0; u < 5; ++u) acc[u] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int64_t s0 = c0; s0 < c1; s0 += kSub) {
    // stage: thread t loads 16 consecutive features of one sample row
    {
      const int row = threadIdx.x >> 2, part16 = (threadIdx.x & 3) * 16;
      const int64_t s = s0 + row;
      const bool ok = s < c1;
      for (int k = 0; k < 16; ++k) {
        const int col = part16 + k;
        Hs[row][col] = (ok && col < ldh) ? H[s * ldh + col] : (short)0;
        short g = 0;
        if (ok) {
          if (layer == 3) g = col < 2 ? f2bf(tb.g4[2 * s + col]) : (short)0;
          else g = tb.g[layer][s * 64 + col];
        }
        Gs[row][col] = g;
      }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 5; ++u) {
      const int j = wv + 4 * u;
      if (j >= njobs) break;
      const bool bias = j >= KT * MT;
      const int kt = bias ? 0 : j / MT, mt = bias ? j - KT * MT : j % MT;
#pragma unroll
      for (int t = 0; t < kSub / 32; ++t) {
        bf16x8 a, b;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const int sr = 32 * t + 8 * q + j;
          a[j] = bias ? (short)0x3F80 : Hs[sr][16 * kt + r];   // 0x3F80 = 1.0
          b[j] = Gs[sr][16 * mt + r];
        }
        acc[u] = mfma32(a, b, acc[u]);
      }
    }
    __syncthreads();
  }
  // D[row][col]: row 4q + i of the tile, column r
  float* out = part + (int64_t)chunk * kNParams;
  const int offW = layer == 0 ? kW1 : layer == 1 ? kW2 : layer == 2 ? kW3 : kW4;
  const int offB = layer == 0 ? kB1 : layer == 1 ? kB2 : layer == 2 ? kB3 : kB4;
#pragma unroll
  for (int u = 0; u < 5; ++u) {
    const int j = wv + 4 * u;
    if (j >= njobs) break;
    const bool bias = j >= KT * MT;
    const int kt = bias ? 0 : j / MT, mt = bias ? j - KT * MT : j % MT;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int row = 4 * q + i, m = 16 * mt + r;
      if (m >= M) continue;
      if (bias) {
        if (row == 0) out[offB + m] = acc[u][i];
      } else {
        const int k = 16 * kt + row;
        if (k < K) out[offW + k * M + m] = acc[u][i];
      }
    }
  }
}

// fixed-order sum of the squared errors (one block)
__global__ __launch_bounds__(256) void k_mlp_loss(const float* err, int64_t B, float* loss) {
  __shared__ float sh[256];
  float a = 0.f;
  for (int64_t s = threadIdx.x; s < B; s += 256) a += err[s];
  sh[threadIdx.x] = a;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss = sh[0] / (2.0f * (float)B);
}

// gradient = fixed-order sum over chunks; optional Adam step on the FP32
// master parameters, then the BF16 copy
__global__ void k_mlp_reduce_adam(const float* part, int nchunk, float* grad, float* p, float* m, float* v,
                                  short* wb, int do_adam, float lr, float bc1, float bc2) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= kNParams) return;
  // chunk partials in order; eight loads in flight per round
  float g = 0.f;
  int c = 0;
  for (; c + 8 <= nchunk; c += 8) {
    float v8[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v8[u] = part[(int64_t)(c + u) * kNParams + k];
#pragma unroll
    for (int u = 0; u < 8; ++u) g += v8[u];
  }
  for (; c < nchunk; ++c) g += part[(int64_t)c * kNParams + k];
  grad[k] = g;
  if (!do_adam) return;
  const float mk = 0.9f * m[k] + 0.1f * g;
  const float vk = 0.999f * v[k] + 0.001f * g * g;
  m[k] = mk;
  v[k] = vk;
  const float pk = p[k] - lr * (mk / bc1) / (sqrtf(vk / bc2) + 1e-8f);
  p[k] = pk;
  wb[k] = f2bf(pk);
}

__global__ void k_mlp_to_bf16(const float* p, short* wb) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < kNParams) wb[k] = f2bf(p[k]);
}

// ---------------------------------------------------------------------------
// closure inference inside the DEM: features (FP64, n x 6) -> normalised ->
// network -> factors c = exp(clip(y, -ln 2, ln 2)) into cdrag, ccoh
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_closure_infer(const DevState* __restrict__ dp) {
  const DevState& d = *dp;
  if (*d.abort) return;
  const int lane = threadIdx.x & 63, q = lane >> 4, r = lane & 15;
  const int64_t nt = (d.n + 15) / 16;
  const int64_t w0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
  const short* wb = (const short*)d.cl_wb;
  const float* pf = d.cl_pf;
  MlpTrainBuf none{};
  const float L2 = 0.69314718055994531f;
  const WeightFrags W = load_frags(wb, pf, q, r);
  for (int64_t t = w0; t < nt; t += nw) {
    const int64_t s = t * 16 + r;
    bf16x4 a;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      int k = 4 * q + i;
      a[i] = (s < d.n && k < 6) ? f2bf((float)((d.cfeat[6 * s + k] - d.cl_norm[k]) / d.cl_norm[6 + k]))
                                : (short)0;
    }
    f32x4 y = forward_tile<false>(W, a, q, r, t * 16, d.n, none);
    if (q == 0 && s < d.n) {
      float y0 = fminf(fmaxf(y[0], -L2), L2), y1 = fminf(fmaxf(y[1], -L2), L2);
      d.cdrag[s] = (double)expf(y0);
      d.ccoh[s] = (double)expf(y1);
    }
  }
}

// blocks of 4 wavefronts, a tile of 16 samples per wavefront and round; at
// most 4 wavefronts per SIMD, so that each keeps its weight fragments over
// several tiles
inline int mlp_grid(int64_t B) {
  int64_t tiles = (B + 15) / 16;
  int64_t blocks = (tiles + 3) / 4;
  return (int)std::max<int64_t>(1, std::min<int64_t>(blocks, 1024));
}

void launch_closure_infer(DevState& d, hipStream_t s) {
  if (d.n > 0) hipLaunchKernelGGL(k_closure_infer, dim3((unsigned)mlp_grid(d.n)), dim3(256), 0, s, d.self);
}

}  // namespace dem

// ---------------------------------------------------------------------------
// C-ABI: the network object
// ---------------------------------------------------------------------------
using namespace dem;

struct dem_mlp {
  int device = 0;
  hipStream_t stream = nullptr;
  float *p = nullptr, *m = nullptr, *v = nullptr, *grad = nullptr, *loss = nullptr;
  short* wb = nullptr;
  int64_t step = 0;
  int64_t cap = 0;            // batch capacity of the training buffers
  MlpTrainBuf tb{};
  float* part = nullptr;
  int64_t part_chunks = 0;
  std::vector<void*> batch_allocs;
};

namespace {
void free_batch(dem_mlp* n) {
  for (void* q : n->batch_allocs) (void)hipFree(q);
  n->batch_allocs.clear();
  n->tb = MlpTrainBuf{};
  n->part = nullptr;
  n->cap = 0;
}
template <typename T> hipError_t balloc(dem_mlp* n, T** q, int64_t count) {
  hipError_t e = hipMalloc((void**)q, sizeof(T) * (size_t)(count > 0 ? count : 1));
  if (e == hipSuccess) n->batch_allocs.push_back((void*)*q);
  return e;
}
dem_status ensure_batch(dem_mlp* n, int64_t B) {
  if (B <= n->cap) return DEM_OK;
  if (hipStreamSynchronize(n->stream) != hipSuccess) return DEM_E_DEVICE;
  free_batch(n);
  int64_t cap = std::max<int64_t>(B, 1024);
  int64_t nch = (cap + kChunk - 1) / kChunk;
  bool ok = balloc(n, &n->tb.h0, cap * 16) == hipSuccess;
  for (int l = 0; l < 3; ++l) {
    ok &= balloc(n, &n->tb.h[l], cap * 64) == hipSuccess;
    ok &= balloc(n, &n->tb.z[l], cap * 64) == hipSuccess;
    ok &= balloc(n, &n->tb.g[l], cap * 64) == hipSuccess;
  }
  ok &= balloc(n, &n->tb.g4, cap * 2) == hipSuccess;
  ok &= balloc(n, &n->tb.err, cap) == hipSuccess;
  ok &= balloc(n, &n->part, nch * kNParams) == hipSuccess;
  if (!ok) {
    free_batch(n);
    return DEM_E_NOMEM;
  }
  n->cap = cap;
  n->part_chunks = nch;
  return DEM_OK;
}
int grid_for(int64_t B) { return mlp_grid(B); }
// forward + backward + chunk gradients + fixed-order reduction (+ Adam), with
// the batch buffers tb and the chunk partials `part` given (every location
// read is written earlier in the same pass: nothing needs clearing)
dem_status train_pass_bufs(dem_mlp* n, const float* x, const float* t, int64_t B, int adam, float lr,
                           float* loss_host, const MlpTrainBuf& tb, float* part) {
  hipStream_t s = n->stream;
  int g = grid_for(B);
  hipLaunchKernelGGL(k_mlp_forward_train, dim3(g), dim3(256), 0, s, n->wb, n->p, x, t, B, tb);
  hipLaunchKernelGGL(k_mlp_backward, dim3(g), dim3(256), 0, s, n->wb, B, tb);
  int nch = (int)((B + kChunk - 1) / kChunk);
  hipLaunchKernelGGL(k_mlp_wgrad, dim3(4 * nch), dim3(256), 0, s, B, tb, part);
  hipLaunchKernelGGL(k_mlp_loss, dim3(1), dim3(256), 0, s, tb.err, B, n->loss);
  float bc1 = 1.f, bc2 = 1.f;
  if (adam) {
    n->step += 1;
    bc1 = (float)(1.0 - std::pow(0.9, (double)n->step));
    bc2 = (float)(1.0 - std::pow(0.999, (double)n->step));
  }
  hipLaunchKernelGGL(k_mlp_reduce_adam, dim3((kNParams + 255) / 256), dim3(256), 0, s, part, nch, n->grad, n->p,
                     n->m, n->v, n->wb, adam, lr, bc1, bc2);
  if (hipGetLastError() != hipSuccess) return DEM_E_DEVICE;
  if (loss_host) {
    if (hipMemcpyAsync(loss_host, n->loss, sizeof(float), hipMemcpyDeviceToHost, s) != hipSuccess) return DEM_E_DEVICE;
    if (hipStreamSynchronize(s) != hipSuccess) return DEM_E_DEVICE;
  }
  return DEM_OK;
}

// the same pass with buffers the network object owns (grown on demand)
dem_status train_pass(dem_mlp* n, const float* x, const float* t, int64_t B, int adam, float lr, float* loss_host) {
  if (!n || !x || !t || B <= 0) return DEM_E_INVAL;
  if (hipSetDevice(n->device) != hipSuccess) return DEM_E_DEVICE;
  dem_status st = ensure_batch(n, B);
  if (st != DEM_OK) return st;
  return train_pass_bufs(n, x, t, B, adam, lr, loss_host, n->tb, n->part);
}

// ---------------------------------------------------------------------------
// Scratch of the training step that allocates nothing: the batch buffers for
// up to DEM_MLP_NOALLOC_MAX_BATCH samples and their chunk partials, in one
// file-scope device array.  Each GPU holds its own copy at its own address,
// looked up once per device (hipGetSymbolAddress) when a network is created
// there; host code uses only that address, never the array's name.
// ---------------------------------------------------------------------------
constexpr int64_t kNoAllocBatch = DEM_MLP_NOALLOC_MAX_BATCH;
constexpr int64_t kNoAllocChunks = (kNoAllocBatch + kChunk - 1) / kChunk;
constexpr size_t al256(size_t b) { return (b + 255) / 256 * 256; }
constexpr size_t kScrH0 = al256(sizeof(short) * kNoAllocBatch * 16);
constexpr size_t kScrH = al256(sizeof(short) * kNoAllocBatch * 64);
constexpr size_t kScrZ = al256(sizeof(float) * kNoAllocBatch * 64);
constexpr size_t kScrG4 = al256(sizeof(float) * kNoAllocBatch * 2);
constexpr size_t kScrErr = al256(sizeof(float) * kNoAllocBatch);
constexpr size_t kScrPart = al256(sizeof(float) * kNoAllocChunks * kNParams);
constexpr size_t kScratchBytes = kScrH0 + 3 * (kScrH + kScrZ + kScrH) + kScrG4 + kScrErr + kScrPart;

static __device__ __align__(256) char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
char* g_scratch[kMaxDevices] = {};   // device address of `scratch` on each device (null: not looked up)
std::mutex g_scratch_mu;

// with `device` current
dem_status scratch_lookup(int device) {
  if (device < 0 || device >= kMaxDevices) return DEM_E_DEVICE;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch[device]) return DEM_OK;
  void* ptr = nullptr;
  if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return DEM_E_DEVICE;
  g_scratch[device] = (char*)ptr;
  return DEM_OK;
}

void scratch_buffers(char* base, MlpTrainBuf& tb, float*& part) {
  char* q = base;
  tb.h0 = (short*)q; q += kScrH0;
  for (int l = 0; l < 3; ++l) {
    tb.h[l] = (short*)q; q += kScrH;
    tb.z[l] = (float*)q; q += kScrZ;
    tb.g[l] = (short*)q; q += kScrH;
  }
  tb.g4 = (float*)q; q += kScrG4;
  tb.err = (float*)q; q += kScrErr;
  part = (float*)q;
}
}  // namespace

namespace dem {
const short* mlp_weights_bf16(const dem_mlp* n) { return n ? n->wb : nullptr; }
const float* mlp_params_f32(const dem_mlp* n) { return n ? n->p : nullptr; }
hipStream_t mlp_stream(const dem_mlp* n) { return n ? n->stream : nullptr; }
}  // namespace dem

extern "C" {

dem_status dem_mlp_create(dem_mlp** out, int32_t device, void* hip_stream) {
  if (!out) return DEM_E_INVAL;
  *out = nullptr;
  if (hipSetDevice(device) != hipSuccess) return DEM_E_DEVICE;
  dem_mlp* n = new dem_mlp();
  n->device = device;
  n->stream = (hipStream_t)hip_stream;
  if (scratch_lookup(device) != DEM_OK) {
    delete n;
    return DEM_E_DEVICE;
  }
  bool ok = hipMalloc((void**)&n->p, sizeof(float) * kNParams) == hipSuccess;
  ok &= hipMalloc((void**)&n->m, sizeof(float) * kNParams) == hipSuccess;
  ok &= hipMalloc((void**)&n->v, sizeof(float) * kNParams) == hipSuccess;
  ok &= hipMalloc((void**)&n->grad, sizeof(float) * kNParams) == hipSuccess;
  ok &= hipMalloc((void**)&n->loss, sizeof(float)) == hipSuccess;
  ok &= hipMalloc((void**)&n->wb, sizeof(short) * kNParams) == hipSuccess;
  if (!ok) {
    dem_mlp_destroy(n);
    return DEM_E_NOMEM;
  }
  ok &= hipMemsetAsync(n->p, 0, sizeof(float) * kNParams, n->stream) == hipSuccess;
  ok &= hipMemsetAsync(n->m, 0, sizeof(float) * kNParams, n->stream) == hipSuccess;
  ok &= hipMemsetAsync(n->v, 0, sizeof(float) * kNParams, n->stream) == hipSuccess;
  ok &= hipMemsetAsync(n->wb, 0, sizeof(short) * kNParams, n->stream) == hipSuccess;
  if (!ok) {
    dem_mlp_destroy(n);
    return DEM_E_DEVICE;
  }
  *out = n;
  return DEM_OK;
}

void dem_mlp_destroy(dem_mlp* n) {
  if (!n) return;
  (void)hipSetDevice(n->device);
  (void)hipStreamSynchronize(n->stream);
  free_batch(n);
  (void)hipFree(n->p); (void)hipFree(n->m); (void)hipFree(n->v);
  (void)hipFree(n->grad); (void)hipFree(n->loss); (void)hipFree(n->wb);
  delete n;
}

dem_status dem_mlp_set_params(dem_mlp* n, const float* params) {
  if (!n || !params) return DEM_E_INVAL;
  if (hipSetDevice(n->device) != hipSuccess) return DEM_E_DEVICE;
  hipStream_t s = n->stream;
  if (hipMemcpyAsync(n->p, params, sizeof(float) * kNParams, hipMemcpyDefault, s) != hipSuccess) return DEM_E_DEVICE;
  if (hipMemsetAsync(n->m, 0, sizeof(float) * kNParams, s) != hipSuccess) return DEM_E_DEVICE;
  if (hipMemsetAsync(n->v, 0, sizeof(float) * kNParams, s) != hipSuccess) return DEM_E_DEVICE;
  n->step = 0;
  hipLaunchKernelGGL(k_mlp_to_bf16, dim3((kNParams + 255) / 256), dim3(256), 0, s, n->p, n->wb);
  if (hipStreamSynchronize(s) != hipSuccess) return DEM_E_DEVICE;
  return DEM_OK;
}

dem_status dem_mlp_get_params(dem_mlp* n, float* params) {
  if (!n || !params) return DEM_E_INVAL;
  if (hipSetDevice(n->device) != hipSuccess) return DEM_E_DEVICE;
  if (hipMemcpyAsync(params, n->p, sizeof(float) * kNParams, hipMemcpyDefault, n->stream) != hipSuccess)
    return DEM_E_DEVICE;
  if (hipStreamSynchronize(n->stream) != hipSuccess) return DEM_E_DEVICE;
  return DEM_OK;
}

dem_status dem_mlp_forward(dem_mlp* n, const float* x, float* y, int64_t batch) {
  if (!n || batch < 0 || (batch > 0 && (!x || !y))) return DEM_E_INVAL;
  if (batch == 0) return DEM_OK;
  if (hipSetDevice(n->device) != hipSuccess) return DEM_E_DEVICE;
  hipLaunchKernelGGL(k_mlp_forward, dim3(grid_for(batch)), dim3(256), 0, n->stream, n->wb, n->p, x, batch, y);
  return hipGetLastError() == hipSuccess ? DEM_OK : DEM_E_DEVICE;
}

dem_status dem_mlp_grad(dem_mlp* n, const float* x, const float* t, int64_t batch, float* grad, float* loss) {
  dem_status st = train_pass(n, x, t, batch, 0, 0.f, loss);
  if (st != DEM_OK) return st;
  if (grad) {
    if (hipMemcpyAsync(grad, n->grad, sizeof(float) * kNParams, hipMemcpyDefault, n->stream) != hipSuccess)
      return DEM_E_DEVICE;
    if (hipStreamSynchronize(n->stream) != hipSuccess) return DEM_E_DEVICE;
  }
  return DEM_OK;
}

dem_status dem_mlp_train_step(dem_mlp* n, const float* x, const float* t, int64_t batch, float lr, float* loss) {
  if (!(lr > 0.f)) return DEM_E_INVAL;
  return train_pass(n, x, t, batch, 1, lr, loss);
}

dem_status dem_mlp_train_step_noalloc(dem_mlp* n, const float* x, const float* t, int64_t batch, float lr,
                                      float* loss) {
  if (!n || !x || !t || batch <= 0 || batch > DEM_MLP_NOALLOC_MAX_BATCH || !(lr > 0.f)) return DEM_E_INVAL;
  if (n->device < 0 || n->device >= kMaxDevices) return DEM_E_DEVICE;
  if (hipSetDevice(n->device) != hipSuccess) return DEM_E_DEVICE;
  char* base = g_scratch[n->device];   // looked up when the network was created on this device
  if (!base) return DEM_E_DEVICE;
  MlpTrainBuf tb{};
  float* part = nullptr;
  scratch_buffers(base, tb, part);
  return train_pass_bufs(n, x, t, batch, 1, lr, loss, tb, part);
}

}  // extern "C"
