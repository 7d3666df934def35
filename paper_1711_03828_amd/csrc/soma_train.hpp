// soma_train.hpp -- training of the learned proposal's network on the matrix
// cores: forward, Gaussian negative log-likelihood of observed displacements,
// back-propagation and Adam, all with BF16 MFMA inputs and FP32 accumulation.
//
// One wavefront (a 64-thread block) handles chunks of 64 samples (lane =
// sample).  Every matrix product is a v_mfma_f32_16x16x32_bf16 tile: the
// forward and the error propagation contract over units (activations and
// errors in sample-major LDS tiles are the B operand), the weight gradients
// contract over the 64 samples of a chunk (unit-major, transposed LDS tiles).
// Gradients accumulate in registers over all chunks of the wave and are
// written once as a per-wave partial; a second kernel sums the partials in a
// fixed order and applies Adam to the FP32 master parameters.
#pragma once

#include "soma_mlp.hpp"

namespace soma {

constexpr int kTStride = 72;  // bf16 per row of a transposed (unit-major) tile

struct TrainArgs {
  const NetDev *net;
  const float *feat;     // [n][60] raw features
  const float *target;   // [n][3] displacements
  uint32_t n;
  HeadArgs head;
  float *partials;       // [waves][kPSize] gradient partials (sums over samples)
  float *loss_partials;  // [waves]
};

__device__ __forceinline__ bf16x8 lds8(const __bf16 *p) { return *reinterpret_cast<const bf16x8 *>(p); }

__device__ __forceinline__ float drelu(float a) { return a > 0.0f ? 1.0f : 0.0f; }

// out[mt][t] += W[16 mt + row][k] * act[sample][k] over K = 64 (two blocks):
// rows of W (global, [64][64] bf16), act sample-major LDS [64][72].
__device__ __forceinline__ void mm_units(const __bf16 *__restrict__ w, int w_stride, int m_tiles,
                                         int k_blocks, const __bf16 *act, f32x4 (&acc)[4][4]) {
  const int lane = threadIdx.x & 63, col = lane & 15, g = lane >> 4;
  for (int kb = 0; kb < k_blocks; ++kb) {
    bf16x8 b[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) b[t] = lds8(act + (16 * t + col) * kActStride + 32 * kb + 8 * g);
    for (int mt = 0; mt < m_tiles; ++mt) {
      const bf16x8 av = *reinterpret_cast<const bf16x8 *>(w + (16 * mt + col) * w_stride + 32 * kb + 8 * g);
#pragma unroll
      for (int t = 0; t < 4; ++t)
        acc[mt][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, b[t], acc[mt][t], 0, 0, 0);
    }
  }
}

// acc[mt][nt] += A[16 mt + row][s] * B[16 nt + col][s] over the 64 samples s,
// both unit-major LDS tiles [units][kTStride].
__device__ __forceinline__ void mm_samples(const __bf16 *a_t, int m_tiles, const __bf16 *b_t,
                                           int n_tiles, f32x4 (&acc)[4][4]) {
  const int lane = threadIdx.x & 63, col = lane & 15, g = lane >> 4;
#pragma unroll
  for (int kb = 0; kb < 2; ++kb) {
    bf16x8 b[4];
    for (int nt = 0; nt < n_tiles; ++nt) b[nt] = lds8(b_t + (16 * nt + col) * kTStride + 32 * kb + 8 * g);
    for (int mt = 0; mt < m_tiles; ++mt) {
      const bf16x8 av = lds8(a_t + (16 * mt + col) * kTStride + 32 * kb + 8 * g);
      for (int nt = 0; nt < n_tiles; ++nt)
        acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, b[nt], acc[mt][nt], 0, 0, 0);
    }
  }
}

__device__ __forceinline__ void zero_acc(f32x4 (&acc)[4][4]) {
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
}

__global__ __launch_bounds__(64) void mlp_grad_kernel(const TrainArgs a) {
  __shared__ __bf16 x_s[64 * kActStride], h1_s[64 * kActStride], h2_s[64 * kActStride];
  __shared__ __bf16 d2_s[64 * kActStride];
  __shared__ __bf16 x_t[64 * kTStride], h1_t[64 * kTStride], h2_t[64 * kTStride];
  __shared__ __bf16 d1_t[64 * kTStride], d2_t[64 * kTStride], dz_t[16 * kTStride];
  __shared__ __bf16 dz_s[64 * 32];
  __shared__ float a1_f[64 * 64], a2_f[64 * 64], z_f[64 * 8];
  const int lane = threadIdx.x & 63, col = lane & 15, g = lane >> 4;
  const NetDev *net = a.net;

  f32x4 gw1[4][4], gw2[4][4], gw3[4][4];
  zero_acc(gw1);
  zero_acc(gw2);
  zero_acc(gw3);
  float gb1[4][4], gb2[4][4], gb3[kNO] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f}, loss = 0.0f;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) gb1[i][j] = gb2[i][j] = 0.0f;

  const uint32_t n_chunks = (a.n + 63u) / 64u;
  for (uint32_t chunk = blockIdx.x; chunk < n_chunks; chunk += gridDim.x) {
    const uint32_t s = chunk * 64u + (uint32_t)lane;
    const bool valid = s < a.n;
    // standardised inputs, sample-major and unit-major
    for (int k = 0; k < 64; ++k) {
      const float raw = (valid && k < kNF) ? a.feat[(size_t)s * kNF + k] : 0.0f;
      const __bf16 v = k < kNF ? (__bf16)((raw - net->shift[k]) * net->scale[k]) : (__bf16)0.0f;
      x_s[lane * kActStride + k] = v;
      x_t[k * kTStride + lane] = v;
    }
    // layer 1
    f32x4 acc[4][4];
    zero_acc(acc);
    mm_units(net->w1, 64, 4, 2, x_s, acc);
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int u = 16 * mt + 4 * g + r, sm = 16 * t + col;
          const float pre = acc[mt][t][r] + net->b1[u];
          const __bf16 h = (__bf16)relu(pre);
          a1_f[sm * 64 + u] = pre;
          h1_s[sm * kActStride + u] = h;
          h1_t[u * kTStride + sm] = h;
        }
    // layer 2
    zero_acc(acc);
    mm_units(net->w2, 64, 4, 2, h1_s, acc);
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int u = 16 * mt + 4 * g + r, sm = 16 * t + col;
          const float pre = acc[mt][t][r] + net->b2[u];
          const __bf16 h = (__bf16)relu(pre);
          a2_f[sm * 64 + u] = pre;
          h2_s[sm * kActStride + u] = h;
          h2_t[u * kTStride + sm] = h;
        }
    // layer 3 -> z (rows 0..5 of one M tile)
    zero_acc(acc);
    mm_units(net->w3, 64, 1, 2, h2_s, acc);
    if (g < 2)
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) z_f[(16 * t + col) * 8 + 4 * g + r] = acc[0][t][r] + net->b3[4 * g + r];
    // loss and dL/dz of this lane's sample
    float dz[kNO];
    {
      const float *z = z_f + lane * 8;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const float tgt = valid ? a.target[(size_t)s * 3 + d] : 0.0f;
        const float mu = a.head.m_max * tanhf(z[d] / a.head.m_max);
        const float sg = fast_rcp(1.0f + __expf(-z[3 + d]));
        const float ls = a.head.lo + (a.head.hi - a.head.lo) * sg;
        const float inv_var = __expf(-2.0f * ls);
        const float e = tgt - mu;
        if (valid) loss += 0.5f * e * e * inv_var + ls;
        const float dmu = -e * inv_var, dls = 1.0f - e * e * inv_var;
        dz[d] = valid ? dmu * (1.0f - (mu / a.head.m_max) * (mu / a.head.m_max)) : 0.0f;
        dz[3 + d] = valid ? dls * (a.head.hi - a.head.lo) * sg * (1.0f - sg) : 0.0f;
      }
    }
    for (int k = 0; k < 32; ++k) {
      const __bf16 v = k < kNO ? (__bf16)dz[k < kNO ? k : 0] : (__bf16)0.0f;
      dz_s[lane * 32 + k] = v;
      if (k < 16) dz_t[k * kTStride + lane] = v;
    }
    // output-bias gradient: FP32 sum of dz over the chunk's samples
#pragma unroll
    for (int o = 0; o < kNO; ++o) {
      float v = dz[o];
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
      gb3[o] += v;
    }
    // delta2 = (W3^T dz) * relu'(a2)
    zero_acc(acc);
    {
      // K = 32 (6 used): one block; B operand from dz_s rows
      bf16x8 b[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) b[t] = lds8(dz_s + (16 * t + col) * 32 + 8 * g);
#pragma unroll
      for (int mt = 0; mt < 4; ++mt) {
        const bf16x8 av = *reinterpret_cast<const bf16x8 *>(net->w3t + (16 * mt + col) * 32 + 8 * g);
#pragma unroll
        for (int t = 0; t < 4; ++t)
          acc[mt][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, b[t], acc[mt][t], 0, 0, 0);
      }
    }
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int u = 16 * mt + 4 * g + r, sm = 16 * t + col;
          const float d = acc[mt][t][r] * drelu(a2_f[sm * 64 + u]);
          gb2[mt][r] += d;
          const __bf16 db = (__bf16)d;
          d2_s[sm * kActStride + u] = db;
          d2_t[u * kTStride + sm] = db;
        }
    // delta1 = (W2^T delta2) * relu'(a1)
    zero_acc(acc);
    mm_units(net->w2t, 64, 4, 2, d2_s, acc);
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int u = 16 * mt + 4 * g + r, sm = 16 * t + col;
          const float d = acc[mt][t][r] * drelu(a1_f[sm * 64 + u]);
          gb1[mt][r] += d;
          d1_t[u * kTStride + sm] = (__bf16)d;
        }
    // weight gradients, contracted over the chunk's samples
    mm_samples(d1_t, 4, x_t, 4, gw1);
    mm_samples(d2_t, 4, h1_t, 4, gw2);
    mm_samples(dz_t, 1, h2_t, 4, gw3);
  }

  // write this wave's partial gradient in the parameter layout
  float *out = a.partials + (size_t)blockIdx.x * kPSize;
#pragma unroll
  for (int mt = 0; mt < 4; ++mt)
#pragma unroll
    for (int nt = 0; nt < 4; ++nt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int o = 16 * mt + 4 * g + r, i = 16 * nt + col;
        if (i < kNF) out[kPW1 + o * kNF + i] = gw1[mt][nt][r];
        out[kPW2 + o * kNH + i] = gw2[mt][nt][r];
        if (mt == 0 && o < kNO) out[kPW3 + o * kNH + i] = gw3[0][nt][r];
      }
  // bias partials: sum the per-lane values over the 16 lanes sharing g
#pragma unroll
  for (int mt = 0; mt < 4; ++mt)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      float v1 = gb1[mt][r], v2 = gb2[mt][r];
#pragma unroll
      for (int off = 8; off > 0; off >>= 1) {
        v1 += __shfl_xor(v1, off, 16);
        v2 += __shfl_xor(v2, off, 16);
      }
      if (col == 0) {
        out[kPB1 + 16 * mt + 4 * g + r] = v1;
        out[kPB2 + 16 * mt + 4 * g + r] = v2;
      }
    }
#pragma unroll
  for (int o = 0; o < kNO; ++o)
    if (lane == o) out[kPB3 + o] = gb3[o];
  if (lane < kPW1) out[lane] = 0.0f;       // no gradient for the standardisation
  if (lane + 64 < kPW1) out[lane + 64] = 0.0f;
  if (lane < kPSize - kPB3 - kNO) out[kPB3 + kNO + lane] = 0.0f;
  // loss partial
  for (int off = 32; off > 0; off >>= 1) loss += __shfl_down(loss, off, 64);
  if (lane == 0) a.loss_partials[blockIdx.x] = loss;
}

struct AdamArgs {
  const float *partials;
  const float *loss_partials;
  uint32_t waves, n;
  float *params, *m, *v;
  float lr, beta1, beta2, eps;
  float bc1, bc2;        // 1 - beta^t
  int apply;
  float *grad_out;       // may be null
  float *loss_out;       // may be null
};

// Mean gradient over the batch and the Adam step on the FP32 master
// parameters (standardisation constants untouched).  A block covers 64
// parameters; its four waves sum the partials of waves q, q+4, q+8, ... (q the
// wave in the block), eight loads in flight, and the four sums are combined
// in a fixed order: the result does not depend on timing.
constexpr uint32_t kAdamParamsPerBlock = 64;

__global__ __launch_bounds__(256) void mlp_adam_kernel(const AdamArgs a) {
  __shared__ float s_part[4][kAdamParamsPerBlock];
  const uint32_t lane = threadIdx.x & 63u, q = threadIdx.x >> 6;
  const uint32_t p = blockIdx.x * kAdamParamsPerBlock + lane;
  float gsum = 0.0f;
  if (p < (uint32_t)kPSize) {
    float acc[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    uint32_t w = q;
    for (; w + 28u < a.waves; w += 32u) {
#pragma unroll
      for (int u = 0; u < 8; ++u) acc[u] += a.partials[(size_t)(w + 4u * u) * kPSize + p];
    }
    for (; w < a.waves; w += 4u) acc[0] += a.partials[(size_t)w * kPSize + p];
    gsum = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
  }
  s_part[q][lane] = gsum;
  __syncthreads();
  if (blockIdx.x == 0 && threadIdx.x == 64 && a.loss_out) {
    float l = 0.0f;
    for (uint32_t w = 0; w < a.waves; ++w) l += a.loss_partials[w];
    *a.loss_out = l / (float)a.n;
  }
  if (q != 0 || p >= (uint32_t)kPSize) return;
  const float grad = ((s_part[0][lane] + s_part[1][lane]) + (s_part[2][lane] + s_part[3][lane])) /
                     (float)a.n;
  if (a.grad_out) a.grad_out[p] = grad;
  if (!a.apply || p < (uint32_t)kPW1 || p >= (uint32_t)(kPB3 + kNO)) return;
  const float m = a.beta1 * a.m[p] + (1.0f - a.beta1) * grad;
  const float v = a.beta2 * a.v[p] + (1.0f - a.beta2) * grad * grad;
  a.m[p] = m;
  a.v[p] = v;
  a.params[p] -= a.lr * (m / a.bc1) / (sqrtf(v / a.bc2) + a.eps);
}

}  // namespace soma
