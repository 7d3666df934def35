// soma_mlp.hpp -- the learned proposal's network on the gfx950 matrix cores.
//
// A learned move proposes r' = r + mu(r) + sigma(r) xi from a small network
// (60 -> 64 -> 64 -> 6, ReLU) fed with the fields around the bead and its two
// bond vectors, and is accepted by Metropolis-Hastings with the exact ratio
// of the Gaussian proposal densities, so the sampled distribution of the
// method (Sec. 2.2) is unchanged; the move is an addition to the paper's local
// and smart-MC moves.
//
// One wavefront evaluates the network for 64 samples (its 64 lanes) with
// v_mfma_f32_16x16x32_bf16: activations are the B operand (K = units, N =
// samples), weights the A operand (M = output units); BF16 inputs, FP32
// accumulation.  The input features come from a per-wave LDS tile
// [64 samples][72] bf16 in natural unit order; the hidden activations stay
// in registers: an output tile of one layer becomes the next layer's B
// operand through the gfx950 lane swaps (v_permlane32_swap,
// v_permlane16_swap), without a trip through LDS.
#pragma once

#include "soma_device.hpp"

namespace soma {

constexpr int kNF = 60, kNH = 64, kNO = 6;
// FP32 parameter blob (interface format): shift[60] scale[60] W1[64][60] b1[64]
// W2[64][64] b2[64] W3[6][64] b3[6], padded to 8576 floats.
constexpr int kPShift = 0, kPScale = 60, kPW1 = 120, kPB1 = 3960, kPW2 = 4024, kPB2 = 8120,
              kPW3 = 8184, kPB3 = 8568, kPSize = 8576;
constexpr int kActStride = 72;  // bf16 per LDS row: 64 units + 8 padding

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// Device copy of the network, ready for the MFMA tiles.  The learned move
// evaluates the first layer with the input standardisation folded in (w1f,
// b1f: W1'[o][k] = W1[o][k] scale[k], b1'[o] = b1[o] - sum_k W1'[o][k] shift[k]
// in FP32, k ascending), so raw features go straight to BF16; training uses
// the standardised form (shift, scale, w1, b1).
struct NetDev {
  float shift[64], scale[64];  // entries 60..63: shift 0, scale 0 (feature 0)
  float b1[64], b2[64], b3[16];
  __bf16 w1[64 * 64];          // [out][in], in >= 60 zero
  __bf16 w2[64 * 64];          // [out][in]
  __bf16 w3[16 * 64];          // rows >= 6 zero
  __bf16 w2t[64 * 64];         // W2 transposed: [in][out]
  __bf16 w3t[64 * 32];         // [hidden][k]: W3[k][hidden] for k < 6, else 0
  float b1f[64];               // folded first-layer bias
  __bf16 w1f[64 * 64];         // folded first-layer weights [out][in], in >= 60 zero
};

struct HeadArgs {
  float m_max, lo, hi;         // mu = m tanh(z/m); log sigma = lo + (hi-lo) sigmoid(z)
};

// One thread per weight index i < 64*64 (launched with kNetPrepareBlocks
// blocks of 256 threads).
constexpr uint32_t kNetPrepareBlocks = 16;

__global__ __launch_bounds__(256) void net_prepare_kernel(const float *__restrict__ p,
                                                          NetDev *__restrict__ net) {
  const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (i >= 64 * 64) return;
  if (i < 64) {
    net->shift[i] = i < kNF ? p[kPShift + i] : 0.0f;
    net->scale[i] = i < kNF ? p[kPScale + i] : 0.0f;
    net->b1[i] = p[kPB1 + i];
    net->b2[i] = p[kPB2 + i];
    if (i < 16) net->b3[i] = i < kNO ? p[kPB3 + i] : 0.0f;
    float b = p[kPB1 + i];   // folded bias of unit i (built without FP contraction)
    for (int k = 0; k < kNF; ++k) {
      const float w = p[kPW1 + i * kNF + k] * p[kPScale + k];
      const float t = w * p[kPShift + k];
      b = b - t;
    }
    net->b1f[i] = b;
  }
  const int o = i >> 6, k = i & 63;
  net->w1[i] = (__bf16)(k < kNF ? p[kPW1 + o * kNF + k] : 0.0f);
  net->w1f[i] = (__bf16)(k < kNF ? p[kPW1 + o * kNF + k] * p[kPScale + k] : 0.0f);
  net->w2[i] = (__bf16)p[kPW2 + o * kNH + k];
  net->w2t[i] = (__bf16)p[kPW2 + k * kNH + o];
  if (o < 16) net->w3[i] = (__bf16)(o < kNO ? p[kPW3 + o * kNH + k] : 0.0f);
  if (i < 64 * 32) {
    const int h = i >> 5, kk = i & 31;
    net->w3t[i] = (__bf16)(kk < kNO ? p[kPW3 + kk * kNH + h] : 0.0f);
  }
}

// Hardware reciprocal (1 ulp): ample where the result feeds a bfloat16 tile
// or a Metropolis-Hastings log ratio.
__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
// Hidden activation: ReLU (one VALU operation per unit).
__device__ __forceinline__ float relu(float a) { return fmaxf(a, 0.0f); }

__device__ __forceinline__ bf16x8 lds_b8(const __bf16 *p) {
  return *reinterpret_cast<const bf16x8 *>(p);
}

// LDS copy of the weights a block's waves read for every network pass:
// rows 0..63 W1' (folded), 64..127 W2, 128..143 W3 (rows >= 6 zero), kWStride
// bf16 per row (64 + 8 padding: the 16 rows one MFMA A operand reads land in
// different banks).
constexpr int kWStride = 72, kWRows = 144;

// Copies the network's weights to `sw` (all threads of the block; the caller
// synchronises before the first read).
__device__ __forceinline__ void net_weights_to_lds(const NetDev *__restrict__ net, __bf16 *sw) {
  for (uint32_t i = threadIdx.x; i < (uint32_t)kWRows * 8u; i += blockDim.x) {
    const uint32_t r = i >> 3, c = i & 7u;
    const __bf16 *src = r < 64u ? net->w1f + r * 64u : (r < 128u ? net->w2 + (r - 64u) * 64u
                                                                 : net->w3 + (r - 128u) * 64u);
    *reinterpret_cast<uint4 *>(sw + r * kWStride + 8u * c) =
        *reinterpret_cast<const uint4 *>(src + 8u * c);
  }
}

// B-operand fragments of a layer's input for the wave's 64 samples: [kb][t]
// holds units 32 kb + 8 g .. + 7 of sample 16 t + col (lane = 16 g + col).
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
struct Frag {
  bf16x8 b[2][4];
};

// The input features of the wave's samples from LDS tile `act` (row = sample).
__device__ __forceinline__ void frag_from_lds(const __bf16 *act, Frag &f) {
  const int lane = threadIdx.x & 63, col = lane & 15, g = lane >> 4;
#pragma unroll
  for (int kb = 0; kb < 2; ++kb)
#pragma unroll
    for (int t = 0; t < 4; ++t)
      f.b[kb][t] = lds_b8(act + (16 * t + col) * kActStride + 32 * kb + 8 * g);
}

// One fully connected layer of 64 outputs with ReLU for the wave's 64
// samples, inputs and outputs as B-operand fragments.  Output units come 16
// at a time (one MFMA row tile: lane 16 g' + col holds units 4 g' .. + 3 of
// sample 16 t + col).  The accumulators start at the bias; the outputs are
// rounded to BF16 and then clipped at zero on the BF16 bit patterns (a
// negative BF16 is a negative 16-bit integer), which gives the same values as
// rounding the clipped FP32 sum.  The output tiles of units 32 kb .. + 15 (X)
// and 32 kb + 16 .. + 31 (Y) hold, in lane row g' (16 lanes each), units
// 4 g' .. + 3 of their tile; the next layer wants in lane row g units
// 32 kb + 8 g .. + 7, i.e. rows 2 (g % 2) and 2 (g % 2) + 1 of X (g < 2) or of
// Y (g >= 2).  v_permlane32_swap(X, Y) gives [X0 X1 Y0 Y1] and [X2 X3 Y2 Y3]
// (rows), v_permlane16_swap of those gives [X0 X2 Y0 Y2] (the first four
// units) and [X1 X3 Y1 Y3] (the last four).
__device__ __forceinline__ void hidden_layer(const __bf16 *w, const float *__restrict__ bias,
                                             const Frag &in, Frag &out) {
  const int lane = threadIdx.x & 63, col = lane & 15, g = lane >> 4;
  typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
  typedef short i16x4 __attribute__((ext_vector_type(4)));
  u32x2 p[4][4];   // [output tile mt][sample tile t]: 4 BF16 units per lane
#pragma unroll
  for (int mt = 0; mt < 4; ++mt) {
    const f32x4 b = *reinterpret_cast<const f32x4 *>(bias + 16 * mt + 4 * g);
    f32x4 acc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = b;
#pragma unroll
    for (int kb = 0; kb < 2; ++kb) {
      const bf16x8 av = lds_b8(w + (16 * mt + col) * kWStride + 32 * kb + 8 * g);
#pragma unroll
      for (int t = 0; t < 4; ++t)
        acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, in.b[kb][t], acc[t], 0, 0, 0);
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const bf16x4 v = __builtin_convertvector(acc[t], bf16x4);
      const i16x4 h = __builtin_elementwise_max(__builtin_bit_cast(i16x4, v), (i16x4)0);
      p[mt][t] = __builtin_bit_cast(u32x2, h);
    }
  }
#pragma unroll
  for (int kb = 0; kb < 2; ++kb)
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      u32x4 o;
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        const auto r = __builtin_amdgcn_permlane32_swap(p[2 * kb][t][c], p[2 * kb + 1][t][c],
                                                        false, false);
        const auto q = __builtin_amdgcn_permlane16_swap(r[0], r[1], false, false);
        o[c] = q[0];       // units 8 g + 2 c, + 1
        o[2 + c] = q[1];   // units 8 g + 4 + 2 c, + 1
      }
      out.b[kb][t] = __builtin_bit_cast(bf16x8, o);
    }
}

// Network output z (6 per sample) for the 64 samples whose raw inputs are in
// LDS tile `act` (row = lane); weights from the block's LDS copy `sw`
// (net_weights_to_lds), biases from `net`.  z of sample s lands in
// zout[8 s .. 8 s + 5] (zout may alias `act`: it is written after the last
// read of `act`).
__device__ __forceinline__ void wave_forward(const NetDev *__restrict__ net, const __bf16 *sw,
                                             const __bf16 *act, float *zout) {
  Frag f0, f1;
  frag_from_lds(act, f0);
  hidden_layer(sw, net->b1f, f0, f1);
  hidden_layer(sw + 64 * kWStride, net->b2, f1, f0);
  const int lane = threadIdx.x & 63, col = lane & 15, g = lane >> 4;
  f32x4 acc[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int kb = 0; kb < 2; ++kb) {
    const bf16x8 av = lds_b8(sw + (128 + col) * kWStride + 32 * kb + 8 * g);
#pragma unroll
    for (int t = 0; t < 4; ++t)
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, f0.b[kb][t], acc[t], 0, 0, 0);
  }
  __builtin_amdgcn_wave_barrier();
  if (g < 2) {
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) zout[(16 * t + col) * 8 + 4 * g + r] = acc[t][r] + net->b3[4 * g + r];
  }
}

// Cell-neighbourhood addressing of a bead: the 3 x 3 x 3 cells around the
// cell that holds r, as 9 row bases (dz, dy) and 3 column offsets (dx).
struct Neighbourhood {
  uint32_t base[9];
  uint32_t xs[3];
  uint32_t centre;
};

__device__ __forceinline__ Neighbourhood neighbourhood(const Grid &g, F3 r) {
  uint32_t cx, cy, cz;
  cell3(g, r.x, r.y, r.z, cx, cy, cz);
  Neighbourhood nb;
  nb.xs[0] = cx == 0 ? g.nx - 1u : cx - 1u;
  nb.xs[1] = cx;
  nb.xs[2] = cx + 1 == (uint32_t)g.nx ? 0u : cx + 1u;
  const uint32_t ys[3] = {cy == 0 ? g.ny - 1u : cy - 1u, cy, cy + 1 == (uint32_t)g.ny ? 0u : cy + 1u};
  const uint32_t zs[3] = {cz == 0 ? g.nz - 1u : cz - 1u, cz, cz + 1 == (uint32_t)g.nz ? 0u : cz + 1u};
#pragma unroll
  for (int dz = 0; dz < 3; ++dz)
#pragma unroll
    for (int dy = 0; dy < 3; ++dy)
      nb.base[3 * dz + dy] = __umul24(__umul24(zs[dz], (uint32_t)g.ny) + ys[dy], (uint32_t)g.nx);
  nb.centre = nb.base[4] + cx;
  return nb;
}

// Field value at cell index c of the plane starting `pl` floats into omega:
// a 32-bit byte offset from the uniform base (fields < 4 GiB, host-checked),
// so the load needs no 64-bit address arithmetic per lane.
__device__ __forceinline__ float field_at(const float *__restrict__ omega, uint32_t pl,
                                          uint32_t c) {
  return *reinterpret_cast<const float *>(reinterpret_cast<const char *>(omega) +
                                          ((pl + c) << 2));
}

// Three x-consecutive cells (periodic in x) of one grid row of the plane at
// `pl`: one 12-byte load of an in-range triple plus, in the first and last
// column, one more value from the other end of the row.  Needs nx >= 3.
typedef float f32x3u __attribute__((ext_vector_type(3), aligned(4)));

__device__ __forceinline__ void row3(const float *__restrict__ omega, uint32_t pl, uint32_t base,
                                     uint32_t cx, uint32_t nx, float &v0, float &v1, float &v2) {
  const bool lo = cx == 0u, hi = cx + 1u == nx;
  const uint32_t start = lo ? 0u : (hi ? nx - 3u : cx - 1u);
  const f32x3u t = *reinterpret_cast<const f32x3u *>(reinterpret_cast<const char *>(omega) +
                                                      ((pl + base + start) << 2));
  float extra = 0.0f;
  if (lo || hi) extra = field_at(omega, pl, base + (lo ? nx - 1u : 0u));
  v0 = lo ? extra : (hi ? t.y : t.x);
  v1 = lo ? t.x : (hi ? t.z : t.y);
  v2 = lo ? t.y : (hi ? extra : t.z);
}

// The 60 raw features of a bead: fields of its own type (plane `own`) at the
// 27 cells around its cell ((dz, dy, dx) order, periodic), then the other
// type's (plane `oth`), then the bond vectors to the previous and next bead
// (zero where absent).  Gathered row by row.
__device__ __forceinline__ void gather_features(const Grid &g, const Neighbourhood &nb,
                                                const float *__restrict__ omega, uint32_t own,
                                                uint32_t oth, F3 bp, F3 bn, float (&f)[kNF]) {
  if (g.nx >= 3) {
    const uint32_t cx = nb.xs[1];
#pragma unroll
    for (int q = 0; q < 9; ++q) {
      row3(omega, own, nb.base[q], cx, (uint32_t)g.nx, f[3 * q], f[3 * q + 1], f[3 * q + 2]);
      row3(omega, oth, nb.base[q], cx, (uint32_t)g.nx, f[27 + 3 * q], f[28 + 3 * q],
           f[29 + 3 * q]);
    }
  } else {
#pragma unroll
    for (int k = 0; k < 27; ++k) {
      f[k] = field_at(omega, own, nb.base[k / 3] + nb.xs[k % 3]);
      f[27 + k] = field_at(omega, oth, nb.base[k / 3] + nb.xs[k % 3]);
    }
  }
  f[54] = bp.x; f[55] = bp.y; f[56] = bp.z;
  f[57] = bn.x; f[58] = bn.y; f[59] = bn.z;
}

// The 60 raw features of a row as BF16 (entries 60..63 zero), 8 at a time:
// the learned move's first layer holds the standardisation.
__device__ __forceinline__ void store_row(const float (&f)[kNF], __bf16 *row) {
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    bf16x8 v;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int k = 8 * c + j;
      v[j] = k < kNF ? (__bf16)f[k < kNF ? k : 0] : (__bf16)0.0f;
    }
    *reinterpret_cast<bf16x8 *>(row + 8 * c) = v;
  }
}

// Rewrites only the bond features (54..59) of a row, whose field features are
// current.
__device__ __forceinline__ void bond_features_to_row(F3 bp, F3 bn, __bf16 *row) {
  typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
  bf16x2 lo;
  lo[0] = (__bf16)bp.x;
  lo[1] = (__bf16)bp.y;
  bf16x8 hi;
  hi[0] = (__bf16)bp.z;
  hi[1] = (__bf16)bn.x;
  hi[2] = (__bf16)bn.y;
  hi[3] = (__bf16)bn.z;
  hi[4] = hi[5] = hi[6] = hi[7] = (__bf16)0.0f;
  *reinterpret_cast<bf16x2 *>(row + 54) = lo;
  *reinterpret_cast<bf16x8 *>(row + 56) = hi;
}

// Gathers the 60 features of a bead at r into one LDS row of bf16.  Returns
// the bead's own field in its cell; `cell` receives that cell's index.
__device__ __forceinline__ float features_to_row(const Grid &g, const float *__restrict__ omega,
                                                 bool is_b, F3 r, F3 bp, F3 bn, __bf16 *row,
                                                 uint32_t &cell) {
  const Neighbourhood nb = neighbourhood(g, r);
  float f[kNF];
  gather_features(g, nb, omega, is_b ? g.n_cells : 0u, is_b ? 0u : g.n_cells, bp, bn, f);
  store_row(f, row);
  cell = nb.centre;
  return f[13];   // own field at (dz, dy, dx) = (0, 0, 0)
}

// features_to_row from the halo copy of the fields ([2][nz*ny][nx + 2], plane
// size `halo_plane`): each of the 18 rows of three cells is one 12-byte load.
__device__ __forceinline__ float features_to_row_halo(const Grid &g, const float *__restrict__ halo,
                                                      uint32_t halo_plane, bool is_b, F3 r,
                                                      F3 bp, F3 bn, __bf16 *row, uint32_t &cell) {
  uint32_t cx, cy, cz;
  cell3(g, r.x, r.y, r.z, cx, cy, cz);
  const uint32_t w = (uint32_t)g.nx + 2u;
  const uint32_t ys[3] = {cy == 0 ? g.ny - 1u : cy - 1u, cy, cy + 1 == (uint32_t)g.ny ? 0u : cy + 1u};
  const uint32_t zs[3] = {cz == 0 ? g.nz - 1u : cz - 1u, cz, cz + 1 == (uint32_t)g.nz ? 0u : cz + 1u};
  const uint32_t own = is_b ? halo_plane : 0u, oth = is_b ? 0u : halo_plane;
  float f[kNF];
#pragma unroll
  for (int q = 0; q < 9; ++q) {
    const uint32_t rowb = (zs[q / 3] * (uint32_t)g.ny + ys[q % 3]) * w + cx;
    const f32x3u a = *reinterpret_cast<const f32x3u *>(reinterpret_cast<const char *>(halo) +
                                                      ((own + rowb) << 2));
    const f32x3u b = *reinterpret_cast<const f32x3u *>(reinterpret_cast<const char *>(halo) +
                                                      ((oth + rowb) << 2));
    f[3 * q] = a.x; f[3 * q + 1] = a.y; f[3 * q + 2] = a.z;
    f[27 + 3 * q] = b.x; f[28 + 3 * q] = b.y; f[29 + 3 * q] = b.z;
  }
  f[54] = bp.x; f[55] = bp.y; f[56] = bp.z;
  f[57] = bn.x; f[58] = bn.y; f[59] = bn.z;
  store_row(f, row);
  cell = cell_index(g, cx, cy, cz);
  return f[13];   // own field at (dz, dy, dx) = (0, 0, 0)
}

// Gaussian head of one sample: mean, sigma and log sigma.
__device__ __forceinline__ void head(const float *z, const HeadArgs &h, float (&mu)[3],
                                     float (&sig)[3], float (&lsig)[3]) {
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    mu[d] = h.m_max * tanhf(z[d] / h.m_max);
    const float s = fast_rcp(1.0f + __expf(-z[3 + d]));
    lsig[d] = h.lo + (h.hi - h.lo) * s;
    sig[d] = __expf(lsig[d]);
  }
}

// Stand-alone forward pass as the learned move evaluates the network (first
// layer with the standardisation folded in): raw features [n][60] -> z [n][6];
// one wave per 64 samples.
__global__ __launch_bounds__(256) void mlp_forward_kernel(const NetDev *__restrict__ net,
                                                          const float *__restrict__ feat,
                                                          uint32_t n, float *__restrict__ z) {
  __shared__ __bf16 s_act[4][64 * kActStride];
  __shared__ float s_z[4][64 * 8];
  const uint32_t wv = threadIdx.x >> 6, lane = threadIdx.x & 63u;
  const uint32_t s = (blockIdx.x * 4u + wv) * 64u + lane;
  __bf16 *row = &s_act[wv][lane * kActStride];
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    bf16x8 v;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int k = 8 * c + j;
      const float x = (k < kNF && s < n) ? feat[(size_t)s * kNF + (k < kNF ? k : 0)] : 0.0f;
      v[j] = (__bf16)x;
    }
    *reinterpret_cast<bf16x8 *>(row + 8 * c) = v;
  }
  __shared__ __bf16 s_w[kWRows * kWStride];
  net_weights_to_lds(net, s_w);
  __syncthreads();
  wave_forward(net, s_w, s_act[wv], s_z[wv]);
  if (s < n)
#pragma unroll
    for (int o = 0; o < kNO; ++o) z[(size_t)s * kNO + o] = s_z[wv][lane * 8 + o];
}

}  // namespace soma

namespace soma {

// Species table for kernels that address beads by (global chain, bead).
struct SpeciesTable {
  uint32_t n_species, total_chains;
  uint32_t chain_off[8], n[8], n_a[8];
  uint64_t bead_off[8];
};

// Species of global chain c and the chain's first bead (c < total_chains).
__device__ __forceinline__ const float *chain_start(const float *pos, const SpeciesTable &st,
                                                    uint32_t c, uint32_t *sp_out) {
  uint32_t sp = 0;
  for (uint32_t k = 1; k < st.n_species; ++k)
    if (c >= st.chain_off[k]) sp = k;
  *sp_out = sp;
  return pos + 3 * (st.bead_off[sp] + (uint64_t)(c - st.chain_off[sp]) * st.n[sp]);
}

// Raw features (FP32) of bead i of a chain of species sp starting at `chain`.
__device__ __forceinline__ void bead_features(const float *chain, const float *omega,
                                              const Grid &g, const SpeciesTable &st, uint32_t sp,
                                              uint32_t i, float *row) {
  const uint32_t nn = st.n[sp];
  const F3 r = {chain[3 * i], chain[3 * i + 1], chain[3 * i + 2]};
  const F3 zero3 = F3{0.f, 0.f, 0.f};
  const F3 bp = i > 0 ? F3{chain[3 * i - 3], chain[3 * i - 2], chain[3 * i - 1]} - r : zero3;
  const F3 bn = i + 1 < nn ? F3{chain[3 * i + 3], chain[3 * i + 4], chain[3 * i + 5]} - r : zero3;
  const Neighbourhood nb = neighbourhood(g, r);
  const bool is_b = i >= st.n_a[sp];
  float f[kNF];
  gather_features(g, nb, omega, is_b ? g.n_cells : 0u, is_b ? 0u : g.n_cells, bp, bn, f);
#pragma unroll
  for (int k = 0; k < kNF; ++k) row[k] = f[k];
}

// Raw features (FP32) of bead `beads[s]` of global chain `chains[s]` at the
// current positions, for training data: out [n][60].  One thread per sample.
__global__ __launch_bounds__(256) void features_kernel(const float *__restrict__ pos,
                                                       const float *__restrict__ omega, Grid g,
                                                       SpeciesTable st,
                                                       const uint32_t *__restrict__ chains,
                                                       const uint32_t *__restrict__ beads,
                                                       uint32_t n, float *__restrict__ out) {
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const uint32_t c = chains[s];
  float *row = out + (size_t)s * kNF;
  if (c >= st.total_chains) {  // out of range: zeros, never a stray read
    for (int k = 0; k < kNF; ++k) row[k] = 0.0f;
    return;
  }
  uint32_t sp;
  const float *chain = chain_start(pos, st, c, &sp);
  bead_features(chain, omega, g, st, sp, min(beads[s], st.n[sp] - 1u), row);
}

// Training samples drawn from the running melt.  Sample s of a round picks a
// chain uniformly among the chains of one species (or of all species) and a
// bead uniformly along it, from the Philox block (s, purpose 5, round, replica).  Phase 0 records the bead's
// features (optional) and position; phase 1, later in the run, the
// displacement from that recorded position.
struct CollectArgs {
  const float *pos;
  const float *omega;
  Grid grid;
  SpeciesTable st;
  uint32_t seed_lo, seed_hi, replica, round, n, phase;
  uint32_t chain_lo, chain_count;  // chains drawn from [chain_lo, chain_lo + chain_count)
  float *features;   // [n][60] or null (phase 0)
  float *r0;         // [n][3]
  float *dr;         // [n][3] (phase 1)
  uint32_t *picked;  // [n][2] (chain, bead) or null (phase 0)
};

__global__ __launch_bounds__(256) void collect_kernel(const CollectArgs a) {
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= a.n) return;
  const Rand4 q = philox(s, kPurposeCollect << 16, a.round, a.replica, a.seed_lo, a.seed_hi);
  const uint32_t c = a.chain_lo + __umulhi(q.x, a.chain_count);
  uint32_t sp;
  const float *chain = chain_start(a.pos, a.st, c, &sp);
  const uint32_t i = __umulhi(q.y, a.st.n[sp]);
  const float *r = chain + 3 * i;
  const size_t o = 3 * (size_t)s;
  if (a.phase == 0) {
    if (a.features) bead_features(chain, a.omega, a.grid, a.st, sp, i, a.features + (size_t)s * kNF);
    a.r0[o] = r[0];
    a.r0[o + 1] = r[1];
    a.r0[o + 2] = r[2];
    if (a.picked) {
      a.picked[2 * (size_t)s] = c;
      a.picked[2 * (size_t)s + 1] = i;
    }
  } else {
    a.dr[o] = r[0] - a.r0[o];
    a.dr[o + 1] = r[1] - a.r0[o + 1];
    a.dr[o + 2] = r[2] - a.r0[o + 2];
  }
}

}  // namespace soma
