// soma_grid.hpp -- stage 1 of the SCMF cycle (Sec. 2.2): the per-type
// occupation histogram of the grid cells (Eq. (4)) and the quasi-instantaneous
// fields (Eq. (12), K^1 form), plus the initial Gaussian-walk configuration.
#pragma once

#include "soma_device.hpp"

namespace soma {

constexpr uint32_t kFieldBlocks = 1024u;  // fixed grid of the field kernel

struct FieldPartial {
  unsigned long long sum_a, sum_b;
  double h_nb;
  double pad;
};

// ---------------------------------------------------------------------------
// Stand-alone histogram: one thread per bead, one packed atomic per bead.
// ---------------------------------------------------------------------------
template <bool COUNT64>
__global__ __launch_bounds__(256) void density_hist_kernel(
    const float *pos, uint64_t n_beads, uint32_t n, uint32_t n_a, Grid g,
    void *counts, const ArchDev *arch) {
  const uint64_t b = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= n_beads) return;
  const float *r = pos + 3 * b;
  const uint32_t cell = cell_of(g, r[0], r[1], r[2]);
  const uint32_t i = n_beads <= 0xFFFFFFFFull ? (uint32_t)b % n : (uint32_t)(b % n);
  const uint32_t t = bead_type(arch, i, n_a);
  const size_t w = (size_t)(t >> 1) * g.n_cells + cell;   // count plane of the type
  if (COUNT64) {
    const unsigned long long inc = 1ull << ((t & 1u) ? 32u : 0u);
    atomicAdd(reinterpret_cast<unsigned long long *>(counts) + w, inc);
  } else {
    const unsigned int inc = 1u << ((t & 1u) ? 16u : 0u);
    atomicAdd(reinterpret_cast<unsigned int *>(counts) + w, inc);
  }
}

// Throughput probe of scattered 32-bit updates (measurement only): thread i
// updates word addr(i) of `words`.  mode 0: atomicAdd at a uniformly random
// word; mode 1: atomicAdd at a word chosen within a window of 4096 words that
// moves with the thread index (the locality of a sweep's count updates,
// whose waves work on compact regions); mode 2: a plain store at a uniformly
// random word.  Addresses from a 32-bit integer hash of (i, seed).
__global__ __launch_bounds__(256) void probe_atomics_kernel(uint32_t *words, uint64_t n_words,
                                                            uint64_t n_updates, uint32_t mode,
                                                            uint32_t seed) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_updates) return;
  uint32_t h = (uint32_t)i * 0x9E3779B1u ^ seed;
  h ^= h >> 15; h *= 0x85EBCA77u; h ^= h >> 13; h *= 0xC2B2AE3Du; h ^= h >> 16;
  uint64_t addr;
  if (mode == 1) {
    const uint64_t base = (i * 7u) % n_words;           // moves slowly with i
    addr = (base + (h & 4095u)) % n_words;
  } else {
    addr = (((uint64_t)h << 32) | (h * 0x27D4EB2Fu)) % n_words;
  }
  if (mode == 2) words[addr] = (uint32_t)i;
  else atomicAdd(words + addr, 1u);
}

// Fill a buffer of n_words 32-bit words with zeros (a kernel, not a memset
// node, so that it can live inside a captured graph).
__global__ __launch_bounds__(256) void zero_kernel(uint32_t *p, uint64_t n_words) {
  const uint64_t n4 = n_words >> 2;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  uint4 *p4 = reinterpret_cast<uint4 *>(p);
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += stride)
    p4[i] = make_uint4(0u, 0u, 0u, 0u);
  const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < (n_words & 3u)) p[n4 * 4 + t] = 0u;
}

// ---------------------------------------------------------------------------
// Fields from counts, Eq. (12) with Eq. (8):
//   phi_t = n_t * inv_rho,  s = (phi_A + phi_B) - 1,  t = kappaN * s,
//   omega_A = fma(chiN, phi_B, t),  omega_B = fma(chiN, phi_A, t)
// in this FP32 order (the library is built without FP contraction).
// Optionally clears the counts in the same pass and accumulates the count
// sums and H_nb (Eqs. (5), (6), (8), FP64) per block.
// ---------------------------------------------------------------------------
struct FieldArgs {
  void *counts;
  float *omega;
  uint32_t n_cells;
  float inv_rho, chi_n, kappa_n;
  double inv_rho_d, chi_n_d, kappa_n_d;
  FieldPartial *partials;  // may be null
  int clear;
  // optional copy of the fields with one periodic halo cell at each end of every
  // x row: [2][nz*ny][nx + 2] (null: not kept)
  float *halo;
  uint32_t nx, halo_plane;
  // external fields (null: none): ext [2][n_cells] added to the fields;
  // forbid one bit per cell (bit c % 32 of word c / 32): impenetrable cells get
  // the field 0 and are left out of H_nb
  const float *ext;
  const uint32_t *forbid;
  // interaction term of the grid Hamiltonian: 1 = chiN phi_A phi_B (default),
  // 0 = -chiN/4 (phi_A - phi_B)^2
  uint32_t form;
};

__device__ __forceinline__ bool cell_forbidden(const uint32_t *m, uint32_t c) {
  return m != nullptr && ((m[c >> 5] >> (c & 31u)) & 1u) != 0u;
}

// External terms of cell c on top of its interaction fields.
__device__ __forceinline__ void field_extras(const FieldArgs &a, uint32_t c, bool off, float &va,
                                             float &vb) {
  if (a.ext) {
    va = va + a.ext[c];
    vb = vb + a.ext[a.n_cells + c];
  }
  if (off) va = vb = 0.0f;
}

// Writes the two field values of the cell at column x of row r into the halo
// copy (and into the halo cell that mirrors it when x is at either end).
__device__ __forceinline__ void halo_put_rx(const FieldArgs &a, uint32_t r, uint32_t x, float va,
                                            float vb) {
  const uint32_t w = a.nx + 2u;
  float *ha = a.halo + (size_t)r * w, *hb = ha + a.halo_plane;
  ha[x + 1u] = va;
  hb[x + 1u] = vb;
  if (x == 0u) { ha[a.nx + 1u] = va; hb[a.nx + 1u] = vb; }
  if (x + 1u == a.nx) { ha[0] = va; hb[0] = vb; }
}

__device__ __forceinline__ void halo_put(const FieldArgs &a, uint32_t c, float va, float vb) {
  const uint32_t r = c / a.nx;
  halo_put_rx(a, r, c - r * a.nx, va, vb);
}

__device__ __forceinline__ void field_cell(uint32_t na, uint32_t nb,
                                           const FieldArgs &a, float &oa,
                                           float &ob) {
  const float phi_a = (float)na * a.inv_rho;
  const float phi_b = (float)nb * a.inv_rho;
  const float s = (phi_a + phi_b) - 1.0f;
  const float t = a.kappa_n * s;
  if (a.form == 0) {   // Eq. (12), first form: t -+ chiN/2 (phi_A - phi_B)
    const float d = phi_a - phi_b;
    oa = fmaf(-0.5f * a.chi_n, d, t);
    ob = fmaf(0.5f * a.chi_n, d, t);
  } else {
    oa = fmaf(a.chi_n, phi_b, t);
    ob = fmaf(a.chi_n, phi_a, t);
  }
}

__device__ __forceinline__ double hnb_cell(uint32_t na, uint32_t nb,
                                           const FieldArgs &a) {
  const double pa = (double)na * a.inv_rho_d, pb = (double)nb * a.inv_rho_d;
  const double dev = pa + pb - 1.0;
  const double inter = a.form == 0 ? -0.25 * a.chi_n_d * (pa - pb) * (pa - pb) : a.chi_n_d * pa * pb;
  return 0.5 * a.kappa_n_d * dev * dev + inter;
}

// NT: the counts are read with the non-temporal hint (grids whose counts
// outgrow the caches: the fields written here, which the next sweep gathers,
// then keep their place in the last-level cache).  A compile-time choice:
// loads that differ only in the hint would be merged, dropping it.
template <bool COUNT64, bool NT = false>
__device__ __forceinline__ void load4(const void *counts, uint32_t q,
                                      uint32_t na[4], uint32_t nb[4]) {
  if (COUNT64) {
    typedef unsigned long long u64x2 __attribute__((ext_vector_type(2)));
    const u64x2 *c = reinterpret_cast<const u64x2 *>(counts) + 2 * (size_t)q;
    u64x2 v0, v1;
    if (NT) {
      v0 = __builtin_nontemporal_load(c);
      v1 = __builtin_nontemporal_load(c + 1);
    } else {
      v0 = c[0];
      v1 = c[1];
    }
    const unsigned long long w[4] = {v0.x, v0.y, v1.x, v1.y};
#pragma unroll
    for (int j = 0; j < 4; ++j) { na[j] = (uint32_t)w[j]; nb[j] = (uint32_t)(w[j] >> 32); }
  } else {
    typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
    const u32x4 *c = reinterpret_cast<const u32x4 *>(counts) + q;
    const u32x4 v = NT ? __builtin_nontemporal_load(c) : c[0];
    const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int j = 0; j < 4; ++j) { na[j] = w[j] & 0xFFFFu; nb[j] = w[j] >> 16; }
  }
}

// Block `blk` of the `nblk` blocks that serve one grid: a grid-stride loop
// over groups of four cells, then the block's partial sums (FP64 H_nb).
template <bool COUNT64, bool NT = false>
__device__ __forceinline__ void field_body(const FieldArgs &a, uint32_t blk, uint32_t nblk) {
  __shared__ unsigned long long s_a[4], s_b[4];
  __shared__ double s_h[4];
  const uint32_t n4 = a.n_cells >> 2;
  const uint32_t stride = nblk * blockDim.x;
  const uint32_t tid = blk * blockDim.x + threadIdx.x;
  unsigned long long sum_a = 0, sum_b = 0;
  double h = 0.0;
  const bool stats = a.partials != nullptr;
  float4 *oa4 = reinterpret_cast<float4 *>(a.omega);
  const bool b_aligned = (a.n_cells & 3u) == 0u;
  float4 *ob4 = reinterpret_cast<float4 *>(a.omega + (b_aligned ? a.n_cells : 0u));
  for (uint32_t q = tid; q < n4; q += stride) {
    uint32_t na[4], nb[4];
    load4<COUNT64, NT>(a.counts, q, na, nb);
    // the four cells 4q..4q+3 share one mask word
    const uint32_t fb = a.forbid ? (a.forbid[q >> 3] >> ((4u * q) & 31u)) & 0xFu : 0u;
    float va[4], vb[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      field_cell(na[j], nb[j], a, va[j], vb[j]);
      const bool off = ((fb >> j) & 1u) != 0u;
      if (a.ext || a.forbid) field_extras(a, 4u * q + j, off, va[j], vb[j]);
      if (stats) {
        sum_a += na[j];
        sum_b += nb[j];
        if (!off) h += hnb_cell(na[j], nb[j], a);
      }
    }
    oa4[q] = make_float4(va[0], va[1], va[2], va[3]);
    if (a.halo) {   // four consecutive cells: one division, then step along the row
      uint32_t r = (4u * q) / a.nx, x = 4u * q - r * a.nx;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        halo_put_rx(a, r, x, va[j], vb[j]);
        if (++x == a.nx) { x = 0; ++r; }
      }
    }
    if (b_aligned) {
      ob4[q] = make_float4(vb[0], vb[1], vb[2], vb[3]);
    } else {  // the B plane starts n_cells floats in: 16-byte stores only if n_cells % 4 == 0
      float *ob = a.omega + a.n_cells + 4 * (size_t)q;
      ob[0] = vb[0]; ob[1] = vb[1]; ob[2] = vb[2]; ob[3] = vb[3];
    }
    if (a.clear) {
      if (COUNT64) {
        ulonglong2 *c = reinterpret_cast<ulonglong2 *>(a.counts) + 2 * (size_t)q;
        c[0] = make_ulonglong2(0ull, 0ull);
        c[1] = make_ulonglong2(0ull, 0ull);
      } else {
        reinterpret_cast<uint4 *>(a.counts)[q] = make_uint4(0u, 0u, 0u, 0u);
      }
    }
  }
  // ragged tail (n_cells not a multiple of 4)
  const uint32_t tail = a.n_cells & 3u;
  if (tid < tail) {
    const uint32_t c = n4 * 4 + tid;
    uint32_t na, nb;
    if (COUNT64) {
      const unsigned long long w = reinterpret_cast<const unsigned long long *>(a.counts)[c];
      na = (uint32_t)w; nb = (uint32_t)(w >> 32);
      if (a.clear) reinterpret_cast<unsigned long long *>(a.counts)[c] = 0ull;
    } else {
      const uint32_t w = reinterpret_cast<const uint32_t *>(a.counts)[c];
      na = w & 0xFFFFu; nb = w >> 16;
      if (a.clear) reinterpret_cast<uint32_t *>(a.counts)[c] = 0u;
    }
    float va, vb;
    field_cell(na, nb, a, va, vb);
    const bool off = cell_forbidden(a.forbid, c);
    if (a.ext || a.forbid) field_extras(a, c, off, va, vb);
    a.omega[c] = va;
    a.omega[a.n_cells + c] = vb;
    if (a.halo) halo_put(a, c, va, vb);
    if (stats) {
      sum_a += na;
      sum_b += nb;
      if (!off) h += hnb_cell(na, nb, a);
    }
  }
  if (!stats) return;
  // block reduction: wave shuffles, then four waves through LDS
  for (int off = 32; off > 0; off >>= 1) {
    sum_a += __shfl_down(sum_a, off, 64);
    sum_b += __shfl_down(sum_b, off, 64);
    h += __shfl_down(h, off, 64);
  }
  const uint32_t lane = threadIdx.x & 63u, wv = threadIdx.x >> 6;
  if (lane == 0) { s_a[wv] = sum_a; s_b[wv] = sum_b; s_h[wv] = h; }
  __syncthreads();
  if (threadIdx.x == 0) {
    FieldPartial p;
    p.sum_a = s_a[0] + s_a[1] + s_a[2] + s_a[3];
    p.sum_b = s_b[0] + s_b[1] + s_b[2] + s_b[3];
    p.h_nb = ((s_h[0] + s_h[1]) + s_h[2]) + s_h[3];
    p.pad = 0.0;
    a.partials[blk] = p;
  }
}

template <bool COUNT64, bool NT = false>
__global__ __launch_bounds__(256) void field_update_kernel(const FieldArgs a) {
  field_body<COUNT64, NT>(a, blockIdx.x, gridDim.x);
}

// ---------------------------------------------------------------------------
// n_t bead types (Sec. 2.1) with a symmetric matrix of chi_ij N, Eq. (12):
//   K^1: omega_i = kappaN (sum_k phi_k - 1) + sum_{k != i} chi_ik N phi_k
//   K^0: omega_i = kappaN (sum_k phi_k - 1) - sum_{k != i} chi_ik N/2 (phi_i - phi_k)
// FP32 order: s = (((phi_0 + phi_1) + phi_2) + ...) - 1, t = kappaN * s, then
// t = fma(chi_ik, phi_k, t) (K^1) or fma(-chi_ik/2, phi_i - phi_k, t) (K^0)
// for k = 0, 1, ... (k != i); with two types this is field_cell's order.
// Counts: plane p holds types 2p (low half) and 2p + 1 (high half) of every
// cell.  One thread per cell in a grid-stride loop; the FP64 partials are
// sum_a = the type-0 count, sum_b = the other types, and H_nb (Eqs. (5), (6),
// (8), pairs i < j).
// ---------------------------------------------------------------------------
constexpr uint32_t kMaxTypes = 8u;

struct MultiFieldArgs {
  void *counts;
  float *omega;
  uint32_t n_cells, n_t, form, clear;
  float inv_rho, kappa_n;
  double inv_rho_d, kappa_n_d;
  float chi[kMaxTypes * kMaxTypes];   // chi_ik N at [i * kMaxTypes + k]
  FieldPartial *partials;              // may be null
};

template <bool COUNT64>
__device__ __forceinline__ void load_types(const MultiFieldArgs &a, uint32_t c, uint32_t (&n)[kMaxTypes]) {
  const uint32_t n_pl = (a.n_t + 1u) >> 1;
#pragma unroll
  for (uint32_t p = 0; p < kMaxTypes / 2; ++p) {
    n[2 * p] = n[2 * p + 1] = 0u;
    if (p < n_pl) {
      const size_t w = (size_t)p * a.n_cells + c;
      if (COUNT64) {
        unsigned long long *q = reinterpret_cast<unsigned long long *>(a.counts) + w;
        const unsigned long long v = *q;
        n[2 * p] = (uint32_t)v;
        n[2 * p + 1] = (uint32_t)(v >> 32);
        if (a.clear) *q = 0ull;
      } else {
        uint32_t *q = reinterpret_cast<uint32_t *>(a.counts) + w;
        const uint32_t v = *q;
        n[2 * p] = v & 0xFFFFu;
        n[2 * p + 1] = v >> 16;
        if (a.clear) *q = 0u;
      }
    }
  }
}

// Fields of one cell of NT types from its counts (the order stated above), and
// its contribution to the count sums and H_nb.
template <uint32_t NT>
__device__ __forceinline__ void multi_cell(const MultiFieldArgs &a, const uint32_t (&n)[NT],
                                           float (&w)[NT], bool stats,
                                           unsigned long long &sum_a, unsigned long long &sum_b,
                                           double &h) {
  float phi[NT];
#pragma unroll
  for (uint32_t i = 0; i < NT; ++i) phi[i] = (float)n[i] * a.inv_rho;
  float s = phi[0];
#pragma unroll
  for (uint32_t i = 1; i < NT; ++i) s = s + phi[i];
  s = s - 1.0f;
  const float t0 = a.kappa_n * s;
#pragma unroll
  for (uint32_t i = 0; i < NT; ++i) {
    float t = t0;
#pragma unroll
    for (uint32_t k = 0; k < NT; ++k) {
      if (k == i) continue;
      const float x = a.chi[i * kMaxTypes + k];
      t = a.form == 0 ? fmaf(-0.5f * x, phi[i] - phi[k], t) : fmaf(x, phi[k], t);
    }
    w[i] = t;
  }
  if (!stats) return;
  double pd[NT], tot = 0.0, inter = 0.0;
#pragma unroll
  for (uint32_t i = 0; i < NT; ++i) {
    pd[i] = (double)n[i] * a.inv_rho_d;
    tot += pd[i];
    if (i == 0) sum_a += n[i];
    else sum_b += n[i];
  }
#pragma unroll
  for (uint32_t i = 0; i < NT; ++i)
#pragma unroll
    for (uint32_t j = i + 1; j < NT; ++j) {
      const double x = (double)a.chi[i * kMaxTypes + j], d = pd[i] - pd[j];
      inter += a.form == 0 ? -0.25 * x * d * d : x * pd[i] * pd[j];
    }
  const double dev = tot - 1.0;
  h += 0.5 * a.kappa_n_d * dev * dev + inter;
}

// One kernel per number of types NT (3..8; a.n_t == NT).  With n_cells % 4 == 0
// every plane starts on a 16-byte boundary: for NT <= 4 a thread then takes
// four consecutive cells per step (16-byte loads and stores per plane); more
// types, or other grids, one cell per step (fewer registers).
template <bool COUNT64, uint32_t NT>
__global__ __launch_bounds__(256) void field_multi_kernel(const MultiFieldArgs a) {
  constexpr uint32_t NP = (NT + 1u) / 2u;   // count planes
  __shared__ unsigned long long s_a[4], s_b[4];
  __shared__ double s_h[4];
  const bool stats = a.partials != nullptr;
  const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x, stride = gridDim.x * blockDim.x;
  unsigned long long sum_a = 0, sum_b = 0;
  double h = 0.0;
  if (NT <= 4u && (a.n_cells & 3u) == 0u) {
    const uint32_t n4 = a.n_cells >> 2;
    for (uint32_t q = tid; q < n4; q += stride) {
      uint32_t n[4][NT];
#pragma unroll
      for (uint32_t p = 0; p < NP; ++p) {
        uint32_t lo[4], hi[4];
        if (COUNT64) {
          ulonglong2 *c = reinterpret_cast<ulonglong2 *>(reinterpret_cast<unsigned long long *>(a.counts) +
                                                         (size_t)p * a.n_cells) + 2 * (size_t)q;
          const ulonglong2 v0 = c[0], v1 = c[1];
          const unsigned long long wv[4] = {v0.x, v0.y, v1.x, v1.y};
#pragma unroll
          for (int j = 0; j < 4; ++j) { lo[j] = (uint32_t)wv[j]; hi[j] = (uint32_t)(wv[j] >> 32); }
          if (a.clear) { c[0] = make_ulonglong2(0ull, 0ull); c[1] = make_ulonglong2(0ull, 0ull); }
        } else {
          uint4 *c = reinterpret_cast<uint4 *>(reinterpret_cast<uint32_t *>(a.counts) +
                                               (size_t)p * a.n_cells) + q;
          const uint4 v = *c;
          const uint32_t wv[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
          for (int j = 0; j < 4; ++j) { lo[j] = wv[j] & 0xFFFFu; hi[j] = wv[j] >> 16; }
          if (a.clear) *c = make_uint4(0u, 0u, 0u, 0u);
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          n[j][2 * p] = lo[j];
          if (2 * p + 1 < NT) n[j][2 * p + 1] = hi[j];
        }
      }
      float w[4][NT];
#pragma unroll
      for (int j = 0; j < 4; ++j) multi_cell<NT>(a, n[j], w[j], stats, sum_a, sum_b, h);
#pragma unroll
      for (uint32_t i = 0; i < NT; ++i)
        reinterpret_cast<float4 *>(a.omega + (size_t)i * a.n_cells)[q] =
            make_float4(w[0][i], w[1][i], w[2][i], w[3][i]);
    }
  } else {
    for (uint32_t c = tid; c < a.n_cells; c += stride) {
      uint32_t nn[kMaxTypes];
      load_types<COUNT64>(a, c, nn);
      uint32_t n[NT];
#pragma unroll
      for (uint32_t i = 0; i < NT; ++i) n[i] = nn[i];
      float w[NT];
      multi_cell<NT>(a, n, w, stats, sum_a, sum_b, h);
#pragma unroll
      for (uint32_t i = 0; i < NT; ++i) a.omega[(size_t)i * a.n_cells + c] = w[i];
    }
  }
  if (!stats) return;
  for (int off = 32; off > 0; off >>= 1) {
    sum_a += __shfl_down(sum_a, off, 64);
    sum_b += __shfl_down(sum_b, off, 64);
    h += __shfl_down(h, off, 64);
  }
  const uint32_t lane = threadIdx.x & 63u, wv = threadIdx.x >> 6;
  if (lane == 0) { s_a[wv] = sum_a; s_b[wv] = sum_b; s_h[wv] = h; }
  __syncthreads();
  if (threadIdx.x == 0) {
    FieldPartial p;
    p.sum_a = s_a[0] + s_a[1] + s_a[2] + s_a[3];
    p.sum_b = s_b[0] + s_b[1] + s_b[2] + s_b[3];
    p.h_nb = ((s_h[0] + s_h[1]) + s_h[2]) + s_h[3];
    p.pad = 0.0;
    a.partials[blockIdx.x] = p;
  }
}

// Per-type totals of the counts: block b writes out[b * kMaxTypes + t].
template <bool COUNT64>
__global__ __launch_bounds__(256) void type_count_kernel(const void *counts, uint32_t n_cells,
                                                         uint32_t n_t, unsigned long long *out) {
  __shared__ unsigned long long s[4][kMaxTypes];
  unsigned long long v[kMaxTypes] = {};
  const uint32_t n_pl = (n_t + 1u) >> 1;
  for (uint32_t c = blockIdx.x * blockDim.x + threadIdx.x; c < n_cells; c += gridDim.x * blockDim.x) {
#pragma unroll
    for (uint32_t p = 0; p < kMaxTypes / 2; ++p)
      if (p < n_pl) {
        const size_t w = (size_t)p * n_cells + c;
        if (COUNT64) {
          const unsigned long long x = reinterpret_cast<const unsigned long long *>(counts)[w];
          v[2 * p] += (uint32_t)x;
          v[2 * p + 1] += (uint32_t)(x >> 32);
        } else {
          const uint32_t x = reinterpret_cast<const uint32_t *>(counts)[w];
          v[2 * p] += x & 0xFFFFu;
          v[2 * p + 1] += x >> 16;
        }
      }
  }
#pragma unroll
  for (uint32_t t = 0; t < kMaxTypes; ++t)
    for (int off = 32; off > 0; off >>= 1) v[t] += __shfl_down(v[t], off, 64);
  const uint32_t lane = threadIdx.x & 63u, wv = threadIdx.x >> 6;
  if (lane == 0)
#pragma unroll
    for (uint32_t t = 0; t < kMaxTypes; ++t) s[wv][t] = v[t];
  __syncthreads();
  if (threadIdx.x < kMaxTypes) {
    const uint32_t t = threadIdx.x;
    out[(size_t)blockIdx.x * kMaxTypes + t] = s[0][t] + s[1][t] + s[2][t] + s[3][t];
  }
}

// Blocks of the grid-field update for a number of systems are given out in
// contiguous ranges: system s owns blocks [first[s], first[s+1]).
__device__ __forceinline__ uint32_t range_of(const uint32_t *first, uint32_t n, uint32_t x) {
  uint32_t lo = 0, hi = n;  // first[lo] <= x < first[hi]
  while (hi - lo > 1u) {
    const uint32_t mid = (lo + hi) >> 1;
    if (first[mid] <= x) lo = mid;
    else hi = mid;
  }
  return lo;
}

template <bool COUNT64>
__global__ __launch_bounds__(256) void batched_field_kernel(const FieldArgs *fa,
                                                            const uint32_t *first, uint32_t n_sys) {
  const uint32_t s = range_of(first, n_sys, blockIdx.x);
  field_body<COUNT64>(fa[s], blockIdx.x - first[s], first[s + 1] - first[s]);
}

// Halo copy of the fields rebuilt from the field planes (after the caller has
// written the fields directly).  One thread per cell.
__global__ __launch_bounds__(256) void halo_from_fields_kernel(const FieldArgs a) {
  const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= a.n_cells) return;
  halo_put(a, c, a.omega[c], a.omega[a.n_cells + c]);
}

// Gradient field for smart-MC moves: for each type and cell, the field and its
// central differences 0.5 (omega(c + e) - omega(c - e)) over the periodic
// neighbours, in the arithmetic the sweep uses when it gathers them itself.
__global__ __launch_bounds__(256) void grad_field_kernel(const float *__restrict__ omega,
                                                         float4 *__restrict__ grad, Grid g) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 2u * g.n_cells) return;
  const uint32_t t = i >= g.n_cells ? 1u : 0u;
  const uint32_t c = i - t * g.n_cells;
  const uint32_t nxy = (uint32_t)g.nx * (uint32_t)g.ny;
  const uint32_t cz = c / nxy, rem = c - cz * nxy;
  const uint32_t cy = rem / (uint32_t)g.nx, cx = rem - cy * (uint32_t)g.nx;
  const float *om = omega + t * g.n_cells;
  const uint32_t xp = cx + 1 == (uint32_t)g.nx ? 0 : cx + 1;
  const uint32_t xm = cx == 0 ? g.nx - 1 : cx - 1;
  const uint32_t yp = cy + 1 == (uint32_t)g.ny ? 0 : cy + 1;
  const uint32_t ym = cy == 0 ? g.ny - 1 : cy - 1;
  const uint32_t zp = cz + 1 == (uint32_t)g.nz ? 0 : cz + 1;
  const uint32_t zm = cz == 0 ? g.nz - 1 : cz - 1;
  float4 v;
  v.x = om[c];
  v.y = 0.5f * (om[cell_index(g, xp, cy, cz)] - om[cell_index(g, xm, cy, cz)]);
  v.z = 0.5f * (om[cell_index(g, cx, yp, cz)] - om[cell_index(g, cx, ym, cz)]);
  v.w = 0.5f * (om[cell_index(g, cx, cy, zp)] - om[cell_index(g, cx, cy, zm)]);
  grad[i] = v;
}

// Device sweep counters: add `by` to each (or set them to `value`).
__global__ __launch_bounds__(64) void sweep_counter_kernel(uint32_t *const *ctrs, uint32_t n,
                                                           uint32_t by, uint32_t set,
                                                           uint32_t value) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint32_t *c = ctrs[i];
  c[0] = set ? value : c[0] + by;
}

__global__ __launch_bounds__(64) void sweep_counter_one_kernel(uint32_t *ctr, uint32_t by,
                                                               uint32_t set, uint32_t value) {
  if (threadIdx.x == 0) ctr[0] = set ? value : ctr[0] + by;
}

// ---------------------------------------------------------------------------
// Initial configuration: Gaussian random walks, bonds N(0, sigma^2) per
// component with sigma^2 = 1/k0 (the ideal chain of Eq. (2); b0^2 = 3/k0,
// Sec. 2.1).  One thread per chain.  Origins:
//   mode 0: uniform in the box, r0_d = u_d * n_d;
//   mode 1: stratified -- chain g of G sits in the cell of rank
//           floor(n_cells (g + u_3) / G) of the bricked order (bricks of 8^3
//           cells row-major in z,y,x, the last brick per axis taking the
//           remainder; cells row-major in z,y,x inside a brick), at a uniform
//           point inside it.
// Draws: Philox block (g, j | 4 << 16, 0xFFFFFFFF, replica) for bead j.
// ---------------------------------------------------------------------------
struct InitArgs {
  float *pos;
  uint32_t n_chains, n;
  uint32_t chain_base, total_chains;
  float sigma;
  Grid grid;
  uint32_t seed_lo, seed_hi, replica, origin_mode;
};

// floor((hi:lo) / d) for a 128-bit dividend whose quotient fits in 64 bits.
__device__ inline uint64_t div128_64(uint64_t hi, uint64_t lo, uint64_t d) {
  uint64_t q = 0;
  for (int i = 63; i >= 0; --i) {
    // shift (hi:lo) left by one into hi, remainder kept in hi
    const uint64_t top = hi >> 63;
    hi = (hi << 1) | (lo >> 63);
    lo <<= 1;
    if (top || hi >= d) { hi -= d; q |= 1ull << i; }
  }
  return q;
}

__device__ inline void brick_cell(uint64_t k, const Grid &g, uint32_t &x,
                                  uint32_t &y, uint32_t &z) {
  const uint64_t B = 8, nx = g.nx, ny = g.ny, nz = g.nz;
  const uint64_t nbx = nx >= B ? nx / B : 1, nby = ny >= B ? ny / B : 1,
                 nbz = nz >= B ? nz / B : 1;
  uint64_t bz = k / (B * nx * ny);
  bz = bz < nbz - 1 ? bz : nbz - 1;
  k -= bz * B * nx * ny;
  const uint64_t wz = bz + 1 < nbz ? B : nz - B * (nbz - 1);
  uint64_t by = k / (wz * B * nx);
  by = by < nby - 1 ? by : nby - 1;
  k -= by * wz * B * nx;
  const uint64_t wy = by + 1 < nby ? B : ny - B * (nby - 1);
  uint64_t bx = k / (wz * wy * B);
  bx = bx < nbx - 1 ? bx : nbx - 1;
  k -= bx * wz * wy * B;
  const uint64_t wx = bx + 1 < nbx ? B : nx - B * (nbx - 1);
  const uint64_t inner = k % (wy * wx);
  x = (uint32_t)(bx * B + inner % wx);
  y = (uint32_t)(by * B + inner / wx);
  z = (uint32_t)(bz * B + k / (wy * wx));
}

__global__ __launch_bounds__(256) void init_chains_kernel(const InitArgs a) {
  const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= a.n_chains) return;
  const uint32_t g = a.chain_base + c;
  float *p = a.pos + (size_t)c * a.n * 3;
  Rand4 w = philox(g, kPurposeInit << 16, kSweepInit, a.replica, a.seed_lo, a.seed_hi);
  float x, y, z;
  if (a.origin_mode == 1) {
    const uint64_t num = ((uint64_t)g << 24) + 2ull * (w.w >> 9) + 1ull;
    const uint64_t nc = a.grid.n_cells;
    const uint64_t lo = nc * num;
    const uint64_t hi = __umul64hi(nc, num);
    const uint64_t k = div128_64(hi, lo, (uint64_t)a.total_chains << 24);
    uint32_t cx, cy, cz;
    brick_cell(k, a.grid, cx, cy, cz);
    x = (float)cx + uniform01(w.x);
    y = (float)cy + uniform01(w.y);
    z = (float)cz + uniform01(w.z);
  } else {
    x = uniform01(w.x) * (float)a.grid.nx;
    y = uniform01(w.y) * (float)a.grid.ny;
    z = uniform01(w.z) * (float)a.grid.nz;
  }
  p[0] = x; p[1] = y; p[2] = z;
  for (uint32_t j = 1; j < a.n; ++j) {
    w = philox(g, j | (kPurposeInit << 16), kSweepInit, a.replica, a.seed_lo, a.seed_hi);
    float n0, n1, n2, n3;
    box_muller(w.x, w.y, n0, n1);
    box_muller(w.z, w.w, n2, n3);
    x = fmaf(a.sigma, n0, x);
    y = fmaf(a.sigma, n1, y);
    z = fmaf(a.sigma, n2, z);
    p[3 * j] = x; p[3 * j + 1] = y; p[3 * j + 2] = z;
  }
}

}  // namespace soma
