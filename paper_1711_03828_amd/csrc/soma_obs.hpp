// soma_obs.hpp -- FP64 global reductions: chain observables, energies,
// acceptance counters and the count sums of the last field update.
#pragma once

#include "soma_grid.hpp"

namespace soma {

constexpr uint32_t SOMA_FLAG_POSITION_BIT = 1u;  // a position non-finite or |x| >= 2^22

struct ObsPartial {
  double re2, rg2, b2, e_bond, e_field, pad;
};

struct Totals {
  unsigned long long accepted[4];   // local, smart MC, learned, bond-Gibbs
  unsigned long long attempted_learned;
  unsigned long long sum_a, sum_b;
  double re2, rg2, b2, e_bond, e_field, h_nb;
  uint32_t err, pad;
};

struct ObsArgs {
  const float *pos;
  const float *omega;
  uint32_t n_chains, n, n_a;
  uint32_t seg;      // lanes per chain: smallest power of two >= n, at most 64
  double inv_n;      // 1 / n
  double half_k0;
  double inv_nref;
  Grid grid;
  ObsPartial *partials;
  uint32_t *err;
  const ArchDev *arch;   // general architecture (types, bonds), or null: linear chain
};

template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double (*s)[NV]) {
  for (int off = 32; off > 0; off >>= 1)
#pragma unroll
    for (int j = 0; j < NV; ++j) v[j] += __shfl_down(v[j], off, 64);
  const uint32_t lane = threadIdx.x & 63u, wv = threadIdx.x >> 6;
  if (lane == 0)
#pragma unroll
    for (int j = 0; j < NV; ++j) s[wv][j] = v[j];
  __syncthreads();
  if (threadIdx.x == 0)
#pragma unroll
    for (int j = 0; j < NV; ++j) v[j] = ((s[0][j] + s[1][j]) + s[2][j]) + s[3][j];
}

// Per-chain observables, Eqs. (1)-(2) and (13): Re^2 = |r_{N-1} - r_0|^2,
// Rg^2 = (1/N) sum |r_i - r_cm|^2, sum of squared bond lengths, bond energy
// (k0/2) sum b^2 (over the bond list for a general architecture) and field
// energy sum_i omega_t(c_i) / N. A chain occupies a
// segment of `seg` lanes (the smallest power of two >= N, at most 64) and bead
// i sits on lane i mod seg, so a wave reads 64/seg whole chains with adjacent
// lanes on adjacent beads. A block of four waves covers 256 consecutive chains
// (wave w the 64 from 64 w, seg groups of 64/seg chains). Per-lane FP64 sums,
// one fixed-order block reduction into a partial per block.
__global__ __launch_bounds__(256) void chain_obs_kernel(const ObsArgs a) {
  __shared__ double s[4][5];
  const uint32_t lane = threadIdx.x & 63u, wv = threadIdx.x >> 6;
  const uint32_t seg = a.seg, sl = lane & (seg - 1u), per = 64u / seg;
  const uint32_t first = blockIdx.x * 256u + wv * 64u + lane / seg;
  double re2 = 0, rg = 0, b2 = 0, ef = 0;
  bool bad = false;
  for (uint32_t g = 0; g < seg; ++g) {
    const uint32_t c = first + g * per;
    const bool live = c < a.n_chains;
    const float *p = a.pos + (size_t)(live ? c : 0u) * a.n * 3;
    double sx = 0, sy = 0, sz = 0;
    if (live) {
      for (uint32_t i = sl; i < a.n; i += seg) {
        const float x = p[3 * i], y = p[3 * i + 1], z = p[3 * i + 2];
        bad |= !(coord_ok(x) && coord_ok(y) && coord_ok(z));
        sx += x; sy += y; sz += z;
        if (a.arch) {   // each bond once, from its lower-numbered end
          for (uint32_t q = a.arch->nb_start[i]; q < a.arch->nb_start[i + 1]; ++q) {
            const uint32_t j = a.arch->nb[q];
            if (j < i) continue;
            const double dx = (double)x - p[3 * j], dy = (double)y - p[3 * j + 1],
                         dz = (double)z - p[3 * j + 2];
            b2 += dx * dx + dy * dy + dz * dz;
          }
        } else if (i > 0) {
          const double dx = (double)x - p[3 * i - 3], dy = (double)y - p[3 * i - 2],
                       dz = (double)z - p[3 * i - 1];
          b2 += dx * dx + dy * dy + dz * dz;
        }
        if (i == a.n - 1) {
          const double ex = (double)x - p[0], ey = (double)y - p[1], ez = (double)z - p[2];
          re2 += ex * ex + ey * ey + ez * ez;
        }
        const uint32_t cell = cell_of(a.grid, x, y, z);
        ef += (double)a.omega[(size_t)bead_type(a.arch, i, a.n_a) * a.grid.n_cells + cell];
      }
    }
    for (uint32_t off = seg >> 1; off > 0; off >>= 1) {   // sums within the segment
      sx += __shfl_xor(sx, off, 64);
      sy += __shfl_xor(sy, off, 64);
      sz += __shfl_xor(sz, off, 64);
    }
    if (live) {
      const double cx = sx * a.inv_n, cy = sy * a.inv_n, cz = sz * a.inv_n;
      for (uint32_t i = sl; i < a.n; i += seg) {
        const double dx = p[3 * i] - cx, dy = p[3 * i + 1] - cy, dz = p[3 * i + 2] - cz;
        rg += dx * dx + dy * dy + dz * dz;
      }
    }
  }
  if (bad) atomicOr(a.err, SOMA_FLAG_POSITION_BIT);
  double v[5] = {re2, rg * a.inv_n, b2, a.half_k0 * b2, ef * a.inv_nref};
  block_sum<5>(v, s);
  if (threadIdx.x == 0) {
    ObsPartial o;
    o.re2 = v[0]; o.rg2 = v[1]; o.b2 = v[2]; o.e_bond = v[3]; o.e_field = v[4]; o.pad = 0;
    a.partials[blockIdx.x] = o;
  }
}

// Single block: fixed-order reduction of all partials into one Totals record.
// acc_slots holds kAccSlots counters for each of local, smart-MC, learned and
// bond-Gibbs moves; att_slots the attempted learned moves.
__global__ __launch_bounds__(256) void reduce_totals_kernel(
    const ObsPartial *op, uint32_t n_op, const FieldPartial *fp, uint32_t n_fp,
    const unsigned long long *acc_slots, const unsigned long long *att_slots,
    const uint32_t *err, Totals *out) {
  __shared__ double s[4][6];
  __shared__ unsigned long long su[4][7];
  double v[6] = {0, 0, 0, 0, 0, 0};
  unsigned long long u[7] = {0, 0, 0, 0, 0, 0, 0};
  for (uint32_t i = threadIdx.x; i < n_op; i += blockDim.x) {
    v[0] += op[i].re2; v[1] += op[i].rg2; v[2] += op[i].b2;
    v[3] += op[i].e_bond; v[4] += op[i].e_field;
  }
  for (uint32_t i = threadIdx.x; i < n_fp; i += blockDim.x) {
    u[3] += fp[i].sum_a; u[4] += fp[i].sum_b; v[5] += fp[i].h_nb;
  }
  for (uint32_t i = threadIdx.x; i < kAccSlots; i += blockDim.x) {
    u[0] += acc_slots[i];
    u[1] += acc_slots[kAccSlots + i];
    u[2] += acc_slots[2 * kAccSlots + i];
    u[5] += att_slots[i];
    u[6] += acc_slots[3 * kAccSlots + i];
  }
  block_sum<6>(v, s);
  for (int off = 32; off > 0; off >>= 1)
#pragma unroll
    for (int j = 0; j < 7; ++j) u[j] += __shfl_down(u[j], off, 64);
  const uint32_t lane = threadIdx.x & 63u, wv = threadIdx.x >> 6;
  if (lane == 0)
#pragma unroll
    for (int j = 0; j < 7; ++j) su[wv][j] = u[j];
  __syncthreads();
  if (threadIdx.x == 0) {
    Totals t;
#pragma unroll
    for (int j = 0; j < 3; ++j) t.accepted[j] = su[0][j] + su[1][j] + su[2][j] + su[3][j];
    t.accepted[3] = su[0][6] + su[1][6] + su[2][6] + su[3][6];
    t.sum_a = su[0][3] + su[1][3] + su[2][3] + su[3][3];
    t.sum_b = su[0][4] + su[1][4] + su[2][4] + su[3][4];
    t.attempted_learned = su[0][5] + su[1][5] + su[2][5] + su[3][5];
    t.re2 = v[0]; t.rg2 = v[1]; t.b2 = v[2]; t.e_bond = v[3]; t.e_field = v[4];
    t.h_nb = v[5];
    t.err = *err;
    t.pad = 0;
    *out = t;
  }
}

}  // namespace soma
