// soma_sweep.hpp -- the MC sweep kernel (stage 2 of the SCMF cycle, Sec. 2.2)
// with the occupation histogram of the final positions fused as its epilogue.
//
// Work decomposition (the "SET" scheme of Sec. 3.1.2 mapped on wave64):
// a chain of N beads occupies ceil(N/2) consecutive lanes of one wavefront;
// lane k holds beads 2k (even set) and 2k+1 (odd set) in registers for the
// whole sweep.  The two sets are moved one after the other in a random order
// per chain; within a set every lane moves its bead at once, since the beads
// of one set are not bonded to each other.  The neighbour a moving bead needs
// from the adjacent lane is exchanged through the cross-lane network, so each
// bead is read from and written to HBM exactly once per sweep.
#pragma once

#include "soma_device.hpp"

namespace soma {

struct SweepArgs {
  float *pos;                      // first bead of the species
  const float *omega;              // [2][n_cells]
  void *counts;                    // packed per-cell counts
  unsigned long long *acc_slots;   // [kAccSlots] accepted-move counters
  uint32_t *err;                   // device error word
  Grid grid;
  uint32_t n_chains, n, n_a;
  uint32_t lanes_per_chain, chains_per_wave;
  uint32_t chain_base;             // global index of the species' first chain
  float half_k0, k0;
  float step;                      // local: a; smart MC: A
  float sqrt_2a, inv_4a;           // smart MC only
  float inv_nref;
  uint32_t seed_lo, seed_hi, sweep, replica;
  uint32_t set_order;              // 0 random per chain and sweep, 1 even first
};

struct F3 {
  float x, y, z;
};

__device__ __forceinline__ F3 sel(bool c, F3 a, F3 b) {
  return {c ? a.x : b.x, c ? a.y : b.y, c ? a.z : b.z};
}

__device__ __forceinline__ float shfl_f(float v, int src) {
  return __int_as_float(__builtin_amdgcn_ds_bpermute(src << 2, __float_as_int(v)));
}

// Central-difference gradient of one field plane at cell (cx,cy,cz), the
// force of the grid field on a bead being -(1/N) grad omega.
__device__ __forceinline__ F3 field_grad(const Grid &g, const float *om,
                                         uint32_t cx, uint32_t cy,
                                         uint32_t cz) {
  const uint32_t xp = cx + 1 == (uint32_t)g.nx ? 0 : cx + 1;
  const uint32_t xm = cx == 0 ? g.nx - 1 : cx - 1;
  const uint32_t yp = cy + 1 == (uint32_t)g.ny ? 0 : cy + 1;
  const uint32_t ym = cy == 0 ? g.ny - 1 : cy - 1;
  const uint32_t zp = cz + 1 == (uint32_t)g.nz ? 0 : cz + 1;
  const uint32_t zm = cz == 0 ? g.nz - 1 : cz - 1;
  F3 r;
  r.x = 0.5f * (om[cell_index(g, xp, cy, cz)] - om[cell_index(g, xm, cy, cz)]);
  r.y = 0.5f * (om[cell_index(g, cx, yp, cz)] - om[cell_index(g, cx, ym, cz)]);
  r.z = 0.5f * (om[cell_index(g, cx, cy, zp)] - om[cell_index(g, cx, cy, zm)]);
  return r;
}

template <bool SMC, bool COUNT64, bool VEC2, bool HIST>
__global__ __launch_bounds__(256) void mc_sweep_kernel(const SweepArgs a) {
  __shared__ uint32_t s_acc[4];
  const int lane = (int)(threadIdx.x & 63u);
  const uint32_t wib = threadIdx.x >> 6;
  const uint32_t tile = xcd_remap(blockIdx.x, gridDim.x);
  const uint32_t L = a.lanes_per_chain;
  const uint32_t slot = (uint32_t)lane / L;
  const uint32_t k = (uint32_t)lane - slot * L;
  const uint32_t chain = (tile * 4u + wib) * a.chains_per_wave + slot;
  const bool active = slot < a.chains_per_wave && chain < a.n_chains;
  const uint32_t N = a.n;
  const uint32_t i0 = 2u * k, i1 = 2u * k + 1u;
  const bool has0 = active;            // 2k < N for every k < ceil(N/2)
  const bool has1 = active && i1 < N;
  float *cp = a.pos + (size_t)(active ? chain : 0u) * N * 3u + 6u * k;

  F3 r0 = {0.f, 0.f, 0.f}, r1 = {0.f, 0.f, 0.f};
  if (VEC2) {
    if (has0) {
      const float2 p0 = reinterpret_cast<const float2 *>(cp)[0];
      const float2 p1 = reinterpret_cast<const float2 *>(cp)[1];
      const float2 p2 = reinterpret_cast<const float2 *>(cp)[2];
      r0 = {p0.x, p0.y, p1.x};
      r1 = {p1.y, p2.x, p2.y};
    }
  } else {
    if (has0) r0 = {cp[0], cp[1], cp[2]};
    if (has1) r1 = {cp[3], cp[4], cp[5]};
  }

  const uint32_t gchain = a.chain_base + chain;
  const Rand4 wa0 = philox(gchain, i0 | (kPurposeMoveA << 16), a.sweep, a.replica, a.seed_lo, a.seed_hi);
  const Rand4 wa1 = philox(gchain, i1 | (kPurposeMoveA << 16), a.sweep, a.replica, a.seed_lo, a.seed_hi);
  Rand4 wb0 = {0, 0, 0, 0}, wb1 = {0, 0, 0, 0};
  if (SMC) {
    wb0 = philox(gchain, i0 | (kPurposeMoveB << 16), a.sweep, a.replica, a.seed_lo, a.seed_hi);
    wb1 = philox(gchain, i1 | (kPurposeMoveB << 16), a.sweep, a.replica, a.seed_lo, a.seed_hi);
  }
  // Set order: bit 0 of the first word of bead 0's draw, broadcast from the
  // chain's first lane (the displacement uses only bits 9..31 of that word).
  uint32_t first = 0;
  if (a.set_order == 0) {
    const int src = lane - (int)k;
    first = (uint32_t)__builtin_amdgcn_ds_bpermute(src << 2, (int)(wa0.x & 1u));
  }

  uint32_t cell0 = 0, cell1 = 0;
  uint32_t n_acc = 0;
#pragma unroll
  for (int pass = 0; pass < 2; ++pass) {
    const bool odd = (pass == 0 ? first : first ^ 1u) != 0u;
    // neighbour from the adjacent lane: even pass needs bead 2k-1 (odd bead of
    // lane k-1), odd pass needs bead 2k+2 (even bead of lane k+1)
    const F3 send = sel(odd, r0, r1);
    const int src = odd ? (lane < 63 ? lane + 1 : lane) : (lane > 0 ? lane - 1 : lane);
    const F3 nb = {shfl_f(send.x, src), shfl_f(send.y, src), shfl_f(send.z, src)};
    const F3 left = sel(odd, r0, nb);
    const F3 right = sel(odd, nb, r1);
    const bool moving = odd ? has1 : has0;
    const float wl = (odd || k > 0) ? 1.0f : 0.0f;
    const float wr = (odd ? (i1 + 1u < N) : (i1 < N)) ? 1.0f : 0.0f;
    const uint32_t mi = odd ? i1 : i0;
    const F3 r = sel(odd, r1, r0);
    const Rand4 w = odd ? wa1 : wa0;
    const float *om = a.omega + (mi < a.n_a ? 0u : a.grid.n_cells);

    bool acc = false;
    uint32_t cell_final = 0;
    if (moving) {
      uint32_t ox, oy, oz;
      cell3(a.grid, r.x, r.y, r.z, ox, oy, oz);
      const uint32_t co = cell_index(a.grid, ox, oy, oz);
      const F3 el = {r.x - left.x, r.y - left.y, r.z - left.z};
      const F3 er = {r.x - right.x, r.y - right.y, r.z - right.z};
      F3 rn;
      float log_q = 0.0f;
      float u;
      F3 f_old = {0.f, 0.f, 0.f}, g_old = {0.f, 0.f, 0.f};
      if (!SMC) {
        rn = {fmaf(a.step, uniform11(w.x), r.x), fmaf(a.step, uniform11(w.y), r.y),
              fmaf(a.step, uniform11(w.z), r.z)};
        u = uniform01(w.w);
      } else {
        const Rand4 wb = odd ? wb1 : wb0;
        float xi0, xi1, xi2, xi3;
        box_muller(w.x, w.y, xi0, xi1);
        box_muller(w.z, w.w, xi2, xi3);
        g_old = field_grad(a.grid, om, ox, oy, oz);
        f_old = {-a.k0 * (wl * el.x + wr * er.x) - a.inv_nref * g_old.x,
                 -a.k0 * (wl * el.y + wr * er.y) - a.inv_nref * g_old.y,
                 -a.k0 * (wl * el.z + wr * er.z) - a.inv_nref * g_old.z};
        rn = {fmaf(a.sqrt_2a, xi0, fmaf(a.step, f_old.x, r.x)),
              fmaf(a.sqrt_2a, xi1, fmaf(a.step, f_old.y, r.y)),
              fmaf(a.sqrt_2a, xi2, fmaf(a.step, f_old.z, r.z))};
        u = uniform01(wb.x);
      }
      uint32_t nx_, ny_, nz_;
      cell3(a.grid, rn.x, rn.y, rn.z, nx_, ny_, nz_);
      const uint32_t cn = cell_index(a.grid, nx_, ny_, nz_);
      const F3 d = {rn.x - r.x, rn.y - r.y, rn.z - r.z};
      if (SMC) {
        // force at the trial position with the same bonded neighbours; the
        // field gradient is constant inside a cell
        const F3 g_new = cn == co ? g_old : field_grad(a.grid, om, nx_, ny_, nz_);
        const F3 nl = {rn.x - left.x, rn.y - left.y, rn.z - left.z};
        const F3 nr = {rn.x - right.x, rn.y - right.y, rn.z - right.z};
        const F3 f_new = {-a.k0 * (wl * nl.x + wr * nr.x) - a.inv_nref * g_new.x,
                          -a.k0 * (wl * nl.y + wr * nr.y) - a.inv_nref * g_new.y,
                          -a.k0 * (wl * nl.z + wr * nr.z) - a.inv_nref * g_new.z};
        const F3 fw = {d.x - a.step * f_old.x, d.y - a.step * f_old.y, d.z - a.step * f_old.z};
        const F3 rv = {-d.x - a.step * f_new.x, -d.y - a.step * f_new.y, -d.z - a.step * f_new.z};
        const float fw2 = fw.x * fw.x + fw.y * fw.y + fw.z * fw.z;
        const float rv2 = rv.x * rv.x + rv.y * rv.y + rv.z * rv.z;
        log_q = (fw2 - rv2) * a.inv_4a;  // log q(r|r') - log q(r'|r)
      }
      // bond energy change in the difference form: sum_j d.(2 (r - r_j) + d)
      const float qx = wl * (2.0f * el.x + d.x) + wr * (2.0f * er.x + d.x);
      const float qy = wl * (2.0f * el.y + d.y) + wr * (2.0f * er.y + d.y);
      const float qz = wl * (2.0f * el.z + d.z) + wr * (2.0f * er.z + d.z);
      const float d_bond = a.half_k0 * (d.x * qx + d.y * qy + d.z * qz);
      const float w_old = om[co];
      const float w_new = cn == co ? w_old : om[cn];
      const float d_e = d_bond + (w_new - w_old) * a.inv_nref;
      if (!SMC) {
        acc = d_e <= 0.0f || u < __expf(-d_e);
      } else {
        const float lr = log_q - d_e;
        acc = lr >= 0.0f || u < __expf(lr);
      }
      cell_final = acc ? cn : co;
      if (acc) {
        if (odd) r1 = rn; else r0 = rn;
      }
    }
    if (odd) cell1 = cell_final; else cell0 = cell_final;
    n_acc += (uint32_t)__popcll(__ballot(acc));
  }

  if (VEC2) {
    if (has0) {
      reinterpret_cast<float2 *>(cp)[0] = make_float2(r0.x, r0.y);
      reinterpret_cast<float2 *>(cp)[1] = make_float2(r0.z, r1.x);
      reinterpret_cast<float2 *>(cp)[2] = make_float2(r1.y, r1.z);
    }
  } else {
    if (has0) { cp[0] = r0.x; cp[1] = r0.y; cp[2] = r0.z; }
    if (has1) { cp[3] = r1.x; cp[4] = r1.y; cp[5] = r1.z; }
  }

  const bool bad = (has0 && !(coord_ok(r0.x) && coord_ok(r0.y) && coord_ok(r0.z))) ||
                   (has1 && !(coord_ok(r1.x) && coord_ok(r1.y) && coord_ok(r1.z)));
  if (__ballot(bad) != 0ull && lane == 0) atomicOr(a.err, 1u);

  if (HIST) {
    // packed increment: one unit in the A or the B half of the cell word
    const unsigned shift = COUNT64 ? 32u : 16u;
    const unsigned long long inc0 = 1ull << (i0 < a.n_a ? 0u : shift);
    const unsigned long long inc1 = has1 ? 1ull << (i1 < a.n_a ? 0u : shift) : 0ull;
    if (has0) {
      const bool same = has1 && cell1 == cell0;
      const unsigned long long first_inc = same ? inc0 + inc1 : inc0;
      if (COUNT64) {
        unsigned long long *c = reinterpret_cast<unsigned long long *>(a.counts);
        atomicAdd(c + cell0, first_inc);
        if (has1 && !same) atomicAdd(c + cell1, inc1);
      } else {
        unsigned int *c = reinterpret_cast<unsigned int *>(a.counts);
        atomicAdd(c + cell0, (unsigned int)first_inc);
        if (has1 && !same) atomicAdd(c + cell1, (unsigned int)inc1);
      }
    }
  }

  if (lane == 0) s_acc[wib] = n_acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint32_t tot = s_acc[0] + s_acc[1] + s_acc[2] + s_acc[3];
    if (tot) atomicAdd(a.acc_slots + (tile & (kAccSlots - 1u)), (unsigned long long)tot);
  }
}

}  // namespace soma
