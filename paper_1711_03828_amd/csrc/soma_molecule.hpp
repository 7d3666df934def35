// soma_molecule.hpp -- local-move sweep in the molecule-parallel order.
#pragma once

#include "soma_sweep.hpp"

namespace soma {

constexpr uint32_t kPurposeMolecule = 6u;  // attempt s: displacement (words 0-2), acceptance (3)
constexpr uint32_t kPurposePick = 7u;      // block floor(s/4), word s mod 4: bead of attempt s

// Sec. 3.1.2, scheme 1 (parallelization over distinct molecules): one lane
// per chain.  The lane makes N local attempts one after another; attempt s
// moves bead floor(word * N / 2^32), word s mod 4 of the chain's purpose-7
// block floor(s/4), so a bead is attempted once per sweep on average and the
// pick does not depend on the configuration.  The attempt itself is the
// LOCAL move with the SET sweep's FP32 arithmetic (trial position, bond and
// field energy change, Metropolis test), drawn from the purpose-6 block of
// attempt s.  Each lane reads and writes its own chain in place, so a later
// attempt sees every earlier one; the lanes of a wave touch 64 different
// chains (384 B apart for N = 32), so these accesses are not coalesced and
// hit in L2 only while few chains are in flight.  The grid may therefore be
// smaller than one lane per chain: lanes then loop over chains with the
// grid's stride (chains running together on one XCD stay one contiguous,
// spatially compact range).
template <bool COUNT64>
__global__ __launch_bounds__(256) void mc_sweep_molecule_kernel(const SweepArgs a_in) {
  const SweepArgs a = resolve_sweep(a_in, 0u);
  const uint64_t stride = (uint64_t)gridDim.x * 256u;
  uint32_t n_acc = 0;
  for (uint64_t c64 = (uint64_t)xcd_remap(blockIdx.x, gridDim.x) * 256u + threadIdx.x;
       __ballot(c64 < a.n_sub) != 0ull; c64 += stride) {
    if (c64 >= a.n_sub) continue;
    const uint32_t cl = (uint32_t)c64;
    const uint32_t N = a.n;
    const uint32_t chain = cl * a.sub_k + a.sub_j;
    const uint32_t gchain = a.chain_base + chain;
    float *cp = a.pos + (size_t)chain * N * 3u;
    Rand4 pick = {0u, 0u, 0u, 0u};
    for (uint32_t s = 0; s < N; ++s) {
      if ((s & 3u) == 0u)
        pick = philox(gchain, (s >> 2) | (kPurposePick << 16), a.sweep, a.replica, a.seed_lo, a.seed_hi);
      const uint32_t q = s & 3u;
      const uint32_t word = q == 0u ? pick.x : (q == 1u ? pick.y : (q == 2u ? pick.z : pick.w));
      const uint32_t i = __umulhi(word, N);
      float *p = cp + 3u * i;
      const F3 r = {p[0], p[1], p[2]};
      const bool has_l = i > 0u, has_r = i + 1u < N;
      F3 left = r, right = r;
      if (has_l) left = F3{p[-3], p[-2], p[-1]};
      if (has_r) right = F3{p[3], p[4], p[5]};
      const Rand4 w = philox(gchain, s | (kPurposeMolecule << 16), a.sweep, a.replica, a.seed_lo, a.seed_hi);
      const F3 t = {fmaf(a.step, uniform11(w.x), r.x), fmaf(a.step, uniform11(w.y), r.y),
                    fmaf(a.step, uniform11(w.z), r.z)};
      uint32_t x, y, z;
      cell3(a.grid, r.x, r.y, r.z, x, y, z);
      const uint32_t co = cell_index(a.grid, x, y, z);
      const uint32_t cn = cell_index(a.grid, shift_cell(x, r.x, t.x, a.grid.nx),
                                     shift_cell(y, r.y, t.y, a.grid.ny),
                                     shift_cell(z, r.z, t.z, a.grid.nz));
      const bool is_b = i >= a.n_a;
      const uint32_t pl = is_b ? a.grid.n_cells : 0u;
      const float wo = field_at(a.omega, pl, co);
      const float wn = cn == co ? wo : field_at(a.omega, pl, cn);
      const F3 d = t - r;
      const float wl = has_l ? 1.0f : 0.0f, wr = has_r ? 1.0f : 0.0f;
      const F3 qv = wl * (2.0f * (r - left) + d) + wr * (2.0f * (r - right) + d);
      const float d_e = a.half_k0 * (d.x * qv.x + d.y * qv.y + d.z * qv.z) + (wn - wo) * a.inv_nref;
      const bool acc = move_allowed(a, co, cn) && (d_e <= 0.0f || uniform01(w.w) < __expf(-d_e));
      if (acc) {
        p[0] = t.x;
        p[1] = t.y;
        p[2] = t.z;
        if (cn != co) move_count<COUNT64>(a.counts, co, cn, is_b);
      }
      n_acc += (uint32_t)__popcll(__ballot(acc));
    }
  }
  finish_block(a, n_acc);
}

}  // namespace soma
