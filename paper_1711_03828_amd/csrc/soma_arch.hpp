// soma_arch.hpp -- general molecular architectures: device tables and the SET
// sweep over arbitrary bond graphs.
#pragma once

#include "soma_sweep.hpp"

namespace soma {

constexpr uint32_t kPurposeSetOrder = 8u; // Philox purpose of the shuffled set order

// Sec. 3.1.2, scheme 2, for any architecture: a wave holds A->per_wave
// molecules (consecutive in the launch's chain subset), each on 64/per_wave
// lanes, their positions staged in LDS; every molecule walks its independent
// sets in its own order for this sweep (two sets: set 1 first iff bit 0 of
// word 0 of monomer 0's move draw, as for linear chains; more: a Fisher-Yates
// shuffle from the purpose-8 blocks; set_order = 1: numerical order), the
// members of a set on the molecule's lanes at once.  A move is the LOCAL move
// of the linear kernel, the bond term summed over the monomer's bond list in
// list order, so a linear chain given as an architecture moves bit for bit as
// in mc_sweep_local_kernel.  A monomer of type t sees field plane t and
// counts in half t & 1 of count plane t >> 1 (any number of types).
template <bool COUNT64>
__global__ __launch_bounds__(256) void mc_sweep_arch_kernel(const SweepArgs a_in,
                                                            const ArchDev *__restrict__ A) {
  __shared__ float s_pos[4][3 * kArchMaxN];
  __shared__ uint8_t s_order[4][64][kArchMaxSets];   // per wave and molecule slot
  const SweepArgs a = resolve_sweep(a_in, 0u);
  const uint32_t lane = threadIdx.x & 63u, wv = threadIdx.x >> 6;
  const uint32_t N = A->n, k = A->n_sets, M = A->per_wave, L = 64u / M;
  const uint32_t mi = lane / L, li = lane - mi * L;
  const uint32_t wave = xcd_remap(blockIdx.x, gridDim.x) * 4u + wv;
  const uint32_t cl0 = wave * M;                       // first molecule of the wave
  const uint32_t n_here = cl0 < a.n_sub ? min(M, a.n_sub - cl0) : 0u;
  const bool mine = mi < n_here;                       // this lane's molecule exists
  const uint32_t cl = cl0 + mi;
  const uint32_t chain = cl * a.sub_k + a.sub_j;
  const uint32_t gchain = a.chain_base + chain;
  float *sp = s_pos[wv] + 3u * N * mi;                 // this lane's molecule in LDS
  float *cp = a.pos + (size_t)(mine ? chain : 0u) * N * 3u;
  uint32_t n_acc = 0;
  if (n_here > 0) {
    for (uint32_t q = li; q < 3u * N; q += L)
      if (mine) sp[q] = cp[q];
    if (mine && li == 0) {
      uint8_t *ord = s_order[wv][mi];
      for (uint32_t s = 0; s < k; ++s) ord[s] = (uint8_t)s;
      if (a.set_order == 0 && k == 2) {
        const Rand4 d = philox(gchain, 0u, a.sweep, a.replica, a.seed_lo, a.seed_hi);
        if (d.x & 1u) { ord[0] = 1; ord[1] = 0; }
      } else if (a.set_order == 0 && k > 2) {
        Rand4 d = {0u, 0u, 0u, 0u};
        for (uint32_t t = k - 1, st = 0; t >= 1; --t, ++st) {
          if ((st & 3u) == 0u)
            d = philox(gchain, (st >> 2) | (kPurposeSetOrder << 16), a.sweep, a.replica, a.seed_lo,
                       a.seed_hi);
          const uint32_t q = st & 3u;
          const uint32_t word = q == 0u ? d.x : (q == 1u ? d.y : (q == 2u ? d.z : d.w));
          const uint32_t j = __umulhi(word, t + 1u);
          const uint8_t tmp = ord[t];
          ord[t] = ord[j];
          ord[j] = tmp;
        }
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    for (uint32_t s = 0; s < k; ++s) {
      const uint32_t set = mine ? s_order[wv][mi][s] : 0u;
      const uint32_t m0 = A->set_start[set], m1 = A->set_start[set + 1];
      // the wave loops as long as any of its molecules has members left
      uint32_t span = mine ? m1 - m0 : 0u;
      for (uint32_t off = 32u; off >= 1u; off >>= 1) span = max(span, (uint32_t)__shfl_xor((int)span, (int)off, 64));
      for (uint32_t base = 0; base < span; base += L) {
        const uint32_t idx = m0 + base + li;
        bool acc = false;
        if (mine && idx < m1) {
          const uint32_t i = A->member[idx];
          const F3 r = {sp[3 * i], sp[3 * i + 1], sp[3 * i + 2]};
          const Rand4 w = philox(gchain, i | (kPurposeMoveA << 16), a.sweep, a.replica, a.seed_lo,
                                 a.seed_hi);
          const F3 t = {fmaf(a.step, uniform11(w.x), r.x), fmaf(a.step, uniform11(w.y), r.y),
                        fmaf(a.step, uniform11(w.z), r.z)};
          const F3 d = t - r;
          F3 qv = {0.f, 0.f, 0.f};
          for (uint32_t b = A->nb_start[i]; b < A->nb_start[i + 1]; ++b) {
            const uint32_t j = A->nb[b];
            const F3 rj = {sp[3 * j], sp[3 * j + 1], sp[3 * j + 2]};
            qv = qv + (2.0f * (r - rj) + d);
          }
          uint32_t x, y, z;
          cell3(a.grid, r.x, r.y, r.z, x, y, z);
          const uint32_t co = cell_index(a.grid, x, y, z);
          const uint32_t cn = cell_index(a.grid, shift_cell(x, r.x, t.x, a.grid.nx),
                                         shift_cell(y, r.y, t.y, a.grid.ny),
                                         shift_cell(z, r.z, t.z, a.grid.nz));
          const uint32_t ty = A->type[i];
          const uint32_t pl = ty * a.grid.n_cells;          // field plane of the type
          const float wo = field_at(a.omega, pl, co);
          const float wn = cn == co ? wo : field_at(a.omega, pl, cn);
          const float d_e = a.half_k0 * (d.x * qv.x + d.y * qv.y + d.z * qv.z) + (wn - wo) * a.inv_nref;
          acc = move_allowed(a, co, cn) && (d_e <= 0.0f || uniform01(w.w) < __expf(-d_e));
          if (acc) {
            sp[3 * i] = t.x;
            sp[3 * i + 1] = t.y;
            sp[3 * i + 2] = t.z;
            if (cn != co) {   // count plane ty >> 1, half ty & 1
              const uint32_t pw = (ty >> 1) * a.grid.n_cells;
              move_count<COUNT64>(a.counts, co + pw, cn + pw, (ty & 1u) != 0u);
            }
          }
        }
        n_acc += (uint32_t)__popcll(__ballot(acc));
      }
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    }
    for (uint32_t q = li; q < 3u * N; q += L)
      if (mine) cp[q] = sp[q];
  }
  finish_block(a, n_acc);
}

}  // namespace soma
