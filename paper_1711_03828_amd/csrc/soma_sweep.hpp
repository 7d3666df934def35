// soma_sweep.hpp -- the MC sweep kernels (stage 2 of the SCMF cycle, Sec. 2.2)
// with the occupation histogram kept current in the same pass.
//
// Work decomposition (the "SET" scheme of Sec. 3.1.2 mapped on wave64):
// a chain of N beads occupies ceil(N/2) consecutive lanes of one wavefront;
// lane k holds beads 2k (even set) and 2k+1 (odd set) in registers for the
// whole sweep.  The two sets are moved one after the other in a random order
// per chain; within a set every lane moves its bead at once, since the beads
// of one set are not bonded to each other.  The neighbour a moving bead needs
// from the adjacent lane comes through the cross-lane network, so each bead is
// read from and written to HBM exactly once per sweep.
//
// Histogram: the counts always hold the occupation numbers of the current
// positions (Eq. (4)).  A sweep moves every bead once, so the histogram of the
// final positions is the old one minus each bead at its old cell plus each
// bead at its new cell; only beads that changed cell need the two integer
// atomics.  Integer addition is exact and order-independent, so the result is
// bit-identical to counting the final positions from scratch.
#pragma once

#include "soma_bins.hpp"
#include "soma_device.hpp"
#include "soma_mlp.hpp"

namespace soma {

struct SweepArgs {
  float *pos;                      // first bead of the species
  const float *omega;              // [2][n_cells]
  void *counts;                    // packed per-cell counts
  unsigned long long *acc_slots;   // [kAccSlots] accepted-move counters
  Grid grid;
  uint32_t n_chains, n, n_a;
  uint32_t lanes_per_chain, chains_per_wave;
  uint32_t chain_base;             // global index of the species' first chain
  float half_k0, k0;
  float step;                      // local: a; smart MC: A
  float sqrt_2a, inv_4a;           // smart MC only
  float inv_nref;
  uint32_t seed_lo, seed_hi;
  uint32_t sweep;                  // offset added to the device sweep counter
  uint32_t replica;
  uint32_t set_order;              // 0 random per chain and sweep, 1 even first
  const uint32_t *sweep_ctr;       // device sweep counter of the system
  // chain subset of this launch: chains sub_j, sub_j + sub_k, ... (n_sub of them);
  // sub_k = 1 moves every chain
  uint32_t sub_k, sub_j, n_sub;
  // optional [2][n_cells] (omega, d omega/dx, d omega/dy, d omega/dz) per type and
  // cell, refreshed with the fields; null: smart-MC gathers the 6 neighbours
  const float4 *grad;
  // optional impenetrable cells, one bit per cell (null: none): a trial position
  // in such a cell, other than the bead's own, is rejected
  const uint32_t *forbid;
  // bond-Gibbs moves: standard deviation of the trial around the mean of two
  // bonded neighbours, 1/sqrt(2 k0) (also the step of a bead without bonds),
  // and around one, 1/sqrt(k0)
  float gibbs_s2, gibbs_s1;
  // per-brick bins of count updates (kernels instantiated with BINNED); the
  // counts are current only after bin_apply_kernel has run
  BinArgs bin;
  // energy added to every move that changes cell (0: the quasi-instantaneous
  // field alone); see soma_set_self_term
  float self_term;
  // persistent local sweeps: kQueueParts x kQueueSub tile counters, kQueueStride
  // words apart, zeroed before the launch (null: the static tile order)
  uint32_t *queue;
  // waves per block of the launch (blockDim.x / 64), as a kernel argument: it
  // loads with the other arguments, while the block size itself is a 16-bit
  // field that costs a vector load ahead of everything that depends on it
  uint32_t wpb;
  // ceil(2^16 / lanes_per_chain): lane / lanes_per_chain = (lane lpc_magic) >> 16
  // for every lane < 64 (exact while lanes_per_chain < 1024)
  uint32_t lpc_magic;
  // binned local sweeps read and write positions with the non-temporal hint
  // (1: melts whose positions outgrow the last-level cache; each is touched
  // once per sweep, and the hint keeps the field and count lines cached instead)
  uint32_t stream_pos;
};

constexpr uint32_t kQueueParts = 8u, kQueueSub = 16u, kQueueStride = 32u;

// Zeroes the tile counters of a persistent sweep (a kernel, not a memset, so
// that it can sit in a captured graph).
__global__ __launch_bounds__(256) void queue_reset_kernel(uint32_t *q) {
  for (uint32_t i = threadIdx.x; i < kQueueParts * kQueueSub; i += blockDim.x)
    q[i * kQueueStride] = 0u;
}

// Tiles of a persistent SET sweep (PERSIST instances; SweepArgs::queue set).  The tiles (one
// wave's chains each) are dealt XCD by XCD when the grid is a multiple of 8
// blocks: part x owns the contiguous range [x T/8, (x+1) T/8), so the waves
// running together on one XCD share one compact region of the grid.  Each
// part hands out its tiles through S = min(kQueueSub, waves of the part)
// counters; a wave draws from counter (wave mod S), which owns the tiles
// sub + S j of the part (every counter has a wave), so that the part's waves
// stay on one moving window of tiles however their speeds differ.  (With a
// fixed stride per wave, waves drift apart over their ~200 tiles and the
// window they cover outgrows L2: half again as many HBM reads.)
struct TileIter {
  uint32_t *q;
  uint32_t t_begin, t_end, n_sq, sq;
  bool lead;
};

__device__ __forceinline__ TileIter tile_iter(const SweepArgs &a) {
  TileIter it;
  const uint32_t n_tiles = (a.n_sub + a.chains_per_wave - 1u) / a.chains_per_wave;
  const uint32_t blocks = gridDim.x;
  const uint32_t parts = (blocks & 7u) == 0u ? 8u : 1u;
  const uint32_t part = blockIdx.x % parts;
  const uint32_t wpb = a.wpb;
  const uint32_t waves_per_part = (blocks / parts) * wpb;
  const uint32_t wave_in_part = (blockIdx.x / parts) * wpb + (threadIdx.x >> 6);
  it.t_begin = (uint32_t)(((uint64_t)n_tiles * part) / parts);
  it.t_end = (uint32_t)(((uint64_t)n_tiles * (part + 1u)) / parts);
  it.n_sq = waves_per_part < kQueueSub ? waves_per_part : kQueueSub;
  it.sq = wave_in_part % it.n_sq;
  it.q = a.queue + (part * kQueueSub + it.sq) * kQueueStride;
  it.lead = (threadIdx.x & 63u) == 0u;
  return it;
}

// Draws the wave's next tile index (lane 0; the value may still be in flight).
__device__ __forceinline__ uint32_t tile_draw(const TileIter &it) {
  uint32_t v = 0u;
  if (it.lead) v = atomicAdd(it.q, 1u);
  return v;
}

// The tile of a draw (>= t_end: no tiles left for this wave).
__device__ __forceinline__ uint32_t tile_of(const TileIter &it, uint32_t v) {
  return it.t_begin + it.sq + it.n_sq * (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
}

// A move from cell `from` to cell `to` that the impenetrable cells allow.
__device__ __forceinline__ bool move_allowed(const SweepArgs &a, uint32_t from, uint32_t to) {
  return a.forbid == nullptr || to == from || ((a.forbid[to >> 5] >> (to & 31u)) & 1u) == 0u;
}

// With impenetrable cells set, a trial more than one cell away from the bead
// along any axis is rejected as well (floor(x') - floor(x) outside {-1, 0, 1}
// on the unwrapped coordinates), so that no move can jump over a wall.  The
// condition is symmetric in (r, r'): detailed balance holds for the
// restricted move.  Local moves (half-width below one cell) always pass.
__device__ __forceinline__ bool step_allowed(const SweepArgs &a, F3 r, F3 rn) {
  return a.forbid == nullptr ||
         (fabsf(floorf(rn.x) - floorf(r.x)) <= 1.0f && fabsf(floorf(rn.y) - floorf(r.y)) <= 1.0f &&
          fabsf(floorf(rn.z) - floorf(r.z)) <= 1.0f);
}

// Arguments with the Philox sweep word resolved: the system's device counter
// plus the launch's offset, so that a launch recorded once (a captured graph)
// still draws fresh numbers on every replay.
__device__ __forceinline__ SweepArgs resolve_sweep(const SweepArgs &in, uint32_t extra) {
  SweepArgs a = in;
  a.sweep = in.sweep + extra + *in.sweep_ctr;
  return a;
}

__device__ __forceinline__ F3 sel(bool c, F3 a, F3 b) { return c ? a : b; }

__device__ __forceinline__ float shfl_f(float v, int src) {
  return __int_as_float(__builtin_amdgcn_ds_bpermute(src << 2, __float_as_int(v)));
}

// Lane geometry of one wave: which chain and which bead pair a lane holds.
struct LaneMap {
  int lane;
  uint32_t k;           // pair index in the chain
  uint32_t chain;       // chain index within the species
  bool has0, has1;      // beads 2k and 2k+1 exist
  uint32_t tile;
  uint32_t wib;
};

__device__ __forceinline__ LaneMap lane_map_tile(const SweepArgs &a, uint32_t tile, bool valid) {
  LaneMap m;
  m.lane = (int)(threadIdx.x & 63u);
  m.wib = threadIdx.x >> 6;
  m.tile = tile;
  const uint32_t L = a.lanes_per_chain;
  const uint32_t slot = __umul24((uint32_t)m.lane, a.lpc_magic) >> 16;
  m.k = (uint32_t)m.lane - slot * L;
  const uint32_t cl = tile * a.chains_per_wave + slot;   // index within the subset
  m.chain = cl * a.sub_k + a.sub_j;
  const bool active = valid && slot < a.chains_per_wave && cl < a.n_sub;
  m.has0 = active;  // 2k < N for every k < ceil(N/2)
  m.has1 = active && 2u * m.k + 1u < a.n;
  return m;
}

__device__ __forceinline__ LaneMap lane_map(const SweepArgs &a) {
  const uint32_t tile = xcd_remap(blockIdx.x, gridDim.x) * a.wpb + (threadIdx.x >> 6);
  return lane_map_tile(a, tile, true);
}

typedef float f32x2 __attribute__((ext_vector_type(2)));

// NT: the non-temporal hint (a compile-time choice: loads that differ only in
// the hint would be merged by the compiler, dropping it).
template <bool VEC2, bool NT = false>
__device__ __forceinline__ void load_pair(const float *cp, const LaneMap &m, F3 &r0, F3 &r1) {
  r0 = F3{0.f, 0.f, 0.f};
  r1 = F3{0.f, 0.f, 0.f};
  if (VEC2) {
    if (m.has0) {
      const f32x2 *q = reinterpret_cast<const f32x2 *>(cp);
      f32x2 p0, p1, p2;
      if (NT) {
        p0 = __builtin_nontemporal_load(q);
        p1 = __builtin_nontemporal_load(q + 1);
        p2 = __builtin_nontemporal_load(q + 2);
      } else {
        p0 = q[0];
        p1 = q[1];
        p2 = q[2];
      }
      r0 = F3{p0.x, p0.y, p1.x};
      r1 = F3{p1.y, p2.x, p2.y};
    }
  } else {
    if (m.has0) r0 = F3{cp[0], cp[1], cp[2]};
    if (m.has1) r1 = F3{cp[3], cp[4], cp[5]};
  }
}

template <bool VEC2, bool NT = false>
__device__ __forceinline__ void store_pair(float *cp, const LaneMap &m, F3 r0, F3 r1) {
  if (VEC2) {
    if (m.has0) {
      f32x2 *q = reinterpret_cast<f32x2 *>(cp);
      const f32x2 p0 = {r0.x, r0.y}, p1 = {r0.z, r1.x}, p2 = {r1.y, r1.z};
      if (NT) {
        __builtin_nontemporal_store(p0, q);
        __builtin_nontemporal_store(p1, q + 1);
        __builtin_nontemporal_store(p2, q + 2);
      } else {
        q[0] = p0;
        q[1] = p1;
        q[2] = p2;
      }
    }
  } else {
    if (m.has0) { cp[0] = r0.x; cp[1] = r0.y; cp[2] = r0.z; }
    if (m.has1) { cp[3] = r1.x; cp[4] = r1.y; cp[5] = r1.z; }
  }
}

// Move one bead's unit from cell `from` to cell `to` in the packed counts
// (32-bit byte offsets from the uniform base: counts < 4 GiB, host-checked).
// A count stays below 2^16 (u16 pairs) or 2^32 (u32 pairs), so adding -1 or +1
// to one half never carries into the other.
template <bool COUNT64>
__device__ __forceinline__ void move_count(void *counts, uint32_t from, uint32_t to, bool is_b) {
  char *base = reinterpret_cast<char *>(counts);
  if (COUNT64) {   // a bead changes only its own type's 32-bit half of the word
    const uint32_t half = is_b ? 4u : 0u;
    atomicAdd(reinterpret_cast<unsigned int *>(base + (from << 3) + half), 0xFFFFFFFFu);
    atomicAdd(reinterpret_cast<unsigned int *>(base + (to << 3) + half), 1u);
  } else {
    const unsigned int inc = is_b ? (1u << 16) : 1u;
    atomicAdd(reinterpret_cast<unsigned int *>(base + (from << 2)), 0u - inc);
    atomicAdd(reinterpret_cast<unsigned int *>(base + (to << 2)), inc);
  }
}

// Accepted-move count of the block (up to 16 waves) into one of kAccSlots
// counters (integer sums: the totals do not depend on the block size).
__device__ __forceinline__ void finish_block(const SweepArgs &a, uint32_t n_acc) {
  __shared__ uint32_t s_acc[16];
  if ((threadIdx.x & 63u) == 0u) s_acc[threadIdx.x >> 6] = n_acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t tot = 0;
    for (uint32_t w = 0; w < a.wpb; ++w) tot += s_acc[w];
    if (tot) atomicAdd(a.acc_slots + (blockIdx.x & (kAccSlots - 1u)), (unsigned long long)tot);
  }
  __syncthreads();
}

// Order of the two sets for this chain and sweep: bit 0 of the first word of
// bead 0's draw, broadcast from the chain's first lane (the displacement uses
// only bits 9..31 of that word).
__device__ __forceinline__ uint32_t set_order_bit(const SweepArgs &a, const LaneMap &m,
                                                  uint32_t w0x) {
  if (a.set_order != 0) return 0u;
  const int src = m.lane - (int)m.k;
  return (uint32_t)__builtin_amdgcn_ds_bpermute(src << 2, (int)(w0x & 1u));
}

// ---------------------------------------------------------------------------
// Local moves (Sec. 2.2, move (i)): uniform trial displacement in [-a,a] per
// Cartesian direction, Metropolis acceptance of
//   dE = (k0/2) sum_bonds (|r'-r_j|^2 - |r-r_j|^2) + (omega_t(c') - omega_t(c))/N.
// A trial position depends only on the bead itself, so both trial positions of
// a lane and the field values they need are fetched before either set moves;
// only the bond term waits for the other set.  Per lane the two beads are
// relabelled once by the chain's set order ("a" moves first, "b" second), so
// the passes need no per-pass selection.  Requires a < 1 cell (host-checked):
// a trial position is then at most one cell away along each axis.
// ---------------------------------------------------------------------------
// One wave's tile of local moves: positions r0/r1 already loaded for lane map m.
template <bool COUNT64, bool VEC2, bool BINNED, bool NT = false>
__device__ __forceinline__ uint32_t local_tile(const SweepArgs &a, const LaneMap &m, float *cp,
                                               F3 r0, F3 r1) {
  const uint32_t N = a.n;
  const uint32_t i0 = 2u * m.k, i1 = i0 + 1u;
  const uint32_t gchain = a.chain_base + m.chain;
  // old cells and their field values first: they need only the positions
  uint32_t x0, y0, z0, x1, y1, z1;
  cell3(a.grid, r0.x, r0.y, r0.z, x0, y0, z0);
  cell3(a.grid, r1.x, r1.y, r1.z, x1, y1, z1);
  const uint32_t c0 = cell_index(a.grid, x0, y0, z0);
  const uint32_t c1 = cell_index(a.grid, x1, y1, z1);
  const bool b0 = i0 >= a.n_a, b1 = i1 >= a.n_a;
  const uint32_t pl0 = b0 ? a.grid.n_cells : 0u, pl1 = b1 ? a.grid.n_cells : 0u;
  const float wo0 = field_at(a.omega, pl0, c0), wo1 = field_at(a.omega, pl1, c1);

  const Rand4 w0 = philox(gchain, i0 | (kPurposeMoveA << 16), a.sweep, a.replica, a.seed_lo, a.seed_hi);
  const Rand4 w1 = philox(gchain, i1 | (kPurposeMoveA << 16), a.sweep, a.replica, a.seed_lo, a.seed_hi);
  const bool odd_first = set_order_bit(a, m, w0.x) != 0u;

  // trial positions r' = fma(a, v, r) and their cells (at most one cell away)
  const F3 t0 = {fmaf(a.step, uniform11(w0.x), r0.x), fmaf(a.step, uniform11(w0.y), r0.y),
                 fmaf(a.step, uniform11(w0.z), r0.z)};
  const F3 t1 = {fmaf(a.step, uniform11(w1.x), r1.x), fmaf(a.step, uniform11(w1.y), r1.y),
                 fmaf(a.step, uniform11(w1.z), r1.z)};
  const uint32_t sx0 = shift_cell(x0, r0.x, t0.x, a.grid.nx),
                 sy0 = shift_cell(y0, r0.y, t0.y, a.grid.ny),
                 sz0 = shift_cell(z0, r0.z, t0.z, a.grid.nz);
  const uint32_t sx1 = shift_cell(x1, r1.x, t1.x, a.grid.nx),
                 sy1 = shift_cell(y1, r1.y, t1.y, a.grid.ny),
                 sz1 = shift_cell(z1, r1.z, t1.z, a.grid.nz);
  const uint32_t n0 = cell_index(a.grid, sx0, sy0, sz0);
  const uint32_t n1 = cell_index(a.grid, sx1, sy1, sz1);
  // brick keys of the four cells now, so that the coordinates die here
  const uint32_t kf0 = BINNED ? brick_key(a.bin, x0, y0, z0) : 0u;
  const uint32_t kt0 = BINNED ? brick_key(a.bin, sx0, sy0, sz0) : 0u;
  const uint32_t kf1 = BINNED ? brick_key(a.bin, x1, y1, z1) : 0u;
  const uint32_t kt1 = BINNED ? brick_key(a.bin, sx1, sy1, sz1) : 0u;
  // trial-cell values only where the trial leaves the cell, chosen afterwards.
  // With the old-cell value as the default of the load (which the compiler
  // makes of a plain choice unless the empty asm hides the loaded registers)
  // every gather waits for the one before it; this way all four are in flight
  // together.
  float g0 = 0.0f, g1 = 0.0f;
  if (n0 != c0) g0 = field_at(a.omega, pl0, n0);
  if (n1 != c1) g1 = field_at(a.omega, pl1, n1);
  asm volatile("" : "+v"(g0), "+v"(g1));
  const float wn0 = n0 != c0 ? g0 : wo0, wn1 = n1 != c1 ? g1 : wo1;
  const bool ok0 = move_allowed(a, c0, n0), ok1 = move_allowed(a, c1, n1);

  // relabel by set order: a moves first, b second
  const F3 ra0 = sel(odd_first, r1, r0), rb0 = sel(odd_first, r0, r1);
  const F3 ta = sel(odd_first, t1, t0), tb = sel(odd_first, t0, t1);
  const Rand4 wa = odd_first ? w1 : w0, wb = odd_first ? w0 : w1;
  const bool has_a = odd_first ? m.has1 : m.has0, has_b = odd_first ? m.has0 : m.has1;
  const bool ok_a = odd_first ? ok1 : ok0, ok_b = odd_first ? ok0 : ok1;
  const float sa = (odd_first ? n1 != c1 : n0 != c0) ? a.self_term : 0.0f;
  const float sb = (odd_first ? n0 != c0 : n1 != c1) ? a.self_term : 0.0f;
  const float dfa = ((odd_first ? wn1 : wn0) - (odd_first ? wo1 : wo0)) * a.inv_nref + sa;
  const float dfb = ((odd_first ? wn0 : wn1) - (odd_first ? wo0 : wo1)) * a.inv_nref + sb;
  // bonded neighbours of a: own b and b of the adjacent lane (lane k-1 if a is
  // even, lane k+1 if a is odd); of b: own a and a of the other adjacent lane
  const int up = m.lane < 63 ? m.lane + 1 : m.lane, dn = m.lane > 0 ? m.lane - 1 : m.lane;
  const int src_a = odd_first ? up : dn, src_b = odd_first ? dn : up;
  const bool lo_ok = m.k > 0, hi_ok = i1 + 1u < N;   // beads 2k-1 and 2k+2 exist
  const float wadj_a = (odd_first ? hi_ok : lo_ok) ? 1.0f : 0.0f;
  const float wadj_b = (odd_first ? lo_ok : hi_ok) ? 1.0f : 0.0f;
  const float wown_a = has_b ? 1.0f : 0.0f, wown_b = has_a ? 1.0f : 0.0f;

  // pass 1: set of a
  F3 ra = ra0;
  bool acc_a;
  {
    const F3 nb = {shfl_f(rb0.x, src_a), shfl_f(rb0.y, src_a), shfl_f(rb0.z, src_a)};
    const F3 d = ta - ra;
    const F3 q = wown_a * (2.0f * (ra - rb0) + d) + wadj_a * (2.0f * (ra - nb) + d);
    const float d_e = a.half_k0 * (d.x * q.x + d.y * q.y + d.z * q.z) + dfa;
    acc_a = has_a && ok_a && (d_e <= 0.0f || uniform01(wa.w) < __expf(-d_e));
    ra = acc_a ? ta : ra;
  }
  // pass 2: set of b, against the updated a beads
  F3 rb = rb0;
  bool acc_b;
  {
    const F3 nb = {shfl_f(ra.x, src_b), shfl_f(ra.y, src_b), shfl_f(ra.z, src_b)};
    const F3 d = tb - rb;
    const F3 q = wown_b * (2.0f * (rb - ra) + d) + wadj_b * (2.0f * (rb - nb) + d);
    const float d_e = a.half_k0 * (d.x * q.x + d.y * q.y + d.z * q.z) + dfb;
    acc_b = has_b && ok_b && (d_e <= 0.0f || uniform01(wb.w) < __expf(-d_e));
    rb = acc_b ? tb : rb;
  }
  store_pair<VEC2, NT>(cp, m, sel(odd_first, rb, ra), sel(odd_first, ra, rb));
  const bool acc0 = odd_first ? acc_b : acc_a, acc1 = odd_first ? acc_a : acc_b;
  if (BINNED) {
    bin_moves<COUNT64>(a.bin, a.grid, a.counts, wave_sub_bin(a.wpb), kf0, kt0, b0 ? 1u : 0u,
                       acc0 && n0 != c0, kf1, kt1, b1 ? 1u : 0u, acc1 && n1 != c1);
  } else {
    if (acc0 && n0 != c0) move_count<COUNT64>(a.counts, c0, n0, b0);
    if (acc1 && n1 != c1) move_count<COUNT64>(a.counts, c1, n1, b1);
  }
  return (uint32_t)(__popcll(__ballot(acc_a)) + __popcll(__ballot(acc_b)));
}

// ---------------------------------------------------------------------------
// Local moves (Sec. 2.2, move (i)): uniform trial displacement in [-a,a] per
// Cartesian direction, Metropolis acceptance of
//   dE = (k0/2) sum_bonds (|r'-r_j|^2 - |r-r_j|^2) + (omega_t(c') - omega_t(c))/N.
// A trial position depends only on the bead itself, so both trial positions of
// a lane and the field values they need are fetched before either set moves;
// only the bond term waits for the other set.  Per lane the two beads are
// relabelled once by the chain's set order ("a" moves first, "b" second), so
// the passes need no per-pass selection.  Requires a < 1 cell (host-checked):
// a trial position is then at most one cell away along each axis.
//
// Tiles (one wave's chains): one per wave, or drawn from per-XCD counters in
// a persistent grid (TileIter).
// ---------------------------------------------------------------------------
// Registers capped for five waves per SIMD (96 VGPRs, no spills), so that the
// persistent grid holds enough waves to cover the latency of its gathers and
// of the bin reservations.
template <bool COUNT64, bool VEC2, bool BINNED, bool PERSIST = false, bool NT = false>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(5)))
void mc_sweep_local_kernel(const SweepArgs a_in) {
  const SweepArgs a = resolve_sweep(a_in, 0u);
  if (!PERSIST) {   // one tile per wave
    const LaneMap m = lane_map(a);
    float *cp = a.pos + (size_t)(m.has0 ? m.chain : 0u) * a.n * 3u + 6u * m.k;
    F3 r0, r1;
    load_pair<VEC2, NT>(cp, m, r0, r1);
    finish_block(a, local_tile<COUNT64, VEC2, BINNED, NT>(a, m, cp, r0, r1));
    return;
  }
  const TileIter it = tile_iter(a);
  uint32_t n_acc = 0;
  uint32_t t = tile_of(it, tile_draw(it));
  while (t < it.t_end) {
    const uint32_t vn = tile_draw(it);   // the next tile, drawn while this one runs
    const LaneMap m = lane_map_tile(a, t, true);
    float *cp = a.pos + (size_t)(m.has0 ? m.chain : 0u) * a.n * 3u + 6u * m.k;
    F3 r0, r1;
    load_pair<VEC2, NT>(cp, m, r0, r1);
    n_acc += local_tile<COUNT64, VEC2, BINNED, NT>(a, m, cp, r0, r1);
    t = tile_of(it, vn);
  }
  finish_block(a, n_acc);
}

// Central-difference gradient of one field plane at cell (cx,cy,cz); the
// force of the grid field on a bead is -(1/N) grad omega.
__device__ __forceinline__ F3 field_grad(const Grid &g, const float *omega, uint32_t pl,
                                         uint32_t cx, uint32_t cy,
                                         uint32_t cz) {
  const uint32_t xp = cx + 1 == (uint32_t)g.nx ? 0 : cx + 1;
  const uint32_t xm = cx == 0 ? g.nx - 1 : cx - 1;
  const uint32_t yp = cy + 1 == (uint32_t)g.ny ? 0 : cy + 1;
  const uint32_t ym = cy == 0 ? g.ny - 1 : cy - 1;
  const uint32_t zp = cz + 1 == (uint32_t)g.nz ? 0 : cz + 1;
  const uint32_t zm = cz == 0 ? g.nz - 1 : cz - 1;
  F3 r;
  r.x = 0.5f * (field_at(omega, pl, cell_index(g, xp, cy, cz)) - field_at(omega, pl, cell_index(g, xm, cy, cz)));
  r.y = 0.5f * (field_at(omega, pl, cell_index(g, cx, yp, cz)) - field_at(omega, pl, cell_index(g, cx, ym, cz)));
  r.z = 0.5f * (field_at(omega, pl, cell_index(g, cx, cy, zp)) - field_at(omega, pl, cell_index(g, cx, cy, zm)));
  return r;
}

// Field value and central-difference gradient of plane `pl` at cell c = (cx,cy,cz):
// one 16-byte gather from the gradient field when it is kept, else 7 gathers.
__device__ __forceinline__ float field_and_grad(const SweepArgs &a, uint32_t pl, uint32_t c,
                                                uint32_t cx, uint32_t cy, uint32_t cz, F3 &g) {
  if (a.grad) {
    const float4 v = a.grad[pl + c];
    g = F3{v.y, v.z, v.w};
    return v.x;
  }
  g = field_grad(a.grid, a.omega, pl, cx, cy, cz);
  return field_at(a.omega, pl, c);
}

// ---------------------------------------------------------------------------
// Smart-MC moves (Sec. 2.2, move (ii)): r' = r + A F(r) + sqrt(2A) xi with the
// bonded force plus the grid-field force -(1/N) grad omega; accepted with
// min(1, exp(-dE) q(r|r')/q(r'|r)), q the Gaussian proposal density.  The
// trial position of the second set depends on the first set's outcome through
// the bonded force, so the sets are handled one after the other.
//
// GIBBS: bond-Gibbs moves instead.  The trial is drawn from the bead's law
// given its bonded neighbours under the bond energy (Eqs. (1)-(2)):
// r' = fma(s, xi, mu), mu = 0.5 (r_l + r_r) and s = 1/sqrt(2 k0) between two
// neighbours, mu = the neighbour and s = 1/sqrt(k0) at a chain end, mu = r and
// s = 1/sqrt(2 k0) without bonds.  The bond energy and the proposal densities
// then cancel in the Metropolis-Hastings ratio, which leaves
// exp(-(omega(c') - omega(c))/N).  Same draws as smart MC.
// ---------------------------------------------------------------------------
template <bool COUNT64, bool VEC2, bool BINNED, bool GIBBS = false>
__device__ __forceinline__ uint32_t smc_wave(const SweepArgs &a, const LaneMap &m) {
  const uint32_t N = a.n;
  const uint32_t i0 = 2u * m.k, i1 = i0 + 1u;
  float *cp = a.pos + (size_t)(m.has0 ? m.chain : 0u) * N * 3u + 6u * m.k;
  F3 r0, r1;
  load_pair<VEC2>(cp, m, r0, r1);

  const uint32_t gchain = a.chain_base + m.chain;
  const Rand4 wa0 = philox(gchain, i0 | (kPurposeMoveA << 16), a.sweep, a.replica, a.seed_lo, a.seed_hi);
  const Rand4 wa1 = philox(gchain, i1 | (kPurposeMoveA << 16), a.sweep, a.replica, a.seed_lo, a.seed_hi);
  const Rand4 wb0 = philox(gchain, i0 | (kPurposeMoveB << 16), a.sweep, a.replica, a.seed_lo, a.seed_hi);
  const Rand4 wb1 = philox(gchain, i1 | (kPurposeMoveB << 16), a.sweep, a.replica, a.seed_lo, a.seed_hi);
  const uint32_t first = set_order_bit(a, m, wa0.x);
  const bool b0 = i0 >= a.n_a, b1 = i1 >= a.n_a;

  // A bead's position does not change before its own pass, so the old cells
  // of both beads are known up front, and with the kept gradient field (one
  // gather per cell) so are their field values and gradients.
  uint32_t ox0, oy0, oz0, ox1, oy1, oz1;
  cell3(a.grid, r0.x, r0.y, r0.z, ox0, oy0, oz0);
  cell3(a.grid, r1.x, r1.y, r1.z, ox1, oy1, oz1);
  const uint32_t co0 = cell_index(a.grid, ox0, oy0, oz0), co1 = cell_index(a.grid, ox1, oy1, oz1);
  F3 g0 = {0.f, 0.f, 0.f}, g1 = {0.f, 0.f, 0.f};
  float f0 = 0.f, f1 = 0.f;
  if (GIBBS) {   // only the field values at the old cells
    if (m.has0) f0 = field_at(a.omega, b0 ? a.grid.n_cells : 0u, co0);
    if (m.has1) f1 = field_at(a.omega, b1 ? a.grid.n_cells : 0u, co1);
  } else if (a.grad) {
    if (m.has0) f0 = field_and_grad(a, b0 ? a.grid.n_cells : 0u, co0, ox0, oy0, oz0, g0);
    if (m.has1) f1 = field_and_grad(a, b1 ? a.grid.n_cells : 0u, co1, ox1, oy1, oz1, g1);
  }

  uint32_t from0 = 0, to0 = 0, from1 = 0, to1 = 0;
  bool moved0 = false, moved1 = false;
  uint32_t n_acc = 0;
#pragma unroll
  for (int pass = 0; pass < 2; ++pass) {
    const bool odd = (first ^ (uint32_t)pass) != 0u;
    const F3 send = sel(odd, r0, r1);
    const int src = odd ? (m.lane < 63 ? m.lane + 1 : m.lane) : (m.lane > 0 ? m.lane - 1 : m.lane);
    const F3 nb = {shfl_f(send.x, src), shfl_f(send.y, src), shfl_f(send.z, src)};
    const F3 left = sel(odd, r0, nb);
    const F3 right = sel(odd, nb, r1);
    const bool moving = odd ? m.has1 : m.has0;
    const float wl = (odd || m.k > 0) ? 1.0f : 0.0f;
    const float wr = (odd ? (i1 + 1u < N) : m.has1) ? 1.0f : 0.0f;
    const F3 r = sel(odd, r1, r0);
    const Rand4 w = odd ? wa1 : wa0;
    const float u = uniform01(odd ? wb1.x : wb0.x);
    const uint32_t pl = (odd ? b1 : b0) ? a.grid.n_cells : 0u;

    bool acc = false;
    uint32_t co = 0, cn = 0, ko = 0, kn = 0;
    F3 rn = r;
    if (GIBBS && moving) {
      co = odd ? co1 : co0;
      float xi0, xi1, xi2, xi3;
      box_muller(w.x, w.y, xi0, xi1);
      box_muller(w.z, w.w, xi2, xi3);
      F3 mu = r;
      float sg = a.gibbs_s2;
      if (wl > 0.0f && wr > 0.0f) {
        mu = {0.5f * (left.x + right.x), 0.5f * (left.y + right.y), 0.5f * (left.z + right.z)};
      } else if (wl > 0.0f || wr > 0.0f) {
        mu = wl > 0.0f ? left : right;
        sg = a.gibbs_s1;
      }
      rn = {fmaf(sg, xi0, mu.x), fmaf(sg, xi1, mu.y), fmaf(sg, xi2, mu.z)};
      uint32_t nx_, ny_, nz_;
      cell3(a.grid, rn.x, rn.y, rn.z, nx_, ny_, nz_);
      cn = cell_index(a.grid, nx_, ny_, nz_);
      if (BINNED) {
        ko = brick_key(a.bin, odd ? ox1 : ox0, odd ? oy1 : oy0, odd ? oz1 : oz0);
        kn = brick_key(a.bin, nx_, ny_, nz_);
      }
      const float w_old = odd ? f1 : f0;
      const float w_new = cn == co ? w_old : field_at(a.omega, pl, cn);
      const float d_e = (w_new - w_old) * a.inv_nref + (cn != co ? a.self_term : 0.0f);
      acc = move_allowed(a, co, cn) && step_allowed(a, r, rn) && (d_e <= 0.0f || u < __expf(-d_e));
    } else if (moving) {
      co = odd ? co1 : co0;
      const F3 el = {r.x - left.x, r.y - left.y, r.z - left.z};
      const F3 er = {r.x - right.x, r.y - right.y, r.z - right.z};
      float xi0, xi1, xi2, xi3;
      box_muller(w.x, w.y, xi0, xi1);
      box_muller(w.z, w.w, xi2, xi3);
      F3 g_old = sel(odd, g1, g0);
      float w_old = odd ? f1 : f0;
      if (!a.grad) w_old = field_and_grad(a, pl, co, odd ? ox1 : ox0, odd ? oy1 : oy0, odd ? oz1 : oz0, g_old);
      const F3 f_old = {-a.k0 * (wl * el.x + wr * er.x) - a.inv_nref * g_old.x,
                        -a.k0 * (wl * el.y + wr * er.y) - a.inv_nref * g_old.y,
                        -a.k0 * (wl * el.z + wr * er.z) - a.inv_nref * g_old.z};
      rn = {fmaf(a.sqrt_2a, xi0, fmaf(a.step, f_old.x, r.x)),
            fmaf(a.sqrt_2a, xi1, fmaf(a.step, f_old.y, r.y)),
            fmaf(a.sqrt_2a, xi2, fmaf(a.step, f_old.z, r.z))};
      uint32_t nx_, ny_, nz_;
      cell3(a.grid, rn.x, rn.y, rn.z, nx_, ny_, nz_);
      cn = cell_index(a.grid, nx_, ny_, nz_);
      if (BINNED) {
        ko = brick_key(a.bin, odd ? ox1 : ox0, odd ? oy1 : oy0, odd ? oz1 : oz0);
        kn = brick_key(a.bin, nx_, ny_, nz_);
      }
      // force at the trial position with the same bonded neighbours; the
      // field gradient is constant inside a cell
      F3 g_new = g_old;
      float w_new = w_old;
      if (cn != co) w_new = field_and_grad(a, pl, cn, nx_, ny_, nz_, g_new);
      const bool ok = move_allowed(a, co, cn) && step_allowed(a, r, rn);
      const F3 d = {rn.x - r.x, rn.y - r.y, rn.z - r.z};
      const F3 nl = {rn.x - left.x, rn.y - left.y, rn.z - left.z};
      const F3 nr = {rn.x - right.x, rn.y - right.y, rn.z - right.z};
      const F3 f_new = {-a.k0 * (wl * nl.x + wr * nr.x) - a.inv_nref * g_new.x,
                        -a.k0 * (wl * nl.y + wr * nr.y) - a.inv_nref * g_new.y,
                        -a.k0 * (wl * nl.z + wr * nr.z) - a.inv_nref * g_new.z};
      const F3 fw = {d.x - a.step * f_old.x, d.y - a.step * f_old.y, d.z - a.step * f_old.z};
      const F3 rv = {-d.x - a.step * f_new.x, -d.y - a.step * f_new.y, -d.z - a.step * f_new.z};
      const float log_q = ((fw.x * fw.x + fw.y * fw.y + fw.z * fw.z) -
                           (rv.x * rv.x + rv.y * rv.y + rv.z * rv.z)) * a.inv_4a;
      const float qx = wl * (2.0f * el.x + d.x) + wr * (2.0f * er.x + d.x);
      const float qy = wl * (2.0f * el.y + d.y) + wr * (2.0f * er.y + d.y);
      const float qz = wl * (2.0f * el.z + d.z) + wr * (2.0f * er.z + d.z);
      const float d_e = a.half_k0 * (d.x * qx + d.y * qy + d.z * qz) + (w_new - w_old) * a.inv_nref +
                        (cn != co ? a.self_term : 0.0f);
      const float lr = log_q - d_e;
      acc = ok && (lr >= 0.0f || u < __expf(lr));
    }
    if (BINNED) { co = ko; cn = kn; }   // cells as brick keys from here on
    if (odd) { r1 = acc ? rn : r1; moved1 = acc && cn != co; from1 = co; to1 = cn; }
    else     { r0 = acc ? rn : r0; moved0 = acc && cn != co; from0 = co; to0 = cn; }
    n_acc += (uint32_t)__popcll(__ballot(acc));
  }

  store_pair<VEC2>(cp, m, r0, r1);
  if (BINNED) {
    bin_moves<COUNT64>(a.bin, a.grid, a.counts, wave_sub_bin(a.wpb), from0, to0, b0 ? 1u : 0u,
                       moved0, from1, to1, b1 ? 1u : 0u, moved1);
  } else {
    if (moved0) move_count<COUNT64>(a.counts, from0, to0, b0);
    if (moved1) move_count<COUNT64>(a.counts, from1, to1, b1);
  }
  return n_acc;
}

// Smart-MC or bond-Gibbs waves over one tile each, or over the tiles of a
// persistent grid (SweepArgs::queue).
template <bool COUNT64, bool VEC2, bool BINNED, bool GIBBS, bool PERSIST>
__device__ __forceinline__ void smc_tiles(const SweepArgs &a) {
  if (!PERSIST) {   // one tile per wave
    finish_block(a, smc_wave<COUNT64, VEC2, BINNED, GIBBS>(a, lane_map(a)));
    return;
  }
  const TileIter it = tile_iter(a);
  uint32_t n_acc = 0;
  uint32_t t = tile_of(it, tile_draw(it));
  while (t < it.t_end) {
    const uint32_t vn = tile_draw(it);
    n_acc += smc_wave<COUNT64, VEC2, BINNED, GIBBS>(a, lane_map_tile(a, t, true));
    t = tile_of(it, vn);
  }
  finish_block(a, n_acc);
}

// PERSIST: the persistent-grid instance (SweepArgs::queue set); its loop over
// tiles needs more registers than a single tile, so single-tile launches use
// their own instance.
template <bool COUNT64, bool VEC2, bool BINNED, bool PERSIST = false>
__global__ __launch_bounds__(512) void mc_sweep_smc_kernel(const SweepArgs a_in) {
  smc_tiles<COUNT64, VEC2, BINNED, false, PERSIST>(resolve_sweep(a_in, 0u));
}

template <bool COUNT64, bool VEC2, bool BINNED, bool PERSIST = false>
__global__ __launch_bounds__(512) void mc_sweep_gibbs_kernel(const SweepArgs a_in) {
  smc_tiles<COUNT64, VEC2, BINNED, true, PERSIST>(resolve_sweep(a_in, 0u));
}

}  // namespace soma

namespace soma {

// Extra arguments of the mixed local / learned sweep.
struct MixArgs {
  const NetDev *net;
  HeadArgs head;
  float p_learn;                   // probability of the learned move (state-independent)
  unsigned long long *att_slots;   // [kAccSlots] attempted learned moves
  uint32_t *err;                   // device error word (bit 2: non-finite network output)
  const float *halo;               // fields with x halos [2][nz*ny][nx + 2] (p_learn > 0)
  uint32_t halo_plane;
};

// ---------------------------------------------------------------------------
// Mixed moves: each bead makes the learned move with probability p_learn
// (word 1 of its purpose-1 draw, independent of the configuration) and the
// local move otherwise.  A learned move draws xi by Box-Muller from the
// purpose-0 block, proposes r' = r + mu(r) + sigma(r) xi and accepts with
// min(1, exp(-dE) q(r|r')/q(r'|r)) (word 0 of the purpose-1 block); a
// non-finite network output rejects it and raises error bit 2.  The network
// needs the bond vectors, so the two sets are handled one after the other.
// ---------------------------------------------------------------------------
// One wave's chains; act is the wave's LDS feature tile, zb its LDS tile of
// network outputs ([64][8] floats), sw the block's LDS copy of the network's
// weights.  Returns through cnt the wave's accepted local moves, accepted
// learned moves and learned attempts.
template <bool COUNT64, bool VEC2, bool BINNED>
__device__ __forceinline__ void mixed_wave(const SweepArgs &a, const MixArgs &mx, const LaneMap &m,
                                           __bf16 *act, float *zb, const __bf16 *sw,
                                           uint32_t cnt[3]) {
  __bf16 *row = act + m.lane * kActStride;
  const uint32_t N = a.n;
  const uint32_t i0 = 2u * m.k, i1 = i0 + 1u;
  float *cp = a.pos + (size_t)(m.has0 ? m.chain : 0u) * N * 3u + 6u * m.k;
  F3 r0, r1;
  load_pair<VEC2>(cp, m, r0, r1);

  const uint32_t gchain = a.chain_base + m.chain;
  const Rand4 wa0 = philox(gchain, i0 | (kPurposeMoveA << 16), a.sweep, a.replica, a.seed_lo, a.seed_hi);
  const Rand4 wa1 = philox(gchain, i1 | (kPurposeMoveA << 16), a.sweep, a.replica, a.seed_lo, a.seed_hi);
  const Rand4 wb0 = philox(gchain, i0 | (kPurposeMoveB << 16), a.sweep, a.replica, a.seed_lo, a.seed_hi);
  const Rand4 wb1 = philox(gchain, i1 | (kPurposeMoveB << 16), a.sweep, a.replica, a.seed_lo, a.seed_hi);
  const uint32_t first = set_order_bit(a, m, wa0.x);
  const bool b0 = i0 >= a.n_a, b1 = i1 >= a.n_a;

  uint32_t from0 = 0, to0 = 0, from1 = 0, to1 = 0;
  bool moved0 = false, moved1 = false;
  uint32_t n_acc = 0, n_acc_l = 0, n_att_l = 0;
  bool net_bad_any = false;
#pragma unroll
  for (int pass = 0; pass < 2; ++pass) {
    const bool odd = (first ^ (uint32_t)pass) != 0u;
    const F3 send = sel(odd, r0, r1);
    const int src = odd ? (m.lane < 63 ? m.lane + 1 : m.lane) : (m.lane > 0 ? m.lane - 1 : m.lane);
    const F3 nb = {shfl_f(send.x, src), shfl_f(send.y, src), shfl_f(send.z, src)};
    const F3 left = sel(odd, r0, nb);     // bead i-1
    const F3 right = sel(odd, nb, r1);    // bead i+1
    const bool moving = odd ? m.has1 : m.has0;
    const bool has_l = odd || m.k > 0;
    const bool has_r = odd ? (i1 + 1u < N) : m.has1;
    const float wl = has_l ? 1.0f : 0.0f, wr = has_r ? 1.0f : 0.0f;
    const F3 r = sel(odd, r1, r0);
    const Rand4 w = odd ? wa1 : wa0;
    const Rand4 wb = odd ? wb1 : wb0;
    const bool is_b = odd ? b1 : b0;
    const bool learned = moving && uniform01(wb.y) < mx.p_learn;
    const uint32_t pl = is_b ? a.grid.n_cells : 0u;
    const F3 zero3 = F3{0.f, 0.f, 0.f};

    F3 rn;
    uint32_t co, cn;
    float w_old, w_new, log_q = 0.0f;
    bool net_bad = false;
    if (__ballot(learned) != 0ull) {
      features_to_row_halo(a.grid, mx.halo, mx.halo_plane, is_b, r, has_l ? left - r : zero3,
                           has_r ? right - r : zero3, row, co);
      w_old = field_at(a.omega, pl, co);   // energies from the field itself
      wave_forward(mx.net, sw, act, zb);
      float mu[3], sig[3], lsig[3];
      head(zb + m.lane * 8, mx.head, mu, sig, lsig);
      float xi0, xi1, xi2, xi3;
      box_muller(w.x, w.y, xi0, xi1);
      box_muller(w.z, w.w, xi2, xi3);
      const F3 tl = {r.x + fmaf(sig[0], xi0, mu[0]), r.y + fmaf(sig[1], xi1, mu[1]),
                     r.z + fmaf(sig[2], xi2, mu[2])};
      const F3 tp = {fmaf(a.step, uniform11(w.x), r.x), fmaf(a.step, uniform11(w.y), r.y),
                     fmaf(a.step, uniform11(w.z), r.z)};
      rn = sel(learned, tl, tp);
      // features at r': in the same cell the 27 field values are those at r
      // (still in the row), so only the bond vectors change
      cn = cell_of(a.grid, rn.x, rn.y, rn.z);
      const F3 bpn = has_l ? left - rn : zero3, bnn = has_r ? right - rn : zero3;
      if (cn != co) {
        uint32_t c2;
        features_to_row_halo(a.grid, mx.halo, mx.halo_plane, is_b, rn, bpn, bnn, row, c2);
      } else {
        bond_features_to_row(bpn, bnn, row);
      }
      w_new = cn == co ? w_old : field_at(a.omega, pl, cn);
      wave_forward(mx.net, sw, act, zb);
      float mun[3], sign[3], lsign[3];
      head(zb + m.lane * 8, mx.head, mun, sign, lsign);
      float lq = 0.0f;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const float rd = d == 0 ? r.x : (d == 1 ? r.y : r.z);
        const float td = d == 0 ? rn.x : (d == 1 ? rn.y : rn.z);
        const float ef = td - rd - mu[d];
        const float er = rd - td - mun[d];
        lq += 0.5f * ef * ef * fast_rcp(sig[d] * sig[d]) + lsig[d] -
              0.5f * er * er * fast_rcp(sign[d] * sign[d]) - lsign[d];
        net_bad |= !(isfinite(mu[d]) && isfinite(sig[d]) && isfinite(mun[d]) && isfinite(sign[d]));
      }
      log_q = lq;   // log q(r|r') - log q(r'|r)
      net_bad = net_bad && learned;
    } else {
      rn = F3{fmaf(a.step, uniform11(w.x), r.x), fmaf(a.step, uniform11(w.y), r.y),
              fmaf(a.step, uniform11(w.z), r.z)};
      co = cell_of(a.grid, r.x, r.y, r.z);
      cn = cell_of(a.grid, rn.x, rn.y, rn.z);
      w_old = field_at(a.omega, pl, co);
      w_new = cn == co ? w_old : field_at(a.omega, pl, cn);
    }
    const F3 d = rn - r;
    const F3 q = wl * (2.0f * (r - left) + d) + wr * (2.0f * (r - right) + d);
    const float d_e = a.half_k0 * (d.x * q.x + d.y * q.y + d.z * q.z) + (w_new - w_old) * a.inv_nref +
                      (cn != co ? a.self_term : 0.0f);
    bool acc;
    if (learned) {
      const float lr = log_q - d_e;
      acc = !net_bad && (lr >= 0.0f || uniform01(wb.x) < __expf(lr));
    } else {
      acc = moving && (d_e <= 0.0f || uniform01(w.w) < __expf(-d_e));
    }
    acc = acc && move_allowed(a, co, cn) && step_allowed(a, r, rn);
    net_bad_any |= net_bad;
    if (odd) { r1 = acc ? rn : r1; moved1 = acc && cn != co; from1 = co; to1 = cn; }
    else     { r0 = acc ? rn : r0; moved0 = acc && cn != co; from0 = co; to0 = cn; }
    n_acc += (uint32_t)__popcll(__ballot(acc));
    n_acc_l += (uint32_t)__popcll(__ballot(acc && learned));
    n_att_l += (uint32_t)__popcll(__ballot(learned));
  }
  store_pair<VEC2>(cp, m, r0, r1);
  if (BINNED) {
    bin_moves<COUNT64>(a.bin, a.grid, a.counts, wave_sub_bin(a.wpb),
                       cell_brick_key(a.bin, a.grid, from0),
                       cell_brick_key(a.bin, a.grid, to0), b0 ? 1u : 0u, moved0,
                       cell_brick_key(a.bin, a.grid, from1), cell_brick_key(a.bin, a.grid, to1),
                       b1 ? 1u : 0u, moved1);
  } else {
    if (moved0) move_count<COUNT64>(a.counts, from0, to0, b0);
    if (moved1) move_count<COUNT64>(a.counts, from1, to1, b1);
  }
  if (__ballot(net_bad_any) != 0ull && m.lane == 0) atomicOr(mx.err, 2u);
  cnt[0] = n_acc - n_acc_l;
  cnt[1] = n_acc_l;
  cnt[2] = n_att_l;
}

// Block totals of the mixed sweep: local and learned acceptances go to separate
// slot arrays, learned attempts to their own.
__device__ __forceinline__ void mixed_finish(const SweepArgs &a, const MixArgs &mx,
                                             const uint32_t cnt[3]) {
  __shared__ uint32_t s_cnt[4][3];
  const uint32_t wib = threadIdx.x >> 6;
  if ((threadIdx.x & 63u) == 0u) { s_cnt[wib][0] = cnt[0]; s_cnt[wib][1] = cnt[1]; s_cnt[wib][2] = cnt[2]; }
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint32_t slot = blockIdx.x & (kAccSlots - 1u);
    const uint32_t loc = s_cnt[0][0] + s_cnt[1][0] + s_cnt[2][0] + s_cnt[3][0];
    const uint32_t lrn = s_cnt[0][1] + s_cnt[1][1] + s_cnt[2][1] + s_cnt[3][1];
    const uint32_t att = s_cnt[0][2] + s_cnt[1][2] + s_cnt[2][2] + s_cnt[3][2];
    if (loc) atomicAdd(a.acc_slots + slot, (unsigned long long)loc);
    if (lrn) atomicAdd(a.acc_slots + 2u * kAccSlots + slot, (unsigned long long)lrn);
    if (att) atomicAdd(mx.att_slots + slot, (unsigned long long)att);
  }
  __syncthreads();
}

template <bool COUNT64, bool VEC2, bool BINNED, bool PERSIST = false>
__global__ __launch_bounds__(256) void mc_sweep_mixed_kernel(const SweepArgs a_in,
                                                             const MixArgs mx) {
  __shared__ __bf16 s_act[4][64 * kActStride];
  __shared__ float s_z[4][64 * 8];
  __shared__ __bf16 s_w[kWRows * kWStride];
  net_weights_to_lds(mx.net, s_w);
  __syncthreads();
  const SweepArgs a = resolve_sweep(a_in, 0u);
  const uint32_t wib = threadIdx.x >> 6;
  uint32_t cnt[3] = {0u, 0u, 0u};
  if (!PERSIST) {   // one tile per wave
    mixed_wave<COUNT64, VEC2, BINNED>(a, mx, lane_map(a), s_act[wib], s_z[wib], s_w, cnt);
    mixed_finish(a, mx, cnt);
    return;
  }
  // a persistent grid copies the weights once per block for all its tiles
  const TileIter it = tile_iter(a);
  uint32_t t = tile_of(it, tile_draw(it));
  while (t < it.t_end) {
    const uint32_t vn = tile_draw(it);
    uint32_t c[3];
    mixed_wave<COUNT64, VEC2, BINNED>(a, mx, lane_map_tile(a, t, true), s_act[wib], s_z[wib],
                                      s_w, c);
    cnt[0] += c[0];
    cnt[1] += c[1];
    cnt[2] += c[2];
    t = tile_of(it, vn);
  }
  mixed_finish(a, mx, cnt);
}

}  // namespace soma
