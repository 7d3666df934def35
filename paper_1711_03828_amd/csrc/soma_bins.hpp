// soma_bins.hpp -- the occupation histogram (Eq. (4), Sec. 3.1.1) kept current
// through per-brick bins of count updates instead of one memory-side atomic
// per update.
//
// The grid is cut into bricks of 16 x 16 x 8 cells.  A wave that moves beads
// to other cells groups its +-1 updates by brick, reserves room in each
// brick's bin with one atomic per (wave, brick) and writes the updates there
// with plain stores; a bin that is full takes the rest as direct atomics on
// the counts.  Afterwards `bin_apply_kernel` gives every brick one workgroup:
// the brick's count words go to LDS, the bin's updates are added with LDS
// atomics, and the words go back.  Integer additions are exact and
// order-independent, so the counts are bit-identical to direct atomics (and
// to a recount of the final positions).
//
// An update is 16 bits: bit 15 present, bit 14 minus (-1, else +1), bits
// 11..13 the bead type, bits 0..10 the cell inside the brick
// ((z & 7) * 16 + (y & 15)) * 16 + (x & 15).  A bin entry holds two updates
// (low and high half), typically the -1 at the old cell and the +1 at the new
// cell of one bead; a half with bit 15 clear is empty.
#pragma once

#include "soma_device.hpp"

namespace soma {

constexpr uint32_t kBrickCells = 2048u;      // 16 x 16 x 8
constexpr uint32_t kHistDirect = 0u;         // one atomic per update
constexpr uint32_t kHistBinned = 1u;         // per-brick bins, applied by bin_apply_kernel
constexpr uint32_t kUpdPresent = 0x8000u;
constexpr uint32_t kUpdMinus = 0x4000u;

struct BinArgs {
  uint32_t *bins;        // [n_bricks][cap] entries
  uint32_t *bin_count;   // [n_bricks] entries written (may exceed cap: the rest went direct)
  uint32_t cap;          // entries per bin
  uint32_t nbx, nby, nbz;
};

// Brick key of cell (x, y, z): brick index << 11 | cell inside the brick.
__device__ __forceinline__ uint32_t brick_key(const BinArgs &b, uint32_t x, uint32_t y,
                                              uint32_t z) {
  const uint32_t brick = __umul24(__umul24(z >> 3, b.nby) + (y >> 4), b.nbx) + (x >> 4);
  return (brick << 11) | ((z & 7u) << 8) | ((y & 15u) << 4) | (x & 15u);
}

// q = floor(c / d) for c < 2^29: an FP32 estimate, refined once with the
// exact remainder (|error| of the estimate far below 2^23), then fixed by one.
__device__ __forceinline__ uint32_t div_small(uint32_t c, uint32_t d, float inv_d) {
  int q = (int)((float)c * inv_d);
  int r = (int)c - q * (int)d;
  q += (int)floorf((float)r * inv_d);
  r = (int)c - q * (int)d;
  q += r >= (int)d ? 1 : (r < 0 ? -1 : 0);
  return (uint32_t)q;
}

// Brick key of the linear cell c = (z ny + y) nx + x.
__device__ __forceinline__ uint32_t cell_brick_key(const BinArgs &b, const Grid &g, uint32_t c) {
  const uint32_t yz = div_small(c, (uint32_t)g.nx, g.inv_nx);
  const uint32_t x = c - yz * (uint32_t)g.nx;
  const uint32_t z = div_small(yz, (uint32_t)g.ny, g.inv_ny);
  const uint32_t y = yz - z * (uint32_t)g.ny;
  return brick_key(b, x, y, z);
}

// Linear cell index of the cell inside brick `brick` at `local` (slow path only).
__device__ __forceinline__ uint32_t brick_cell(const BinArgs &b, const Grid &g, uint32_t brick,
                                               uint32_t local) {
  const uint32_t bx = brick % b.nbx, rest = brick / b.nbx;
  const uint32_t by = rest % b.nby, bz = rest / b.nby;
  const uint32_t x = bx * 16u + (local & 15u), y = by * 16u + ((local >> 4) & 15u),
                 z = bz * 8u + (local >> 8);
  return (z * (uint32_t)g.ny + y) * (uint32_t)g.nx + x;
}

// One update applied directly to the packed counts (the overflow path).
template <bool COUNT64>
__device__ __forceinline__ void apply_update_direct(void *counts, uint32_t n_cells, uint32_t cell,
                                                    uint32_t upd) {
  const uint32_t t = (upd >> 11) & 7u;
  const bool minus = (upd & kUpdMinus) != 0u;
  const size_t w = (size_t)(t >> 1) * n_cells + cell;
  if (COUNT64) {
    unsigned int *p = reinterpret_cast<unsigned int *>(counts) + 2 * w + (t & 1u);
    atomicAdd(p, minus ? 0xFFFFFFFFu : 1u);
  } else {
    const unsigned int inc = (t & 1u) ? (1u << 16) : 1u;
    atomicAdd(reinterpret_cast<unsigned int *>(counts) + w, minus ? 0u - inc : inc);
  }
}

template <bool COUNT64>
__device__ __forceinline__ void apply_entry_direct(const BinArgs &b, const Grid &g, void *counts,
                                                   uint32_t key, uint32_t entry) {
  const uint32_t brick = key;
  for (int h = 0; h < 2; ++h) {
    const uint32_t upd = (entry >> (16 * h)) & 0xFFFFu;
    if (upd & kUpdPresent)
      apply_update_direct<COUNT64>(counts, g.n_cells, brick_cell(b, g, brick, upd & 2047u), upd);
  }
}

// Appends the entries of a wave to their bricks' bins.  Each lane offers up
// to four entries (slot s: brick key[s], value val[s], wanted if bit s of
// `want`).  All lanes of the wave must call this together.  Entries are
// grouped by brick; the first four groups reserve their room with atomics
// issued back to back (one wait for all), further groups one at a time.
template <bool COUNT64>
__device__ __forceinline__ void bin_append(const BinArgs &b, const Grid &g, void *counts,
                                           const uint32_t key[4], const uint32_t val[4],
                                           uint32_t want) {
  const uint32_t lane = __lane_id();
  const uint64_t lanes_below = (1ull << lane) - 1ull;
  uint32_t grp[4] = {4u, 4u, 4u, 4u};   // group of each slot (4: later groups)
  uint32_t off[4] = {0u, 0u, 0u, 0u};   // rank inside the group
  uint32_t gkey[4] = {0u, 0u, 0u, 0u};  // brick of each group (wave-uniform)
  uint32_t gbase[4] = {0u, 0u, 0u, 0u}; // returned bin count (leader lane only)
  uint32_t glead[4] = {0u, 0u, 0u, 0u};
  uint32_t n_groups = 0;
#pragma unroll
  for (uint32_t j = 0; j < 4; ++j) {
    const uint64_t any = __ballot(want != 0u);
    if (any == 0ull) break;
    const uint32_t leader = (uint32_t)__ffsll((long long)any) - 1u;
    const uint32_t first = (want & 1u) ? key[0] : (want & 2u) ? key[1] : (want & 4u) ? key[2] : key[3];
    const uint32_t k = (uint32_t)__builtin_amdgcn_readlane((int)first, (int)leader);
    uint32_t tot = 0;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const bool mt = ((want >> s) & 1u) && key[s] == k;
      const uint64_t bm = __ballot(mt);
      if (mt) { grp[s] = j; off[s] = tot + (uint32_t)__popcll(bm & lanes_below); }
      tot += (uint32_t)__popcll(bm);
      want &= mt ? ~(1u << s) : ~0u;
    }
    if (lane == leader) gbase[j] = atomicAdd(b.bin_count + k, tot);
    gkey[j] = k;
    glead[j] = leader;
    n_groups = j + 1u;
  }
  uint32_t base[4];
#pragma unroll
  for (uint32_t j = 0; j < 4; ++j)
    base[j] = j < n_groups ? (uint32_t)__builtin_amdgcn_readlane((int)gbase[j], (int)glead[j]) : 0u;
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    if (grp[s] < 4u) {
      const uint32_t j = grp[s];
      const uint32_t bk = j == 0 ? gkey[0] : j == 1 ? gkey[1] : j == 2 ? gkey[2] : gkey[3];
      const uint32_t pos = (j == 0 ? base[0] : j == 1 ? base[1] : j == 2 ? base[2] : base[3]) + off[s];
      if (pos < b.cap) b.bins[(size_t)bk * b.cap + pos] = val[s];
      else apply_entry_direct<COUNT64>(b, g, counts, bk, val[s]);
    }
  }
  // rare: more than four bricks in one wave
  while (true) {
    const uint64_t any = __ballot(want != 0u);
    if (any == 0ull) break;
    const uint32_t leader = (uint32_t)__ffsll((long long)any) - 1u;
    const uint32_t first = (want & 1u) ? key[0] : (want & 2u) ? key[1] : (want & 4u) ? key[2] : key[3];
    const uint32_t k = (uint32_t)__builtin_amdgcn_readlane((int)first, (int)leader);
    uint32_t tot = 0, my_off[4] = {0u, 0u, 0u, 0u}, mine = 0u;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const bool mt = ((want >> s) & 1u) && key[s] == k;
      const uint64_t bm = __ballot(mt);
      if (mt) { my_off[s] = tot + (uint32_t)__popcll(bm & lanes_below); mine |= 1u << s; }
      tot += (uint32_t)__popcll(bm);
    }
    want &= ~mine;
    uint32_t bs = 0;
    if (lane == leader) bs = atomicAdd(b.bin_count + k, tot);
    bs = (uint32_t)__builtin_amdgcn_readlane((int)bs, (int)leader);
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      if ((mine >> s) & 1u) {
        const uint32_t pos = bs + my_off[s];
        if (pos < b.cap) b.bins[(size_t)k * b.cap + pos] = val[s];
        else apply_entry_direct<COUNT64>(b, g, counts, k, val[s]);
      }
    }
  }
}

// The count updates of a lane's two beads (bead e moved from the cell with
// brick key from[e] to to[e] if moved[e]; t[e] its type), as bin entries:
// one entry when both cells lie in one brick, else one entry per brick.
template <bool COUNT64>
__device__ __forceinline__ void bin_moves(const BinArgs &b, const Grid &g, void *counts,
                                          uint32_t from0, uint32_t to0, uint32_t t0, bool moved0,
                                          uint32_t from1, uint32_t to1, uint32_t t1, bool moved1) {
  uint32_t key[4], val[4], want = 0u;
  const uint32_t from[2] = {from0, from1}, to[2] = {to0, to1}, ty[2] = {t0, t1};
  const bool mv[2] = {moved0, moved1};
#pragma unroll
  for (int e = 0; e < 2; ++e) {
    const uint32_t hm = kUpdPresent | kUpdMinus | (ty[e] << 11) | (from[e] & 2047u);
    const uint32_t hp = kUpdPresent | (ty[e] << 11) | (to[e] & 2047u);
    const bool same = (from[e] >> 11) == (to[e] >> 11);
    key[2 * e] = from[e] >> 11;
    val[2 * e] = same ? (hm | (hp << 16)) : hm;
    key[2 * e + 1] = to[e] >> 11;
    val[2 * e + 1] = hp << 16;
    if (mv[e]) want |= (same ? 1u : 3u) << (2 * e);
  }
  bin_append<COUNT64>(b, g, counts, key, val, want);
}

// Applies the bins to the counts: one workgroup per brick.  The brick's count
// words (every plane) are staged in LDS, the bin's updates added with LDS
// atomics, the words written back, and the bin emptied for the next sweep.
// LDS: planes x 2048 words (u16 pairs) or 2 x planes x 2048 halves (u32 pairs).
template <bool COUNT64>
__global__ __launch_bounds__(256) void bin_apply_kernel(BinArgs b, Grid g, void *counts,
                                                        uint32_t planes) {
  extern __shared__ uint32_t s_cnt[];
  const uint32_t brick = blockIdx.x;
  const uint32_t bx = brick % b.nbx, rest = brick / b.nbx;
  const uint32_t by = rest % b.nby, bz = rest / b.nby;
  const uint32_t x0 = bx * 16u, y0 = by * 16u, z0 = bz * 8u;
  for (uint32_t i = threadIdx.x; i < planes * kBrickCells; i += blockDim.x) {
    const uint32_t p = i / kBrickCells, l = i % kBrickCells;
    const uint32_t x = x0 + (l & 15u), y = y0 + ((l >> 4) & 15u), z = z0 + (l >> 8);
    uint32_t lo = 0u, hi = 0u;
    if (x < (uint32_t)g.nx && y < (uint32_t)g.ny && z < (uint32_t)g.nz) {
      const size_t w = (size_t)p * g.n_cells + ((size_t)z * g.ny + y) * g.nx + x;
      if (COUNT64) {
        const uint2 v = reinterpret_cast<const uint2 *>(counts)[w];
        lo = v.x;
        hi = v.y;
      } else {
        lo = reinterpret_cast<const uint32_t *>(counts)[w];
      }
    }
    if (COUNT64) reinterpret_cast<uint2 *>(s_cnt)[i] = make_uint2(lo, hi);
    else s_cnt[i] = lo;
  }
  __syncthreads();
  const uint32_t n = min(b.bin_count[brick], b.cap);
  const uint32_t *bin = b.bins + (size_t)brick * b.cap;
  for (uint32_t j = threadIdx.x; j < n; j += blockDim.x) {
    const uint32_t e = bin[j];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const uint32_t upd = (e >> (16 * h)) & 0xFFFFu;
      const uint32_t t = (upd >> 11) & 7u;
      if ((upd & kUpdPresent) && (t >> 1) < planes) {
        const uint32_t i = (t >> 1) * kBrickCells + (upd & 2047u);
        const bool minus = (upd & kUpdMinus) != 0u;
        if (COUNT64) {
          atomicAdd(&s_cnt[i * 2 + (t & 1u)], minus ? 0xFFFFFFFFu : 1u);
        } else {
          const uint32_t inc = (t & 1u) ? (1u << 16) : 1u;
          atomicAdd(&s_cnt[i], minus ? 0u - inc : inc);
        }
      }
    }
  }
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < planes * kBrickCells; i += blockDim.x) {
    const uint32_t p = i / kBrickCells, l = i % kBrickCells;
    const uint32_t x = x0 + (l & 15u), y = y0 + ((l >> 4) & 15u), z = z0 + (l >> 8);
    if (x < (uint32_t)g.nx && y < (uint32_t)g.ny && z < (uint32_t)g.nz) {
      const size_t w = (size_t)p * g.n_cells + ((size_t)z * g.ny + y) * g.nx + x;
      if (COUNT64)
        reinterpret_cast<uint2 *>(counts)[w] = reinterpret_cast<const uint2 *>(s_cnt)[i];
      else
        reinterpret_cast<uint32_t *>(counts)[w] = s_cnt[i];
    }
  }
  if (threadIdx.x == 0) b.bin_count[brick] = 0u;
}

}  // namespace soma
