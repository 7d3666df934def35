// soma_bins.hpp -- the occupation histogram (Eq. (4), Sec. 3.1.1) kept current
// through per-brick bins of count updates instead of one memory-side atomic
// per update.
//
// The grid is cut into bricks of 16 x 16 x 8 cells.  A wave that moves beads
// to other cells counts its +-1 updates per brick in a small LDS table,
// reserves room in each brick's bin with one atomic per (wave, brick) and
// writes the updates there with plain stores; a bin that is full takes the
// rest as direct atomics on the counts.  Afterwards `bin_apply_kernel` gives
// every brick one workgroup: the brick's count words go to LDS, the bin's
// updates are added with LDS atomics, and the words go back.  Integer additions are exact and
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

// Every brick has kSubBins sub-bins; a wave appends to sub-bin (wave index
// mod kSubBins), so that the waves working on one region of the grid at the
// same time (they share its bricks) spread their reservations over
// different counters instead of queueing on one.
constexpr uint32_t kSubShift = 4u, kSubBins = 1u << kSubShift;

struct BinArgs {
  uint32_t *bins;        // [n_bricks][kSubBins][cap] entries
  uint32_t *bin_count;   // [n_bricks][kSubBins] entries written (beyond cap: went direct)
  uint32_t cap;          // entries per sub-bin
  uint32_t nbx, nby, nbz;
};

// Sub-bin of the calling wave (wpb waves per block).
__device__ __forceinline__ uint32_t wave_sub_bin(uint32_t wpb) {
  return ((blockIdx.x * wpb) + (threadIdx.x >> 6)) & (kSubBins - 1u);
}

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

// Per-wave table of the bricks a wave's updates fall in: kTabSlots slots of
// {brick, count} in LDS, open addressing with linear probing.  Built for one
// bin_append call and discarded after it.
constexpr uint32_t kTabSlots = 32u;
constexpr uint32_t kTabEmpty = 0xFFFFFFFFu;   // no brick (brick indices are below 2^21)
constexpr uint32_t kNoSlot = 0xFFu;
constexpr uint32_t kMaxWaves = 8u;            // waves per block that may call bin_append

__device__ __forceinline__ uint32_t tab_hash(uint32_t brick) {
  return (__umul24(brick, 0x9E3779u) >> 11) & (kTabSlots - 1u);
}

// Slot of `brick` in the wave's table (claimed if new) << 16 | the entry's
// rank among the wave's entries for that brick; kNoSlot << 16 if the table is
// full.
__device__ __forceinline__ uint32_t tab_insert(uint2 *tab, uint32_t brick) {
  uint32_t h = tab_hash(brick);
  uint32_t probe = 0;
#pragma unroll 1
  for (; probe < kTabSlots; ++probe) {
    const uint32_t old = atomicCAS(&tab[h].x, kTabEmpty, brick);
    if (old == kTabEmpty || old == brick) break;
    h = (h + 1u) & (kTabSlots - 1u);
  }
  if (probe == kTabSlots) return kNoSlot << 16;
  return (h << 16) | atomicAdd(&tab[h].y, 1u);
}

// Stores entry v (brick k, table slot and rank q) at its reserved place, or
// applies it directly if its sub-bin is full or the wave's table was.
template <bool COUNT64>
__device__ __forceinline__ void tab_put(const BinArgs &b, const Grid &g, void *counts,
                                        const uint2 *tab, uint32_t sub, uint32_t k, uint32_t q,
                                        uint32_t v) {
  const uint32_t h = q >> 16;
  const uint32_t pos = h != kNoSlot ? tab[h].y + (q & 0xFFFFu) : 0xFFFFFFFFu;
  if (pos < b.cap) b.bins[(size_t)((k << kSubShift) | sub) * b.cap + pos] = v;
  else apply_entry_direct<COUNT64>(b, g, counts, k, v);
}

// Set bits of mask m in the lanes below the calling one.
__device__ __forceinline__ uint32_t mbcnt64(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                   __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Appends the entries of a wave to their bricks' bins.  Each lane offers up
// to four entries (slot s: brick ks, value vs, wanted if bit s of `want`).
// All lanes of the wave must call this together (wave-uniform control flow).
// The wanted entries are first packed into a wave-private LDS list (slot 0 of
// every lane, then slot 1, ...), so that the steps below run once per 64
// entries with every lane busy, rather than once per slot with the few lanes
// whose bead changed cell.  The entries are counted per brick in the wave's
// LDS table (the rank of an entry is its place among the wave's entries for
// its brick), one lane per brick reserves that many places in the brick's
// sub-bin `sub` with one atomic, and every entry is stored at reserved base +
// rank.  LDS operations of one wave execute in issue order, so neither the
// list nor the table needs a barrier between the steps.
constexpr uint32_t kListSlots = 4u * 64u;

template <bool COUNT64>
__device__ __forceinline__ void bin_append(const BinArgs &b, const Grid &g, void *counts,
                                           uint32_t sub, uint32_t k0, uint32_t k1, uint32_t k2,
                                           uint32_t k3, uint32_t v0, uint32_t v1, uint32_t v2,
                                           uint32_t v3, uint32_t want) {
  __shared__ uint2 s_tab[kMaxWaves * kTabSlots];
  __shared__ uint2 s_list[kMaxWaves * kListSlots];
  const uint32_t lane = __lane_id();
  uint2 *tab = s_tab + (threadIdx.x >> 6) * kTabSlots;
  uint2 *list = s_list + (threadIdx.x >> 6) * kListSlots;
  if (lane < kTabSlots) tab[lane] = make_uint2(kTabEmpty, 0u);
  const uint64_t m0 = __ballot((want & 1u) != 0u), m1 = __ballot((want & 2u) != 0u);
  const uint64_t m2 = __ballot((want & 4u) != 0u), m3 = __ballot((want & 8u) != 0u);
  const uint32_t o1 = (uint32_t)__popcll(m0), o2 = o1 + (uint32_t)__popcll(m1);
  const uint32_t o3 = o2 + (uint32_t)__popcll(m2), n = o3 + (uint32_t)__popcll(m3);
  if (want & 1u) list[mbcnt64(m0)] = make_uint2(k0, v0);
  if (want & 2u) list[o1 + mbcnt64(m1)] = make_uint2(k1, v1);
  if (want & 4u) list[o2 + mbcnt64(m2)] = make_uint2(k2, v2);
  if (want & 8u) list[o3 + mbcnt64(m3)] = make_uint2(k3, v3);
  __builtin_amdgcn_wave_barrier();
  // entry lane + 64 p of the list in pass p (n is wave-uniform)
  uint2 e[4];
  uint32_t q[4];   // slot << 16 | rank
#pragma unroll
  for (uint32_t p = 0; p < 4u; ++p) {
    e[p] = make_uint2(0u, 0u);
    q[p] = 0u;
    if (64u * p < n) {
      const uint32_t j = 64u * p + lane;
      if (j < n) {
        e[p] = list[j];
        q[p] = tab_insert(tab, e[p].x);
      }
    }
  }
  __builtin_amdgcn_wave_barrier();
  if (lane < kTabSlots) {   // one reservation per brick; the slot keeps its base
    const uint2 t = tab[lane];
    if (t.x != kTabEmpty) tab[lane].y = atomicAdd(b.bin_count + ((t.x << kSubShift) | sub), t.y);
  }
  __builtin_amdgcn_wave_barrier();
#pragma unroll
  for (uint32_t p = 0; p < 4u; ++p) {
    if (64u * p < n && 64u * p + lane < n)
      tab_put<COUNT64>(b, g, counts, tab, sub, e[p].x, q[p], e[p].y);
  }
  __builtin_amdgcn_wave_barrier();
}

// The count updates of a lane's two beads (bead e moved from the cell with
// brick key from[e] to to[e] if moved[e]; t[e] its type), as bin entries of
// sub-bin `sub`:
// one entry when both cells lie in one brick, else one entry per brick.
template <bool COUNT64>
__device__ __forceinline__ void bin_moves(const BinArgs &b, const Grid &g, void *counts,
                                          uint32_t sub, uint32_t from0, uint32_t to0, uint32_t t0,
                                          bool moved0, uint32_t from1, uint32_t to1, uint32_t t1,
                                          bool moved1) {
  const uint32_t hm0 = kUpdPresent | kUpdMinus | (t0 << 11) | (from0 & 2047u);
  const uint32_t hp0 = kUpdPresent | (t0 << 11) | (to0 & 2047u);
  const uint32_t hm1 = kUpdPresent | kUpdMinus | (t1 << 11) | (from1 & 2047u);
  const uint32_t hp1 = kUpdPresent | (t1 << 11) | (to1 & 2047u);
  const bool same0 = (from0 >> 11) == (to0 >> 11), same1 = (from1 >> 11) == (to1 >> 11);
  const uint32_t want = (moved0 ? (same0 ? 1u : 3u) : 0u) | (moved1 ? (same1 ? 4u : 12u) : 0u);
  bin_append<COUNT64>(b, g, counts, sub, from0 >> 11, to0 >> 11, from1 >> 11, to1 >> 11,
                      same0 ? (hm0 | (hp0 << 16)) : hm0, hp0 << 16,
                      same1 ? (hm1 | (hp1 << 16)) : hm1, hp1 << 16, want);
}

// From-scratch histogram of one species through the bins (counts cleared
// before): lane q of the grid takes beads 2q and 2q+1 of the species (one
// entry when both lie in one brick), so that a wave of 128 consecutive beads
// reserves room once per brick it touches.  Positions are read as three
// 8-byte pairs when `vec2` (8-byte aligned species start).
template <bool COUNT64>
__global__ __launch_bounds__(256) void density_hist_binned_kernel(
    const float *pos, uint64_t n_beads, uint32_t n, uint32_t n_a, Grid g, void *counts,
    const ArchDev *arch, BinArgs b, uint32_t vec2) {
  const uint64_t q = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t i0 = 2 * q, i1 = 2 * q + 1;
  const bool has0 = i0 < n_beads, has1 = i1 < n_beads;
  float r[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  if (has1 && vec2) {
    const float2 *p2 = reinterpret_cast<const float2 *>(pos + 3 * i0);
    const float2 a = p2[0], c = p2[1], d = p2[2];
    r[0] = a.x; r[1] = a.y; r[2] = c.x; r[3] = c.y; r[4] = d.x; r[5] = d.y;
  } else {
    if (has0) { r[0] = pos[3 * i0]; r[1] = pos[3 * i0 + 1]; r[2] = pos[3 * i0 + 2]; }
    if (has1) { r[3] = pos[3 * i1]; r[4] = pos[3 * i1 + 1]; r[5] = pos[3 * i1 + 2]; }
  }
  uint32_t x0, y0, z0, x1, y1, z1;
  cell3(g, r[0], r[1], r[2], x0, y0, z0);
  cell3(g, r[3], r[4], r[5], x1, y1, z1);
  const uint32_t k0 = brick_key(b, x0, y0, z0), k1 = brick_key(b, x1, y1, z1);
  const uint32_t j0 = n_beads <= 0xFFFFFFFFull ? (uint32_t)i0 % n : (uint32_t)(i0 % n);
  const uint32_t j1 = j0 + 1u == n ? 0u : j0 + 1u;
  const uint32_t t0 = bead_type(arch, j0, n_a), t1 = bead_type(arch, j1, n_a);
  const uint32_t h0 = kUpdPresent | (t0 << 11) | (k0 & 2047u);
  const uint32_t h1 = kUpdPresent | (t1 << 11) | (k1 & 2047u);
  const bool same = (k0 >> 11) == (k1 >> 11);
  uint32_t want = 0u;
  if (has0) want |= 1u;
  if (has1) want |= same ? 0u : 2u;
  const uint32_t v0 = (has1 && same) ? (h0 | (h1 << 16)) : h0;
  const uint32_t v1 = h1 << 16;
  // a lane without bead 2q has only bead 2q+1 absent too (n_beads is the end)
  bin_append<COUNT64>(b, g, counts, wave_sub_bin(blockDim.x >> 6), k0 >> 11, k1 >> 11, 0u, 0u,
                      v0, v1, 0u, 0u, want);
}

// Applies the bins to the counts: one workgroup of kApplyThreads per brick.
// The brick's count words (every plane) are staged in LDS, the bin's updates
// added with LDS atomics, the words written back, and the bin emptied for the
// next sweep.  The sub-bins' fill levels load together with the counts, and
// their entries are taken as one flat index range, kApplyBatch independent
// loads per thread at a time, so that a block waits on memory a few times
// rather than twice per sub-bin.
// LDS: planes x 2048 words (u16 pairs) or 2 x planes x 2048 halves (u32 pairs).
constexpr uint32_t kApplyThreads = 256u;
constexpr uint32_t kApplyBatch = 4u;
constexpr uint32_t kApplyPerThread = kBrickCells / kApplyThreads;   // cells per thread and plane

template <bool COUNT64>
__device__ __forceinline__ void apply_entry_lds(uint32_t *s_cnt, uint32_t planes, uint32_t e) {
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

// The body of one brick's workgroup (s_cnt: the dynamic LDS of the counts).
template <bool COUNT64>
__device__ __forceinline__ void bin_apply_brick(const BinArgs &b, const Grid &g, void *counts,
                                                uint32_t planes, uint32_t brick, uint32_t *s_cnt) {
  __shared__ uint32_t s_fill[kSubBins];
  const uint32_t tid = threadIdx.x;
  uint32_t fill = 0u;
  if (tid < kSubBins) fill = b.bin_count[(brick << kSubShift) | tid];
  const uint32_t bx = brick % b.nbx, rest = brick / b.nbx;
  const uint32_t by = rest % b.nby, bz = rest / b.nby;
  const uint32_t x0 = bx * 16u, y0 = by * 16u, z0 = bz * 8u;
  // cell l = tid + u * kApplyThreads of the brick: a thread keeps x = x0 + (tid & 15)
  const uint32_t x = x0 + (tid & 15u);
  for (uint32_t p = 0; p < planes; ++p) {
    uint2 v[kApplyPerThread];
#pragma unroll
    for (uint32_t u = 0; u < kApplyPerThread; ++u) {
      const uint32_t l = tid + u * kApplyThreads;
      const uint32_t y = y0 + ((l >> 4) & 15u), z = z0 + (l >> 8);
      v[u] = make_uint2(0u, 0u);
      if (x < (uint32_t)g.nx && y < (uint32_t)g.ny && z < (uint32_t)g.nz) {
        const size_t w = (size_t)p * g.n_cells + ((size_t)z * g.ny + y) * g.nx + x;
        if (COUNT64) v[u] = reinterpret_cast<const uint2 *>(counts)[w];
        else v[u].x = reinterpret_cast<const uint32_t *>(counts)[w];
      }
    }
#pragma unroll
    for (uint32_t u = 0; u < kApplyPerThread; ++u) {
      const uint32_t i = p * kBrickCells + tid + u * kApplyThreads;
      if (COUNT64) reinterpret_cast<uint2 *>(s_cnt)[i] = v[u];
      else s_cnt[i] = v[u].x;
    }
  }
  if (tid < kSubBins) s_fill[tid] = min(fill, b.cap);
  __syncthreads();
  // sub-bin s holds the flat indices [start[s], start[s] + fill of s)
  uint32_t start[kSubBins];
  uint32_t total = 0u;
#pragma unroll
  for (uint32_t s = 0; s < kSubBins; ++s) {
    start[s] = total;
    total += s_fill[s];
  }
  const uint32_t *bins = b.bins + (size_t)(brick << kSubShift) * b.cap;
  for (uint32_t j0 = 0; j0 < total; j0 += kApplyBatch * kApplyThreads) {
    uint32_t e[kApplyBatch];
#pragma unroll
    for (uint32_t u = 0; u < kApplyBatch; ++u) {
      const uint32_t j = j0 + u * kApplyThreads + tid;
      e[u] = 0u;
      if (j < total) {
        uint32_t sb = 0u, base = 0u;
#pragma unroll
        for (uint32_t s = 1; s < kSubBins; ++s) {
          const bool past = j >= start[s];
          sb = past ? s : sb;
          base = past ? start[s] : base;
        }
        e[u] = bins[(size_t)sb * b.cap + (j - base)];
      }
    }
#pragma unroll
    for (uint32_t u = 0; u < kApplyBatch; ++u) apply_entry_lds<COUNT64>(s_cnt, planes, e[u]);
  }
  __syncthreads();
  for (uint32_t p = 0; p < planes; ++p) {
#pragma unroll
    for (uint32_t u = 0; u < kApplyPerThread; ++u) {
      const uint32_t l = tid + u * kApplyThreads;
      const uint32_t y = y0 + ((l >> 4) & 15u), z = z0 + (l >> 8);
      if (x < (uint32_t)g.nx && y < (uint32_t)g.ny && z < (uint32_t)g.nz) {
        const size_t w = (size_t)p * g.n_cells + ((size_t)z * g.ny + y) * g.nx + x;
        const uint32_t i = p * kBrickCells + l;
        if (COUNT64)
          reinterpret_cast<uint2 *>(counts)[w] = reinterpret_cast<const uint2 *>(s_cnt)[i];
        else
          reinterpret_cast<uint32_t *>(counts)[w] = s_cnt[i];
      }
    }
  }
  if (tid < kSubBins) b.bin_count[(brick << kSubShift) | tid] = 0u;
}

template <bool COUNT64>
__global__ __launch_bounds__(kApplyThreads) void bin_apply_kernel(BinArgs b, Grid g, void *counts,
                                                                  uint32_t planes) {
  extern __shared__ uint32_t s_cnt[];
  bin_apply_brick<COUNT64>(b, g, counts, planes, blockIdx.x, s_cnt);
}

}  // namespace soma
