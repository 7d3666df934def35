// soma_batch.hpp -- one sweep launch over many melts (replicas of different
// size, chain length and interaction strength).
//
// Small melts alone cannot fill 256 compute units (Secs. 5.1-5.2: small systems
// leave the GPU idle), so the chain tiles of all melts of a batch form one
// work list.  An item is one block's worth of chains (four wave tiles) of one
// (melt, species) segment; segments are listed largest first and the list is
// cut into eight equal contiguous ranges, one per XCD, so that the blocks
// running on one XCD touch few melts and their grids stay in that XCD's L2.
// Every item costs about the same (each wave moves 2 x 64 beads whatever the
// chain length), so equal ranges are balanced ranges.  Each segment carries
// its own arguments (positions, grids, constants, counters); the Philox
// counters of a bead are those of an unbatched sweep of its melt, so a
// batched sweep gives bit-identical results.
#pragma once

#include "soma_grid.hpp"
#include "soma_sweep.hpp"

namespace soma {

struct BatchSeg {
  SweepArgs a;   // sweep offset 0: the melt's device counter decides
  MixArgs mx;
};

struct BatchLaunch {
  const BatchSeg *segs;
  const uint32_t *seg_first;   // [n_segs + 1] first item of each segment
  uint32_t n_segs, n_items;
  uint32_t per_xcd;            // items per XCD range (mode 0)
  uint32_t mode;               // 0: XCD ranges; 1: items dealt round-robin
  uint32_t sweep_off;          // offset of this launch within a captured cycle
  uint32_t sub_k, sub_j;       // chain subset of this launch (see SweepArgs)
};

// BINNED: count updates through the melts' own per-brick bins (each segment's
// SweepArgs carry its melt's BinArgs), applied afterwards by
// batched_bin_apply_kernel; else direct atomics.
template <bool COUNT64, bool VEC2, uint32_t KIND, bool BINNED>
__global__ __launch_bounds__(256, 2) void batched_sweep_kernel(const BatchLaunch L) {
  __shared__ __bf16 s_act[KIND == 2 ? 4 : 1][KIND == 2 ? 64 * kActStride : 1];
  __shared__ float s_z[KIND == 2 ? 4 : 1][KIND == 2 ? 64 * 8 : 1];
  __shared__ __bf16 s_w[KIND == 2 ? kWRows * kWStride : 1];
  uint32_t net_sg = 0xFFFFFFFFu;   // segment whose weights s_w holds (mixed sweeps)
  uint32_t item, end, stride;
  if (L.mode == 0) {   // grid is a multiple of 8 blocks (host-checked)
    const uint32_t x = blockIdx.x & 7u;
    item = x * L.per_xcd + (blockIdx.x >> 3);
    end = min((x + 1u) * L.per_xcd, L.n_items);
    stride = gridDim.x >> 3;
  } else {
    item = blockIdx.x;
    end = L.n_items;
    stride = gridDim.x;
  }
  for (; item < end; item += stride) {   // block-uniform loop
    const uint32_t sg = range_of(L.seg_first, L.n_segs, item);
    SweepArgs a = resolve_sweep(L.segs[sg].a, L.sweep_off);
    a.sub_k = L.sub_k;
    a.sub_j = L.sub_j;
    a.n_sub = a.n_chains > L.sub_j ? (a.n_chains - L.sub_j + L.sub_k - 1u) / L.sub_k : 0u;
    const uint32_t tile = (item - L.seg_first[sg]) * 4u + (threadIdx.x >> 6);
    const LaneMap m = lane_map_tile(a, tile, true);
    if (KIND == 0) {
      float *cp = a.pos + (size_t)(m.has0 ? m.chain : 0u) * a.n * 3u + 6u * m.k;
      F3 r0, r1;
      load_pair<VEC2>(cp, m, r0, r1);
      finish_block(a, local_tile<COUNT64, VEC2, BINNED>(a, m, cp, r0, r1));
    } else if (KIND == 1) {
      finish_block(a, smc_wave<COUNT64, VEC2, BINNED>(a, m));
    } else if (KIND == 3) {
      finish_block(a, smc_wave<COUNT64, VEC2, BINNED, true>(a, m));
    } else {
      const MixArgs mx = L.segs[sg].mx;
      if (sg != net_sg) {   // block-uniform: a new segment's network
        __syncthreads();
        net_weights_to_lds(mx.net, s_w);
        __syncthreads();
        net_sg = sg;
      }
      uint32_t cnt[3];
      mixed_wave<COUNT64, VEC2, BINNED>(a, mx, m, s_act[KIND == 2 ? m.wib : 0],
                                       s_z[KIND == 2 ? m.wib : 0], s_w, cnt);
      mixed_finish(a, mx, cnt);
    }
  }
}

// The bins of every melt of a batch applied in one launch: one workgroup per
// brick of every melt (melt s owns the blocks [brick_first[s],
// brick_first[s + 1])), each the brick workgroup of bin_apply_kernel.
struct BinApplySeg {
  BinArgs b;
  Grid g;
  void *counts;
};

template <bool COUNT64>
__global__ __launch_bounds__(kApplyThreads) void batched_bin_apply_kernel(
    const BinApplySeg *__restrict__ segs, const uint32_t *__restrict__ brick_first,
    uint32_t n_sys) {
  extern __shared__ uint32_t s_cnt[];
  const uint32_t s = range_of(brick_first, n_sys, blockIdx.x);
  const BinApplySeg x = segs[s];
  bin_apply_brick<COUNT64>(x.b, x.g, x.counts, 1u, blockIdx.x - brick_first[s], s_cnt);
}

}  // namespace soma
