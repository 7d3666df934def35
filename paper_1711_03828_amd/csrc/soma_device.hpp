// soma_device.hpp -- device helpers of the SCMF hot path for gfx950:
// counter-based random numbers, uniform conversions, periodic cell indices.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace soma {

constexpr uint32_t kPurposeMoveA = 0u;
constexpr uint32_t kPurposeMoveB = 1u;
constexpr uint32_t kPurposeInit = 4u;
constexpr uint32_t kPurposeCollect = 5u;
constexpr uint32_t kSweepInit = 0xFFFFFFFFu;
constexpr uint32_t kAccSlots = 1024u;  // acceptance counter slots per move kind
constexpr float kMaxCoord = 4194304.0f;  // 2^22: cell arithmetic stays exact below

// Three-component vector kept in registers (a native vector type, so that
// selects between vectors never go through private memory).
typedef float F3 __attribute__((ext_vector_type(3)));

struct Rand4 {
  uint32_t x, y, z, w;
};

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).  The paper keeps a PCG
// state per thread in memory (Sec. 3.2.3); a counter-based generator needs no
// state at all, so the draws cost ALU work only.  The key schedule is
// wave-uniform and lands in scalar registers.
__device__ __forceinline__ Rand4 philox(uint32_t c0, uint32_t c1, uint32_t c2,
                                        uint32_t c3, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    // one v_mad_u64_u32 per product gives both halves
    const uint64_t p0 = (uint64_t)c0 * 0xD2511F53u;
    const uint64_t p1 = (uint64_t)c2 * 0xCD9E8D57u;
    // three-input XOR in one v_bitop3_b32 (truth table 0x96)
    c0 = __builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), c1, k0, 0x96);
    c1 = (uint32_t)p1;
    c2 = __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), c3, k1, 0x96);
    c3 = (uint32_t)p0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return {c0, c1, c2, c3};
}

// u = (2k+1) 2^-24 from the top 23 bits k: exact in FP32, in (0,1), symmetric.
// Built from the bit pattern 1 + k 2^-23 of [1,2): (f - 1) + 2^-24, both exact.
__device__ __forceinline__ float uniform01(uint32_t x) {
  const float f = __uint_as_float((x >> 9) | 0x3F800000u);
  return (f - 1.0f) + 0x1p-24f;
}
// v = 2u - 1 = (2f - 3) + 2^-23 in (-1,1), both steps exact.
__device__ __forceinline__ float uniform11(uint32_t x) {
  const float f = __uint_as_float((x >> 9) | 0x3F800000u);
  return fmaf(2.0f, f, -3.0f) + 0x1p-23f;
}

// Two standard normals from two words (Box-Muller).
__device__ __forceinline__ void box_muller(uint32_t w0, uint32_t w1, float &n0,
                                           float &n1) {
  const float rad = sqrtf(-2.0f * logf(uniform01(w0)));
  float s, c;
  sincospif(2.0f * uniform01(w1), &s, &c);
  n0 = rad * c;
  n1 = rad * s;
}

// floor(x) mod n, exact for |x| < 2^22; NaN and larger values are clamped
// first so the index is always inside [0, n).  The quotient estimate
// floor(f/n) may be off by one; the two unsigned minima fix either case.
__device__ __forceinline__ uint32_t wrap_cell(float x, int n, float inv_n) {
  const float f = fminf(fmaxf(floorf(x), -kMaxCoord), kMaxCoord);
  const float q = floorf(f * inv_n);
  const int r = (int)fmaf(-q, (float)n, f);  // exact: integers below 2^24
  // r in [-n, 0) -> r + n, r in [n, 2n) -> r - n: as unsigned words the one
  // candidate in [0, n) is the smallest of the three
  const uint32_t u = (uint32_t)r;
  return min(u, min(u + (uint32_t)n, u - (uint32_t)n));
}

// Cell coordinate of x' given the cell coordinate c of x and |x' - x| < 1:
// floor moves by -1, 0 or +1, then wraps at the box faces.
__device__ __forceinline__ uint32_t shift_cell(uint32_t c, float x, float xn, int n) {
  const int d = (int)(floorf(xn) - floorf(x));
  const uint32_t u = c + (uint32_t)d;   // -1 -> n-1 and n -> 0 as in wrap_cell
  return min(u, min(u + (uint32_t)n, u - (uint32_t)n));
}

struct Grid {
  int nx, ny, nz;
  float inv_nx, inv_ny, inv_nz;
  uint32_t n_cells;
};

__device__ __forceinline__ void cell3(const Grid &g, float x, float y, float z,
                                      uint32_t &cx, uint32_t &cy,
                                      uint32_t &cz) {
  cx = wrap_cell(x, g.nx, g.inv_nx);
  cy = wrap_cell(y, g.ny, g.inv_ny);
  cz = wrap_cell(z, g.nz, g.inv_nz);
}

// (z ny + y) nx + x with 24-bit multiplies (every factor is below 2^24).
__device__ __forceinline__ uint32_t cell_index(const Grid &g, uint32_t cx,
                                               uint32_t cy, uint32_t cz) {
  return __umul24(__umul24(cz, (uint32_t)g.ny) + cy, (uint32_t)g.nx) + cx;
}

__device__ __forceinline__ uint32_t cell_of(const Grid &g, float x, float y,
                                            float z) {
  uint32_t cx, cy, cz;
  cell3(g, x, y, z, cx, cy, cz);
  return cell_index(g, cx, cy, cz);
}

__device__ __forceinline__ bool coord_ok(float x) {
  return fabsf(x) < kMaxCoord;  // false for NaN and +-inf
}

// Consecutive logical tiles on one XCD: the hardware deals workgroups to the
// eight XCDs round-robin, so tile t runs on XCD t % 8.  Remapping gives XCD x
// the contiguous range [x n/8, (x+1) n/8) and keeps neighbouring chains (which
// share grid cells) in one L2.
__device__ __forceinline__ uint32_t xcd_remap(uint32_t b, uint32_t n) {
  const uint32_t n8 = n & ~7u;
  if (b >= n8) return b;
  return (b & 7u) * (n8 >> 3) + (b >> 3);
}

// ---------------------------------------------------------------------------
// General molecular architectures (decoded on the host).
// ---------------------------------------------------------------------------
constexpr uint32_t kArchMaxN = 128;       // monomers per molecule
constexpr uint32_t kArchMaxBonds = 2048;  // bond-list entries (each bond twice)
constexpr uint32_t kArchMaxSets = 16;

// One molecule type, decoded from the 32-bit architecture array (Sec. 3.2.1)
// on the host: types, the bond lists (partners in the array's order) and the
// independent sets (members of set s: member[set_start[s] .. set_start[s+1])).
struct ArchDev {
  uint32_t n, n_sets, n_type0;
  uint32_t per_wave;   // molecules per wave: min(64 / largest set, 128 / n), at least 1
  uint8_t type[kArchMaxN];
  uint8_t member[kArchMaxN];
  uint16_t set_start[kArchMaxSets + 1];
  uint16_t nb_start[kArchMaxN + 1];
  uint8_t nb[kArchMaxBonds];
};

// Type code of monomer i (0 .. n_t - 1): from the architecture, else 0 (A) for
// i < n_a and 1 (B).  Counts of type t live in the half t & 1 of the words of
// count plane t >> 1; its field is plane t.
__device__ __forceinline__ uint32_t bead_type(const ArchDev *arch, uint32_t i, uint32_t n_a) {
  return arch ? (uint32_t)arch->type[i] : (i >= n_a ? 1u : 0u);
}

}  // namespace soma
