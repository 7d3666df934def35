/*
 * soma_oracle.c -- plain, slow CPU oracle for the SCMF hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, header, table or constant generator
 * with the HIP path: both sides implement the same written specification
 * independently.
 *
 * Paper: L. Schneider and M. Mueller, "Multi-Architecture Monte-Carlo (MC)
 * Simulation of Soft Coarse-Grained Polymeric Materials: SOft coarse grained
 * Monte-carlo Acceleration (SOMA)", arXiv:1711.03828.
 *
 * Every function cites the passage it follows.  Conventions (readings of the
 * paper that it leaves open) are the ones documented with the project:
 *   - lengths in grid units (Delta L = 1); positions FP32, unwrapped;
 *   - a cell is the half-open unit cube [i, i+1), the index is floor(x) mod n;
 *   - two bead types A (0) and B (1); a linear species A_{NA} B_{N-NA};
 *   - counts held as one uint32 plane per type, omega as one FP32 plane per
 *     type, planes ordered A then B; a cell's linear index is (z*ny + y)*nx + x;
 *   - energies, forces and the Metropolis / Metropolis-Hastings ratio are
 *     evaluated in FP64 from the FP32 state.
 *
 * Parity status: every function below is pinned by a CPU test
 * (tests/test_oracle_*.py) except where its header says "parity unpinned".
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_TYPE_A 0u
#define ORC_TYPE_B 1u

#define ORC_MOVE_LOCAL 0u
#define ORC_MOVE_SMC 1u
#define ORC_MOVE_GIBBS 3u

#define ORC_PURPOSE_MOVE_A 0u
#define ORC_PURPOSE_MOVE_B 1u
#define ORC_PURPOSE_INIT 4u

#define ORC_SWEEP_INIT 0xFFFFFFFFu

/* ------------------------------------------------------------------------- */
/* Philox4x32-10, from its published definition (Salmon, Moraes, Dror, Shaw,  */
/* "Parallel random numbers: as easy as 1, 2, 3", SC'11).  The paper itself   */
/* stores a PCG state per thread (Sec. 3.2.3); a stateless counter-based      */
/* generator replaces it here so that no generator state lives in memory.     */
/* ------------------------------------------------------------------------- */
void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2],
                       uint32_t out[4]) {
  uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
  uint32_t k0 = key_in[0], k1 = key_in[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += 0x9E3779B9u; /* golden ratio Weyl increment */
      k1 += 0xBB67AE85u; /* sqrt(3)-1 Weyl increment */
    }
    uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c1 ^ k0;
    uint32_t n1 = lo1;
    uint32_t n2 = hi0 ^ c3 ^ k1;
    uint32_t n3 = lo0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Batch form for the tests. */
void orc_philox_batch(uint64_t n, const uint32_t *ctr, const uint32_t *key,
                      uint32_t *out) {
  for (uint64_t i = 0; i < n; ++i)
    orc_philox4x32_10(ctr + 4 * i, key + 2 * i, out + 4 * i);
}

static void orc_draw(uint64_t seed, uint32_t chain, uint32_t bead,
                     uint32_t purpose, uint32_t sweep, uint32_t replica,
                     uint32_t out[4]) {
  uint32_t ctr[4] = {chain, bead | (purpose << 16), sweep, replica};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  orc_philox4x32_10(ctr, key, out);
}

/* Uniform on the open interval (0,1): the top 23 bits k of a word give
 * u = (2k+1) / 2^24, which FP32 holds exactly and which is symmetric about
 * 1/2.  v = 2u - 1 lies in (-1,1), is exact and never 0. */
float orc_u01(uint32_t x) { return (float)(2u * (x >> 9) + 1u) * 0x1p-24f; }
float orc_v11(uint32_t x) {
  return (float)((int32_t)(2u * (x >> 9) + 1u) - (int32_t)(1u << 23)) * 0x1p-23f;
}

/* Box-Muller in FP64 from two FP32 uniforms. */
static void orc_box_muller(uint32_t w0, uint32_t w1, double *n0, double *n1) {
  double u1 = (double)orc_u01(w0), u2 = (double)orc_u01(w1);
  double r = sqrt(-2.0 * log(u1));
  double ang = 2.0 * M_PI * u2;
  *n0 = r * cos(ang);
  *n1 = r * sin(ang);
}

/* ------------------------------------------------------------------------- */
/* Grid geometry: cubic collocation grid with spacing Delta L (Sec. 2.1,      */
/* Eq. (4) and the characteristic function of a cell that follows it).        */
/* ------------------------------------------------------------------------- */
static int64_t orc_wrap(double x, uint32_t n) {
  double f = floor(x);
  int64_t i = (int64_t)f;
  int64_t m = i % (int64_t)n;
  if (m < 0) m += n;
  return m;
}

static uint64_t orc_cell(const float *r, uint32_t nx, uint32_t ny,
                         uint32_t nz) {
  int64_t cx = orc_wrap((double)r[0], nx);
  int64_t cy = orc_wrap((double)r[1], ny);
  int64_t cz = orc_wrap((double)r[2], nz);
  return ((uint64_t)cz * ny + (uint64_t)cy) * nx + (uint64_t)cx;
}

static uint64_t orc_cell_shift(const float *r, int dim, int s, uint32_t nx,
                               uint32_t ny, uint32_t nz) {
  int64_t c[3] = {orc_wrap((double)r[0], nx), orc_wrap((double)r[1], ny),
                  orc_wrap((double)r[2], nz)};
  int64_t n[3] = {nx, ny, nz};
  c[dim] = ((c[dim] + s) % n[dim] + n[dim]) % n[dim];
  return ((uint64_t)c[2] * ny + (uint64_t)c[1]) * nx + (uint64_t)c[0];
}

/* Bead type inside a linear species A_{NA} B_{N-NA} (Sec. 2.1: every bead
 * has one of n_t types; here n_t = 2). */
static uint32_t orc_type(uint32_t i, uint32_t n_a) {
  return i < n_a ? ORC_TYPE_A : ORC_TYPE_B;
}

/* ------------------------------------------------------------------------- */
/* Density histogram: occupation numbers n_i(c) of every type in every cell,   */
/* Eq. (4) with the characteristic-function assignment; counted once per MC   */
/* step (Sec. 3.1.1).  counts[t * n_cells + c] is zeroed here.                 */
/* ------------------------------------------------------------------------- */
void orc_density_hist(const float *pos, uint32_t n_species,
                      const uint32_t *n_chains, const uint32_t *n_per_chain,
                      const uint32_t *n_a, uint32_t nx, uint32_t ny,
                      uint32_t nz, uint32_t *counts) {
  uint64_t n_cells = (uint64_t)nx * ny * nz;
  memset(counts, 0, 2 * n_cells * sizeof(uint32_t));
  uint64_t bead = 0;
  for (uint32_t s = 0; s < n_species; ++s)
    for (uint32_t c = 0; c < n_chains[s]; ++c)
      for (uint32_t i = 0; i < n_per_chain[s]; ++i, ++bead) {
        uint64_t cell = orc_cell(pos + 3 * bead, nx, ny, nz);
        counts[orc_type(i, n_a[s]) * n_cells + cell] += 1u;
      }
}

/* ------------------------------------------------------------------------- */
/* Quasi-instantaneous fields, Eq. (12), K^1 form of the interaction (Eq. (8)) */
/* for two types:                                                              */
/*   phi_t = n_t / (rho0 dL^3),   omega_A = kappaN (phi_A+phi_B-1) + chiN phi_B */
/*                                omega_B = kappaN (phi_A+phi_B-1) + chiN phi_A */
/* omega is the per-chain (xN) field; the energy of one bead is omega/N with   */
/* N the reference chain length (Sec. 2.1, the paragraph on N-invariance).     */
/* inv_rho = 1/(rho0 dL^3) = n_cells / n_beads.                                */
/* ------------------------------------------------------------------------- */
/* External fields (Sec. 4): ext (may be NULL) holds per type and cell an
 * energy in the units of omega, added to the interaction field; a cell whose
 * bit is set in forbid (may be NULL) is impenetrable and gets the field 0
 * (no bead enters it).  With forbidden cells the reference density counts
 * the free cells only (inv_rho = n_free / n_beads, chosen by the caller). */
#define ORC_MAX_TYPES 8
static int orc_bit(const uint32_t *mask, uint64_t c) {
  return mask && ((mask[c >> 5] >> (c & 31u)) & 1u);
}

/* form selects the interaction term of Eq. (6): 1 = K^1 (chiN phi_A phi_B, the
 * default), 0 = K^0 (-chiN/4 (phi_A - phi_B)^2), both read over unordered
 * pairs; the K^0 field is kappaN (phi_A+phi_B-1) -+ chiN/2 (phi_A - phi_B)
 * (Eq. (12), its first form). */
void orc_field_f64(const uint32_t *counts, uint64_t n_cells, double inv_rho,
                   double chi_n, double kappa_n, uint32_t form, const float *ext,
                   const uint32_t *forbid, double *omega) {
  for (uint64_t c = 0; c < n_cells; ++c) {
    double phi_a = counts[c] * inv_rho;
    double phi_b = counts[n_cells + c] * inv_rho;
    double incompress = kappa_n * (phi_a + phi_b - 1.0);
    if (form == 0) {
      omega[c] = incompress - 0.5 * chi_n * (phi_a - phi_b);
      omega[n_cells + c] = incompress - 0.5 * chi_n * (phi_b - phi_a);
    } else {
      omega[c] = incompress + chi_n * phi_b;
      omega[n_cells + c] = incompress + chi_n * phi_a;
    }
    if (ext) {
      omega[c] += (double)ext[c];
      omega[n_cells + c] += (double)ext[n_cells + c];
    }
    if (orc_bit(forbid, c)) omega[c] = omega[n_cells + c] = 0.0;
  }
}

/* The same field in a fixed FP32 operation order (products and sums rounded
 * one by one, the chi term fused), used to hold the device result to
 * bit equality.  Compiled with -ffp-contract=off so the order is the one
 * written. */
/* K^0 in FP32: d = phi_A - phi_B, omega_A = fma(-chiN/2, d, t),
 * omega_B = fma(chiN/2, d, t) (chiN/2 is exact). */
void orc_field_f32(const uint32_t *counts, uint64_t n_cells, float inv_rho,
                   float chi_n, float kappa_n, uint32_t form, const float *ext,
                   const uint32_t *forbid, float *omega) {
  for (uint64_t c = 0; c < n_cells; ++c) {
    float phi_a = (float)counts[c] * inv_rho;
    float phi_b = (float)counts[n_cells + c] * inv_rho;
    float s = (phi_a + phi_b) - 1.0f;
    float t = kappa_n * s;
    float wa, wb;
    if (form == 0) {
      float d = phi_a - phi_b;
      wa = fmaf(-0.5f * chi_n, d, t);
      wb = fmaf(0.5f * chi_n, d, t);
    } else {
      wa = fmaf(chi_n, phi_b, t);
      wb = fmaf(chi_n, phi_a, t);
    }
    if (ext) {
      wa = wa + ext[c];
      wb = wb + ext[n_cells + c];
    }
    if (orc_bit(forbid, c)) wa = wb = 0.0f;
    omega[c] = wa;
    omega[n_cells + c] = wb;
  }
}

/* Non-bonded energy on the grid, Eqs. (5), (6), (8), in units of kT:
 *   H_nb = (rho0 dL^3 / N) sum_c [ kappaN/2 (phi_A+phi_B-1)^2 + chiN phi_A phi_B ]
 * (the i != j sum of Eq. (8) read over unordered pairs, which is the reading
 * that reproduces the field of Eq. (12) as its derivative). */
double orc_h_nb(const uint32_t *counts, uint64_t n_cells, double inv_rho,
                double chi_n, double kappa_n, uint32_t n_ref, uint32_t form,
                const uint32_t *forbid) {
  double sum = 0.0;
  for (uint64_t c = 0; c < n_cells; ++c) {
    if (orc_bit(forbid, c)) continue;   /* impenetrable cells hold no beads */
    double phi_a = counts[c] * inv_rho;
    double phi_b = counts[n_cells + c] * inv_rho;
    double dev = phi_a + phi_b - 1.0;
    double inter = form == 0 ? -0.25 * chi_n * (phi_a - phi_b) * (phi_a - phi_b)
                             : chi_n * phi_a * phi_b;
    sum += 0.5 * kappa_n * dev * dev + inter;
  }
  return sum / (inv_rho * (double)n_ref);
}

/* ------------------------------------------------------------------------- */
/* n_t bead types (Sec. 2.1).  counts: n_t planes of n_cells (type i in plane  */
/* i); chi: the symmetric n_t x n_t matrix of chi_ij N (diagonal unused).      */
/* Fields, Eq. (12):                                                           */
/*   K^1: omega_i = kappaN (sum_k phi_k - 1) + sum_{k != i} chi_ik N phi_k      */
/*   K^0: omega_i = kappaN (sum_k phi_k - 1)                                   */
/*                  - sum_{k != i} (chi_ik N / 2) (phi_i - phi_k)               */
/* For n_t = 2 these are the two-type fields above.                            */
/* ------------------------------------------------------------------------- */
void orc_field_multi_f64(const uint32_t *counts, uint64_t n_cells, uint32_t n_t,
                         double inv_rho, const double *chi, double kappa_n, uint32_t form,
                         double *omega) {
  for (uint64_t c = 0; c < n_cells; ++c) {
    double phi[ORC_MAX_TYPES], total = 0.0;
    for (uint32_t i = 0; i < n_t; ++i) {
      phi[i] = counts[(uint64_t)i * n_cells + c] * inv_rho;
      total += phi[i];
    }
    for (uint32_t i = 0; i < n_t; ++i) {
      double w = kappa_n * (total - 1.0);
      for (uint32_t k = 0; k < n_t; ++k) {
        if (k == i) continue;
        if (form == 0) w -= 0.5 * chi[i * n_t + k] * (phi[i] - phi[k]);
        else w += chi[i * n_t + k] * phi[k];
      }
      omega[(uint64_t)i * n_cells + c] = w;
    }
  }
}

/* The same in FP32, operation by operation:
 *   s = (((phi_0 + phi_1) + phi_2) + ...) - 1,  t = kappaN * s,
 *   then for k = 0, 1, ... (k != i): t = fma(chi_ik, phi_k, t) (K^1) or
 *   t = fma(-chi_ik / 2, phi_i - phi_k, t) (K^0); omega_i = t.
 * With two types this is the two-type FP32 order above. */
void orc_field_multi_f32(const uint32_t *counts, uint64_t n_cells, uint32_t n_t,
                         float inv_rho, const float *chi, float kappa_n, uint32_t form,
                         float *omega) {
  for (uint64_t c = 0; c < n_cells; ++c) {
    float phi[ORC_MAX_TYPES];
    for (uint32_t i = 0; i < n_t; ++i) phi[i] = (float)counts[(uint64_t)i * n_cells + c] * inv_rho;
    float s = phi[0];
    for (uint32_t i = 1; i < n_t; ++i) s = s + phi[i];
    s = s - 1.0f;
    for (uint32_t i = 0; i < n_t; ++i) {
      float t = kappa_n * s;
      for (uint32_t k = 0; k < n_t; ++k) {
        if (k == i) continue;
        if (form == 0) t = fmaf(-0.5f * chi[i * n_t + k], phi[i] - phi[k], t);
        else t = fmaf(chi[i * n_t + k], phi[k], t);
      }
      omega[(uint64_t)i * n_cells + c] = t;
    }
  }
}

/* H_nb / kT for n_t types, Eqs. (5), (6), (8), the i != j sums over
 * unordered pairs i < j:
 *   (rho0 dL^3 / N) sum_c [ kappaN/2 (sum phi - 1)^2 + sum_{i<j} K_ij ],
 *   K_ij = chi_ij N phi_i phi_j (K^1) or -(chi_ij N / 4)(phi_i - phi_j)^2 (K^0). */
double orc_h_nb_multi(const uint32_t *counts, uint64_t n_cells, uint32_t n_t, double inv_rho,
                      const double *chi, double kappa_n, uint32_t n_ref, uint32_t form) {
  double sum = 0.0;
  for (uint64_t c = 0; c < n_cells; ++c) {
    double phi[ORC_MAX_TYPES], total = 0.0, inter = 0.0;
    for (uint32_t i = 0; i < n_t; ++i) {
      phi[i] = counts[(uint64_t)i * n_cells + c] * inv_rho;
      total += phi[i];
    }
    for (uint32_t i = 0; i < n_t; ++i)
      for (uint32_t j = i + 1; j < n_t; ++j) {
        double x = chi[i * n_t + j];
        inter += form == 0 ? -0.25 * x * (phi[i] - phi[j]) * (phi[i] - phi[j]) : x * phi[i] * phi[j];
      }
    sum += 0.5 * kappa_n * (total - 1.0) * (total - 1.0) + inter;
  }
  return sum / (inv_rho * (double)n_ref);
}

/* ------------------------------------------------------------------------- */
/* Bonded energy of one bead with its chain neighbours, Eqs. (1)-(2):          */
/* V = (k0/2) r^2 per bond.                                                    */
/* ------------------------------------------------------------------------- */
static double orc_bond_energy(const float *r, const float *chain, uint32_t i,
                              uint32_t n, double k0) {
  double e = 0.0;
  for (int nb = -1; nb <= 1; nb += 2) {
    int64_t j = (int64_t)i + nb;
    if (j < 0 || j >= (int64_t)n) continue;
    const float *rj = chain + 3 * j;
    for (int d = 0; d < 3; ++d) {
      double dx = (double)r[d] - (double)rj[d];
      e += 0.5 * k0 * dx * dx;
    }
  }
  return e;
}

/* Force on a bead used by the force-biased proposal (Sec. 2.2, smart MC):
 * the bonded force -dH_b/dr plus the grid-field force -(1/N) grad omega_t,
 * with the gradient taken as the central difference of omega between the two
 * neighbouring cells of the cell that holds r (piecewise constant in a cell). */
static void orc_force(const float *r, const float *chain, uint32_t i,
                      uint32_t n, double k0, const float *omega_t,
                      uint32_t nx, uint32_t ny, uint32_t nz, uint32_t n_ref,
                      double f[3]) {
  f[0] = f[1] = f[2] = 0.0;
  for (int nb = -1; nb <= 1; nb += 2) {
    int64_t j = (int64_t)i + nb;
    if (j < 0 || j >= (int64_t)n) continue;
    const float *rj = chain + 3 * j;
    for (int d = 0; d < 3; ++d) f[d] += k0 * ((double)rj[d] - (double)r[d]);
  }
  if (omega_t) {
    for (int d = 0; d < 3; ++d) {
      double up = omega_t[orc_cell_shift(r, d, +1, nx, ny, nz)];
      double dn = omega_t[orc_cell_shift(r, d, -1, nx, ny, nz)];
      f[d] -= 0.5 * (up - dn) / (double)n_ref;
    }
  }
}

/* ------------------------------------------------------------------------- */
/* One MC sweep of one linear species with the fields held fixed (stage 2 of   */
/* the SCMF cycle, Sec. 2.2).                                                  */
/*                                                                             */
/* Order of attempts: the "SET" scheme of Sec. 3.1.2 -- for a linear chain the */
/* even and the odd beads are the two independent sets; per chain and sweep    */
/* the order of the two sets is random (bit 0 of the first word of bead 0's   */
/* move draw), or even-first when set_order == 1.  Inside a set the moves do  */
/* not interact, so doing them one after another equals doing them at once.   */
/*                                                                             */
/* LOCAL (Sec. 2.2, move (i)): trial displacement uniform in [-a,a] per        */
/* Cartesian direction, r' = fmaf(a, v, r) in FP32; Metropolis acceptance      */
/* min(1, exp(-dE)) with dE = dE_bond + (omega_t(c') - omega_t(c))/N           */
/* (the non-bonded change of Eq. (15), per bead).                              */
/*                                                                             */
/* SMC (Sec. 2.2, move (ii), force-biased): r' = r + A F(r) + sqrt(2A) xi,     */
/* xi ~ N(0,1)^3, accepted by Metropolis-Hastings with the ratio of the        */
/* Gaussian proposal densities q(r|r') / q(r'|r).                              */
/*                                                                             */
/* Random numbers: Philox4x32-10, key = seed, counter = (chain_base + chain,   */
/* bead | purpose << 16, sweep, replica).  LOCAL uses one block (words 0-2:    */
/* displacement, word 3: acceptance).  SMC uses block A (purpose 0) for four   */
/* normals and block B (purpose 1), word 0, for acceptance.                    */
/*                                                                             */
/* accept_flags (n_chains * N bytes, may be NULL) records 1 for an accepted    */
/* move.  Returns the number of accepted moves.                                */
/* ------------------------------------------------------------------------- */
/* Impenetrable cells for the moves (Sec. 4, geometric confinement): a trial
 * position in a set cell other than the bead's own cell is rejected (an
 * infinite energy).  With impenetrable cells set, a trial more than one cell
 * away from the bead along any axis is rejected as well, so that no move can
 * jump over a wall of impenetrable cells: floor(x') - floor(x) must lie in
 * {-1, 0, 1} per axis on the unwrapped coordinates.  The condition is
 * symmetric in (x, x'), so detailed balance holds for the restricted move.
 * NULL: none.  Set by orc_set_forbidden before a sweep; read-only during it. */
static const uint32_t *orc_forbidden = NULL;
void orc_set_forbidden(const uint32_t *mask) { orc_forbidden = mask; }
static int orc_blocked(const float *r, const float *trial, uint32_t nx, uint32_t ny,
                       uint32_t nz) {
  if (!orc_forbidden) return 0;
  for (int d = 0; d < 3; ++d)
    if (fabs(floor((double)trial[d]) - floor((double)r[d])) > 1.0) return 1;
  uint64_t to = orc_cell(trial, nx, ny, nz);
  return to != orc_cell(r, nx, ny, nz) && orc_bit(orc_forbidden, to);
}

/* Energy added to every move that changes cell (0: the quasi-instantaneous
 * field alone).  Moving one bead of type t from cell c to c' changes the grid
 * Hamiltonian of Eqs. (5), (6), (8) (quadratic in the counts) by
 * (omega_t(c') - omega_t(c))/N plus its second difference in n_t, which the
 * caller passes here (kappaN/(N rho) for the K^1 form). */
static double orc_self = 0.0;
void orc_set_self_term(double s) { orc_self = s; }
static double orc_self_extra(const float *r, const float *trial, uint32_t nx, uint32_t ny,
                             uint32_t nz) {
  return orc_cell(r, nx, ny, nz) != orc_cell(trial, nx, ny, nz) ? orc_self : 0.0;
}

/* One local attempt on bead i from the four words w of its draw. */
static int orc_local_attempt(float *chain, uint32_t i, uint32_t n, uint32_t n_a,
                             double k0, const float *omega, uint64_t n_cells,
                             uint32_t nx, uint32_t ny, uint32_t nz,
                             uint32_t n_ref, float a, const uint32_t w[4]) {
  float *r = chain + 3 * i;
  float trial[3];
  for (int d = 0; d < 3; ++d) trial[d] = fmaf(a, orc_v11(w[d]), r[d]);
  if (orc_blocked(r, trial, nx, ny, nz)) return 0;
  double d_bond = orc_bond_energy(trial, chain, i, n, k0) -
                  orc_bond_energy(r, chain, i, n, k0);
  const float *om = omega + (uint64_t)orc_type(i, n_a) * n_cells;
  double d_field = ((double)om[orc_cell(trial, nx, ny, nz)] -
                    (double)om[orc_cell(r, nx, ny, nz)]) /
                   (double)n_ref + orc_self_extra(r, trial, nx, ny, nz);
  double d_e = d_bond + d_field;
  double u = (double)orc_u01(w[3]);
  int accept = (d_e <= 0.0) || (u < exp(-d_e));
  if (accept) memcpy(r, trial, sizeof trial);
  return accept;
}

static int orc_move_local(float *chain, uint32_t c_id, uint32_t i, uint32_t n,
                          uint32_t n_a, double k0, const float *omega,
                          uint64_t n_cells, uint32_t nx, uint32_t ny,
                          uint32_t nz, uint32_t n_ref, float a, uint64_t seed,
                          uint32_t sweep, uint32_t replica) {
  uint32_t w[4];
  orc_draw(seed, c_id, i, ORC_PURPOSE_MOVE_A, sweep, replica, w);
  return orc_local_attempt(chain, i, n, n_a, k0, omega, n_cells, nx, ny, nz,
                           n_ref, a, w);
}

static int orc_move_smc(float *chain, uint32_t c_id, uint32_t i, uint32_t n,
                        uint32_t n_a, double k0, const float *omega,
                        uint64_t n_cells, uint32_t nx, uint32_t ny,
                        uint32_t nz, uint32_t n_ref, float a_smc,
                        uint64_t seed, uint32_t sweep, uint32_t replica) {
  uint32_t wa[4], wb[4];
  orc_draw(seed, c_id, i, ORC_PURPOSE_MOVE_A, sweep, replica, wa);
  orc_draw(seed, c_id, i, ORC_PURPOSE_MOVE_B, sweep, replica, wb);
  double xi[4];
  orc_box_muller(wa[0], wa[1], &xi[0], &xi[1]);
  orc_box_muller(wa[2], wa[3], &xi[2], &xi[3]);
  const float *om = omega + (uint64_t)orc_type(i, n_a) * n_cells;
  double A = (double)a_smc;
  float *r = chain + 3 * i;
  double f_old[3], f_new[3];
  orc_force(r, chain, i, n, k0, om, nx, ny, nz, n_ref, f_old);
  float trial[3];
  for (int d = 0; d < 3; ++d)
    trial[d] = (float)((double)r[d] + A * f_old[d] + sqrt(2.0 * A) * xi[d]);
  if (orc_blocked(r, trial, nx, ny, nz)) return 0;
  orc_force(trial, chain, i, n, k0, om, nx, ny, nz, n_ref, f_new);
  double log_fwd = 0.0, log_rev = 0.0;
  for (int d = 0; d < 3; ++d) {
    double x_f = (double)trial[d] - (double)r[d] - A * f_old[d];
    double x_r = (double)r[d] - (double)trial[d] - A * f_new[d];
    log_fwd -= x_f * x_f / (4.0 * A);
    log_rev -= x_r * x_r / (4.0 * A);
  }
  double d_bond = orc_bond_energy(trial, chain, i, n, k0) -
                  orc_bond_energy(r, chain, i, n, k0);
  double d_field = ((double)om[orc_cell(trial, nx, ny, nz)] -
                    (double)om[orc_cell(r, nx, ny, nz)]) /
                   (double)n_ref + orc_self_extra(r, trial, nx, ny, nz);
  double log_ratio = -(d_bond + d_field) + log_rev - log_fwd;
  double u = (double)orc_u01(wb[0]);
  int accept = (log_ratio >= 0.0) || (u < exp(log_ratio));
  if (accept) memcpy(r, trial, sizeof trial);
  return accept;
}

/* Bond-Gibbs move: the trial position is drawn from the distribution of the
 * bead given its bonded neighbours under the bond energy alone, Eqs. (1)-(2):
 * a Gaussian around the mean of the neighbours with variance 1/(n_b k0) per
 * component (n_b = 1 or 2 neighbours); a bead without bonds makes a symmetric
 * Gaussian step of variance 1/(2 k0).  Accepted by the Metropolis-Hastings
 * ratio exp(-dE) q(r|r') / q(r'|r), evaluated here term by term (the bond and
 * proposal terms cancel in exact arithmetic, leaving the field term).  Draws:
 * block A (purpose 0) for four normals (three used), block B (purpose 1), word
 * 0, for acceptance -- the smart-MC layout. */
static int orc_move_gibbs(float *chain, uint32_t c_id, uint32_t i, uint32_t n,
                          uint32_t n_a, double k0, const float *omega,
                          uint64_t n_cells, uint32_t nx, uint32_t ny,
                          uint32_t nz, uint32_t n_ref, uint64_t seed,
                          uint32_t sweep, uint32_t replica) {
  uint32_t wa[4], wb[4];
  orc_draw(seed, c_id, i, ORC_PURPOSE_MOVE_A, sweep, replica, wa);
  orc_draw(seed, c_id, i, ORC_PURPOSE_MOVE_B, sweep, replica, wb);
  double xi[4];
  orc_box_muller(wa[0], wa[1], &xi[0], &xi[1]);
  orc_box_muller(wa[2], wa[3], &xi[2], &xi[3]);
  float *r = chain + 3 * i;
  int n_b = (i > 0) + (i + 1 < n);
  double mu[3], var;
  for (int d = 0; d < 3; ++d) {
    double s = 0.0;
    if (i > 0) s += (double)chain[3 * (i - 1) + d];
    if (i + 1 < n) s += (double)chain[3 * (i + 1) + d];
    mu[d] = n_b > 0 ? s / n_b : (double)r[d];
  }
  var = 1.0 / ((n_b > 0 ? n_b : 2) * k0);
  float trial[3];
  for (int d = 0; d < 3; ++d) trial[d] = (float)(mu[d] + sqrt(var) * xi[d]);
  if (orc_blocked(r, trial, nx, ny, nz)) return 0;
  /* log q(x | y): the Gaussian around mu (n_b > 0, independent of y) or around y */
  double log_fwd = 0.0, log_rev = 0.0;
  for (int d = 0; d < 3; ++d) {
    double cf = n_b > 0 ? mu[d] : (double)r[d];
    double cr = n_b > 0 ? mu[d] : (double)trial[d];
    log_fwd -= ((double)trial[d] - cf) * ((double)trial[d] - cf) / (2.0 * var);
    log_rev -= ((double)r[d] - cr) * ((double)r[d] - cr) / (2.0 * var);
  }
  const float *om = omega + (uint64_t)orc_type(i, n_a) * n_cells;
  double d_bond = orc_bond_energy(trial, chain, i, n, k0) - orc_bond_energy(r, chain, i, n, k0);
  double d_field = ((double)om[orc_cell(trial, nx, ny, nz)] -
                    (double)om[orc_cell(r, nx, ny, nz)]) / (double)n_ref +
                   orc_self_extra(r, trial, nx, ny, nz);
  double log_ratio = -(d_bond + d_field) + log_rev - log_fwd;
  double u = (double)orc_u01(wb[0]);
  int accept = (log_ratio >= 0.0) || (u < exp(log_ratio));
  if (accept) memcpy(r, trial, sizeof trial);
  return accept;
}

uint64_t orc_mc_sweep(float *pos, uint32_t n_chains, uint32_t n,
                      uint32_t n_a, float k0, uint32_t n_ref,
                      const float *omega, uint32_t nx, uint32_t ny,
                      uint32_t nz, uint32_t move_kind, float step,
                      uint64_t seed, uint32_t sweep, uint32_t replica,
                      uint32_t chain_base, uint32_t set_order,
                      uint8_t *accept_flags, int n_threads) {
  uint64_t n_cells = (uint64_t)nx * ny * nz;
  uint64_t accepted = 0;
  (void)n_threads;
#pragma omp parallel for schedule(static) reduction(+ : accepted) num_threads(n_threads > 0 ? n_threads : 1)
  for (int64_t c = 0; c < (int64_t)n_chains; ++c) {
    float *chain = pos + (uint64_t)c * n * 3;
    uint32_t c_id = chain_base + (uint32_t)c;
    uint32_t first = 0;
    if (set_order == 0) {
      uint32_t w[4];
      orc_draw(seed, c_id, 0, ORC_PURPOSE_MOVE_A, sweep, replica, w);
      first = w[0] & 1u;
    }
    for (uint32_t pass = 0; pass < 2; ++pass) {
      uint32_t parity = pass == 0 ? first : 1u - first;
      for (uint32_t i = parity; i < n; i += 2) {
        int acc;
        if (move_kind == ORC_MOVE_SMC)
          acc = orc_move_smc(chain, c_id, i, n, n_a, (double)k0, omega,
                             n_cells, nx, ny, nz, n_ref, step, seed, sweep,
                             replica);
        else if (move_kind == ORC_MOVE_GIBBS)
          acc = orc_move_gibbs(chain, c_id, i, n, n_a, (double)k0, omega, n_cells, nx, ny, nz,
                               n_ref, seed, sweep, replica);
        else
          acc = orc_move_local(chain, c_id, i, n, n_a, (double)k0, omega,
                               n_cells, nx, ny, nz, n_ref, step, seed, sweep,
                               replica);
        accepted += (uint64_t)acc;
        if (accept_flags) accept_flags[(uint64_t)c * n + i] = (uint8_t)acc;
      }
    }
  }
  return accepted;
}

/* ------------------------------------------------------------------------- */
/* One MC sweep with local moves in the molecule-parallel order (Sec. 3.1.2,   */
/* scheme 1, "parallelization over distinct molecules"): every chain makes N  */
/* attempts one after another; attempt s picks its bead uniformly at random,  */
/* independently of the configuration, so a bead is attempted once per sweep */
/* on average and each attempt satisfies detailed balance.                    */
/*                                                                             */
/* Random numbers (this project's counter layout, Philox as above):           */
/*   bead of attempt s: word s mod 4 of the purpose-7 block with bead field   */
/*     floor(s/4), mapped to i = floor(word * N / 2^32);                      */
/*   the attempt itself: the purpose-6 block with bead field s, words 0-2     */
/*     the displacement, word 3 the acceptance, as for a LOCAL move.          */
/* accept_flags and picked (n_chains * N entries each, may be NULL) record    */
/* per attempt whether it was accepted and which bead it moved.              */
/* ------------------------------------------------------------------------- */
#define ORC_PURPOSE_MOLECULE 6u
#define ORC_PURPOSE_PICK 7u

uint32_t orc_pick_bead(uint32_t word, uint32_t n) {
  return (uint32_t)(((uint64_t)word * (uint64_t)n) >> 32);
}

uint64_t orc_mc_sweep_molecule(float *pos, uint32_t n_chains, uint32_t n,
                               uint32_t n_a, float k0, uint32_t n_ref,
                               const float *omega, uint32_t nx, uint32_t ny,
                               uint32_t nz, float step, uint64_t seed,
                               uint32_t sweep, uint32_t replica,
                               uint32_t chain_base, uint8_t *accept_flags,
                               uint32_t *picked, int n_threads) {
  uint64_t n_cells = (uint64_t)nx * ny * nz;
  uint64_t accepted = 0;
#pragma omp parallel for schedule(static) reduction(+ : accepted) num_threads(n_threads > 0 ? n_threads : 1)
  for (int64_t c = 0; c < (int64_t)n_chains; ++c) {
    float *chain = pos + (uint64_t)c * n * 3;
    uint32_t c_id = chain_base + (uint32_t)c;
    uint32_t sel[4] = {0, 0, 0, 0};
    for (uint32_t s = 0; s < n; ++s) {
      if (s % 4u == 0u)
        orc_draw(seed, c_id, s / 4u, ORC_PURPOSE_PICK, sweep, replica, sel);
      uint32_t i = orc_pick_bead(sel[s % 4u], n);
      uint32_t w[4];
      orc_draw(seed, c_id, s, ORC_PURPOSE_MOLECULE, sweep, replica, w);
      int acc = orc_local_attempt(chain, i, n, n_a, (double)k0, omega, n_cells,
                                  nx, ny, nz, n_ref, step, w);
      accepted += (uint64_t)acc;
      if (accept_flags) accept_flags[(uint64_t)c * n + s] = (uint8_t)acc;
      if (picked) picked[(uint64_t)c * n + s] = i;
    }
  }
  return accepted;
}

/* ------------------------------------------------------------------------- */
/* Initial configuration (the paper does not prescribe one): every chain is a */
/* Gaussian random walk -- the ideal chain of the harmonic bond model, bond   */
/* components i.i.d. N(0, 1/k0), so that b0^2 = 3/k0 (Sec. 2.1, after Eq. (9)) */
/* -- started from an origin uniform in the box.                               */
/*                                                                             */
/* origin_mode 0: origin i.i.d. uniform in the box, r0_d = u_d * n_d.          */
/* origin_mode 1: stratified uniform -- chain g of G falls in the cell of rank */
/*   k = floor(n_cells (g + u_3) / G) along the bricked cell order below, at a */
/*   uniform point of that cell; neighbouring chain numbers are then           */
/*   neighbours in space.                                                      */
/* Bricked order: bricks of 8 cells per side (the last brick along a direction */
/* takes the remainder), bricks row-major in (z, y, x), cells row-major in     */
/* (z, y, x) inside a brick.                                                   */
/* Draws: block (g, j | 4 << 16, 0xFFFFFFFF, replica) for bead j; bead 0 gives  */
/* the origin, bead j >= 1 the bond j via Box-Muller (words 0,1 -> x,y;        */
/* words 2,3 -> z from the cosine branch).                                     */
/* ------------------------------------------------------------------------- */
static void orc_brick_cell(uint64_t k, uint32_t nx, uint32_t ny, uint32_t nz,
                           uint64_t out[3]) {
  const uint64_t B = 8;
  uint64_t nbx = nx / B ? nx / B : 1, nby = ny / B ? ny / B : 1,
           nbz = nz / B ? nz / B : 1;
#define ORC_W(b, nb, n) ((b) + 1 < (nb) ? B : (n) - B * ((nb) - 1))
  uint64_t slab = B * (uint64_t)nx * ny;
  uint64_t bz = k / slab;
  if (bz > nbz - 1) bz = nbz - 1;
  k -= bz * slab;
  uint64_t wz = ORC_W(bz, nbz, nz);
  uint64_t row = wz * B * nx;
  uint64_t by = k / row;
  if (by > nby - 1) by = nby - 1;
  k -= by * row;
  uint64_t wy = ORC_W(by, nby, ny);
  uint64_t brick = wz * wy * B;
  uint64_t bx = k / brick;
  if (bx > nbx - 1) bx = nbx - 1;
  k -= bx * brick;
  uint64_t wx = ORC_W(bx, nbx, nx);
#undef ORC_W
  uint64_t z = k / (wy * wx);
  uint64_t rem = k % (wy * wx);
  out[0] = bx * B + rem % wx;
  out[1] = by * B + rem / wx;
  out[2] = bz * B + z;
}

void orc_brick_cell_batch(uint64_t n, const uint64_t *k, uint32_t nx,
                          uint32_t ny, uint32_t nz, uint64_t *out) {
  for (uint64_t i = 0; i < n; ++i) orc_brick_cell(k[i], nx, ny, nz, out + 3 * i);
}

void orc_init_chains(float *pos, uint32_t n_chains, uint32_t n,
                     float bond_sigma, uint32_t nx, uint32_t ny, uint32_t nz,
                     uint64_t seed, uint32_t replica, uint32_t chain_base,
                     uint32_t total_chains, uint32_t origin_mode) {
  uint64_t n_cells = (uint64_t)nx * ny * nz;
  for (uint32_t c = 0; c < n_chains; ++c) {
    uint32_t g = chain_base + c;
    float *chain = pos + (uint64_t)c * n * 3;
    uint32_t w[4];
    orc_draw(seed, g, 0, ORC_PURPOSE_INIT, ORC_SWEEP_INIT, replica, w);
    if (origin_mode == 1) {
      /* k = floor(n_cells * (g + (2m+1)/2^24) / G), exact in 128-bit ints */
      unsigned __int128 num =
          (unsigned __int128)n_cells *
          (((unsigned __int128)g << 24) + 2u * (w[3] >> 9) + 1u);
      unsigned __int128 den = (unsigned __int128)total_chains << 24;
      uint64_t k = (uint64_t)(num / den);
      uint64_t cell[3];
      orc_brick_cell(k, nx, ny, nz, cell);
      for (int d = 0; d < 3; ++d) chain[d] = (float)cell[d] + orc_u01(w[d]);
    } else {
      float dims[3] = {(float)nx, (float)ny, (float)nz};
      for (int d = 0; d < 3; ++d) chain[d] = orc_u01(w[d]) * dims[d];
    }
    for (uint32_t j = 1; j < n; ++j) {
      orc_draw(seed, g, j, ORC_PURPOSE_INIT, ORC_SWEEP_INIT, replica, w);
      double xi[4];
      orc_box_muller(w[0], w[1], &xi[0], &xi[1]);
      orc_box_muller(w[2], w[3], &xi[2], &xi[3]);
      for (int d = 0; d < 3; ++d)
        chain[3 * j + d] =
            (float)((double)chain[3 * (j - 1) + d] + (double)bond_sigma * xi[d]);
    }
  }
}

/* ------------------------------------------------------------------------- */
/* Chain observables (Sec. 5.5 uses <Re^2>; Rg and the bond length follow the  */
/* same ideal-chain definitions of Sec. 2.1): per chain, with unwrapped         */
/* positions,                                                                  */
/*   Re^2 = |r_{N-1} - r_0|^2,  Rg^2 = (1/N) sum_i |r_i - r_cm|^2,              */
/*   b2   = sum over bonds |r_{i+1} - r_i|^2,   E_b = (k0/2) b2.               */
/* Outputs are per-chain FP64 arrays (any may be NULL).                         */
/* ------------------------------------------------------------------------- */
void orc_chain_observables(const float *pos, uint32_t n_chains, uint32_t n,
                           double *re2, double *rg2, double *b2) {
  for (uint32_t c = 0; c < n_chains; ++c) {
    const float *ch = pos + (uint64_t)c * n * 3;
    double cm[3] = {0, 0, 0};
    for (uint32_t i = 0; i < n; ++i)
      for (int d = 0; d < 3; ++d) cm[d] += ch[3 * i + d];
    for (int d = 0; d < 3; ++d) cm[d] /= n;
    double e = 0, g = 0, b = 0;
    for (int d = 0; d < 3; ++d) {
      double x = (double)ch[3 * (n - 1) + d] - (double)ch[d];
      e += x * x;
    }
    for (uint32_t i = 0; i < n; ++i)
      for (int d = 0; d < 3; ++d) {
        double x = (double)ch[3 * i + d] - cm[d];
        g += x * x;
      }
    for (uint32_t i = 0; i + 1 < n; ++i)
      for (int d = 0; d < 3; ++d) {
        double x = (double)ch[3 * (i + 1) + d] - (double)ch[3 * i + d];
        b += x * x;
      }
    if (re2) re2[c] = e;
    if (rg2) rg2[c] = g / n;
    if (b2) b2[c] = b;
  }
}

/* Field energy of the beads in their cells, the right-hand side of Eq. (13)
 * divided by N: sum_j omega_type(j)(c_j) / N. */
double orc_field_energy(const float *pos, uint32_t n_chains, uint32_t n,
                        uint32_t n_a, const float *omega, uint32_t nx,
                        uint32_t ny, uint32_t nz, uint32_t n_ref) {
  uint64_t n_cells = (uint64_t)nx * ny * nz;
  double e = 0.0;
  for (uint32_t c = 0; c < n_chains; ++c)
    for (uint32_t i = 0; i < n; ++i) {
      const float *r = pos + ((uint64_t)c * n + i) * 3;
      e += (double)omega[(uint64_t)orc_type(i, n_a) * n_cells +
                         orc_cell(r, nx, ny, nz)];
    }
  return e / (double)n_ref;
}

/* ========================================================================= */
/* Learned proposal (not part of the paper: an addition to its local and     */
/* smart-MC moves, Sec. 2.2, that keeps the sampled distribution exact by     */
/* Metropolis-Hastings with the proposal ratio).                              */
/*                                                                            */
/* Features of bead i at position r (60): the per-chain fields of the bead's  */
/* own type at the 27 cells around its cell, then those of the other type    */
/* (cells in (dz, dy, dx) order, each -1..1, periodic), then the bond vectors */
/* r_{i-1} - r and r_{i+1} - r (zero where the neighbour does not exist).     */
/* Standardised per feature: (f - shift) * scale.                             */
/* Network: h1 = relu(W1 x + b1), h2 = relu(W2 h1 + b2), z = W3 h2 + b3       */
/* (60 -> 64 -> 64 -> 6).  Head: mu_d = m tanh(z_d / m),                      */
/* log sigma_d = lo + (hi - lo) sigmoid(z_{3+d}).                             */
/* Proposal: r' = r + mu(r) + sigma(r) xi, xi ~ N(0,1)^3.                     */
/* BF16 mode rounds the standardised input, every weight and each hidden      */
/* activation to bfloat16 (round to nearest even) at the points the device    */
/* does, accumulating in FP64.                                                */
/* ========================================================================= */
#define ORC_NF 60
#define ORC_NH 64
#define ORC_NO 6
#define ORC_P_SHIFT 0
#define ORC_P_SCALE 60
#define ORC_P_W1 120
#define ORC_P_B1 3960
#define ORC_P_W2 4024
#define ORC_P_B2 8120
#define ORC_P_W3 8184
#define ORC_P_B3 8568
#define ORC_P_SIZE 8576
#define ORC_MOVE_MIXED 2u
#define ORC_PURPOSE_MIX 1u

uint32_t orc_param_layout(uint32_t which) {
  const uint32_t v[] = {ORC_P_SHIFT, ORC_P_SCALE, ORC_P_W1, ORC_P_B1, ORC_P_W2,
                        ORC_P_B2, ORC_P_W3, ORC_P_B3, ORC_P_SIZE};
  return which < 9 ? v[which] : 0u;
}

/* float -> bfloat16 -> float, round to nearest even */
float orc_bf16(float x) {
  uint32_t u;
  memcpy(&u, &x, 4);
  if ((u & 0x7FFFFFFFu) > 0x7F800000u) return x; /* NaN unchanged */
  u += 0x7FFFu + ((u >> 16) & 1u);
  u &= 0xFFFF0000u;
  memcpy(&x, &u, 4);
  return x;
}

static double orc_relu(double a) { return a > 0.0 ? a : 0.0; }
static double orc_drelu(double a) { return a > 0.0 ? 1.0 : 0.0; }

/* Test hook: with orc_acc_f32 set, the BF16 forward sums its terms in FP32
 * in index order instead of FP64 -- another order of FP32 additions that a
 * device may take, for testing the rounding envelope below.  Off by default. */
static int orc_acc_f32 = 0;
void orc_set_acc_f32(int on) { orc_acc_f32 = on; }
static double orc_acc(double acc, double t, int bf16) {
  return (bf16 && orc_acc_f32) ? (double)((float)acc + (float)t) : acc + t;
}

/* The network as the learned move evaluates it: the input standardisation
 * folded into the first layer.  W1'[m][k] = W1[m][k] scale[k] (one FP32
 * product), b1'[m] = b1[m] - sum_k W1'[m][k] shift[k] in FP32 with k
 * ascending (each product rounded before it is subtracted), shift 0 and
 * scale 1; the other parameters unchanged.  In exact arithmetic the same
 * function, W1' f + b1' = W1 ((f - shift) scale) + b1; in BF16 mode the
 * raw features and W1' are what gets rounded. */
void orc_fold_params(const float *p, float *q) {
  memcpy(q, p, ORC_P_SIZE * sizeof(float));
  for (int m = 0; m < ORC_NH; ++m) {
    float b = p[ORC_P_B1 + m];
    for (int k = 0; k < ORC_NF; ++k) {
      const float w = p[ORC_P_W1 + m * ORC_NF + k] * p[ORC_P_SCALE + k];
      const float t = w * p[ORC_P_SHIFT + k];
      q[ORC_P_W1 + m * ORC_NF + k] = w;
      b = b - t;
    }
    q[ORC_P_B1 + m] = b;
  }
  for (int k = 0; k < ORC_NF; ++k) {
    q[ORC_P_SHIFT + k] = 0.0f;
    q[ORC_P_SCALE + k] = 1.0f;
  }
}

/* cache layout: x[60] a1[64] h1[64] a2[64] h2[64] */
void orc_mlp_forward(const float *p, const double *f, int bf16, double *z,
                     double *cache) {
  double x[ORC_NF], a1[ORC_NH], h1[ORC_NH], a2[ORC_NH], h2[ORC_NH];
  for (int k = 0; k < ORC_NF; ++k) {
    float s = ((float)f[k] - p[ORC_P_SHIFT + k]) * p[ORC_P_SCALE + k];
    x[k] = bf16 ? (double)orc_bf16(s) : (f[k] - p[ORC_P_SHIFT + k]) * p[ORC_P_SCALE + k];
  }
#define ORC_W(off, idx) (bf16 ? (double)orc_bf16(p[(off) + (idx)]) : (double)p[(off) + (idx)])
  for (int m = 0; m < ORC_NH; ++m) {
    double acc = 0.0;
    for (int k = 0; k < ORC_NF; ++k) acc = orc_acc(acc, ORC_W(ORC_P_W1, m * ORC_NF + k) * x[k], bf16);
    a1[m] = orc_acc(acc, p[ORC_P_B1 + m], bf16);
    h1[m] = orc_relu(a1[m]);
    if (bf16) h1[m] = orc_bf16((float)h1[m]);
  }
  for (int m = 0; m < ORC_NH; ++m) {
    double acc = 0.0;
    for (int k = 0; k < ORC_NH; ++k) acc = orc_acc(acc, ORC_W(ORC_P_W2, m * ORC_NH + k) * h1[k], bf16);
    a2[m] = orc_acc(acc, p[ORC_P_B2 + m], bf16);
    h2[m] = orc_relu(a2[m]);
    if (bf16) h2[m] = orc_bf16((float)h2[m]);
  }
  for (int o = 0; o < ORC_NO; ++o) {
    double acc = 0.0;
    for (int k = 0; k < ORC_NH; ++k) acc = orc_acc(acc, ORC_W(ORC_P_W3, o * ORC_NH + k) * h2[k], bf16);
    z[o] = orc_acc(acc, p[ORC_P_B3 + o], bf16);
  }
#undef ORC_W
  if (cache) {
    memcpy(cache, x, sizeof x);
    memcpy(cache + ORC_NF, a1, sizeof a1);
    memcpy(cache + ORC_NF + ORC_NH, h1, sizeof h1);
    memcpy(cache + ORC_NF + 2 * ORC_NH, a2, sizeof a2);
    memcpy(cache + ORC_NF + 3 * ORC_NH, h2, sizeof h2);
  }
}

/* Back-propagation of dL/dz through the network (plain chain rule), adding
 * dL/dparam into grad (ORC_P_SIZE doubles; standardisation constants get no
 * gradient).  Uses the same (possibly bf16-rounded) weights and activations as
 * the forward pass that filled `cache`. */
void orc_mlp_backward(const float *p, const double *cache, const double *dz,
                      int bf16, double *grad) {
  const double *x = cache, *a1 = cache + ORC_NF, *h1 = cache + ORC_NF + ORC_NH,
               *a2 = cache + ORC_NF + 2 * ORC_NH, *h2 = cache + ORC_NF + 3 * ORC_NH;
#define ORC_W(off, idx) (bf16 ? (double)orc_bf16(p[(off) + (idx)]) : (double)p[(off) + (idx)])
  double d2[ORC_NH], d1[ORC_NH];
  for (int o = 0; o < ORC_NO; ++o) {
    grad[ORC_P_B3 + o] += dz[o];
    for (int k = 0; k < ORC_NH; ++k) grad[ORC_P_W3 + o * ORC_NH + k] += dz[o] * h2[k];
  }
  for (int k = 0; k < ORC_NH; ++k) {
    double s = 0.0;
    for (int o = 0; o < ORC_NO; ++o) s += ORC_W(ORC_P_W3, o * ORC_NH + k) * dz[o];
    d2[k] = s * orc_drelu(a2[k]);
  }
  for (int m = 0; m < ORC_NH; ++m) {
    grad[ORC_P_B2 + m] += d2[m];
    for (int k = 0; k < ORC_NH; ++k) grad[ORC_P_W2 + m * ORC_NH + k] += d2[m] * h1[k];
  }
  for (int k = 0; k < ORC_NH; ++k) {
    double s = 0.0;
    for (int m = 0; m < ORC_NH; ++m) s += ORC_W(ORC_P_W2, m * ORC_NH + k) * d2[m];
    d1[k] = s * orc_drelu(a1[k]);
  }
  for (int m = 0; m < ORC_NH; ++m) {
    grad[ORC_P_B1 + m] += d1[m];
    for (int k = 0; k < ORC_NF; ++k) grad[ORC_P_W1 + m * ORC_NF + k] += d1[m] * x[k];
  }
#undef ORC_W
}

/* Gaussian head: mu, sigma, log sigma from z. */
static void orc_head(const double *z, double m_max, double lo, double hi,
                     double *mu, double *sig, double *lsig) {
  for (int d = 0; d < 3; ++d) {
    mu[d] = m_max * tanh(z[d] / m_max);
    double sg = 1.0 / (1.0 + exp(-z[3 + d]));
    lsig[d] = lo + (hi - lo) * sg;
    sig[d] = exp(lsig[d]);
  }
}

/* Negative log-likelihood (without the constant 3/2 log 2 pi) of a
 * displacement dr under the head's Gaussian, and dL/dz. */
double orc_nll(const double *z, const double *dr, double m_max, double lo,
               double hi, double *dz) {
  double loss = 0.0;
  for (int d = 0; d < 3; ++d) {
    double mu = m_max * tanh(z[d] / m_max);
    double sg = 1.0 / (1.0 + exp(-z[3 + d]));
    double ls = lo + (hi - lo) * sg;
    double inv_var = exp(-2.0 * ls);
    double e = dr[d] - mu;
    loss += 0.5 * e * e * inv_var + ls;
    double dmu = -e * inv_var;
    double dls = 1.0 - e * e * inv_var;
    dz[d] = dmu * (1.0 - (mu / m_max) * (mu / m_max));
    dz[3 + d] = dls * (hi - lo) * sg * (1.0 - sg);
  }
  return loss;
}

/* Mean NLL over a batch and its gradient (grad: ORC_P_SIZE doubles,
 * overwritten).  features [n][60], targets [n][3]. */
double orc_nll_batch(const float *p, uint64_t n, const double *features,
                     const double *targets, double m_max, double lo, double hi,
                     int bf16, double *grad, double *z_out) {
  double cache[ORC_NF + 4 * ORC_NH], z[ORC_NO], dz[ORC_NO];
  memset(grad, 0, ORC_P_SIZE * sizeof(double));
  double total = 0.0;
  for (uint64_t s = 0; s < n; ++s) {
    orc_mlp_forward(p, features + s * ORC_NF, bf16, z, cache);
    if (z_out) memcpy(z_out + s * ORC_NO, z, sizeof z);
    total += orc_nll(z, targets + 3 * s, m_max, lo, hi, dz);
    for (int o = 0; o < ORC_NO; ++o) dz[o] /= (double)n;
    orc_mlp_backward(p, cache, dz, bf16, grad);
  }
  return total / (double)n;
}

/* ------------------------------------------------------------------------- */
/* Rounding envelope of the BF16 network -- a test instrument for the parity */
/* of the device's learned proposal and training; the sampler above does    */
/* not use it.  The device evaluates the network with BF16 operands whose    */
/* products it sums in FP32 on the matrix cores, in an order of the          */
/* hardware's, and rounds the hidden activations (and, in training, the      */
/* back-propagated errors) to BF16.  Where the exact value of such a sum     */
/* lies closer to a BF16 rounding boundary (or, under the ReLU, to zero)     */
/* than an FP32 sum of its terms can err, the device may round it the other  */
/* way.  The functions below take one sample through the network with the    */
/* device's rounding points, list every such ambiguous rounding, and can     */
/* re-evaluate the sample with one of them taken the other way, so that a    */
/* test can bound the device's result by the oracle's plus the effect of     */
/* each ambiguous rounding (to first order: one at a time).                  */
/*                                                                           */
/* Error of an FP32 sum of K exact products plus a bias, each addition       */
/* rounded faithfully: at most (K + 2) 2^-23 S, S the sum of the magnitudes  */
/* of the terms.  The matrix-core tiles sum K = 64 (hidden layers, output,   */
/* error of the first layer) or K = 32 (error of the second layer) terms.    */
/* orc_env_scale multiplies every such window (1: the bound as stated).      */
/* ------------------------------------------------------------------------- */
static double orc_env_scale = 1.0;
void orc_set_envelope(double scale) { orc_env_scale = scale; }

static double orc_env_window(int k, double s) { return orc_env_scale * (k + 2) * 0x1p-23 * s; }

static float orc_bf16_bits(uint32_t u) {
  float f;
  memcpy(&f, &u, 4);
  return f;
}

/* The two BF16 values next to q (a BF16 value) in the directions of -inf and +inf. */
static void orc_bf16_neighbours(float q, double *dn, double *up) {
  uint32_t u;
  memcpy(&u, &q, 4);
  if ((u & 0x7FFFFFFFu) == 0u) {           /* +-0 */
    *up = (double)orc_bf16_bits(0x00010000u);
    *dn = -*up;
  } else if (u & 0x80000000u) {            /* negative: magnitude up = toward -inf */
    *dn = (double)orc_bf16_bits(u + 0x10000u);
    *up = (double)orc_bf16_bits(u - 0x10000u);
  } else {
    *up = (double)orc_bf16_bits(u + 0x10000u);
    *dn = (double)orc_bf16_bits(u - 0x10000u);
  }
}

/* Distance of v from the nearest point where BF16 round-to-nearest changes
 * its result (a midpoint between two neighbouring BF16 values), and the BF16
 * value on the other side of that point. */
double orc_bf16_boundary(double v, double *other) {
  float q = orc_bf16((float)v);
  double dn, up;
  orc_bf16_neighbours(q, &dn, &up);
  double m_up = 0.5 * ((double)q + up), m_dn = 0.5 * ((double)q + dn);
  double d_up = fabs(v - m_up), d_dn = fabs(v - m_dn);
  if (other) *other = d_up < d_dn ? up : dn;
  return d_up < d_dn ? d_up : d_dn;
}

/* Stages of the rounding points of one sample. */
enum { ORC_ST_NONE = 0, ORC_ST_X = 1, ORC_ST_H1 = 2, ORC_ST_H2 = 3, ORC_ST_R1 = 4,
       ORC_ST_R2 = 5, ORC_ST_DZ = 6, ORC_ST_D2 = 7, ORC_ST_D1 = 8 };
/* X: a standardised input; H1, H2: a hidden activation's BF16 rounding;
 * R1, R2: a hidden unit's ReLU (pre-activation within the window of zero);
 * DZ, D2, D1: the BF16 rounding of a back-propagated error. */

#define ORC_AMB_MAX 1024
typedef struct {
  int stage[ORC_AMB_MAX], unit[ORC_AMB_MAX];
  int n;
} orc_amb_list;

static void orc_amb_add(orc_amb_list *l, int stage, int unit) {
  if (l && l->n < ORC_AMB_MAX) {
    l->stage[l->n] = stage;
    l->unit[l->n] = unit;
    l->n++;
  }
}

/* One sample as the device evaluates it.  x0: the standardised inputs [60]
 * in FP32 (before their BF16 rounding), xwin: the window of each input
 * (0: known exactly).  Override (ov_stage, ov_unit) takes that rounding the
 * other way.  Writes z [6] and its windows zwin [6]; with `amb`, lists the
 * ambiguous roundings.  With `tgt` (a training target, 3) and `grad`, also
 * the training pass: adds the unnormalised loss gradient into grad[8576] and
 * the bound of the FP32 (unrounded) bias terms into bias_err[8576] and the
 * magnitudes of the gradient terms into gabs[8576] (both may be NULL). */
static void orc_dev_sample(const float *p, const double *x0, const double *xwin,
                           int ov_stage, int ov_unit, double *z, double *zwin,
                           orc_amb_list *amb, const double *tgt, double m_max, double lo,
                           double hi, double *grad, double *bias_err, double *gabs) {
  double x[ORC_NF], a1[ORC_NH], h1[ORC_NH], a2[ORC_NH], h2[ORC_NH];
  int r1[ORC_NH], r2[ORC_NH];
#define ORC_WB(off, idx) ((double)orc_bf16(p[(off) + (idx)]))
  for (int k = 0; k < ORC_NF; ++k) {
    double other;
    double dist = orc_bf16_boundary(x0[k], &other);
    x[k] = (double)orc_bf16((float)x0[k]);
    if (ov_stage == ORC_ST_X && ov_unit == k) x[k] = other;
    else if (xwin && xwin[k] > 0.0 && dist <= xwin[k]) orc_amb_add(amb, ORC_ST_X, k);
  }
  /* hidden layers: pre-activation a, its window, ReLU, BF16 rounding */
  for (int layer = 0; layer < 2; ++layer) {
    const double *in = layer == 0 ? x : h1;
    double *a = layer == 0 ? a1 : a2, *h = layer == 0 ? h1 : h2;
    int *rl = layer == 0 ? r1 : r2;
    int n_in = layer == 0 ? ORC_NF : ORC_NH;
    int w_off = layer == 0 ? ORC_P_W1 : ORC_P_W2, b_off = layer == 0 ? ORC_P_B1 : ORC_P_B2;
    int st_h = layer == 0 ? ORC_ST_H1 : ORC_ST_H2, st_r = layer == 0 ? ORC_ST_R1 : ORC_ST_R2;
    for (int m = 0; m < ORC_NH; ++m) {
      double acc = 0.0, s = fabs((double)p[b_off + m]);
      for (int k = 0; k < n_in; ++k) {
        double t = ORC_WB(w_off, m * n_in + k) * in[k];
        acc += t;
        s += fabs(t);
      }
      a[m] = acc + p[b_off + m];
      double win = orc_env_window(64, s);
      rl[m] = a[m] > 0.0;
      if (fabs(a[m]) <= win) {
        if (ov_stage == st_r && ov_unit == m) {
          rl[m] = !rl[m];
          h[m] = rl[m] ? (double)orc_bf16((float)win) : 0.0;
          continue;
        }
        orc_amb_add(amb, st_r, m);
        h[m] = rl[m] ? (double)orc_bf16((float)a[m]) : 0.0;
        continue;
      }
      if (!rl[m]) { h[m] = 0.0; continue; }
      double other;
      double dist = orc_bf16_boundary(a[m], &other);
      h[m] = (double)orc_bf16((float)a[m]);
      if (ov_stage == st_h && ov_unit == m) h[m] = other;
      else if (dist <= win) orc_amb_add(amb, st_h, m);
    }
  }
  for (int o = 0; o < ORC_NO; ++o) {
    double acc = 0.0, s = fabs((double)p[ORC_P_B3 + o]);
    for (int k = 0; k < ORC_NH; ++k) {
      double t = ORC_WB(ORC_P_W3, o * ORC_NH + k) * h2[k];
      acc += t;
      s += fabs(t);
    }
    z[o] = acc + p[ORC_P_B3 + o];
    if (zwin) zwin[o] = orc_env_window(64, s);
  }
  if (!grad) return;

  /* training: dL/dz in FP32 from z, rounded to BF16 for the tiles */
  double dz[ORC_NO], dzb[ORC_NO], dzw[ORC_NO];
  double zwl[ORC_NO];
  for (int o = 0; o < ORC_NO; ++o) {
    double acc_s = fabs((double)p[ORC_P_B3 + o]);
    for (int k = 0; k < ORC_NH; ++k) acc_s += fabs(ORC_WB(ORC_P_W3, o * ORC_NH + k) * h2[k]);
    zwl[o] = orc_env_window(64, acc_s);
  }
  /* |term| of every gradient entry, for the bound of the FP32 sums over samples */
#define ORC_GABS(idx, v) do { if (gabs) gabs[idx] += fabs(v); } while (0)
  orc_nll(z, tgt, m_max, lo, hi, dz);
  for (int d = 0; d < 3; ++d) {
    /* window of the device's FP32 dz: z within its window (four corners), and
     * 2^-18 of the magnitudes for the FP32 head (transcendentals, cancellation) */
    double zc[ORC_NO], dzc[ORC_NO], dev_mu = 0.0, dev_s = 0.0;
    for (int corner = 0; corner < 4; ++corner) {
      memcpy(zc, z, sizeof zc);
      zc[d] += (corner & 1) ? zwl[d] : -zwl[d];
      zc[3 + d] += (corner & 2) ? zwl[3 + d] : -zwl[3 + d];
      orc_nll(zc, tgt, m_max, lo, hi, dzc);
      if (fabs(dzc[d] - dz[d]) > dev_mu) dev_mu = fabs(dzc[d] - dz[d]);
      if (fabs(dzc[3 + d] - dz[3 + d]) > dev_s) dev_s = fabs(dzc[3 + d] - dz[3 + d]);
    }
    double mu = m_max * tanh(z[d] / m_max);
    double sg = 1.0 / (1.0 + exp(-z[3 + d]));
    double inv_var = exp(-2.0 * (lo + (hi - lo) * sg));
    double e = tgt[d] - mu;
    double mag_mu = (fabs(tgt[d]) + fabs(mu)) * inv_var * 2.0;
    double mag_s = (1.0 + e * e * inv_var) * (hi - lo) * sg * (1.0 - sg) * 2.0;
    dzw[d] = dev_mu + orc_env_scale * 0x1p-18 * mag_mu;
    dzw[3 + d] = dev_s + orc_env_scale * 0x1p-18 * mag_s;
  }
  for (int o = 0; o < ORC_NO; ++o) {
    double other;
    double dist = orc_bf16_boundary(dz[o], &other);
    dzb[o] = (double)orc_bf16((float)dz[o]);
    if (ov_stage == ORC_ST_DZ && ov_unit == o) dzb[o] = other;
    else if (dist <= dzw[o]) orc_amb_add(amb, ORC_ST_DZ, o);
    grad[ORC_P_B3 + o] += dz[o];
    ORC_GABS(ORC_P_B3 + o, dz[o]);
    if (bias_err) bias_err[ORC_P_B3 + o] += dzw[o];
    for (int k = 0; k < ORC_NH; ++k) {
      grad[ORC_P_W3 + o * ORC_NH + k] += dzb[o] * h2[k];
      ORC_GABS(ORC_P_W3 + o * ORC_NH + k, dzb[o] * h2[k]);
    }
  }
  /* error of the second hidden layer: K = 32 tile (6 used) */
  double d2b[ORC_NH];
  for (int k = 0; k < ORC_NH; ++k) {
    double acc = 0.0, s = 0.0;
    for (int o = 0; o < ORC_NO; ++o) {
      double t = ORC_WB(ORC_P_W3, o * ORC_NH + k) * dzb[o];
      acc += t;
      s += fabs(t);
    }
    double d = r2[k] ? acc : 0.0;
    double win = orc_env_window(32, s);
    grad[ORC_P_B2 + k] += d;
    ORC_GABS(ORC_P_B2 + k, d);
    if (bias_err && r2[k]) bias_err[ORC_P_B2 + k] += win;
    double other;
    double dist = orc_bf16_boundary(d, &other);
    d2b[k] = (double)orc_bf16((float)d);
    if (ov_stage == ORC_ST_D2 && ov_unit == k) d2b[k] = other;
    else if (r2[k] && dist <= win) orc_amb_add(amb, ORC_ST_D2, k);
    for (int j = 0; j < ORC_NH; ++j) {
      grad[ORC_P_W2 + k * ORC_NH + j] += d2b[k] * h1[j];
      ORC_GABS(ORC_P_W2 + k * ORC_NH + j, d2b[k] * h1[j]);
    }
  }
  /* error of the first hidden layer: K = 64 */
  for (int k = 0; k < ORC_NH; ++k) {
    double acc = 0.0, s = 0.0;
    for (int m = 0; m < ORC_NH; ++m) {
      double t = ORC_WB(ORC_P_W2, m * ORC_NH + k) * d2b[m];
      acc += t;
      s += fabs(t);
    }
    double d = r1[k] ? acc : 0.0;
    double win = orc_env_window(64, s);
    grad[ORC_P_B1 + k] += d;
    ORC_GABS(ORC_P_B1 + k, d);
    if (bias_err && r1[k]) bias_err[ORC_P_B1 + k] += win;
    double other;
    double dist = orc_bf16_boundary(d, &other);
    double d1b = (double)orc_bf16((float)d);
    if (ov_stage == ORC_ST_D1 && ov_unit == k) d1b = other;
    else if (r1[k] && dist <= win) orc_amb_add(amb, ORC_ST_D1, k);
    for (int j = 0; j < ORC_NF; ++j) {
      grad[ORC_P_W1 + k * ORC_NF + j] += d1b * x[j];
      ORC_GABS(ORC_P_W1 + k * ORC_NF + j, d1b * x[j]);
    }
  }
#undef ORC_GABS
#undef ORC_WB
}

/* Network outputs as the device computes them, with their envelope: z [n][6]
 * (the BF16 forward with FP64 sums) and bound [n][6], the window of each
 * output's own FP32 sum plus, for every ambiguous rounding of the sample, the
 * change of the output when it is taken the other way.  Returns the number of
 * ambiguous roundings. */
uint64_t orc_mlp_forward_envelope(const float *p_in, uint64_t n, const double *features,
                                  double *z, double *bound) {
  float p[ORC_P_SIZE];   /* the learned move's network: standardisation folded */
  orc_fold_params(p_in, p);
  orc_amb_list *amb = malloc(sizeof(orc_amb_list));
  uint64_t na = 0;
  for (uint64_t s = 0; s < n; ++s) {
    double x0[ORC_NF], zw[ORC_NO], za[ORC_NO], zaw[ORC_NO];
    double *zs = z + s * ORC_NO, *bs = bound + s * ORC_NO;
    for (int k = 0; k < ORC_NF; ++k)
      x0[k] = (double)(((float)features[s * ORC_NF + k] - p[ORC_P_SHIFT + k]) * p[ORC_P_SCALE + k]);
    amb->n = 0;
    orc_dev_sample(p, x0, NULL, ORC_ST_NONE, 0, zs, zw, amb, NULL, 0, 0, 0, NULL, NULL, NULL);
    for (int o = 0; o < ORC_NO; ++o) bs[o] = zw[o];
    for (int a = 0; a < amb->n; ++a) {
      orc_dev_sample(p, x0, NULL, amb->stage[a], amb->unit[a], za, zaw, NULL, NULL, 0, 0, 0, NULL,
                     NULL, NULL);
      for (int o = 0; o < ORC_NO; ++o) bs[o] += fabs(za[o] - zs[o]);
    }
    na += (uint64_t)amb->n;
  }
  free(amb);
  return na;
}

/* Training gradient as the device computes it, with its envelope.  Returns
 * the mean loss.  grad [8576]: the mean gradient with the device's rounding
 * points (BF16 inputs, weights, activations and back-propagated errors; FP64
 * sums).  bound [8576]: per parameter, the sum over samples of the change of
 * that sample's term when one ambiguous rounding is taken the other way (one
 * at a time), plus the windows of the FP32 bias terms, plus
 * (64 + n) 2^-23 times the sum of the magnitudes of the terms (the FP32 sums
 * over samples), divided by n.  n_amb: ambiguous roundings found; n_flagged:
 * samples with at least one. */
double orc_nll_batch_envelope(const float *p, uint64_t n, const double *features,
                              const double *targets, double m_max, double lo, double hi,
                              double *grad, double *bound, uint64_t *n_amb,
                              uint64_t *n_flagged) {
  double *g_main = calloc(ORC_P_SIZE, sizeof(double));
  double *g_alt = calloc(ORC_P_SIZE, sizeof(double));
  double *gabs = calloc(ORC_P_SIZE, sizeof(double));
  orc_amb_list *amb = malloc(sizeof(orc_amb_list));
  memset(grad, 0, ORC_P_SIZE * sizeof(double));
  memset(bound, 0, ORC_P_SIZE * sizeof(double));
  double total = 0.0, z[ORC_NO], zw[ORC_NO], dz[ORC_NO];
  uint64_t na = 0, nf = 0;
  for (uint64_t s = 0; s < n; ++s) {
    const double *f = features + s * ORC_NF;
    const double *t = targets + 3 * s;
    double x0[ORC_NF];
    for (int k = 0; k < ORC_NF; ++k)
      x0[k] = (double)(((float)f[k] - p[ORC_P_SHIFT + k]) * p[ORC_P_SCALE + k]);
    memset(g_main, 0, ORC_P_SIZE * sizeof(double));
    amb->n = 0;
    orc_dev_sample(p, x0, NULL, ORC_ST_NONE, 0, z, zw, amb, t, m_max, lo, hi, g_main, bound,
                   gabs);
    total += orc_nll(z, t, m_max, lo, hi, dz);
    for (int j = 0; j < ORC_P_SIZE; ++j) grad[j] += g_main[j];
    na += (uint64_t)amb->n;
    nf += amb->n > 0;
    for (int a = 0; a < amb->n; ++a) {
      memset(g_alt, 0, ORC_P_SIZE * sizeof(double));
      orc_dev_sample(p, x0, NULL, amb->stage[a], amb->unit[a], z, zw, NULL, t, m_max, lo, hi,
                     g_alt, NULL, NULL);
      for (int j = 0; j < ORC_P_SIZE; ++j) bound[j] += fabs(g_alt[j] - g_main[j]);
    }
  }
  const double gamma = orc_env_scale * (64.0 + (double)n) * 0x1p-23;
  for (int j = 0; j < ORC_P_SIZE; ++j) {
    grad[j] /= (double)n;
    bound[j] = (bound[j] + gamma * gabs[j]) / (double)n + 0x1p-22 * fabs(grad[j]);
  }
  free(g_main);
  free(g_alt);
  free(gabs);
  free(amb);
  if (n_amb) *n_amb = na;
  if (n_flagged) *n_flagged = nf;
  return total / (double)n;
}

void orc_features(const float *chain, uint32_t i, uint32_t n, uint32_t n_a,
                  const float *omega, uint32_t nx, uint32_t ny, uint32_t nz,
                  const float *r, double *f) {
  uint64_t n_cells = (uint64_t)nx * ny * nz;
  uint32_t own = orc_type(i, n_a);
  const float *om_own = omega + (uint64_t)own * n_cells;
  const float *om_oth = omega + (uint64_t)(1u - own) * n_cells;
  int64_t c[3] = {orc_wrap((double)r[0], nx), orc_wrap((double)r[1], ny),
                  orc_wrap((double)r[2], nz)};
  int j = 0;
  for (int dz_ = -1; dz_ <= 1; ++dz_)
    for (int dy = -1; dy <= 1; ++dy)
      for (int dx = -1; dx <= 1; ++dx, ++j) {
        int64_t x = ((c[0] + dx) % nx + nx) % nx;
        int64_t y = ((c[1] + dy) % ny + ny) % ny;
        int64_t zz = ((c[2] + dz_) % nz + nz) % nz;
        uint64_t cell = ((uint64_t)zz * ny + (uint64_t)y) * nx + (uint64_t)x;
        f[j] = om_own[cell];
        f[27 + j] = om_oth[cell];
      }
  for (int d = 0; d < 3; ++d) {
    f[54 + d] = i > 0 ? (double)chain[3 * (i - 1) + d] - (double)r[d] : 0.0;
    f[57 + d] = i + 1 < n ? (double)chain[3 * (i + 1) + d] - (double)r[d] : 0.0;
  }
}

/* Features of bead `bead` of every chain of a species (for the training data
 * and the tests): out [n_chains][60]. */
void orc_features_batch(const float *pos, uint32_t n_chains, uint32_t n, uint32_t n_a,
                        const uint32_t *beads, const float *omega, uint32_t nx,
                        uint32_t ny, uint32_t nz, double *out) {
  for (uint32_t c = 0; c < n_chains; ++c) {
    const float *chain = pos + (uint64_t)c * n * 3;
    orc_features(chain, beads[c], n, n_a, omega, nx, ny, nz, chain + 3 * beads[c],
                 out + (uint64_t)c * ORC_NF);
  }
}

/* Log of the Metropolis-Hastings ratio of a learned move r -> trial, from the
 * network outputs z at r and zn at trial (as in orc_move_learned); with
 * `mag`, also the sum of the magnitudes of its terms. */
static double orc_learned_log_ratio(const float *chain, uint32_t i, uint32_t n, uint32_t n_a,
                                    double k0, const float *omega, uint64_t n_cells,
                                    uint32_t nx, uint32_t ny, uint32_t nz, uint32_t n_ref,
                                    const float *r, const float *trial, const double *z,
                                    const double *zn, double m_max, double lo, double hi,
                                    double *mag) {
  double mu[3], sig[3], lsig[3], mun[3], sign[3], lsign[3];
  orc_head(z, m_max, lo, hi, mu, sig, lsig);
  orc_head(zn, m_max, lo, hi, mun, sign, lsign);
  double log_fwd = 0.0, log_rev = 0.0, m = 0.0;
  for (int d = 0; d < 3; ++d) {
    double ef = (double)trial[d] - (double)r[d] - mu[d];
    double er = (double)r[d] - (double)trial[d] - mun[d];
    log_fwd -= ef * ef / (2.0 * sig[d] * sig[d]) + lsig[d];
    log_rev -= er * er / (2.0 * sign[d] * sign[d]) + lsign[d];
    m += ef * ef / (2.0 * sig[d] * sig[d]) + fabs(lsig[d]) + er * er / (2.0 * sign[d] * sign[d]) +
         fabs(lsign[d]);
  }
  double e_new = orc_bond_energy(trial, chain, i, n, k0), e_old = orc_bond_energy(r, chain, i, n, k0);
  const float *om = omega + (uint64_t)orc_type(i, n_a) * n_cells;
  double w_new = om[orc_cell(trial, nx, ny, nz)], w_old = om[orc_cell(r, nx, ny, nz)];
  if (mag) *mag = m + e_new + e_old + (fabs(w_new) + fabs(w_old)) / (double)n_ref;
  return -((e_new - e_old) + (w_new - w_old) / (double)n_ref +
           orc_self_extra(r, trial, nx, ny, nz)) + log_rev - log_fwd;
}

/* Standardised FP32 inputs of the network for raw features f. */
static void orc_std_inputs(const float *p, const double *f, double *x0) {
  for (int k = 0; k < ORC_NF; ++k)
    x0[k] = (double)(((float)f[k] - p[ORC_P_SHIFT + k]) * p[ORC_P_SCALE + k]);
}

/* Trial position of a learned move from z and the normals xi, as the oracle
 * forms it, and the bound dr[3] of the device's FP32 trial: the window of z
 * carried through the head plus 2^-20 of |mu| + |sigma xi| (FP32 head and
 * normals) plus 2^-23 of |r| + |trial| (the additions). */
static void orc_learned_trial(const float *r, const double *z, const double *zw,
                              const double *xi, double m_max, double lo, double hi,
                              float *trial, double *dr) {
  double mu[3], sig[3], lsig[3];
  orc_head(z, m_max, lo, hi, mu, sig, lsig);
  for (int d = 0; d < 3; ++d) {
    trial[d] = (float)((double)r[d] + mu[d] + sig[d] * xi[d]);
    if (!dr) continue;
    double th = tanh(z[d] / m_max);
    double sg = 1.0 / (1.0 + exp(-z[3 + d]));
    double dmu = (1.0 - th * th) * zw[d];
    double dsig = sig[d] * (hi - lo) * sg * (1.0 - sg) * zw[3 + d];
    dr[d] = dmu + fabs(xi[d]) * dsig + 0x1p-20 * (fabs(mu[d]) + fabs(sig[d] * xi[d])) +
            0x1p-23 * (fabs((double)r[d]) + fabs((double)trial[d]));
    dr[d] *= orc_env_scale;
  }
}

/* Whether the device's outcome of a learned move may differ from the
 * oracle's through rounding alone: the trial (within its bound) may lie in
 * another cell, or the log ratio (with the effect of every ambiguous rounding
 * of both network passes, the windows of z, the trial's bound and nb_env, the
 * amount by which the bonded neighbours may already sit elsewhere) may fall
 * on the other side of log u.  *pos_env: how far the device's trial may lie
 * from the oracle's (the trial's bound plus the largest shift of an
 * ambiguous rounding of the pass at r).  The move is the one
 * orc_move_learned makes from the chain's current state. */
static int orc_learned_ambiguous(const float *chain, uint32_t i, uint32_t n, uint32_t n_a,
                                 double k0, const float *omega, uint64_t n_cells,
                                 uint32_t nx, uint32_t ny, uint32_t nz, uint32_t n_ref,
                                 const float *p, double m_max, double lo, double hi,
                                 const double *xi, double log_u, double nb_env,
                                 double *pos_env) {
  const float *r = chain + 3 * i;
  orc_amb_list *amb1 = malloc(sizeof(orc_amb_list)), *amb2 = malloc(sizeof(orc_amb_list));
  double f[ORC_NF], x0[ORC_NF], z[ORC_NO], zw[ORC_NO], dr[3];
  double fn[ORC_NF], xn[ORC_NF], xnw[ORC_NF], zn[ORC_NO], znw[ORC_NO];
  int flag = 0;
  double shift = 0.0;
  *pos_env = 0.0;
  amb1->n = amb2->n = 0;
  orc_features(chain, i, n, n_a, omega, nx, ny, nz, r, f);
  orc_std_inputs(p, f, x0);
  orc_dev_sample(p, x0, NULL, ORC_ST_NONE, 0, z, zw, amb1, NULL, 0, 0, 0, NULL, NULL, NULL);
  float trial[3];
  orc_learned_trial(r, z, zw, xi, m_max, lo, hi, trial, dr);
  /* the trial's cell within its bound, and the bound against the tolerance */
  for (int d = 0; d < 3; ++d) {
    double t = (double)trial[d];
    double frac = t - floor(t);
    if (frac <= dr[d] || 1.0 - frac <= dr[d]) flag = 1;
    if (dr[d] > *pos_env) *pos_env = dr[d];
  }
  orc_features(chain, i, n, n_a, omega, nx, ny, nz, trial, fn);
  orc_std_inputs(p, fn, xn);
  for (int k = 0; k < ORC_NF; ++k)
    xnw[k] = k >= 54 ? fabs((double)p[ORC_P_SCALE + k]) * dr[(k - 54) % 3] + 0x1p-23 * fabs(xn[k])
                     : 0.0;
  orc_dev_sample(p, xn, xnw, ORC_ST_NONE, 0, zn, znw, amb2, NULL, 0, 0, 0, NULL, NULL, NULL);
  double mag;
  const double lr = orc_learned_log_ratio(chain, i, n, n_a, k0, omega, n_cells, nx, ny, nz, n_ref,
                                          r, trial, z, zn, m_max, lo, hi, &mag);
  /* FP32 evaluation of the ratio and of exp; neighbours elsewhere by up to
   * nb_env change the bond terms by k0 |trial - r| nb_env and the network's
   * inputs (bounded generously by nb_env itself) */
  double step = 0.0;
  for (int d = 0; d < 3; ++d) step += fabs((double)trial[d] - (double)r[d]);
  double eps = orc_env_scale * (0x1p-18 * mag + 0x1p-20) + (k0 * step + 1.0) * nb_env;
  /* windows of z at r (through the trial) and at the trial */
  for (int j = 0; j < ORC_NO && !flag; ++j) {
    double zp[ORC_NO];
    float tp[3];
    memcpy(zp, z, sizeof zp);
    zp[j] += zw[j];
    orc_learned_trial(r, zp, zw, xi, m_max, lo, hi, tp, NULL);
    eps += fabs(orc_learned_log_ratio(chain, i, n, n_a, k0, omega, n_cells, nx, ny, nz, n_ref, r,
                                      tp, zp, zn, m_max, lo, hi, NULL) - lr);
    memcpy(zp, zn, sizeof zp);
    zp[j] += znw[j];
    eps += fabs(orc_learned_log_ratio(chain, i, n, n_a, k0, omega, n_cells, nx, ny, nz, n_ref, r,
                                      trial, z, zp, m_max, lo, hi, NULL) - lr);
  }
  /* the trial's bound, axis by axis */
  for (int d = 0; d < 3 && !flag; ++d) {
    float tp[3] = {trial[0], trial[1], trial[2]};
    tp[d] = (float)((double)trial[d] + dr[d]);
    eps += fabs(orc_learned_log_ratio(chain, i, n, n_a, k0, omega, n_cells, nx, ny, nz, n_ref, r,
                                      tp, z, zn, m_max, lo, hi, NULL) - lr);
  }
  /* every ambiguous rounding of the pass at r (moving the trial) ... */
  double rad = 0.0;
  for (int a = 0; a < amb1->n && !flag; ++a) {
    double za[ORC_NO], zaw[ORC_NO], fa[ORC_NF], xa[ORC_NF], zna[ORC_NO], znaw[ORC_NO];
    float ta[3];
    orc_dev_sample(p, x0, NULL, amb1->stage[a], amb1->unit[a], za, zaw, NULL, NULL, 0, 0, 0,
                   NULL, NULL, NULL);
    orc_learned_trial(r, za, zw, xi, m_max, lo, hi, ta, NULL);
    if (orc_cell(ta, nx, ny, nz) != orc_cell(trial, nx, ny, nz)) { flag = 1; break; }
    for (int d = 0; d < 3; ++d) shift = fmax(shift, fabs((double)ta[d] - (double)trial[d]));
    orc_features(chain, i, n, n_a, omega, nx, ny, nz, ta, fa);
    orc_std_inputs(p, fa, xa);
    orc_dev_sample(p, xa, NULL, ORC_ST_NONE, 0, zna, znaw, NULL, NULL, 0, 0, 0, NULL, NULL, NULL);
    rad += fabs(orc_learned_log_ratio(chain, i, n, n_a, k0, omega, n_cells, nx, ny, nz, n_ref, r,
                                      ta, za, zna, m_max, lo, hi, NULL) - lr);
  }
  /* ... and of the pass at the trial */
  for (int a = 0; a < amb2->n && !flag; ++a) {
    double zna[ORC_NO], znaw[ORC_NO];
    orc_dev_sample(p, xn, xnw, amb2->stage[a], amb2->unit[a], zna, znaw, NULL, NULL, 0, 0, 0,
                   NULL, NULL, NULL);
    rad += fabs(orc_learned_log_ratio(chain, i, n, n_a, k0, omega, n_cells, nx, ny, nz, n_ref, r,
                                      trial, z, zna, m_max, lo, hi, NULL) - lr);
  }
  if (!flag && fabs(lr - log_u) <= rad + eps) flag = 1;
  *pos_env += shift;
  free(amb1);
  free(amb2);
  return flag;
}

/* Whether the device's decision on a local move may differ from the oracle's
 * through rounding alone: -dE within the FP32 error of its delta-form
 * evaluation (2^-18 of the magnitudes of its terms) and of exp, plus the
 * change of the bond term when the bonded neighbours sit elsewhere by up to
 * nb_env, from log u. */
static int orc_local_ambiguous(const float *chain, uint32_t i, uint32_t n, uint32_t n_a,
                               double k0, const float *omega, uint64_t n_cells, uint32_t nx,
                               uint32_t ny, uint32_t nz, uint32_t n_ref, float a,
                               const uint32_t w[4], double nb_env) {
  const float *r = chain + 3 * i;
  float trial[3];
  double mag = 0.0;
  for (int d = 0; d < 3; ++d) trial[d] = fmaf(a, orc_v11(w[d]), r[d]);
  for (int d = 0; d < 3; ++d) {
    double dd = fabs((double)trial[d] - (double)r[d]);
    if (i > 0) mag += dd * (2.0 * fabs((double)r[d] - (double)chain[3 * (i - 1) + d]) + dd);
    if (i + 1 < n) mag += dd * (2.0 * fabs((double)r[d] - (double)chain[3 * (i + 1) + d]) + dd);
  }
  mag *= 0.5 * k0;
  double d_bond = orc_bond_energy(trial, chain, i, n, k0) - orc_bond_energy(r, chain, i, n, k0);
  const float *om = omega + (uint64_t)orc_type(i, n_a) * n_cells;
  double w_new = om[orc_cell(trial, nx, ny, nz)], w_old = om[orc_cell(r, nx, ny, nz)];
  double d_e = d_bond + (w_new - w_old) / (double)n_ref + orc_self_extra(r, trial, nx, ny, nz);
  mag += (fabs(w_new) + fabs(w_old)) / (double)n_ref;
  double step = 0.0;
  for (int d = 0; d < 3; ++d) step += fabs((double)trial[d] - (double)r[d]);
  double eps = orc_env_scale * (0x1p-18 * mag + 0x1p-20) + k0 * step * nb_env;
  return fabs(-d_e - log((double)orc_u01(w[3]))) <= eps;
}

/* Mixed sweep: each bead makes the learned move with probability p_learn
 * (uniform from word 1 of its purpose-1 draw, independent of the state) and
 * the local move otherwise.  A learned move draws xi by Box-Muller from the
 * purpose-0 block and accepts with word 0 of the purpose-1 block; a network
 * output that is not finite at r or r' rejects the move (q = 0). */
static int orc_move_learned(float *chain, uint32_t c_id, uint32_t i, uint32_t n,
                            uint32_t n_a, double k0, const float *omega,
                            uint64_t n_cells, uint32_t nx, uint32_t ny, uint32_t nz,
                            uint32_t n_ref, const float *params, double m_max,
                            double lo, double hi, int bf16, uint64_t seed,
                            uint32_t sweep, uint32_t replica, uint32_t *bad_net,
                            uint8_t *ambiguous, double nb_env, double *pos_env) {
  uint32_t wa[4], wb[4];
  orc_draw(seed, c_id, i, ORC_PURPOSE_MOVE_A, sweep, replica, wa);
  orc_draw(seed, c_id, i, ORC_PURPOSE_MOVE_B, sweep, replica, wb);
  double xi[4];
  orc_box_muller(wa[0], wa[1], &xi[0], &xi[1]);
  orc_box_muller(wa[2], wa[3], &xi[2], &xi[3]);
  float *r = chain + 3 * i;
  double f[ORC_NF], z[ORC_NO], mu[3], sig[3], lsig[3];
  orc_features(chain, i, n, n_a, omega, nx, ny, nz, r, f);
  orc_mlp_forward(params, f, bf16, z, NULL);
  orc_head(z, m_max, lo, hi, mu, sig, lsig);
  float trial[3];
  for (int d = 0; d < 3; ++d)
    trial[d] = (float)((double)r[d] + mu[d] + sig[d] * xi[d]);
  double fn[ORC_NF], zn[ORC_NO], mun[3], sign[3], lsign[3];
  orc_features(chain, i, n, n_a, omega, nx, ny, nz, trial, fn);
  orc_mlp_forward(params, fn, bf16, zn, NULL);
  orc_head(zn, m_max, lo, hi, mun, sign, lsign);
  for (int d = 0; d < 6; ++d)
    if (!isfinite(z[d]) || !isfinite(zn[d])) { (*bad_net)++; return 0; }
  if (orc_blocked(r, trial, nx, ny, nz)) return 0;
  double log_fwd = 0.0, log_rev = 0.0;
  for (int d = 0; d < 3; ++d) {
    double ef = (double)trial[d] - (double)r[d] - mu[d];
    double er = (double)r[d] - (double)trial[d] - mun[d];
    log_fwd -= ef * ef / (2.0 * sig[d] * sig[d]) + lsig[d];
    log_rev -= er * er / (2.0 * sign[d] * sign[d]) + lsign[d];
  }
  double d_bond = orc_bond_energy(trial, chain, i, n, k0) - orc_bond_energy(r, chain, i, n, k0);
  const float *om = omega + (uint64_t)orc_type(i, n_a) * n_cells;
  double d_field = ((double)om[orc_cell(trial, nx, ny, nz)] -
                    (double)om[orc_cell(r, nx, ny, nz)]) / (double)n_ref +
                   orc_self_extra(r, trial, nx, ny, nz);
  double log_ratio = -(d_bond + d_field) + log_rev - log_fwd;
  double u = (double)orc_u01(wb[0]);
  int accept = (log_ratio >= 0.0) || (u < exp(log_ratio));
  if (ambiguous && bf16)
    *ambiguous = (uint8_t)orc_learned_ambiguous(chain, i, n, n_a, k0, omega, n_cells, nx, ny, nz,
                                                n_ref, params, m_max, lo, hi, xi, log(u),
                                                nb_env, pos_env);
  if (accept) memcpy(r, trial, sizeof trial);
  return accept;
}

uint64_t orc_mc_sweep_mixed(float *pos, uint32_t n_chains, uint32_t n, uint32_t n_a,
                            float k0, uint32_t n_ref, const float *omega, uint32_t nx,
                            uint32_t ny, uint32_t nz, float local_a, float p_learn,
                            const float *params, float m_max, float lo, float hi, int bf16,
                            uint64_t seed, uint32_t sweep, uint32_t replica,
                            uint32_t chain_base, uint32_t set_order, uint8_t *kind_flags,
                            uint8_t *accept_flags, uint8_t *amb_flags, float *pos_env,
                            uint64_t *accepted_learned, uint32_t *bad_net, int n_threads) {
  uint64_t n_cells = (uint64_t)nx * ny * nz;
  uint64_t acc_total = 0, acc_l = 0;
  uint32_t bad = 0;
  /* BF16 mode evaluates the network as the learned move does (standardisation
   * folded into the first layer); FP64 mode is the definition itself */
  float folded[ORC_P_SIZE];
  const float *net = params;
  if (bf16) {
    orc_fold_params(params, folded);
    net = folded;
  }
#pragma omp parallel for schedule(static) reduction(+ : acc_total, acc_l, bad) num_threads(n_threads > 0 ? n_threads : 1)
  for (int64_t c = 0; c < (int64_t)n_chains; ++c) {
    float *chain = pos + (uint64_t)c * n * 3;
    uint32_t c_id = chain_base + (uint32_t)c;
    uint32_t first = 0;
    if (set_order == 0) {
      uint32_t w[4];
      orc_draw(seed, c_id, 0, ORC_PURPOSE_MOVE_A, sweep, replica, w);
      first = w[0] & 1u;
    }
    for (uint32_t pass = 0; pass < 2; ++pass) {
      uint32_t parity = pass == 0 ? first : 1u - first;
      for (uint32_t i = parity; i < n; i += 2) {
        uint32_t wb[4];
        orc_draw(seed, c_id, i, ORC_PURPOSE_MOVE_B, sweep, replica, wb);
        int learned = (double)orc_u01(wb[1]) < (double)p_learn;
        int acc;
        uint32_t b = 0;
        uint8_t amb = 0;
        double env = 0.0, nb_env = 0.0;
        if (amb_flags) {   /* how far the bonded neighbours may sit elsewhere */
          if (i > 0) nb_env += pos_env[(uint64_t)c * n + i - 1];
          if (i + 1 < n) nb_env += pos_env[(uint64_t)c * n + i + 1];
        }
        if (learned) {
          acc = orc_move_learned(chain, c_id, i, n, n_a, (double)k0, omega, n_cells, nx, ny,
                                 nz, n_ref, net, m_max, lo, hi, bf16, seed, sweep,
                                 replica, &b, amb_flags ? &amb : NULL, nb_env, &env);
        } else {
          if (amb_flags) {
            uint32_t w[4];
            orc_draw(seed, c_id, i, ORC_PURPOSE_MOVE_A, sweep, replica, w);
            amb = (uint8_t)orc_local_ambiguous(chain, i, n, n_a, (double)k0, omega, n_cells,
                                               nx, ny, nz, n_ref, local_a, w, nb_env);
          }
          acc = orc_move_local(chain, c_id, i, n, n_a, (double)k0, omega, n_cells, nx, ny,
                               nz, n_ref, local_a, seed, sweep, replica);
        }
        if (amb_flags) {
          amb_flags[(uint64_t)c * n + i] = amb;
          pos_env[(uint64_t)c * n + i] = acc ? (float)env : 0.0f;
        }
        bad += b;
        acc_total += (uint64_t)acc;
        if (learned) acc_l += (uint64_t)acc;
        if (kind_flags) kind_flags[(uint64_t)c * n + i] = (uint8_t)learned;
        if (accept_flags) accept_flags[(uint64_t)c * n + i] = (uint8_t)acc;
      }
    }
  }
  if (accepted_learned) *accepted_learned = acc_l;
  if (bad_net) *bad_net = bad;
  return acc_total;
}

/* ------------------------------------------------------------------------- */
/* General molecular architectures (Sec. 3.2.1): one array of 32-bit words per */
/* molecule type.  Word 0 holds N; word 1+i describes monomer i: its type in  */
/* the top byte and, in the low 24 bits, the index (from the start of the      */
/* array) of its bond list, 0 for a monomer without bonds.  A bond word holds */
/* the signed offset partner - i in its low 27 bits, the bond type in bits    */
/* 27-30 (0: harmonic, the only kind) and, in bit 31, the flag that ends the  */
/* monomer's list.  Two types (A = 0, B = 1).                                  */
/*                                                                             */
/* Independent sets (Sec. 3.1.2, scheme 2): greedy colouring in index order,  */
/* monomer i gets the smallest set number not used by a bonded monomer of     */
/* lower index (a linear chain gives the even and the odd monomers).  Order   */
/* of the sets per chain and sweep: with two sets, set 1 first iff bit 0 of    */
/* word 0 of monomer 0's move draw is set (as for linear chains); with more,  */
/* a Fisher-Yates shuffle, step t = k-1 .. 1 swapping t with                   */
/* floor(w (t+1) / 2^32), w = word (k-1-t) mod 4 of the Philox block          */
/* (chain, floor((k-1-t)/4) | 8 << 16, sweep, replica); set_order = 1 keeps   */
/* the numerical order.  A move is the LOCAL move with the bond energy summed */
/* over the monomer's bond list.                                              */
/* ------------------------------------------------------------------------- */
#define ORC_MAX_N 128
#define ORC_MAX_BONDS 2048
#define ORC_PURPOSE_SET_ORDER 8u

typedef struct {
  uint32_t n, n_sets, n_bonds;
  uint8_t type[ORC_MAX_N];
  uint32_t color[ORC_MAX_N];
  uint32_t nb_start[ORC_MAX_N + 1];
  uint32_t nb[ORC_MAX_BONDS];
} orc_arch;

/* Decodes and checks an architecture; returns 0, or -1 if it is malformed
 * (a partner out of range or equal to the monomer, a non-harmonic bond, a
 * bond listed on one side only, a list running off the array, a type code of
 * ORC_MAX_TYPES or more). */
static int orc_arch_decode(const uint32_t *w, uint32_t n_words, orc_arch *a) {
  if (n_words < 1) return -1;
  uint32_t n = w[0];
  if (n == 0 || n > ORC_MAX_N || n_words < 1 + n) return -1;
  a->n = n;
  uint32_t nb = 0;
  for (uint32_t i = 0; i < n; ++i) {
    uint32_t m = w[1 + i];
    a->type[i] = (uint8_t)(m >> 24);
    if ((m >> 24) >= ORC_MAX_TYPES) return -1;
    a->nb_start[i] = nb;
    uint32_t k = m & 0xFFFFFFu;
    if (k == 0) continue;
    for (;; ++k) {
      if (k >= n_words || nb >= ORC_MAX_BONDS) return -1;
      uint32_t b = w[k];
      int32_t off = (int32_t)(b << 5) >> 5;          /* sign-extend 27 bits */
      if (((b >> 27) & 0xFu) != 0u) return -1;
      int64_t p = (int64_t)i + off;
      if (off == 0 || p < 0 || p >= (int64_t)n) return -1;
      a->nb[nb++] = (uint32_t)p;
      if (b >> 31) break;
    }
  }
  a->nb_start[n] = nb;
  a->n_bonds = nb;
  /* every bond must be listed at both ends */
  for (uint32_t i = 0; i < n; ++i)
    for (uint32_t q = a->nb_start[i]; q < a->nb_start[i + 1]; ++q) {
      uint32_t j = a->nb[q], found = 0;
      for (uint32_t r = a->nb_start[j]; r < a->nb_start[j + 1]; ++r) found |= a->nb[r] == i;
      if (!found) return -1;
    }
  uint32_t k_max = 0;
  for (uint32_t i = 0; i < n; ++i) {
    uint64_t used = 0;
    for (uint32_t q = a->nb_start[i]; q < a->nb_start[i + 1]; ++q)
      if (a->nb[q] < i) used |= 1ull << a->color[a->nb[q]];
    uint32_t c = 0;
    while (used & (1ull << c)) ++c;
    a->color[i] = c;
    if (c + 1 > k_max) k_max = c + 1;
  }
  a->n_sets = k_max;
  return 0;
}

/* Set numbers of the monomers (set_of[N]); returns the number of sets or -1. */
int orc_arch_sets(const uint32_t *w, uint32_t n_words, uint32_t *set_of) {
  static orc_arch a;
  if (orc_arch_decode(w, n_words, &a)) return -1;
  for (uint32_t i = 0; i < a.n; ++i) set_of[i] = a.color[i];
  return (int)a.n_sets;
}

/* Bond energy of monomer i at position r with its bonded partners, Eqs. (1)-(2). */
static double orc_arch_bond_energy(const float *r, const float *chain, const orc_arch *a,
                                   uint32_t i, double k0) {
  double e = 0.0;
  for (uint32_t q = a->nb_start[i]; q < a->nb_start[i + 1]; ++q) {
    const float *rj = chain + 3 * a->nb[q];
    for (int d = 0; d < 3; ++d) {
      double dx = (double)r[d] - (double)rj[d];
      e += 0.5 * k0 * dx * dx;
    }
  }
  return e;
}

uint64_t orc_mc_sweep_arch(float *pos, uint32_t n_chains, const uint32_t *w,
                           uint32_t n_words, float k0, uint32_t n_ref, const float *omega,
                           uint32_t nx, uint32_t ny, uint32_t nz, float step, uint64_t seed,
                           uint32_t sweep, uint32_t replica, uint32_t chain_base,
                           uint32_t set_order, uint8_t *accept_flags, int n_threads) {
  static orc_arch a;
  if (orc_arch_decode(w, n_words, &a)) return UINT64_MAX;
  const uint32_t n = a.n, k = a.n_sets;
  uint64_t n_cells = (uint64_t)nx * ny * nz;
  uint64_t accepted = 0;
#pragma omp parallel for schedule(static) reduction(+ : accepted) num_threads(n_threads > 0 ? n_threads : 1)
  for (int64_t c = 0; c < (int64_t)n_chains; ++c) {
    float *chain = pos + (uint64_t)c * n * 3;
    uint32_t c_id = chain_base + (uint32_t)c;
    uint32_t order[ORC_MAX_N];
    for (uint32_t s = 0; s < k; ++s) order[s] = s;
    if (set_order == 0 && k == 2) {
      uint32_t d[4];
      orc_draw(seed, c_id, 0, ORC_PURPOSE_MOVE_A, sweep, replica, d);
      if (d[0] & 1u) { order[0] = 1; order[1] = 0; }
    } else if (set_order == 0 && k > 2) {
      uint32_t d[4];
      for (uint32_t t = k - 1, step_i = 0; t >= 1; --t, ++step_i) {
        if (step_i % 4u == 0u)
          orc_draw(seed, c_id, step_i / 4u, ORC_PURPOSE_SET_ORDER, sweep, replica, d);
        uint32_t j = orc_pick_bead(d[step_i % 4u], t + 1);
        uint32_t tmp = order[t]; order[t] = order[j]; order[j] = tmp;
      }
    }
    for (uint32_t s = 0; s < k; ++s)
      for (uint32_t i = 0; i < n; ++i) {
        if (a.color[i] != order[s]) continue;
        uint32_t wd[4];
        orc_draw(seed, c_id, i, ORC_PURPOSE_MOVE_A, sweep, replica, wd);
        float *r = chain + 3 * i;
        float trial[3];
        for (int d = 0; d < 3; ++d) trial[d] = fmaf(step, orc_v11(wd[d]), r[d]);
        int acc = 0;
        if (!orc_blocked(r, trial, nx, ny, nz)) {
          double d_bond = orc_arch_bond_energy(trial, chain, &a, i, (double)k0) -
                          orc_arch_bond_energy(r, chain, &a, i, (double)k0);
          const float *om = omega + (uint64_t)a.type[i] * n_cells;
          double d_field = ((double)om[orc_cell(trial, nx, ny, nz)] -
                            (double)om[orc_cell(r, nx, ny, nz)]) / (double)n_ref;
          double d_e = d_bond + d_field;
          acc = (d_e <= 0.0) || ((double)orc_u01(wd[3]) < exp(-d_e));
          if (acc) memcpy(r, trial, sizeof trial);
        }
        accepted += (uint64_t)acc;
        if (accept_flags) accept_flags[(uint64_t)c * n + i] = (uint8_t)acc;
      }
  }
  return accepted;
}

/* Histogram of chains of one architecture (types from the architecture) into
 * n_t planes; -1 if the architecture is malformed or uses a type >= n_t. */
int orc_density_hist_arch(const float *pos, uint32_t n_chains, const uint32_t *w,
                          uint32_t n_words, uint32_t nx, uint32_t ny, uint32_t nz,
                          uint32_t n_t, uint32_t *counts) {
  static orc_arch a;
  if (orc_arch_decode(w, n_words, &a)) return -1;
  for (uint32_t i = 0; i < a.n; ++i)
    if (a.type[i] >= n_t) return -1;
  uint64_t n_cells = (uint64_t)nx * ny * nz;
  memset(counts, 0, (uint64_t)n_t * n_cells * sizeof(uint32_t));
  for (uint64_t c = 0; c < n_chains; ++c)
    for (uint32_t i = 0; i < a.n; ++i) {
      uint64_t cell = orc_cell(pos + 3 * (c * a.n + i), nx, ny, nz);
      counts[(uint64_t)a.type[i] * n_cells + cell] += 1u;
    }
  return 0;
}
