// soma_api.hip -- the C ABI declared in include/soma.h: configuration checks,
// workspace layout, kernel launches and the SCMF cycle bookkeeping.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "soma.h"
#include "soma_device.hpp"
#include "soma_grid.hpp"
#include "soma_obs.hpp"
#include "soma_sweep.hpp"
#include "soma_molecule.hpp"
#include "soma_arch.hpp"
#include "soma_train.hpp"
#include "soma_batch.hpp"
#include "soma_sq.hpp"

namespace {

thread_local char g_err[512] = "";

int32_t fail(int32_t code, const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
  return code;
}

#define HIP_TRY(expr)                                                        \
  do {                                                                       \
    hipError_t e_ = (expr);                                                  \
    if (e_ != hipSuccess)                                                    \
      return fail(SOMA_E_HIP, "%s failed: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

#define LAUNCH_TRY() HIP_TRY(hipGetLastError())

constexpr uint64_t kAlign = 256;
uint64_t align_up(uint64_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Derived {
  uint64_t n_beads = 0, n_chains = 0, n_cells = 0;
  uint64_t bead_off[SOMA_MAX_SPECIES] = {};
  uint64_t chain_off[SOMA_MAX_SPECIES] = {};
  uint64_t n_a_total = 0;
  uint64_t obs_blocks = 0;
  uint64_t obs_block_off[SOMA_MAX_SPECIES] = {};
  uint64_t pos_bytes = 0, counts_bytes = 0, omega_bytes = 0;
  // workspace layout
  uint64_t off_err = 0, off_acc = 0, off_att = 0, off_net = 0, off_fpart = 0, off_totals = 0,
           off_opart = 0, off_halo = 0, off_arch = 0, off_tcount = 0;
  uint64_t halo_plane = 0;    // floats per plane of the halo copy (0: not kept)
  // external fields (soma_set_external): caller-owned device buffers, null if none;
  // n_free = cells not impenetrable (the reference density counts these)
  const float *ext = nullptr;
  const uint32_t *forbid = nullptr;
  uint64_t n_free = 0;
  // general architectures (soma_set_architecture): device tables per species, null: linear
  const soma::ArchDev *arch[SOMA_MAX_SPECIES] = {};
  uint32_t form = 1;   // interaction term of the Hamiltonian (soma_set_hamiltonian)
  // bead types (soma_set_types): 2 uses chi_n of the config; more use chi_m,
  // chi_ij N at [i * kMaxTypes + j]
  uint32_t n_types = 2;
  float chi_m[soma::kMaxTypes * soma::kMaxTypes] = {};
  uint64_t ws_bytes = 0;
  uint32_t field_blocks = 1;  // blocks of the field update (and its FP64 partial sums)
  // per-brick bins of count updates (soma_set_histogram): bricks of 16 x 16 x 8 cells
  uint32_t nbx = 0, nby = 0, nbz = 0, bin_cap = 0;
  uint64_t n_bricks = 0, off_bin_count = 0, off_bins = 0;
  bool bins_ok = false;
  uint64_t off_queue = 0;   // tile counters of persistent local sweeps
};

int32_t derive(const soma_config *c, Derived *d) {
  if (!c) return fail(SOMA_E_INVAL, "config is NULL");
  if (c->nx == 0 || c->ny == 0 || c->nz == 0)
    return fail(SOMA_E_INVAL, "grid dimensions must be positive");
  const uint64_t n_cells = (uint64_t)c->nx * c->ny * c->nz;
  // field planes are addressed with 32-bit byte offsets: 2 * 4 * n_cells < 2^32
  if (n_cells >= (1ull << 29)) return fail(SOMA_E_UNSUPPORTED, "more than 2^29 - 1 cells");
  if (c->n_species == 0 || c->n_species > SOMA_MAX_SPECIES)
    return fail(SOMA_E_INVAL, "n_species must be in 1..%d", SOMA_MAX_SPECIES);
  if (c->count_width != 16 && c->count_width != 32)
    return fail(SOMA_E_INVAL, "count_width must be 16 or 32");
  if (c->n_ref == 0) return fail(SOMA_E_INVAL, "n_ref must be positive");
  if (c->set_order > 1) return fail(SOMA_E_INVAL, "set_order must be 0 or 1");
  if (c->origin_mode > 1) return fail(SOMA_E_INVAL, "origin_mode must be 0 or 1");
  if (!(c->p_learn >= 0.f && c->p_learn <= 1.f) || !(c->mu_max > 0.f) ||
      !std::isfinite(c->log_sigma_min) || !std::isfinite(c->log_sigma_max) ||
      !(c->log_sigma_min <= c->log_sigma_max))
    return fail(SOMA_E_INVAL, "learned proposal: need 0 <= p_learn <= 1, mu_max > 0, "
                              "finite log_sigma_min <= log_sigma_max");
  if (!std::isfinite(c->chi_n) || !std::isfinite(c->kappa_n) || !std::isfinite(c->local_a) ||
      !std::isfinite(c->smc_a) || c->local_a < 0.f || c->smc_a < 0.f)
    return fail(SOMA_E_INVAL, "chi_n, kappa_n, local_a, smc_a must be finite (steps >= 0)");
  d->n_cells = n_cells;
  d->n_free = n_cells;
  {
    const uint64_t fb = (n_cells + 4095) / 4096;
    d->field_blocks = (uint32_t)(fb < soma::kFieldBlocks ? fb : soma::kFieldBlocks);
  }
  d->n_beads = d->n_chains = d->n_a_total = d->obs_blocks = 0;
  for (uint32_t s = 0; s < c->n_species; ++s) {
    const soma_species &sp = c->species[s];
    if (sp.n == 0 || sp.n > SOMA_MAX_BEADS_PER_CHAIN)
      return fail(SOMA_E_UNSUPPORTED, "species %u: beads per chain must be 1..%d", s,
                  SOMA_MAX_BEADS_PER_CHAIN);
    if (sp.n_a > sp.n) return fail(SOMA_E_INVAL, "species %u: n_a > n", s);
    if (!std::isfinite(sp.k0) || sp.k0 <= 0.f)
      return fail(SOMA_E_INVAL, "species %u: k0 must be positive", s);
    d->bead_off[s] = d->n_beads;
    d->chain_off[s] = d->n_chains;
    d->obs_block_off[s] = d->obs_blocks;
    d->n_beads += (uint64_t)sp.n_chains * sp.n;
    d->n_chains += sp.n_chains;
    d->n_a_total += (uint64_t)sp.n_chains * sp.n_a;
    d->obs_blocks += (sp.n_chains + 255u) / 256u;
  }
  if (d->n_chains >= (1ull << 32)) return fail(SOMA_E_UNSUPPORTED, "2^32 or more chains");
  if (d->n_beads == 0) return fail(SOMA_E_INVAL, "no beads");
  d->pos_bytes = 12ull * d->n_beads;
  d->counts_bytes = (c->count_width == 16 ? 4ull : 8ull) * n_cells;
  d->omega_bytes = 8ull * n_cells;
  d->off_err = 0;
  d->off_acc = align_up(d->off_err + 16);
  d->off_att = align_up(d->off_acc + 4ull * soma::kAccSlots * 8ull);
  d->off_net = align_up(d->off_att + soma::kAccSlots * 8ull);
  d->off_fpart = align_up(d->off_net + SOMA_MAX_SPECIES * align_up(sizeof(soma::NetDev)));
  d->off_totals = align_up(d->off_fpart + soma::kFieldBlocks * sizeof(soma::FieldPartial));
  d->off_opart = align_up(d->off_totals + sizeof(soma::Totals));
  d->off_arch = align_up(d->off_opart + (d->obs_blocks ? d->obs_blocks : 1) * sizeof(soma::ObsPartial));
  d->off_tcount = align_up(d->off_arch + SOMA_MAX_SPECIES * align_up(sizeof(soma::ArchDev)));
  d->off_halo = align_up(d->off_tcount + 8ull * soma::kFieldBlocks * soma::kMaxTypes);
  // the learned proposal reads its 27-cell neighbourhoods from a copy of the
  // fields with one periodic halo cell at both ends of each x row
  d->halo_plane = c->p_learn > 0.f ? (uint64_t)c->nz * c->ny * (c->nx + 2u) : 0u;
  if (8ull * d->halo_plane >= (1ull << 32))
    return fail(SOMA_E_UNSUPPORTED, "grid too large for the learned proposal's field copy");
  d->off_queue = align_up(d->off_halo + 8ull * d->halo_plane);
  d->ws_bytes = align_up(d->off_queue + 4ull * soma::kQueueParts * soma::kQueueSub * soma::kQueueStride);
  // bins: room for the updates of about half the beads of a brick per sweep
  // (entries beyond it go to the counts as direct atomics)
  d->nbx = (c->nx + 15u) / 16u;
  d->nby = (c->ny + 15u) / 16u;
  d->nbz = (c->nz + 7u) / 8u;
  d->n_bricks = (uint64_t)d->nbx * d->nby * d->nbz;
  d->bins_ok = d->n_bricks < (1ull << 21);
  if (d->bins_ok) {
    // per sub-bin: twice its share of about half a brick's beads, plus slack
    // (a recount fills about half a brick's beads, a smart-MC sweep about 0.45)
    const double per_brick = (double)d->n_beads * soma::kBrickCells / (double)n_cells;
    uint64_t cap = (uint64_t)std::ceil(1.1 * per_brick / soma::kSubBins) + 64u;
    cap = (cap + 15u) / 16u * 16u;
    if (cap > (1ull << 22)) cap = 1ull << 22;
    d->bin_cap = (uint32_t)cap;
    d->off_bin_count = d->ws_bytes;
    d->off_bins = align_up(d->off_bin_count + 4ull * d->n_bricks * soma::kSubBins);
    d->ws_bytes = align_up(d->off_bins + 4ull * d->n_bricks * soma::kSubBins * cap);
  }
  return SOMA_OK;
}

soma::Grid make_grid(const soma_config *c, uint64_t n_cells) {
  soma::Grid g;
  g.nx = (int)c->nx; g.ny = (int)c->ny; g.nz = (int)c->nz;
  g.inv_nx = 1.0f / (float)c->nx;
  g.inv_ny = 1.0f / (float)c->ny;
  g.inv_nz = 1.0f / (float)c->nz;
  g.n_cells = (uint32_t)n_cells;
  return g;
}

// 1 / rho_bar: free cells per bead (all cells without impenetrable ones)
double inv_rho_d(const Derived &d) { return (double)d.n_free / (double)d.n_beads; }
float inv_rho_f(const Derived &d) { return (float)inv_rho_d(d); }

int32_t launch_zero(void *p, uint64_t bytes, hipStream_t s) {
  const uint64_t words = bytes / 4;
  uint64_t blocks = (words / 4 + 255) / 256;
  if (blocks < 1) blocks = 1;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(soma::zero_kernel, dim3((uint32_t)blocks), dim3(256), 0, s,
                     reinterpret_cast<uint32_t *>(p), words);
  LAUNCH_TRY();
  return SOMA_OK;
}

// From-scratch histogram.  With bins (`bins` not null: the system's workspace
// holds them), each species' beads go through the per-brick bins and one
// apply pass per brick; otherwise one device atomic per bead.
int32_t launch_hist(const soma_config *c, const Derived &d, const float *pos, void *counts,
                    hipStream_t s, const soma::BinArgs *bins = nullptr) {
  int32_t rc = launch_zero(counts, d.counts_bytes, s);
  if (rc) return rc;
  const soma::Grid g = make_grid(c, d.n_cells);
  if (bins) {
    for (uint32_t sp = 0; sp < c->n_species; ++sp) {
      const soma_species &S = c->species[sp];
      const uint64_t nb = (uint64_t)S.n_chains * S.n;
      if (!nb) continue;
      const uint64_t blocks = ((nb + 1) / 2 + 255) / 256;
      const float *p = pos + 3 * d.bead_off[sp];
      const uint32_t v2 = (reinterpret_cast<uintptr_t>(p) % 8u) == 0u ? 1u : 0u;
      if (c->count_width == 32)
        hipLaunchKernelGGL(soma::density_hist_binned_kernel<true>, dim3((uint32_t)blocks),
                           dim3(256), 0, s, p, nb, S.n, S.n_a, g, counts, d.arch[sp], *bins, v2);
      else
        hipLaunchKernelGGL(soma::density_hist_binned_kernel<false>, dim3((uint32_t)blocks),
                           dim3(256), 0, s, p, nb, S.n, S.n_a, g, counts, d.arch[sp], *bins, v2);
      LAUNCH_TRY();
    }
    const uint32_t planes = (d.n_types + 1u) / 2u;
    const size_t lds = (size_t)planes * soma::kBrickCells * (c->count_width == 32 ? 8u : 4u);
    if (c->count_width == 32)
      hipLaunchKernelGGL(soma::bin_apply_kernel<true>, dim3((uint32_t)d.n_bricks),
                         dim3(soma::kApplyThreads), lds, s, *bins, g, counts, planes);
    else
      hipLaunchKernelGGL(soma::bin_apply_kernel<false>, dim3((uint32_t)d.n_bricks),
                         dim3(soma::kApplyThreads), lds, s, *bins, g, counts, planes);
    LAUNCH_TRY();
    return SOMA_OK;
  }
  for (uint32_t sp = 0; sp < c->n_species; ++sp) {
    const soma_species &S = c->species[sp];
    const uint64_t nb = (uint64_t)S.n_chains * S.n;
    if (!nb) continue;
    const uint64_t blocks = (nb + 255) / 256;
    const float *p = pos + 3 * d.bead_off[sp];
    if (c->count_width == 32)
      hipLaunchKernelGGL(soma::density_hist_kernel<true>, dim3((uint32_t)blocks), dim3(256), 0, s,
                         p, nb, S.n, S.n_a, g, counts, d.arch[sp]);
    else
      hipLaunchKernelGGL(soma::density_hist_kernel<false>, dim3((uint32_t)blocks), dim3(256), 0,
                         s, p, nb, S.n, S.n_a, g, counts, d.arch[sp]);
    LAUNCH_TRY();
  }
  return SOMA_OK;
}

soma::FieldArgs field_args(const soma_config *c, const Derived &d, void *counts, float *omega,
                           soma::FieldPartial *partials, float *halo = nullptr) {
  soma::FieldArgs a;
  a.counts = counts;
  a.omega = omega;
  a.n_cells = (uint32_t)d.n_cells;
  a.inv_rho = inv_rho_f(d);
  a.chi_n = c->chi_n;
  a.kappa_n = c->kappa_n;
  a.inv_rho_d = inv_rho_d(d);
  a.chi_n_d = (double)c->chi_n;
  a.kappa_n_d = (double)c->kappa_n;
  a.partials = partials;
  a.clear = 0;
  a.halo = d.halo_plane ? halo : nullptr;
  a.nx = c->nx;
  a.halo_plane = (uint32_t)d.halo_plane;
  a.ext = d.ext;
  a.forbid = d.forbid;
  a.form = d.form;
  return a;
}

int32_t launch_field(const soma_config *c, const Derived &d, void *counts, float *omega,
                     soma::FieldPartial *partials, hipStream_t s, float *halo = nullptr) {
  const uint32_t blocks = d.field_blocks;
  if (d.n_types > 2) {   // no halo copy, external fields or walls with more than two types
    soma::MultiFieldArgs m;
    m.counts = counts;
    m.omega = omega;
    m.n_cells = (uint32_t)d.n_cells;
    m.n_t = d.n_types;
    m.form = d.form;
    m.clear = 0;
    m.inv_rho = inv_rho_f(d);
    m.kappa_n = c->kappa_n;
    m.inv_rho_d = inv_rho_d(d);
    m.kappa_n_d = (double)c->kappa_n;
    std::memcpy(m.chi, d.chi_m, sizeof m.chi);
    m.partials = partials;
    const bool c64 = c->count_width == 32;
    switch (d.n_types) {
#define SOMA_MULTI_CASE(NT)                                                                       \
  case NT:                                                                                        \
    if (c64) hipLaunchKernelGGL((soma::field_multi_kernel<true, NT>), dim3(blocks), dim3(256), 0, s, m); \
    else hipLaunchKernelGGL((soma::field_multi_kernel<false, NT>), dim3(blocks), dim3(256), 0, s, m);    \
    break;
      SOMA_MULTI_CASE(3)
      SOMA_MULTI_CASE(4)
      SOMA_MULTI_CASE(5)
      SOMA_MULTI_CASE(6)
      SOMA_MULTI_CASE(7)
      SOMA_MULTI_CASE(8)
#undef SOMA_MULTI_CASE
      default:
        return fail(SOMA_E_INVAL, "%u bead types", d.n_types);
    }
    LAUNCH_TRY();
    return SOMA_OK;
  }
  const soma::FieldArgs a = field_args(c, d, counts, omega, partials, halo);
  // counts of 64 MiB and more are read with the non-temporal hint (measured on
  // the 134M-bead melt: 3.7% off the SCMF cycle, the next sweep's field
  // gathers hitting the last-level cache more often)
  const bool c64 = c->count_width == 32;
  const bool nt = (uint64_t)d.n_cells * (c64 ? 8u : 4u) >= (64ull << 20);
  const dim3 grid(blocks), block(256);
  if (c64) {
    if (nt) hipLaunchKernelGGL((soma::field_update_kernel<true, true>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((soma::field_update_kernel<true, false>), grid, block, 0, s, a);
  } else {
    if (nt) hipLaunchKernelGGL((soma::field_update_kernel<false, true>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((soma::field_update_kernel<false, false>), grid, block, 0, s, a);
  }
  LAUNCH_TRY();
  return SOMA_OK;
}

int32_t launch_init(const soma_config *c, const Derived &d, float *pos, hipStream_t s) {
  const soma::Grid g = make_grid(c, d.n_cells);
  for (uint32_t sp = 0; sp < c->n_species; ++sp) {
    const soma_species &S = c->species[sp];
    if (!S.n_chains) continue;
    soma::InitArgs a;
    a.pos = pos + 3 * d.bead_off[sp];
    a.n_chains = S.n_chains;
    a.n = S.n;
    a.chain_base = (uint32_t)d.chain_off[sp];
    a.total_chains = (uint32_t)d.n_chains;
    a.sigma = (float)(1.0 / std::sqrt((double)S.k0));
    a.grid = g;
    a.seed_lo = (uint32_t)c->seed;
    a.seed_hi = (uint32_t)(c->seed >> 32);
    a.replica = c->replica;
    a.origin_mode = c->origin_mode;
    hipLaunchKernelGGL(soma::init_chains_kernel, dim3((S.n_chains + 255) / 256), dim3(256), 0,
                       s, a);
    LAUNCH_TRY();
  }
  return SOMA_OK;
}

bool aligned(const void *p, uintptr_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

}  // namespace

// An instantiated graph of SCMF cycles (sweep, field refresh) x cycles, then
// the advance of the device sweep counters.
struct CycleGraph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  uint32_t cycles = 0, kind = 0;
  void release() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
    cycles = 0;
  }
};

struct soma_system {
  soma_config cfg;
  soma_buffers buf;
  Derived d;
  soma::Grid grid;
  uint64_t sweep = 0;
  uint64_t attempted[4] = {0, 0, 0, 0};   // by move kind (the learned slot unused)
  uint32_t sweep_blocks = 0;  // SET sweep grid: 0 = one tile per wave, else persistent blocks
  uint64_t mixed_moves = 0;   // bead moves made by mixed sweeps (local or learned)
  uint32_t net_mask = 0;      // species with an installed network (bit per species)
  uint32_t arch_mask = 0;     // species with a general architecture (bit per species)
  uint32_t arch_type0[SOMA_MAX_SPECIES] = {};  // A monomers per molecule of those species
  uint32_t arch_per_wave[SOMA_MAX_SPECIES] = {};  // molecules per wave of their sweep
  uint32_t arch_max_type[SOMA_MAX_SPECIES] = {};  // largest type code of their monomers
  uint32_t substeps = 1;      // field refreshes per SCMF cycle (chain subsets)
  uint32_t scheme = SOMA_SCHEME_SET;  // iteration order of local moves
  uint32_t hist_mode = soma::kHistDirect;  // count updates of the SET sweeps (soma_set_histogram)
  uint32_t sweep_threads = 256;  // block size of the local, smart-MC and bond-Gibbs sweeps
  uint32_t self_term = 0;        // add the bead's own share to cell-changing moves (soma_set_self_term)
  float4 *grad = nullptr;     // optional gradient field (caller-owned), see soma_set_grad_field
  unsigned char *ws = nullptr;
  CycleGraph graph;
  ~soma_system() { graph.release(); }
  uint32_t *err() { return reinterpret_cast<uint32_t *>(ws + d.off_err); }
  uint32_t *sweep_ctr() { return reinterpret_cast<uint32_t *>(ws + d.off_err) + 1; }
  void count_sweeps(uint32_t kind, uint64_t n) {
    sweep += n;
    if (kind == SOMA_MOVE_MIXED) mixed_moves += n * d.n_beads;
    else attempted[kind] += n * d.n_beads;
  }
  unsigned long long *acc() { return reinterpret_cast<unsigned long long *>(ws + d.off_acc); }
  soma::FieldPartial *fpart() { return reinterpret_cast<soma::FieldPartial *>(ws + d.off_fpart); }
  soma::Totals *totals() { return reinterpret_cast<soma::Totals *>(ws + d.off_totals); }
  soma::ObsPartial *opart() { return reinterpret_cast<soma::ObsPartial *>(ws + d.off_opart); }
  float *halo() { return d.halo_plane ? reinterpret_cast<float *>(ws + d.off_halo) : nullptr; }
  unsigned long long *att() { return reinterpret_cast<unsigned long long *>(ws + d.off_att); }
  soma::ArchDev *arch(uint32_t sp) {
    return reinterpret_cast<soma::ArchDev *>(ws + d.off_arch + sp * align_up(sizeof(soma::ArchDev)));
  }
  const soma::ArchDev *arch_or_null(uint32_t sp) { return (arch_mask >> sp & 1u) ? arch(sp) : nullptr; }
  soma::BinArgs bins() {
    soma::BinArgs b;
    b.bin_count = reinterpret_cast<uint32_t *>(ws + d.off_bin_count);
    b.bins = reinterpret_cast<uint32_t *>(ws + d.off_bins);
    b.cap = d.bin_cap;
    b.nbx = d.nbx;
    b.nby = d.nby;
    b.nbz = d.nbz;
    return b;
  }
  soma::NetDev *net(uint32_t sp) {
    return reinterpret_cast<soma::NetDev *>(ws + d.off_net + sp * align_up(sizeof(soma::NetDev)));
  }
  bool nets_ready() const {
    for (uint32_t sp = 0; sp < cfg.n_species; ++sp)
      if (cfg.species[sp].n_chains && !(net_mask >> sp & 1u)) return false;
    return true;
  }
};

namespace {

// The system's recount goes through the bins whenever its grid has them.
int32_t launch_hist_sys(soma_system *sys, hipStream_t s) {
  soma::BinArgs b;
  if (sys->d.bins_ok) b = sys->bins();
  return launch_hist(&sys->cfg, sys->d, sys->buf.pos, sys->buf.counts, s,
                     sys->d.bins_ok ? &b : nullptr);
}

// The mixed kernel's LDS tiles are laid out for four waves: it always runs
// 256-thread blocks; the others take `threads` (64..512).
template <bool C64, bool V2, bool B, bool P>
void launch_sweep_p(uint32_t kind, dim3 grid, dim3 threads, hipStream_t s,
                    const soma::SweepArgs &a, const soma::MixArgs &mx) {
  if (kind == SOMA_MOVE_MIXED)
    hipLaunchKernelGGL((soma::mc_sweep_mixed_kernel<C64, V2, B, P>), grid, dim3(256), 0, s, a, mx);
  else if (kind == SOMA_MOVE_SMC)
    hipLaunchKernelGGL((soma::mc_sweep_smc_kernel<C64, V2, B, P>), grid, threads, 0, s, a);
  else if (kind == SOMA_MOVE_GIBBS)
    hipLaunchKernelGGL((soma::mc_sweep_gibbs_kernel<C64, V2, B, P>), grid, threads, 0, s, a);
  else if (B && a.stream_pos)   // measured: no gain with direct atomics
    hipLaunchKernelGGL((soma::mc_sweep_local_kernel<C64, V2, B, P, true>), grid, threads, 0, s, a);
  else
    hipLaunchKernelGGL((soma::mc_sweep_local_kernel<C64, V2, B, P>), grid, threads, 0, s, a);
}

// The mixed kernel's LDS tiles are laid out for four waves: it always runs
// 256-thread blocks; the others take `threads` (64..512).  A set queue
// selects the persistent instance.
template <bool C64, bool V2, bool B>
void launch_sweep_t(uint32_t kind, dim3 grid, dim3 threads, hipStream_t s,
                    const soma::SweepArgs &a, const soma::MixArgs &mx) {
  if (a.queue) launch_sweep_p<C64, V2, B, true>(kind, grid, threads, s, a, mx);
  else launch_sweep_p<C64, V2, B, false>(kind, grid, threads, s, a, mx);
}

// Blocks of a SET sweep kernel (local, smart-MC, bond-Gibbs or mixed; the
// persistent 8-byte-pair instance that the full-size melts use) that the whole device
// holds at once at `threads` per block: occupancy of the kernel's registers
// and LDS times the compute units, the persistent grid whose waves all start
// together.  0 if the runtime cannot tell.
template <bool C64, bool B>
uint32_t resident_blocks_t(uint32_t kind, uint32_t threads) {
  int per_cu = 0, dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0u;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 0u;
  const void *f = kind == SOMA_MOVE_MIXED
                      ? reinterpret_cast<const void *>(&soma::mc_sweep_mixed_kernel<C64, true, B, true>)
                  : kind == SOMA_MOVE_SMC
                      ? reinterpret_cast<const void *>(&soma::mc_sweep_smc_kernel<C64, true, B, true>)
                  : kind == SOMA_MOVE_GIBBS
                      ? reinterpret_cast<const void *>(&soma::mc_sweep_gibbs_kernel<C64, true, B, true>)
                      : reinterpret_cast<const void *>(&soma::mc_sweep_local_kernel<C64, true, B, true>);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, f, (int)threads, 0) != hipSuccess)
    return 0u;
  return per_cu > 0 && cus > 0 ? (uint32_t)per_cu * (uint32_t)cus : 0u;
}

uint32_t resident_blocks(uint32_t kind, bool c64, bool binned, uint32_t threads) {
  if (c64) return binned ? resident_blocks_t<true, true>(kind, threads)
                         : resident_blocks_t<true, false>(kind, threads);
  return binned ? resident_blocks_t<false, true>(kind, threads)
                : resident_blocks_t<false, false>(kind, threads);
}

template <bool C64, bool V2>
void launch_sweep_b(bool binned, uint32_t kind, dim3 grid, dim3 threads, hipStream_t s,
                    const soma::SweepArgs &a, const soma::MixArgs &mx) {
  if (binned) launch_sweep_t<C64, V2, true>(kind, grid, threads, s, a, mx);
  else launch_sweep_t<C64, V2, false>(kind, grid, threads, s, a, mx);
}

// Adds the binned count updates of the sweeps before it to the counts (one
// workgroup per brick; the SET sweep kernels bin updates of types 0 and 1
// only, which live in count plane 0).
int32_t launch_bin_apply(soma_system *sys, hipStream_t s) {
  const soma::BinArgs b = sys->bins();
  const bool c64 = sys->cfg.count_width == 32;
  const uint32_t planes = 1u;
  const size_t lds = (size_t)planes * soma::kBrickCells * (c64 ? 8u : 4u);
  const dim3 grid((uint32_t)sys->d.n_bricks), block(soma::kApplyThreads);
  if (c64)
    hipLaunchKernelGGL(soma::bin_apply_kernel<true>, grid, block, lds, s, b, sys->grid,
                       sys->buf.counts, planes);
  else
    hipLaunchKernelGGL(soma::bin_apply_kernel<false>, grid, block, lds, s, b, sys->grid,
                       sys->buf.counts, planes);
  LAUNCH_TRY();
  return SOMA_OK;
}

// The second difference of the grid Hamiltonian per bead and cell, in kT:
// moving one bead from cell c to c' changes H_nb by (omega(c') - omega(c))/N
// plus this (the bead no longer counts in c and now counts in c').  K^1 form:
// kappaN / (N rho); K^0 form: (kappaN - chiN/2) / (N rho).
float self_energy(const soma_system *sys) {
  const double inv_rho = inv_rho_d(sys->d);
  const double k = sys->d.form == 0 ? (double)sys->cfg.kappa_n - 0.5 * (double)sys->cfg.chi_n
                                    : (double)sys->cfg.kappa_n;
  return (float)(k * inv_rho / (double)sys->cfg.n_ref);
}

// Arguments of species sp's sweep of kind `kind` (sweep offset 0).
void sweep_args(soma_system *sys, uint32_t sp, uint32_t kind, soma::SweepArgs &a,
                soma::MixArgs &mx) {
  const soma_config *c = &sys->cfg;
  const soma_species &S = c->species[sp];
  a.pos = sys->buf.pos + 3 * sys->d.bead_off[sp];
  a.omega = sys->buf.omega;
  a.counts = sys->buf.counts;
  // accepted-move counters: local (and the local part of mixed sweeps), smart MC,
  // learned, bond-Gibbs
  a.acc_slots = sys->acc() + (kind == SOMA_MOVE_SMC ? soma::kAccSlots
                              : kind == SOMA_MOVE_GIBBS ? 3u * soma::kAccSlots : 0u);
  a.grid = sys->grid;
  a.n_chains = S.n_chains;
  a.n = S.n;
  a.n_a = S.n_a;
  a.lanes_per_chain = (S.n + 1) / 2;
  a.chains_per_wave = 64u / a.lanes_per_chain;
  a.lpc_magic = (65536u + a.lanes_per_chain - 1u) / a.lanes_per_chain;
  a.chain_base = (uint32_t)sys->d.chain_off[sp];
  a.k0 = S.k0;
  a.half_k0 = 0.5f * S.k0;
  a.step = kind == SOMA_MOVE_SMC ? c->smc_a : c->local_a;  // mixed: local half-width
  a.sqrt_2a = (float)std::sqrt(2.0 * (double)c->smc_a);
  a.inv_4a = c->smc_a > 0.f ? (float)(1.0 / (4.0 * (double)c->smc_a)) : 0.f;
  a.inv_nref = (float)(1.0 / (double)c->n_ref);
  a.seed_lo = (uint32_t)c->seed;
  a.seed_hi = (uint32_t)(c->seed >> 32);
  a.sweep = 0;
  a.replica = c->replica;
  a.set_order = c->set_order;
  a.sweep_ctr = sys->sweep_ctr();
  a.sub_k = 1;
  a.sub_j = 0;
  a.n_sub = S.n_chains;
  a.grad = sys->grad;
  a.forbid = sys->d.forbid;
  a.gibbs_s2 = (float)(1.0 / std::sqrt(2.0 * (double)S.k0));
  a.gibbs_s1 = (float)(1.0 / std::sqrt((double)S.k0));
  a.bin = sys->d.bins_ok ? sys->bins() : soma::BinArgs{};
  a.self_term = sys->self_term ? self_energy(sys) : 0.0f;
  a.queue = nullptr;   // set by launch_sweep for persistent local grids
  a.wpb = 4u;          // 256-thread blocks unless launch_sweep picks another size
  // positions larger than the last-level cache (256 MB) stream past it
  a.stream_pos = 12ull * sys->d.n_beads > (256ull << 20) ? 1u : 0u;
  mx.net = sys->net(sp);
  mx.head.m_max = c->mu_max;
  mx.head.lo = c->log_sigma_min;
  mx.head.hi = c->log_sigma_max;
  mx.p_learn = c->p_learn;
  mx.att_slots = sys->att();
  mx.err = sys->err();
  mx.halo = sys->halo();
  mx.halo_plane = (uint32_t)sys->d.halo_plane;
}

bool species_vec2(const soma_system *sys, uint32_t sp) {
  const uint64_t off = sys->d.bead_off[sp];
  return (sys->cfg.species[sp].n % 2 == 0) && (off % 2 == 0) &&
         aligned(sys->buf.pos + 3 * off, 8);
}

// Chains sub_j, sub_j + sub_k, ... of a species of n chains.
uint32_t subset_size(uint32_t n, uint32_t k, uint32_t j) { return n > j ? (n - j + k - 1) / k : 0u; }

// One sweep of chain subset j of k of every species (k = 1: all chains); `off`
// is added to the device sweep counter.
int32_t launch_sweep(soma_system *sys, uint32_t kind, hipStream_t s, uint32_t off,
                     uint32_t k = 1, uint32_t j = 0) {
  const soma_config *c = &sys->cfg;
  const bool binned = sys->hist_mode == soma::kHistBinned;
  bool any_binned = false;
  for (uint32_t sp = 0; sp < c->n_species; ++sp) {
    const soma_species &S = c->species[sp];
    if (!S.n_chains) continue;
    soma::SweepArgs a;
    soma::MixArgs mx;
    sweep_args(sys, sp, kind, a, mx);
    a.sweep = off;
    a.sub_k = k;
    a.sub_j = j;
    a.n_sub = subset_size(S.n_chains, k, j);
    if (a.n_sub == 0) continue;
    const bool c64 = c->count_width == 32;
    if (sys->d.arch[sp]) {   // general architecture: per_wave molecules per wave (local moves, SET)
      const uint32_t per_block = 4u * sys->arch_per_wave[sp];
      const dim3 grid((a.n_sub + per_block - 1u) / per_block);
      if (c64) hipLaunchKernelGGL(soma::mc_sweep_arch_kernel<true>, grid, dim3(256), 0, s, a, sys->d.arch[sp]);
      else hipLaunchKernelGGL(soma::mc_sweep_arch_kernel<false>, grid, dim3(256), 0, s, a, sys->d.arch[sp]);
      LAUNCH_TRY();
      continue;
    }
    if (kind == SOMA_MOVE_LOCAL && sys->scheme == SOMA_SCHEME_MOLECULE) {
      uint32_t blocks = (a.n_sub + 255u) / 256u;   // one lane per chain
      if (sys->sweep_blocks && sys->sweep_blocks < blocks) blocks = sys->sweep_blocks;
      const dim3 grid(blocks);
      if (c64) hipLaunchKernelGGL(soma::mc_sweep_molecule_kernel<true>, grid, dim3(256), 0, s, a);
      else hipLaunchKernelGGL(soma::mc_sweep_molecule_kernel<false>, grid, dim3(256), 0, s, a);
      LAUNCH_TRY();
      continue;
    }
    const uint32_t threads = kind == SOMA_MOVE_MIXED ? 256u : sys->sweep_threads;
    a.wpb = threads / 64u;
    const uint64_t chains_per_block = (uint64_t)(threads / 64u) * a.chains_per_wave;
    uint64_t blocks = (a.n_sub + chains_per_block - 1) / chains_per_block;
    if (sys->sweep_blocks && sys->sweep_blocks < blocks) {
      blocks = sys->sweep_blocks;   // persistent: tiles from counters zeroed here
      a.queue = reinterpret_cast<uint32_t *>(sys->ws + sys->d.off_queue);
      hipLaunchKernelGGL(soma::queue_reset_kernel, dim3(1), dim3(256), 0, s, a.queue);
      LAUNCH_TRY();
    }
    const bool v2 = species_vec2(sys, sp);
    const dim3 grid((uint32_t)blocks), block(threads);
    if (c64) {
      if (v2) launch_sweep_b<true, true>(binned, kind, grid, block, s, a, mx);
      else launch_sweep_b<true, false>(binned, kind, grid, block, s, a, mx);
    } else {
      if (v2) launch_sweep_b<false, true>(binned, kind, grid, block, s, a, mx);
      else launch_sweep_b<false, false>(binned, kind, grid, block, s, a, mx);
    }
    LAUNCH_TRY();
    any_binned |= binned;
  }
  if (any_binned) return launch_bin_apply(sys, s);
  return SOMA_OK;
}

int32_t launch_counter(uint32_t *ctr, uint32_t by, uint32_t set, uint32_t value, hipStream_t s) {
  hipLaunchKernelGGL(soma::sweep_counter_one_kernel, dim3(1), dim3(64), 0, s, ctr, by, set, value);
  LAUNCH_TRY();
  return SOMA_OK;
}

int32_t check_kind(soma_system *sys, uint32_t move_kind) {
  if (move_kind != SOMA_MOVE_LOCAL && move_kind != SOMA_MOVE_SMC && move_kind != SOMA_MOVE_MIXED &&
      move_kind != SOMA_MOVE_GIBBS)
    return fail(SOMA_E_UNSUPPORTED, "move kind %u", move_kind);
  if (move_kind == SOMA_MOVE_MIXED && sys->cfg.p_learn > 0.f && !sys->nets_ready())
    return fail(SOMA_E_INVAL, "mixed moves need a network for every species (soma_set_proposal)");
  if (move_kind == SOMA_MOVE_SMC && !(sys->cfg.smc_a > 0.f))
    return fail(SOMA_E_INVAL, "smart-MC moves need smc_a > 0");
  if ((move_kind == SOMA_MOVE_LOCAL || move_kind == SOMA_MOVE_MIXED) && !(sys->cfg.local_a < 1.f))
    return fail(SOMA_E_UNSUPPORTED, "local moves need a half-width below one cell");
  if (move_kind != SOMA_MOVE_LOCAL && sys->scheme != SOMA_SCHEME_SET)
    return fail(SOMA_E_UNSUPPORTED, "the molecule-parallel order has local moves only");
  if (sys->arch_mask && (move_kind != SOMA_MOVE_LOCAL || sys->scheme != SOMA_SCHEME_SET))
    return fail(SOMA_E_UNSUPPORTED, "general architectures have local moves in the SET order only");
  if (sys->d.n_types > 2 && move_kind != SOMA_MOVE_LOCAL)
    return fail(SOMA_E_UNSUPPORTED, "more than two bead types: local moves only");
  if (sys->self_term && (sys->scheme != SOMA_SCHEME_SET || sys->arch_mask || sys->d.n_types > 2))
    return fail(SOMA_E_UNSUPPORTED, "the self term: linear chains of two types, SET order");
  return SOMA_OK;
}

int32_t launch_grad(soma_system *sys, hipStream_t s) {
  const uint32_t n = 2u * (uint32_t)sys->d.n_cells;
  hipLaunchKernelGGL(soma::grad_field_kernel, dim3((n + 255) / 256), dim3(256), 0, s,
                     sys->buf.omega, sys->grad, sys->grid);
  LAUNCH_TRY();
  return SOMA_OK;
}

// Stage 1 of the cycle: fields from the counts, then the gradient field if kept.
int32_t refresh_fields(soma_system *sys, hipStream_t s) {
  int32_t r = launch_field(&sys->cfg, sys->d, sys->buf.counts, sys->buf.omega, sys->fpart(), s,
                           sys->halo());
  if (!r && sys->grad) r = launch_grad(sys, s);
  return r;
}

// One SCMF cycle with sweep offset `off`: for each of the system's k chain
// subsets, its sweep and then the field refresh (k = 1: sweep, refresh).
int32_t enqueue_cycle(soma_system *sys, uint32_t kind, hipStream_t s, uint32_t off) {
  const uint32_t k = sys->substeps;
  for (uint32_t j = 0; j < k; ++j) {
    int32_t r = launch_sweep(sys, kind, s, off, k, j);
    if (!r) r = refresh_fields(sys, s);
    if (r) return r;
  }
  return SOMA_OK;
}

// Records what `enqueue(stream)` launches into a graph and instantiates it.
// Capture runs on a private stream, so nothing executes while recording.
template <class F>
int32_t capture_graph(CycleGraph &g, uint32_t cycles, uint32_t kind, F enqueue) {
  hipStream_t cs = nullptr;
  HIP_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) {
    (void)hipStreamDestroy(cs);
    return fail(SOMA_E_HIP, "hipStreamBeginCapture: %s", hipGetErrorString(e));
  }
  const int32_t rc = enqueue(cs);
  hipGraph_t graph = nullptr;
  e = hipStreamEndCapture(cs, &graph);
  (void)hipStreamDestroy(cs);
  if (rc || e != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    if (rc) return rc;
    return fail(SOMA_E_HIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
  }
  hipGraphExec_t exec = nullptr;
  e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(graph);
    return fail(SOMA_E_HIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
  }
  g.release();
  g.graph = graph;
  g.exec = exec;
  g.cycles = cycles;
  g.kind = kind;
  return SOMA_OK;
}

int32_t check_buffers(const Derived &d, const soma_buffers *b) {
  if (!b) return fail(SOMA_E_INVAL, "buffers is NULL");
  if (!b->pos || !b->counts || !b->omega || !b->workspace)
    return fail(SOMA_E_INVAL, "a buffer pointer is NULL");
  if (b->pos_bytes < d.pos_bytes) return fail(SOMA_E_SIZE, "positions: %llu < %llu bytes",
                                              (unsigned long long)b->pos_bytes, (unsigned long long)d.pos_bytes);
  if (b->counts_bytes < d.counts_bytes) return fail(SOMA_E_SIZE, "counts: %llu < %llu bytes",
                                                    (unsigned long long)b->counts_bytes, (unsigned long long)d.counts_bytes);
  if (b->omega_bytes < d.omega_bytes) return fail(SOMA_E_SIZE, "omega: %llu < %llu bytes",
                                                  (unsigned long long)b->omega_bytes, (unsigned long long)d.omega_bytes);
  if (b->workspace_bytes < d.ws_bytes) return fail(SOMA_E_SIZE, "workspace: %llu < %llu bytes",
                                                   (unsigned long long)b->workspace_bytes, (unsigned long long)d.ws_bytes);
  if (!aligned(b->pos, 4) || !aligned(b->counts, 16) || !aligned(b->omega, 16) ||
      !aligned(b->workspace, 256))
    return fail(SOMA_E_INVAL, "alignment: pos 4, counts 16, omega 16, workspace 256 bytes");
  return SOMA_OK;
}

}  // namespace

extern "C" {

const char *soma_last_error(void) { return g_err; }

int32_t soma_buffer_sizes(const soma_config *cfg, uint64_t *pos_bytes, uint64_t *counts_bytes,
                          uint64_t *omega_bytes, uint64_t *workspace_bytes) {
  Derived d;
  const int32_t rc = derive(cfg, &d);
  if (rc) return rc;
  if (pos_bytes) *pos_bytes = d.pos_bytes;
  if (counts_bytes) *counts_bytes = d.counts_bytes;
  if (omega_bytes) *omega_bytes = d.omega_bytes;
  if (workspace_bytes) *workspace_bytes = d.ws_bytes;
  return SOMA_OK;
}

int32_t soma_workspace_size(const soma_config *cfg, uint64_t *bytes) {
  if (!bytes) return fail(SOMA_E_INVAL, "bytes is NULL");
  return soma_buffer_sizes(cfg, nullptr, nullptr, nullptr, bytes);
}

int32_t soma_init_system(const soma_config *cfg, const soma_buffers *buf, uint32_t init_positions,
                         void *stream, soma_system **out) {
  if (!out) return fail(SOMA_E_INVAL, "out is NULL");
  *out = nullptr;
  Derived d;
  int32_t rc = derive(cfg, &d);
  if (rc) return rc;
  rc = check_buffers(d, buf);
  if (rc) return rc;
  soma_system *sys = new (std::nothrow) soma_system();
  if (!sys) return fail(SOMA_E_INVAL, "out of host memory");
  sys->cfg = *cfg;
  sys->buf = *buf;
  sys->d = d;
  sys->grid = make_grid(cfg, d.n_cells);
  sys->ws = reinterpret_cast<unsigned char *>(buf->workspace);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  rc = launch_zero(sys->ws, d.ws_bytes, s);
  if (!rc && init_positions) rc = launch_init(cfg, d, buf->pos, s);
  if (!rc) rc = launch_hist_sys(sys, s);
  if (!rc) rc = launch_field(cfg, d, buf->counts, buf->omega, sys->fpart(), s, sys->halo());
  if (rc) {
    delete sys;
    return rc;
  }
  *out = sys;
  return SOMA_OK;
}

int32_t soma_mc_sweep(soma_system *sys, uint32_t n_sweeps, uint32_t move_kind, void *stream) {
  if (!sys) return fail(SOMA_E_INVAL, "system is NULL");
  int32_t rc = check_kind(sys, move_kind);
  if (rc) return rc;
  if (n_sweeps == 0) return SOMA_OK;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  for (uint32_t i = 0; i < n_sweeps; ++i) {
    rc = launch_sweep(sys, move_kind, s, i);
    if (rc) return rc;
  }
  rc = launch_counter(sys->sweep_ctr(), n_sweeps, 0, 0, s);
  if (rc) return rc;
  sys->count_sweeps(move_kind, n_sweeps);
  return SOMA_OK;
}

int32_t soma_capture_cycle(soma_system *sys, uint32_t cycles, uint32_t move_kind) {
  if (!sys) return fail(SOMA_E_INVAL, "system is NULL");
  if (cycles == 0) return fail(SOMA_E_INVAL, "cycles must be positive");
  int32_t rc = check_kind(sys, move_kind);
  if (rc) return rc;
  return capture_graph(sys->graph, cycles, move_kind, [&](hipStream_t cs) -> int32_t {
    for (uint32_t i = 0; i < cycles; ++i) {
      const int32_t r = enqueue_cycle(sys, move_kind, cs, i);
      if (r) return r;
    }
    return launch_counter(sys->sweep_ctr(), cycles, 0, 0, cs);
  });
}

int32_t soma_set_substeps(soma_system *sys, uint32_t k) {
  if (!sys) return fail(SOMA_E_INVAL, "system is NULL");
  if (k == 0 || k > 4096) return fail(SOMA_E_INVAL, "substeps must be 1..4096");
  sys->substeps = k;
  return SOMA_OK;
}

int32_t soma_cycle(soma_system *sys, uint32_t n_cycles, uint32_t move_kind, void *stream) {
  if (!sys) return fail(SOMA_E_INVAL, "system is NULL");
  int32_t rc = check_kind(sys, move_kind);
  if (rc || n_cycles == 0) return rc;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  for (uint32_t i = 0; i < n_cycles; ++i) {
    rc = enqueue_cycle(sys, move_kind, s, i);
    if (rc) return rc;
  }
  rc = launch_counter(sys->sweep_ctr(), n_cycles, 0, 0, s);
  if (rc) return rc;
  sys->count_sweeps(move_kind, n_cycles);
  return SOMA_OK;
}

int32_t soma_run_cycle(soma_system *sys, uint32_t n_launches, void *stream) {
  if (!sys) return fail(SOMA_E_INVAL, "system is NULL");
  if (!sys->graph.exec) return fail(SOMA_E_INVAL, "no captured cycle (soma_capture_cycle)");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  for (uint32_t i = 0; i < n_launches; ++i) {
    HIP_TRY(hipGraphLaunch(sys->graph.exec, s));
    sys->count_sweeps(sys->graph.kind, sys->graph.cycles);
  }
  return SOMA_OK;
}

int32_t soma_set_scheme(soma_system *sys, uint32_t scheme) {
  if (!sys) return fail(SOMA_E_INVAL, "system is NULL");
  if (scheme != SOMA_SCHEME_SET && scheme != SOMA_SCHEME_MOLECULE)
    return fail(SOMA_E_INVAL, "scheme %u", scheme);
  sys->scheme = scheme;
  return SOMA_OK;
}

int32_t soma_set_histogram(soma_system *sys, uint32_t mode) {
  if (!sys) return fail(SOMA_E_INVAL, "system is NULL");
  if (mode != SOMA_HIST_DIRECT && mode != SOMA_HIST_BINNED)
    return fail(SOMA_E_INVAL, "histogram mode %u", mode);
  if (mode == SOMA_HIST_BINNED && !sys->d.bins_ok)
    return fail(SOMA_E_UNSUPPORTED, "binned count updates need fewer than 2^21 bricks of 16x16x8 cells");
  sys->hist_mode = mode == SOMA_HIST_BINNED ? soma::kHistBinned : soma::kHistDirect;
  return SOMA_OK;
}

int32_t soma_set_self_term(soma_system *sys, uint32_t on) {
  if (!sys) return fail(SOMA_E_INVAL, "system is NULL");
  if (on > 1) return fail(SOMA_E_INVAL, "self term: 0 or 1");
  if (on && (sys->d.n_types > 2 || sys->arch_mask || sys->scheme != SOMA_SCHEME_SET))
    return fail(SOMA_E_UNSUPPORTED, "the self term: linear chains of two types, SET order");
  sys->self_term = on;
  return SOMA_OK;
}

int32_t soma_probe_atomics(uint32_t *words, uint64_t n_words, uint64_t n_updates,
                           uint32_t mode, uint32_t seed, void *stream) {
  if (!words || n_words == 0) return fail(SOMA_E_INVAL, "empty word array");
  if (mode > 2) return fail(SOMA_E_INVAL, "probe mode %u", mode);
  if (n_updates == 0) return SOMA_OK;
  if (!aligned(words, 4)) return fail(SOMA_E_INVAL, "words must be 4-byte aligned");
  const uint64_t blocks = (n_updates + 255) / 256;
  if (blocks >= (1ull << 31)) return fail(SOMA_E_UNSUPPORTED, "too many updates");
  hipLaunchKernelGGL(soma::probe_atomics_kernel, dim3((uint32_t)blocks), dim3(256), 0,
                     reinterpret_cast<hipStream_t>(stream), words, n_words, n_updates, mode, seed);
  LAUNCH_TRY();
  return SOMA_OK;
}

int32_t soma_set_sweep_blocks(soma_system *sys, uint32_t blocks) {
  if (!sys) return fail(SOMA_E_INVAL, "system is NULL");
  sys->sweep_blocks = blocks;
  return SOMA_OK;
}

int32_t soma_set_sweep_threads(soma_system *sys, uint32_t threads) {
  if (!sys) return fail(SOMA_E_INVAL, "system is NULL");
  if (threads < 64 || threads > 512 || threads % 64)
    return fail(SOMA_E_INVAL, "sweep threads must be 64, 128, ..., 512");
  sys->sweep_threads = threads;
  return SOMA_OK;
}

int32_t soma_rebuild_histogram(soma_system *sys, void *stream) {
  if (!sys) return fail(SOMA_E_INVAL, "system is NULL");
  return launch_hist_sys(sys, reinterpret_cast<hipStream_t>(stream));
}

int32_t soma_update_fields(soma_system *sys, void *stream) {
  if (!sys) return fail(SOMA_E_INVAL, "system is NULL");
  return refresh_fields(sys, reinterpret_cast<hipStream_t>(stream));
}

int32_t soma_sync_fields(soma_system *sys, void *stream) {
  if (!sys) return fail(SOMA_E_INVAL, "system is NULL");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (sys->halo()) {
    const soma::FieldArgs a = field_args(&sys->cfg, sys->d, sys->buf.counts, sys->buf.omega,
                                         nullptr, sys->halo());
    hipLaunchKernelGGL(soma::halo_from_fields_kernel, dim3((uint32_t)((sys->d.n_cells + 255) / 256)),
                       dim3(256), 0, s, a);
    LAUNCH_TRY();
  }
  if (sys->grad) return launch_grad(sys, s);
  return SOMA_OK;
}

int32_t soma_set_grad_field(soma_system *sys, void *grad, uint64_t grad_bytes, void *stream) {
  if (!sys) return fail(SOMA_E_INVAL, "system is NULL");
  if (grad && sys->d.n_types > 2)
    return fail(SOMA_E_UNSUPPORTED, "gradient field with two bead types only");
  if (!grad) {
    sys->grad = nullptr;
    return SOMA_OK;
  }
  const uint64_t need = 32ull * sys->d.n_cells;
  if (grad_bytes < need)
    return fail(SOMA_E_SIZE, "gradient field: %llu < %llu bytes", (unsigned long long)grad_bytes,
                (unsigned long long)need);
  if (!aligned(grad, 16)) return fail(SOMA_E_INVAL, "gradient field must be 16-byte aligned");
  sys->grad = reinterpret_cast<float4 *>(grad);
  return launch_grad(sys, reinterpret_cast<hipStream_t>(stream));
}

int32_t soma_set_hamiltonian(soma_system *sys, uint32_t form, void *stream) {
  if (!sys) return fail(SOMA_E_INVAL, "system is NULL");
  if (form > 1) return fail(SOMA_E_INVAL, "Hamiltonian form %u", form);
  sys->d.form = form;
  sys->graph.release();   // captured launches hold the old arguments
  return refresh_fields(sys, reinterpret_cast<hipStream_t>(stream));
}

int32_t soma_set_external(soma_system *sys, const float *ext, uint64_t ext_bytes,
                          const uint32_t *forbid, uint64_t forbid_bytes, void *stream) {
  if (!sys) return fail(SOMA_E_INVAL, "system is NULL");
  if (sys->d.n_types > 2 && (ext || forbid))
    return fail(SOMA_E_UNSUPPORTED, "external fields with two bead types only");
  const uint64_t n_cells = sys->d.n_cells;
  if (ext && ext_bytes < 8ull * n_cells)
    return fail(SOMA_E_SIZE, "external field: %llu < %llu bytes", (unsigned long long)ext_bytes,
                (unsigned long long)(8ull * n_cells));
  if (ext && !aligned(ext, 4)) return fail(SOMA_E_INVAL, "external field must be 4-byte aligned");
  const uint64_t words = (n_cells + 31) / 32;
  uint64_t n_free = n_cells;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (forbid) {
    if (forbid_bytes < 4ull * words)
      return fail(SOMA_E_SIZE, "impenetrable-cell mask: %llu < %llu bytes",
                  (unsigned long long)forbid_bytes, (unsigned long long)(4ull * words));
    if (!aligned(forbid, 4)) return fail(SOMA_E_INVAL, "mask must be 4-byte aligned");
    std::vector<uint32_t> h(words);
    HIP_TRY(hipMemcpyAsync(h.data(), forbid, 4ull * words, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    uint64_t blocked = 0;
    for (uint64_t w = 0; w < words; ++w) {
      uint32_t v = h[w];
      if (w == words - 1 && (n_cells & 31u)) v &= (1u << (n_cells & 31u)) - 1u;  // bits past the grid
      blocked += (uint64_t)__builtin_popcount(v);
    }
    if (blocked >= n_cells) return fail(SOMA_E_INVAL, "every cell is impenetrable");
    n_free = n_cells - blocked;
  }
  sys->d.ext = ext;
  sys->d.forbid = forbid;
  sys->d.n_free = n_free;
  sys->graph.release();   // captured launches hold the old arguments
  const int32_t rc = refresh_fields(sys, s);
  if (rc) return rc;
  HIP_TRY(hipStreamSynchronize(s));
  return SOMA_OK;
}

}  // extern "C"

namespace {

// Decodes a 32-bit architecture array (Sec. 3.2.1) into the device table:
// types, bond lists and the greedy independent sets (monomer i joins the
// lowest set not holding a bonded monomer of lower index).  Returns 0 or a
// message naming the first defect.
const char *decode_architecture(const uint32_t *w, uint32_t n_words, uint32_t n_expected,
                                uint32_t n_types, soma::ArchDev &t) {
  std::memset(&t, 0, sizeof t);
  if (n_words < 1) return "empty array";
  const uint32_t n = w[0];
  if (n != n_expected) return "N differs from the species' chain length";
  if (n == 0 || n > soma::kArchMaxN || n_words < 1 + n) return "N out of range or array too short";
  t.n = n;
  std::vector<std::vector<uint32_t>> nbrs(n);
  for (uint32_t i = 0; i < n; ++i) {
    const uint32_t m = w[1 + i];
    const uint32_t type = m >> 24;
    if (type >= n_types) return "monomer type code not below the number of types";
    t.type[i] = (uint8_t)type;
    if (type == 0) ++t.n_type0;
    uint32_t k = m & 0xFFFFFFu;
    if (k == 0) continue;   // no bonds
    while (true) {
      if (k >= n_words) return "bond list runs off the array";
      const uint32_t b = w[k++];
      const int32_t off = (int32_t)(b << 5) >> 5;
      if ((b >> 27) & 0xFu) return "bond type other than harmonic";
      const int64_t j = (int64_t)i + off;
      if (off == 0 || j < 0 || j >= (int64_t)n) return "bond partner out of range";
      nbrs[i].push_back((uint32_t)j);
      if (b >> 31) break;
    }
  }
  uint32_t n_nb = 0;
  for (uint32_t i = 0; i < n; ++i) {
    for (uint32_t j : nbrs[i])
      if (std::find(nbrs[j].begin(), nbrs[j].end(), i) == nbrs[j].end())
        return "bond listed at one end only";
    t.nb_start[i] = (uint16_t)n_nb;
    for (uint32_t j : nbrs[i]) {
      if (n_nb >= soma::kArchMaxBonds) return "too many bonds";
      t.nb[n_nb++] = (uint8_t)j;
    }
  }
  t.nb_start[n] = (uint16_t)n_nb;
  std::vector<uint32_t> set(n, 0);
  uint32_t k = 0;
  for (uint32_t i = 0; i < n; ++i) {
    uint32_t used = 0;
    for (uint32_t j : nbrs[i])
      if (j < i) used |= 1u << set[j];
    uint32_t c = 0;
    while (used >> c & 1u) ++c;
    if (c >= soma::kArchMaxSets) return "more than 16 independent sets";
    set[i] = c;
    k = std::max(k, c + 1);
  }
  t.n_sets = k;
  uint32_t pos = 0;
  for (uint32_t c = 0; c < k; ++c) {
    t.set_start[c] = (uint16_t)pos;
    for (uint32_t i = 0; i < n; ++i)
      if (set[i] == c) t.member[pos++] = (uint8_t)i;
  }
  t.set_start[k] = (uint16_t)pos;
  uint32_t largest = 1;
  for (uint32_t c = 0; c < k; ++c) largest = std::max<uint32_t>(largest, t.set_start[c + 1] - t.set_start[c]);
  t.per_wave = std::max(1u, std::min(64u / largest, soma::kArchMaxN / n));
  return nullptr;
}

}  // namespace

extern "C" {

int32_t soma_set_architecture(soma_system *sys, uint32_t species, const uint32_t *words,
                              uint32_t n_words, void *stream) {
  if (!sys) return fail(SOMA_E_INVAL, "system is NULL");
  if (species >= sys->cfg.n_species) return fail(SOMA_E_INVAL, "species %u", species);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const soma_species &S = sys->cfg.species[species];
  if (words) {
    soma::ArchDev t;
    const char *err = decode_architecture(words, n_words, S.n, sys->d.n_types, t);
    if (err) return fail(SOMA_E_INVAL, "architecture of species %u: %s", species, err);
    HIP_TRY(hipMemcpyAsync(sys->arch(species), &t, sizeof t, hipMemcpyHostToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
    sys->arch_mask |= 1u << species;
    sys->arch_type0[species] = t.n_type0;
    sys->arch_per_wave[species] = t.per_wave;
    sys->arch_max_type[species] = *std::max_element(t.type, t.type + t.n);
    sys->d.arch[species] = sys->arch(species);
  } else {
    sys->arch_mask &= ~(1u << species);
    sys->d.arch[species] = nullptr;
  }
  // expected A count for the conservation check
  uint64_t n_a = 0;
  for (uint32_t sp = 0; sp < sys->cfg.n_species; ++sp) {
    const soma_species &X = sys->cfg.species[sp];
    n_a += (uint64_t)X.n_chains * ((sys->arch_mask >> sp & 1u) ? sys->arch_type0[sp] : X.n_a);
  }
  sys->d.n_a_total = n_a;
  sys->graph.release();
  int32_t rc = launch_hist_sys(sys, s);
  if (!rc) rc = refresh_fields(sys, s);
  if (rc) return rc;
  HIP_TRY(hipStreamSynchronize(s));
  return SOMA_OK;
}

int32_t soma_set_types(soma_system *sys, uint32_t n_types, const float *chi_n, void *counts,
                       uint64_t counts_bytes, float *omega, uint64_t omega_bytes, void *stream) {
  if (!sys) return fail(SOMA_E_INVAL, "system is NULL");
  if (n_types < 2 || n_types > soma::kMaxTypes)
    return fail(SOMA_E_INVAL, "n_types must be in 2..%u", soma::kMaxTypes);
  if (!chi_n || !counts || !omega) return fail(SOMA_E_INVAL, "chi_n, counts and omega are required");
  for (uint32_t i = 0; i < n_types; ++i)
    for (uint32_t j = 0; j < n_types; ++j) {
      const float x = chi_n[i * n_types + j], y = chi_n[j * n_types + i];
      if (!std::isfinite(x)) return fail(SOMA_E_INVAL, "chi_n[%u][%u] is not finite", i, j);
      if (x != y) return fail(SOMA_E_INVAL, "chi_n is not symmetric at (%u, %u)", i, j);
    }
  const uint64_t n_cells = sys->d.n_cells, word = sys->cfg.count_width == 32 ? 8u : 4u;
  const uint64_t planes = (n_types + 1) / 2;
  // count and field planes are addressed with 32-bit byte offsets
  if (planes * n_cells * word >= (1ull << 32) || 4ull * n_types * n_cells >= (1ull << 32))
    return fail(SOMA_E_UNSUPPORTED, "%u types on %llu cells exceed 32-bit plane offsets", n_types,
                (unsigned long long)n_cells);
  if (counts_bytes < planes * n_cells * word)
    return fail(SOMA_E_SIZE, "counts: %llu < %llu bytes", (unsigned long long)counts_bytes,
                (unsigned long long)(planes * n_cells * word));
  if (omega_bytes < 4ull * n_types * n_cells)
    return fail(SOMA_E_SIZE, "omega: %llu < %llu bytes", (unsigned long long)omega_bytes,
                (unsigned long long)(4ull * n_types * n_cells));
  if (!aligned(counts, 16) || !aligned(omega, 16))
    return fail(SOMA_E_INVAL, "counts and omega must be 16-byte aligned");
  if (n_types > 2 && (sys->d.ext || sys->d.forbid))
    return fail(SOMA_E_UNSUPPORTED, "external fields with two bead types only");
  if (n_types > 2 && sys->grad)
    return fail(SOMA_E_UNSUPPORTED, "gradient field with two bead types only");
  for (uint32_t sp = 0; sp < sys->cfg.n_species; ++sp)
    if ((sys->arch_mask >> sp & 1u) && sys->arch_max_type[sp] >= n_types)
      return fail(SOMA_E_INVAL, "species %u has monomers of type %u", sp, sys->arch_max_type[sp]);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  sys->d.n_types = n_types;
  std::memset(sys->d.chi_m, 0, sizeof sys->d.chi_m);
  for (uint32_t i = 0; i < n_types; ++i)
    for (uint32_t j = 0; j < n_types; ++j)
      sys->d.chi_m[i * soma::kMaxTypes + j] = i == j ? 0.f : chi_n[i * n_types + j];
  if (n_types == 2) sys->cfg.chi_n = chi_n[1];
  sys->buf.counts = counts;
  sys->buf.counts_bytes = counts_bytes;
  sys->buf.omega = omega;
  sys->buf.omega_bytes = omega_bytes;
  sys->d.counts_bytes = planes * n_cells * word;
  sys->d.omega_bytes = 4ull * n_types * n_cells;
  sys->graph.release();   // captured launches hold the old buffers
  int32_t rc = launch_hist_sys(sys, s);
  if (!rc) rc = refresh_fields(sys, s);
  if (rc) return rc;
  HIP_TRY(hipStreamSynchronize(s));
  return SOMA_OK;
}

int32_t soma_type_counts(soma_system *sys, uint64_t *out, uint32_t n_out, void *stream) {
  if (!sys || !out) return fail(SOMA_E_INVAL, "system or out is NULL");
  if (n_out < sys->d.n_types) return fail(SOMA_E_SIZE, "out holds %u < %u types", n_out, sys->d.n_types);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const uint32_t blocks = sys->d.field_blocks;
  unsigned long long *part = reinterpret_cast<unsigned long long *>(sys->ws + sys->d.off_tcount);
  if (sys->cfg.count_width == 32)
    hipLaunchKernelGGL(soma::type_count_kernel<true>, dim3(blocks), dim3(256), 0, s,
                       sys->buf.counts, (uint32_t)sys->d.n_cells, sys->d.n_types, part);
  else
    hipLaunchKernelGGL(soma::type_count_kernel<false>, dim3(blocks), dim3(256), 0, s,
                       sys->buf.counts, (uint32_t)sys->d.n_cells, sys->d.n_types, part);
  LAUNCH_TRY();
  std::vector<unsigned long long> h((size_t)blocks * soma::kMaxTypes);
  HIP_TRY(hipMemcpyAsync(h.data(), part, 8ull * h.size(), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  for (uint32_t t = 0; t < n_out; ++t) out[t] = 0;
  for (uint32_t b = 0; b < blocks; ++b)
    for (uint32_t t = 0; t < sys->d.n_types; ++t) out[t] += h[(size_t)b * soma::kMaxTypes + t];
  return SOMA_OK;
}

int32_t soma_observables(soma_system *sys, soma_obs *out, void *stream) {
  if (!sys || !out) return fail(SOMA_E_INVAL, "system or out is NULL");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const soma_config *c = &sys->cfg;
  for (uint32_t sp = 0; sp < c->n_species; ++sp) {
    const soma_species &S = c->species[sp];
    if (!S.n_chains) continue;
    soma::ObsArgs a;
    a.pos = sys->buf.pos + 3 * sys->d.bead_off[sp];
    a.omega = sys->buf.omega;
    a.n_chains = S.n_chains;
    a.n = S.n;
    a.n_a = S.n_a;
    a.seg = 1;
    while (a.seg < S.n && a.seg < 64) a.seg <<= 1;
    a.inv_n = 1.0 / (double)S.n;
    a.half_k0 = 0.5 * (double)S.k0;
    a.inv_nref = 1.0 / (double)c->n_ref;
    a.grid = sys->grid;
    a.partials = sys->opart() + sys->d.obs_block_off[sp];
    a.arch = sys->d.arch[sp];
    a.err = sys->err();
    hipLaunchKernelGGL(soma::chain_obs_kernel, dim3((S.n_chains + 255) / 256), dim3(256), 0, s, a);
    LAUNCH_TRY();
  }
  hipLaunchKernelGGL(soma::reduce_totals_kernel, dim3(1), dim3(256), 0, s, sys->opart(),
                     (uint32_t)sys->d.obs_blocks, sys->fpart(), sys->d.field_blocks, sys->acc(),
                     sys->att(), sys->err(), sys->totals());
  LAUNCH_TRY();
  soma::Totals t;
  HIP_TRY(hipMemcpyAsync(&t, sys->totals(), sizeof t, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  std::memset(out, 0, sizeof *out);
  out->sweeps = sys->sweep;
  out->n_beads = sys->d.n_beads;
  out->n_chains = sys->d.n_chains;
  out->count_a = t.sum_a;
  out->count_b = t.sum_b;
  for (int k = 0; k < 4; ++k) out->accepted[k] = t.accepted[k];
  out->attempted[0] = sys->attempted[0] + (sys->mixed_moves - t.attempted_learned);
  out->attempted[1] = sys->attempted[1];
  out->attempted[2] = t.attempted_learned;
  out->attempted[3] = sys->attempted[3];
  out->re2_sum = t.re2;
  out->rg2_sum = t.rg2;
  out->b2_sum = t.b2;
  out->e_bond = t.e_bond;
  out->e_field = t.e_field;
  out->h_nb = t.h_nb / (inv_rho_d(sys->d) * (double)c->n_ref);
  out->error_flags = t.err;
  out->counts_conserved =
      (t.sum_a == sys->d.n_a_total && t.sum_b == sys->d.n_beads - sys->d.n_a_total) ? 1u : 0u;
  if (t.err) return fail(SOMA_E_DEVICE_FLAG, "device error word 0x%x", t.err);
  return SOMA_OK;
}

int32_t soma_check(soma_system *sys, uint32_t *flags, void *stream) {
  if (!sys) return fail(SOMA_E_INVAL, "system is NULL");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  uint32_t f = 0;
  HIP_TRY(hipMemcpyAsync(&f, sys->err(), sizeof f, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (flags) *flags = f;
  if (f) return fail(SOMA_E_DEVICE_FLAG, "device error word 0x%x", f);
  return SOMA_OK;
}

int32_t soma_get_sweep(const soma_system *sys, uint64_t *sweep) {
  if (!sys || !sweep) return fail(SOMA_E_INVAL, "NULL argument");
  *sweep = sys->sweep;
  return SOMA_OK;
}

int32_t soma_set_sweep(soma_system *sys, uint64_t sweep, void *stream) {
  if (!sys) return fail(SOMA_E_INVAL, "system is NULL");
  const int32_t rc = launch_counter(sys->sweep_ctr(), 0, 1, (uint32_t)sweep,
                                    reinterpret_cast<hipStream_t>(stream));
  if (rc) return rc;
  sys->sweep = sweep;
  return SOMA_OK;
}

int32_t soma_density_hist(const soma_config *cfg, const float *pos, void *counts, void *stream) {
  Derived d;
  int32_t rc = derive(cfg, &d);
  if (rc) return rc;
  if (!pos || !counts) return fail(SOMA_E_INVAL, "NULL buffer");
  if (!aligned(counts, 16)) return fail(SOMA_E_INVAL, "counts must be 16-byte aligned");
  return launch_hist(cfg, d, pos, counts, reinterpret_cast<hipStream_t>(stream));
}

int32_t soma_field_from_counts(const soma_config *cfg, const void *counts, float *omega,
                               void *stream) {
  Derived d;
  int32_t rc = derive(cfg, &d);
  if (rc) return rc;
  if (!counts || !omega) return fail(SOMA_E_INVAL, "NULL buffer");
  if (!aligned(counts, 16) || !aligned(omega, 16))
    return fail(SOMA_E_INVAL, "counts and omega must be 16-byte aligned");
  return launch_field(cfg, d, const_cast<void *>(counts), omega, nullptr,
                      reinterpret_cast<hipStream_t>(stream));
}

int32_t soma_init_positions(const soma_config *cfg, float *pos, void *stream) {
  Derived d;
  int32_t rc = derive(cfg, &d);
  if (rc) return rc;
  if (!pos) return fail(SOMA_E_INVAL, "NULL buffer");
  return launch_init(cfg, d, pos, reinterpret_cast<hipStream_t>(stream));
}

uint64_t soma_net_bytes(void) { return sizeof(soma::NetDev); }

int32_t soma_prepare_net(const float *params, void *net, void *stream) {
  if (!params || !net) return fail(SOMA_E_INVAL, "NULL buffer");
  if (!aligned(net, 16)) return fail(SOMA_E_INVAL, "net buffer must be 16-byte aligned");
  hipLaunchKernelGGL(soma::net_prepare_kernel, dim3(soma::kNetPrepareBlocks), dim3(256), 0,
                     reinterpret_cast<hipStream_t>(stream), params,
                     reinterpret_cast<soma::NetDev *>(net));
  LAUNCH_TRY();
  return SOMA_OK;
}

int32_t soma_set_proposal(soma_system *sys, uint32_t species, const float *params,
                          void *stream) {
  if (!sys) return fail(SOMA_E_INVAL, "system is NULL");
  const uint32_t n_sp = sys->cfg.n_species;
  if (species != SOMA_ALL_SPECIES && species >= n_sp)
    return fail(SOMA_E_INVAL, "species %u of %u", species, n_sp);
  const uint32_t lo = species == SOMA_ALL_SPECIES ? 0u : species;
  const uint32_t hi = species == SOMA_ALL_SPECIES ? n_sp : species + 1u;
  for (uint32_t sp = lo; sp < hi; ++sp) {
    const int32_t rc = soma_prepare_net(params, sys->net(sp), stream);
    if (rc) return rc;
    sys->net_mask |= 1u << sp;
  }
  return SOMA_OK;
}

int32_t soma_mlp_forward(const void *net, const float *features, uint32_t n, float *z,
                         void *stream) {
  if (!net || !features || !z) return fail(SOMA_E_INVAL, "NULL buffer");
  if (n == 0) return SOMA_OK;
  hipLaunchKernelGGL(soma::mlp_forward_kernel, dim3((n + 255) / 256), dim3(256), 0,
                     reinterpret_cast<hipStream_t>(stream),
                     reinterpret_cast<const soma::NetDev *>(net), features, n, z);
  LAUNCH_TRY();
  return SOMA_OK;
}

namespace {
soma::SpeciesTable species_table(const soma_system *sys) {
  soma::SpeciesTable st;
  st.n_species = sys->cfg.n_species;
  st.total_chains = (uint32_t)sys->d.n_chains;
  for (uint32_t k = 0; k < 8; ++k) {
    const bool ok = k < sys->cfg.n_species;
    st.chain_off[k] = ok ? (uint32_t)sys->d.chain_off[k] : 0u;
    st.bead_off[k] = ok ? sys->d.bead_off[k] : 0u;
    st.n[k] = ok ? sys->cfg.species[k].n : 1u;
    st.n_a[k] = ok ? sys->cfg.species[k].n_a : 0u;
  }
  return st;
}
}  // namespace

int32_t soma_features(soma_system *sys, const uint32_t *chains, const uint32_t *beads,
                      uint32_t n, float *out, void *stream) {
  if (!sys || !chains || !beads || !out) return fail(SOMA_E_INVAL, "NULL argument");
  if (n == 0) return SOMA_OK;
  hipLaunchKernelGGL(soma::features_kernel, dim3((n + 255) / 256), dim3(256), 0,
                     reinterpret_cast<hipStream_t>(stream), sys->buf.pos, sys->buf.omega,
                     sys->grid, species_table(sys), chains, beads, n, out);
  LAUNCH_TRY();
  return SOMA_OK;
}

int32_t soma_collect_training(soma_system *sys, uint32_t species, uint32_t n, uint32_t round,
                              uint32_t phase, float *features, float *r0, float *dr,
                              uint32_t *picked, void *stream) {
  if (!sys || !r0) return fail(SOMA_E_INVAL, "NULL argument");
  if (phase > 1) return fail(SOMA_E_INVAL, "phase %u", phase);
  if (species != SOMA_ALL_SPECIES &&
      (species >= sys->cfg.n_species || sys->cfg.species[species].n_chains == 0))
    return fail(SOMA_E_INVAL, "species %u has no chains", species);
  if (phase == 1 && !dr) return fail(SOMA_E_INVAL, "phase 1 needs dr");
  if (sys->arch_mask) return fail(SOMA_E_UNSUPPORTED, "training data of linear chains only");
  if (sys->d.n_types > 2) return fail(SOMA_E_UNSUPPORTED, "training data with two bead types only");
  if (n == 0) return SOMA_OK;
  soma::CollectArgs a;
  a.pos = sys->buf.pos;
  a.omega = sys->buf.omega;
  a.grid = sys->grid;
  a.st = species_table(sys);
  a.seed_lo = (uint32_t)sys->cfg.seed;
  a.seed_hi = (uint32_t)(sys->cfg.seed >> 32);
  a.replica = sys->cfg.replica;
  a.round = round;
  a.n = n;
  a.phase = phase;
  a.features = features;
  a.r0 = r0;
  a.dr = dr;
  a.picked = picked;
  a.chain_lo = species == SOMA_ALL_SPECIES ? 0u : (uint32_t)sys->d.chain_off[species];
  a.chain_count = species == SOMA_ALL_SPECIES ? (uint32_t)sys->d.n_chains
                                              : sys->cfg.species[species].n_chains;
  hipLaunchKernelGGL(soma::collect_kernel, dim3((n + 255) / 256), dim3(256), 0,
                     reinterpret_cast<hipStream_t>(stream), a);
  LAUNCH_TRY();
  return SOMA_OK;
}

uint64_t soma_sq_workspace_bytes(const soma_system *sys) {
  if (!sys) return 0;
  const uint64_t n = sys->d.n_cells;
  return align_up(16 * n) * 2 + align_up(16ull * (sys->cfg.nx + sys->cfg.ny + sys->cfg.nz));
}

int32_t soma_structure_factor(soma_system *sys, void *workspace, uint64_t workspace_bytes,
                              double *sq, void *stream) {
  if (!sys || !workspace || !sq) return fail(SOMA_E_INVAL, "NULL argument");
  if (!aligned(workspace, 256) || !aligned(sq, 8))
    return fail(SOMA_E_INVAL, "workspace must be 256-byte aligned, sq 8-byte aligned");
  const uint64_t need = soma_sq_workspace_bytes(sys);
  if (workspace_bytes < need)
    return fail(SOMA_E_SIZE, "structure-factor workspace: %llu < %llu bytes",
                (unsigned long long)workspace_bytes, (unsigned long long)need);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const uint64_t n = sys->d.n_cells;
  unsigned char *ws = reinterpret_cast<unsigned char *>(workspace);
  soma::SqArgs a;
  a.counts = sys->buf.counts;
  a.count64 = sys->cfg.count_width == 32;
  a.nx = sys->cfg.nx;
  a.ny = sys->cfg.ny;
  a.nz = sys->cfg.nz;
  a.a = reinterpret_cast<double2 *>(ws);
  a.b = reinterpret_cast<double2 *>(ws + align_up(16 * n));
  double2 *tw = reinterpret_cast<double2 *>(ws + 2 * align_up(16 * n));
  const uint32_t len[3] = {a.nx, a.ny, a.nz};
  uint32_t off = 0;
  for (int k = 0; k < 3; ++k) {
    hipLaunchKernelGGL(soma::sq_twiddle_kernel, dim3((len[k] + 255) / 256), dim3(256), 0, s,
                       tw + off, len[k]);
    LAUNCH_TRY();
    a.tw[k] = tw + off;
    off += len[k];
  }
  const dim3 grid((uint32_t)((n + 255) / 256));
  hipLaunchKernelGGL(soma::sq_dft_x_kernel, grid, dim3(256), 0, s, a);
  LAUNCH_TRY();
  hipLaunchKernelGGL(soma::sq_dft_axis_kernel, grid, dim3(256), 0, s, a.a, a.b, a.tw[1], a.nx,
                     a.ny, a.nz, 1);
  LAUNCH_TRY();
  hipLaunchKernelGGL(soma::sq_dft_axis_kernel, grid, dim3(256), 0, s, a.b, a.a, a.tw[2], a.nx,
                     a.ny, a.nz, 2);
  LAUNCH_TRY();
  const double nn = (double)sys->cfg.n_ref;
  hipLaunchKernelGGL(soma::sq_power_kernel, grid, dim3(256), 0, s, a.a, sq, n,
                     nn * nn / (4.0 * (double)sys->d.n_beads));
  LAUNCH_TRY();
  return SOMA_OK;
}

}  // extern "C"

namespace {

// Shell average over the lattice vectors of an nx x ny x nz grid (nz = 1: the
// m_z = 0 plane of a 3-D S(q), i.e. the in-plane structure factor), shell
// width 2 pi / lmin.
int32_t soma_sq_shells_impl(const double *sq, uint32_t nx, uint32_t ny, uint32_t nz,
                            uint32_t lmin, uint32_t n_shells, double *q_mid, double *s_avg,
                            uint64_t *count, uint32_t *peak) {
  if (!sq || !s_avg || !count || n_shells == 0) return fail(SOMA_E_INVAL, "NULL argument");
  if (nx == 0 || ny == 0 || nz == 0) return fail(SOMA_E_INVAL, "empty grid");
  const double two_pi = 6.283185307179586476925286766559;
  const double dq = two_pi / (double)lmin;
  for (uint32_t k = 0; k < n_shells; ++k) {
    s_avg[k] = 0.0;
    count[k] = 0;
    if (q_mid) q_mid[k] = dq * k;
  }
  auto wave = [](uint32_t m, uint32_t n) { return (double)(m <= n / 2 ? (int64_t)m : (int64_t)m - n) / n; };
  uint64_t c = 0;
  for (uint32_t z = 0; z < nz; ++z) {
    const double fz = wave(z, nz);
    for (uint32_t y = 0; y < ny; ++y) {
      const double fy = wave(y, ny);
      for (uint32_t x = 0; x < nx; ++x, ++c) {
        const double fx = wave(x, nx);
        const double q = two_pi * std::sqrt(fx * fx + fy * fy + fz * fz);
        const uint64_t k = (uint64_t)std::floor(q / dq + 0.5);
        if (k >= n_shells) continue;
        s_avg[k] += sq[c];
        count[k] += 1;
      }
    }
  }
  uint32_t best = 0;
  for (uint32_t k = 0; k < n_shells; ++k) {
    if (count[k]) s_avg[k] /= (double)count[k];
    if (k >= 1 && count[k] && (best == 0 || s_avg[k] > s_avg[best])) best = k;
  }
  if (peak) *peak = best;
  return SOMA_OK;
}

}  // namespace

extern "C" {

int32_t soma_sq_plane_shells(const double *sq, uint32_t nx, uint32_t ny, uint32_t n_shells,
                             double *q_mid, double *s_avg, uint64_t *count, uint32_t *peak) {
  return soma_sq_shells_impl(sq, nx, ny, 1, std::min(nx, ny), n_shells, q_mid, s_avg, count, peak);
}

int32_t soma_sq_shells(const double *sq, uint32_t nx, uint32_t ny, uint32_t nz,
                       uint32_t n_shells, double *q_mid, double *s_avg, uint64_t *count,
                       uint32_t *peak) {
  return soma_sq_shells_impl(sq, nx, ny, nz, std::min(nx, std::min(ny, nz)), n_shells, q_mid,
                             s_avg, count, peak);
}


uint64_t soma_train_workspace_bytes(uint32_t max_waves) {
  if (max_waves == 0) max_waves = 1;
  return align_up(sizeof(soma::NetDev)) + align_up((uint64_t)max_waves * soma::kPSize * 4ull) +
         align_up((uint64_t)max_waves * 4ull);
}

}  // extern "C"

namespace {

// The training step on a scratch buffer `workspace` of workspace_bytes bytes
// (the prepared network, per-wave partial gradients and loss partials; every
// byte the step reads is written by the step first).
int32_t train_step_impl(const float *features, const float *targets, uint32_t n, float *params,
                        float *adam_m, float *adam_v, uint32_t step, const soma_train_opts *o,
                        void *workspace, uint64_t workspace_bytes, float *grad_out,
                        float *loss_out, void *stream) {
  if (!features || !targets || !params || !o || !workspace)
    return fail(SOMA_E_INVAL, "NULL argument");
  if (n == 0) return fail(SOMA_E_INVAL, "empty batch");
  if (o->apply && (!adam_m || !adam_v || step == 0))
    return fail(SOMA_E_INVAL, "an update needs Adam moments and step >= 1");
  if (!(o->mu_max > 0.f) || !(o->log_sigma_min <= o->log_sigma_max))
    return fail(SOMA_E_INVAL, "head bounds");
  if (!aligned(workspace, 256)) return fail(SOMA_E_INVAL, "workspace must be 256-byte aligned");
  const uint32_t chunks = (n + 63u) / 64u;
  const uint32_t waves = o->max_waves ? (chunks < o->max_waves ? chunks : o->max_waves) : chunks;
  if (workspace_bytes < soma_train_workspace_bytes(waves))
    return fail(SOMA_E_SIZE, "train workspace: %llu < %llu bytes",
                (unsigned long long)workspace_bytes,
                (unsigned long long)soma_train_workspace_bytes(waves));
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  unsigned char *ws = reinterpret_cast<unsigned char *>(workspace);
  soma::NetDev *net = reinterpret_cast<soma::NetDev *>(ws);
  float *partials = reinterpret_cast<float *>(ws + align_up(sizeof(soma::NetDev)));
  float *lossp = reinterpret_cast<float *>(ws + align_up(sizeof(soma::NetDev)) +
                                           align_up((uint64_t)waves * soma::kPSize * 4ull));
  hipLaunchKernelGGL(soma::net_prepare_kernel, dim3(soma::kNetPrepareBlocks), dim3(256), 0, s, params, net);
  LAUNCH_TRY();
  soma::TrainArgs ta;
  ta.net = net;
  ta.feat = features;
  ta.target = targets;
  ta.n = n;
  ta.head.m_max = o->mu_max;
  ta.head.lo = o->log_sigma_min;
  ta.head.hi = o->log_sigma_max;
  ta.partials = partials;
  ta.loss_partials = lossp;
  hipLaunchKernelGGL(soma::mlp_grad_kernel, dim3(waves), dim3(64), 0, s, ta);
  LAUNCH_TRY();
  soma::AdamArgs aa;
  aa.partials = partials;
  aa.loss_partials = lossp;
  aa.waves = waves;
  aa.n = n;
  aa.params = params;
  aa.m = adam_m;
  aa.v = adam_v;
  aa.lr = o->lr;
  aa.beta1 = o->beta1;
  aa.beta2 = o->beta2;
  aa.eps = o->eps;
  aa.bc1 = 1.0f - std::pow(o->beta1, (float)(step ? step : 1));
  aa.bc2 = 1.0f - std::pow(o->beta2, (float)(step ? step : 1));
  aa.apply = o->apply ? 1 : 0;
  aa.grad_out = grad_out;
  aa.loss_out = loss_out;
  hipLaunchKernelGGL(soma::mlp_adam_kernel,
                     dim3((soma::kPSize + soma::kAdamParamsPerBlock - 1) / soma::kAdamParamsPerBlock),
                     dim3(256), 0, s, aa);
  LAUNCH_TRY();
  return SOMA_OK;
}

// Scratch of soma_train_step_noalloc: the prepared network, up to
// kNoAllocWaves partial gradients and their loss partials, in a device array
// of the library (one copy per GPU, held until the process ends).
constexpr uint64_t align256(uint64_t x) { return (x + 255u) / 256u * 256u; }
constexpr uint32_t kNoAllocWaves = SOMA_NOALLOC_TRAIN_WAVES;
constexpr uint64_t kNoAllocBytes = align256(sizeof(soma::NetDev)) +
                                   align256((uint64_t)kNoAllocWaves * soma::kPSize * 4u) +
                                   align256((uint64_t)kNoAllocWaves * 4u);

}  // namespace

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per
// device.  Host code uses only this address, never the array's name.
int32_t scratch_address(void **out) {
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(SOMA_E_UNSUPPORTED, "device %d", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(SOMA_E_HIP, "hipGetSymbolAddress returned NULL");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return SOMA_OK;
}

}  // namespace

extern "C" {

int32_t soma_train_step(const float *features, const float *targets, uint32_t n, float *params,
                        float *adam_m, float *adam_v, uint32_t step, const soma_train_opts *o,
                        void *workspace, uint64_t workspace_bytes, float *grad_out,
                        float *loss_out, void *stream) {
  return train_step_impl(features, targets, n, params, adam_m, adam_v, step, o, workspace,
                         workspace_bytes, grad_out, loss_out, stream);
}

int32_t soma_train_step_noalloc(const float *features, const float *targets, uint32_t n,
                                float *params, float *adam_m, float *adam_v, uint32_t step,
                                const soma_train_opts *o, float *grad_out, float *loss_out,
                                void *stream) {
  if (!o) return fail(SOMA_E_INVAL, "NULL argument");
  if (n == 0) return fail(SOMA_E_INVAL, "empty batch");
  const uint32_t chunks = (n + 63u) / 64u;
  const uint32_t waves = o->max_waves ? (chunks < o->max_waves ? chunks : o->max_waves) : chunks;
  if (waves > kNoAllocWaves)
    return fail(SOMA_E_SIZE, "the batch needs %u partial gradients, more than the %u of the "
                             "fixed scratch; set opts->max_waves <= %u", waves, kNoAllocWaves,
                kNoAllocWaves);
  void *ws = nullptr;
  const int32_t rc = scratch_address(&ws);
  if (rc) return rc;
  return train_step_impl(features, targets, n, params, adam_m, adam_v, step, o, ws,
                         kNoAllocBytes, grad_out, loss_out, stream);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Batches: one launch per sweep (and per field refresh) for many systems.
// ---------------------------------------------------------------------------
struct soma_batch {
  std::vector<soma_system *> sys;
  // host copies of the device tables (kept for the batch's lifetime)
  std::vector<soma::BatchSeg> segs[4];   // by move kind (local, smart MC, mixed, bond-Gibbs)
  std::vector<uint32_t> seg_first;
  std::vector<soma::FieldArgs> fargs;
  std::vector<uint32_t> fb_first;
  std::vector<uint32_t *> ctrs;
  soma::BatchSeg *d_segs[4] = {nullptr, nullptr, nullptr, nullptr};
  uint32_t *d_seg_first = nullptr, *d_fb_first = nullptr;
  soma::FieldArgs *d_fargs = nullptr;
  uint32_t **d_ctrs = nullptr;
  uint32_t n_items = 0, c64 = 0, v2 = 1;
  uint32_t mode = 0, grid_blocks = 0;  // launch shape (results do not depend on it)
  // binned count updates: every system's own bins, one apply launch for all
  uint32_t hist = 0;                    // soma::kHistDirect or soma::kHistBinned
  bool bins_ok = false;                 // every system has bins and two bead types
  std::vector<soma::BinApplySeg> apply;
  std::vector<uint32_t> brick_first;
  soma::BinApplySeg *d_apply = nullptr;
  uint32_t *d_brick_first = nullptr;
  uint32_t substeps = 1;                // chain subsets per cycle (field refresh after each)
  CycleGraph graph;
  ~soma_batch() { graph.release(); }
};

namespace {

struct BatchLayout {
  uint64_t segs[4], seg_first, fargs, fb_first, ctrs, apply, brick_first, total;
};

BatchLayout batch_layout(uint64_t n_segs, uint64_t n_sys) {
  BatchLayout L;
  uint64_t o = 0;
  for (int k = 0; k < 4; ++k) {
    L.segs[k] = o;
    o = align_up(o + n_segs * sizeof(soma::BatchSeg));
  }
  L.seg_first = o;
  o = align_up(o + (n_segs + 1) * 4);
  L.fargs = o;
  o = align_up(o + n_sys * sizeof(soma::FieldArgs));
  L.fb_first = o;
  o = align_up(o + (n_sys + 1) * 4);
  L.ctrs = o;
  o = align_up(o + n_sys * 8);
  L.apply = o;
  o = align_up(o + n_sys * sizeof(soma::BinApplySeg));
  L.brick_first = o;
  o = align_up(o + (n_sys + 1) * 4);
  L.total = o;
  return L;
}

int32_t batch_segments(soma_system *const *systems, uint32_t n, uint64_t *n_segs) {
  if (!systems || n == 0) return fail(SOMA_E_INVAL, "empty batch");
  uint64_t k = 0;
  for (uint32_t i = 0; i < n; ++i) {
    if (!systems[i]) return fail(SOMA_E_INVAL, "system %u is NULL", i);
    for (uint32_t sp = 0; sp < systems[i]->cfg.n_species; ++sp)
      if (systems[i]->cfg.species[sp].n_chains) ++k;
    if (systems[i]->cfg.count_width != systems[0]->cfg.count_width)
      return fail(SOMA_E_UNSUPPORTED, "all systems of a batch need the same count_width");
  }
  *n_segs = k;
  return SOMA_OK;
}

// Items (blocks of four wave tiles) of one segment when its chains are split
// into k subsets: enough for the largest subset.
uint32_t items_of(const soma::SweepArgs &a, uint32_t k) {
  const uint32_t per = 4u * a.chains_per_wave;
  const uint32_t n = (a.n_chains + k - 1u) / k;
  return (n + per - 1u) / per;
}

// Segment prefix of the work list for the batch's current subset count.
int32_t batch_items(soma_batch *b) {
  b->seg_first.assign(1, 0u);
  uint64_t items = 0;
  for (const soma::BatchSeg &seg : b->segs[0]) {
    items += items_of(seg.a, b->substeps);
    if (items >= (1ull << 31)) return fail(SOMA_E_UNSUPPORTED, "batch too large");
    b->seg_first.push_back((uint32_t)items);
  }
  b->n_items = (uint32_t)items;
  return SOMA_OK;
}

template <bool C64, bool V2, bool B>
void launch_batch_k(uint32_t kind, dim3 grid, hipStream_t s, const soma::BatchLaunch &L) {
  if (kind == SOMA_MOVE_MIXED)   // direct atomics only (see launch_batch_sweep)
    hipLaunchKernelGGL((soma::batched_sweep_kernel<C64, V2, 2, false>), grid, dim3(256), 0, s,
                       L);
  else if (kind == SOMA_MOVE_GIBBS)
    hipLaunchKernelGGL((soma::batched_sweep_kernel<C64, V2, 3, B>), grid, dim3(256), 0, s, L);
  else if (kind == SOMA_MOVE_SMC)
    hipLaunchKernelGGL((soma::batched_sweep_kernel<C64, V2, 1, B>), grid, dim3(256), 0, s, L);
  else
    hipLaunchKernelGGL((soma::batched_sweep_kernel<C64, V2, 0, B>), grid, dim3(256), 0, s, L);
}

template <bool C64, bool V2>
void launch_batch_t(bool binned, uint32_t kind, dim3 grid, hipStream_t s,
                    const soma::BatchLaunch &L) {
  if (binned && kind != SOMA_MOVE_MIXED) launch_batch_k<C64, V2, true>(kind, grid, s, L);
  else launch_batch_k<C64, V2, false>(kind, grid, s, L);
}

int32_t launch_batch_sweep(soma_batch *b, uint32_t kind, hipStream_t s, uint32_t off,
                           uint32_t j) {
  soma::BatchLaunch L;
  L.sub_k = b->substeps;
  L.sub_j = j;
  L.segs = b->d_segs[kind];
  L.seg_first = b->d_seg_first;
  L.n_segs = (uint32_t)b->seg_first.size() - 1u;
  L.n_items = b->n_items;
  L.per_xcd = (b->n_items + 7u) / 8u;
  L.mode = b->mode;
  L.sweep_off = off;
  uint32_t blocks;
  if (b->mode == 0) {
    blocks = 8u * L.per_xcd;
    if (b->grid_blocks && b->grid_blocks < blocks) blocks = (b->grid_blocks + 7u) / 8u * 8u;
  } else {
    blocks = b->n_items;
    if (b->grid_blocks && b->grid_blocks < blocks) blocks = b->grid_blocks;
  }
  const dim3 grid(blocks);
  // mixed sweeps keep direct atomics: their LDS tiles leave no room for the
  // bin tables at two blocks per compute unit
  const bool binned = b->hist == soma::kHistBinned && kind != SOMA_MOVE_MIXED;
  if (b->c64) {
    if (b->v2) launch_batch_t<true, true>(binned, kind, grid, s, L);
    else launch_batch_t<true, false>(binned, kind, grid, s, L);
  } else {
    if (b->v2) launch_batch_t<false, true>(binned, kind, grid, s, L);
    else launch_batch_t<false, false>(binned, kind, grid, s, L);
  }
  LAUNCH_TRY();
  if (!binned) return SOMA_OK;
  // every system's bins into its counts: one workgroup per brick of the batch
  const uint32_t n_sys = (uint32_t)b->sys.size();
  const dim3 agrid(b->brick_first[n_sys]), ablock(soma::kApplyThreads);
  const size_t lds = (size_t)soma::kBrickCells * (b->c64 ? 8u : 4u);
  if (b->c64)
    hipLaunchKernelGGL(soma::batched_bin_apply_kernel<true>, agrid, ablock, lds, s, b->d_apply,
                       b->d_brick_first, n_sys);
  else
    hipLaunchKernelGGL(soma::batched_bin_apply_kernel<false>, agrid, ablock, lds, s, b->d_apply,
                       b->d_brick_first, n_sys);
  LAUNCH_TRY();
  return SOMA_OK;
}

int32_t launch_batch_field(soma_batch *b, hipStream_t s) {
  const uint32_t n_sys = (uint32_t)b->sys.size();
  const dim3 grid(b->fb_first[n_sys]);
  if (b->c64)
    hipLaunchKernelGGL(soma::batched_field_kernel<true>, grid, dim3(256), 0, s, b->d_fargs,
                       b->d_fb_first, n_sys);
  else
    hipLaunchKernelGGL(soma::batched_field_kernel<false>, grid, dim3(256), 0, s, b->d_fargs,
                       b->d_fb_first, n_sys);
  LAUNCH_TRY();
  for (soma_system *x : b->sys)   // gradient fields of the systems that keep one
    if (x->grad) {
      const int32_t r = launch_grad(x, s);
      if (r) return r;
    }
  return SOMA_OK;
}

int32_t launch_batch_counter(soma_batch *b, uint32_t by, hipStream_t s) {
  const uint32_t n_sys = (uint32_t)b->sys.size();
  hipLaunchKernelGGL(soma::sweep_counter_kernel, dim3((n_sys + 63) / 64), dim3(64), 0, s,
                     b->d_ctrs, n_sys, by, 0u, 0u);
  LAUNCH_TRY();
  return SOMA_OK;
}

int32_t batch_check_kind(soma_batch *b, uint32_t kind) {
  for (soma_system *x : b->sys) {
    const int32_t rc = check_kind(x, kind);
    if (rc) return rc;
    if (x->scheme != SOMA_SCHEME_SET)
      return fail(SOMA_E_UNSUPPORTED, "batched sweeps use the SET order only");
    if (x->arch_mask) return fail(SOMA_E_UNSUPPORTED, "batched sweeps take linear chains only");
    if (x->d.n_types > 2) return fail(SOMA_E_UNSUPPORTED, "batched sweeps take two bead types");
  }
  return SOMA_OK;
}

void batch_count(soma_batch *b, uint32_t kind, uint64_t n) {
  for (soma_system *x : b->sys) x->count_sweeps(kind, n);
}

}  // namespace

extern "C" {

int32_t soma_batch_workspace_size(soma_system *const *systems, uint32_t n, uint64_t *bytes) {
  if (!bytes) return fail(SOMA_E_INVAL, "bytes is NULL");
  uint64_t n_segs = 0;
  const int32_t rc = batch_segments(systems, n, &n_segs);
  if (rc) return rc;
  *bytes = batch_layout(n_segs, n).total;
  return SOMA_OK;
}

int32_t soma_batch_create(soma_system *const *systems, uint32_t n, void *workspace,
                          uint64_t workspace_bytes, void *stream, soma_batch **out) {
  if (!out) return fail(SOMA_E_INVAL, "out is NULL");
  *out = nullptr;
  uint64_t n_segs = 0;
  int32_t rc = batch_segments(systems, n, &n_segs);
  if (rc) return rc;
  const BatchLayout lay = batch_layout(n_segs, n);
  if (!workspace) return fail(SOMA_E_INVAL, "workspace is NULL");
  if (!aligned(workspace, 256)) return fail(SOMA_E_INVAL, "workspace must be 256-byte aligned");
  if (workspace_bytes < lay.total)
    return fail(SOMA_E_SIZE, "batch workspace: %llu < %llu bytes",
                (unsigned long long)workspace_bytes, (unsigned long long)lay.total);
  soma_batch *b = new (std::nothrow) soma_batch();
  if (!b) return fail(SOMA_E_INVAL, "out of host memory");
  b->sys.assign(systems, systems + n);
  b->c64 = systems[0]->cfg.count_width == 32 ? 1u : 0u;
  // segments, largest first (equal sizes keep their order)
  struct Ref { uint32_t s, sp; uint64_t beads; };
  std::vector<Ref> refs;
  for (uint32_t i = 0; i < n; ++i)
    for (uint32_t sp = 0; sp < systems[i]->cfg.n_species; ++sp) {
      const soma_species &S = systems[i]->cfg.species[sp];
      if (S.n_chains) refs.push_back({i, sp, (uint64_t)S.n_chains * S.n});
    }
  std::stable_sort(refs.begin(), refs.end(),
                   [](const Ref &x, const Ref &y) { return x.beads > y.beads; });
  for (const Ref &r : refs) {
    soma::BatchSeg seg[4];
    for (uint32_t k = 0; k < 4; ++k) sweep_args(systems[r.s], r.sp, k, seg[k].a, seg[k].mx);
    for (uint32_t k = 0; k < 4; ++k) b->segs[k].push_back(seg[k]);
    if (!species_vec2(systems[r.s], r.sp)) b->v2 = 0;
  }
  rc = batch_items(b);
  if (rc) {
    delete b;
    return rc;
  }
  b->fb_first.push_back(0);
  for (uint32_t i = 0; i < n; ++i) {
    soma_system *x = systems[i];
    b->fargs.push_back(field_args(&x->cfg, x->d, x->buf.counts, x->buf.omega, x->fpart(),
                                  x->halo()));
    b->fb_first.push_back(b->fb_first.back() + x->d.field_blocks);
    b->ctrs.push_back(x->sweep_ctr());
  }
  b->bins_ok = true;
  b->brick_first.push_back(0);
  for (uint32_t i = 0; i < n; ++i) {
    soma_system *x = systems[i];
    b->bins_ok = b->bins_ok && x->d.bins_ok && x->d.n_types <= 2;
    soma::BinApplySeg a{};
    if (x->d.bins_ok) a.b = x->bins();
    a.g = x->grid;
    a.counts = x->buf.counts;
    b->apply.push_back(a);
    const uint64_t next = (uint64_t)b->brick_first.back() + (x->d.bins_ok ? x->d.n_bricks : 0u);
    b->bins_ok = b->bins_ok && next < (1ull << 31);
    b->brick_first.push_back((uint32_t)std::min<uint64_t>(next, 1ull << 31));
  }
  unsigned char *ws = reinterpret_cast<unsigned char *>(workspace);
  for (int k = 0; k < 4; ++k) b->d_segs[k] = reinterpret_cast<soma::BatchSeg *>(ws + lay.segs[k]);
  b->d_seg_first = reinterpret_cast<uint32_t *>(ws + lay.seg_first);
  b->d_fargs = reinterpret_cast<soma::FieldArgs *>(ws + lay.fargs);
  b->d_fb_first = reinterpret_cast<uint32_t *>(ws + lay.fb_first);
  b->d_ctrs = reinterpret_cast<uint32_t **>(ws + lay.ctrs);
  b->d_apply = reinterpret_cast<soma::BinApplySeg *>(ws + lay.apply);
  b->d_brick_first = reinterpret_cast<uint32_t *>(ws + lay.brick_first);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  auto put = [&](void *dst, const void *src, size_t bytes) -> int32_t {
    HIP_TRY(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s));
    return SOMA_OK;
  };
  for (int k = 0; k < 4 && !rc; ++k)
    rc = put(b->d_segs[k], b->segs[k].data(), b->segs[k].size() * sizeof(soma::BatchSeg));
  if (!rc) rc = put(b->d_seg_first, b->seg_first.data(), b->seg_first.size() * 4);
  if (!rc) rc = put(b->d_fargs, b->fargs.data(), b->fargs.size() * sizeof(soma::FieldArgs));
  if (!rc) rc = put(b->d_fb_first, b->fb_first.data(), b->fb_first.size() * 4);
  if (!rc) rc = put(b->d_ctrs, b->ctrs.data(), b->ctrs.size() * 8);
  if (!rc) rc = put(b->d_apply, b->apply.data(), b->apply.size() * sizeof(soma::BinApplySeg));
  if (!rc) rc = put(b->d_brick_first, b->brick_first.data(), b->brick_first.size() * 4);
  if (!rc) {  // the host tables must outlive the copies
    const hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) rc = fail(SOMA_E_HIP, "batch tables: %s", hipGetErrorString(e));
  }
  if (rc) {
    delete b;
    return rc;
  }
  *out = b;
  return SOMA_OK;
}

int32_t soma_batch_set_histogram(soma_batch *b, uint32_t mode) {
  if (!b) return fail(SOMA_E_INVAL, "batch is NULL");
  if (mode != SOMA_HIST_DIRECT && mode != SOMA_HIST_BINNED)
    return fail(SOMA_E_INVAL, "histogram mode %u", mode);
  if (mode == SOMA_HIST_BINNED && !b->bins_ok)
    return fail(SOMA_E_UNSUPPORTED,
                "binned count updates need bins in every system and two bead types");
  b->hist = mode == SOMA_HIST_BINNED ? soma::kHistBinned : soma::kHistDirect;
  return SOMA_OK;
}

int32_t soma_batch_set_launch(soma_batch *b, uint32_t mode, uint32_t grid_blocks) {
  if (!b) return fail(SOMA_E_INVAL, "batch is NULL");
  if (mode > 1) return fail(SOMA_E_INVAL, "mode must be 0 or 1");
  b->mode = mode;
  b->grid_blocks = grid_blocks;
  return SOMA_OK;
}

int32_t soma_batch_sweep(soma_batch *b, uint32_t n_sweeps, uint32_t move_kind, void *stream) {
  if (!b) return fail(SOMA_E_INVAL, "batch is NULL");
  int32_t rc = batch_check_kind(b, move_kind);
  if (rc || n_sweeps == 0) return rc;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  for (uint32_t i = 0; i < n_sweeps; ++i)
    for (uint32_t j = 0; j < b->substeps; ++j) {   // fields fixed: subsets in turn = one sweep
      rc = launch_batch_sweep(b, move_kind, s, i, j);
      if (rc) return rc;
    }
  rc = launch_batch_counter(b, n_sweeps, s);
  if (rc) return rc;
  batch_count(b, move_kind, n_sweeps);
  return SOMA_OK;
}

int32_t soma_batch_update_fields(soma_batch *b, void *stream) {
  if (!b) return fail(SOMA_E_INVAL, "batch is NULL");
  return launch_batch_field(b, reinterpret_cast<hipStream_t>(stream));
}

int32_t soma_batch_capture_cycle(soma_batch *b, uint32_t cycles, uint32_t move_kind) {
  if (!b) return fail(SOMA_E_INVAL, "batch is NULL");
  if (cycles == 0) return fail(SOMA_E_INVAL, "cycles must be positive");
  const int32_t rc = batch_check_kind(b, move_kind);
  if (rc) return rc;
  return capture_graph(b->graph, cycles, move_kind, [&](hipStream_t cs) -> int32_t {
    for (uint32_t i = 0; i < cycles; ++i)
      for (uint32_t j = 0; j < b->substeps; ++j) {
        int32_t r = launch_batch_sweep(b, move_kind, cs, i, j);
        if (!r) r = launch_batch_field(b, cs);
        if (r) return r;
      }
    return launch_batch_counter(b, cycles, cs);
  });
}

int32_t soma_batch_set_substeps(soma_batch *b, uint32_t k, void *stream) {
  if (!b) return fail(SOMA_E_INVAL, "batch is NULL");
  if (k == 0 || k > 4096) return fail(SOMA_E_INVAL, "substeps must be 1..4096");
  b->substeps = k;
  int32_t rc = batch_items(b);
  if (rc) return rc;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  HIP_TRY(hipMemcpyAsync(b->d_seg_first, b->seg_first.data(), b->seg_first.size() * 4,
                         hipMemcpyHostToDevice, s));
  HIP_TRY(hipStreamSynchronize(s));   // the host table must outlive the copy
  return SOMA_OK;
}

int32_t soma_batch_cycle(soma_batch *b, uint32_t n_cycles, uint32_t move_kind, void *stream) {
  if (!b) return fail(SOMA_E_INVAL, "batch is NULL");
  int32_t rc = batch_check_kind(b, move_kind);
  if (rc || n_cycles == 0) return rc;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  for (uint32_t i = 0; i < n_cycles; ++i)
    for (uint32_t j = 0; j < b->substeps; ++j) {
      rc = launch_batch_sweep(b, move_kind, s, i, j);
      if (!rc) rc = launch_batch_field(b, s);
      if (rc) return rc;
    }
  rc = launch_batch_counter(b, n_cycles, s);
  if (rc) return rc;
  batch_count(b, move_kind, n_cycles);
  return SOMA_OK;
}

int32_t soma_batch_run_cycle(soma_batch *b, uint32_t n_launches, void *stream) {
  if (!b) return fail(SOMA_E_INVAL, "batch is NULL");
  if (!b->graph.exec) return fail(SOMA_E_INVAL, "no captured cycle (soma_batch_capture_cycle)");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  for (uint32_t i = 0; i < n_launches; ++i) {
    HIP_TRY(hipGraphLaunch(b->graph.exec, s));
    batch_count(b, b->graph.kind, b->graph.cycles);
  }
  return SOMA_OK;
}

}  // extern "C"

namespace {

std::string system_key(const soma_system *x) {
  char buf[128];
  std::string k;
  std::snprintf(buf, sizeof buf, "%ux%ux%u/c%u", x->cfg.nx, x->cfg.ny, x->cfg.nz,
                x->cfg.count_width);
  k += buf;
  for (uint32_t sp = 0; sp < x->cfg.n_species; ++sp) {
    const soma_species &S = x->cfg.species[sp];
    std::snprintf(buf, sizeof buf, ",%u:%u:%u", S.n_chains, S.n, S.n_a);
    k += buf;
  }
  return k;
}

bool cache_lookup(const char *path, const std::string &key, uint32_t *mode, uint32_t *grid) {
  if (!path) return false;
  FILE *f = std::fopen(path, "r");
  if (!f) return false;
  bool found = false;
  char line[8192];
  while (std::fgets(line, sizeof line, f)) {
    char *tab = std::strchr(line, '\t');
    if (!tab) continue;
    *tab = '\0';
    unsigned m = 0, g = 0;
    if (key == line && std::sscanf(tab + 1, "%u %u", &m, &g) == 2 && m < 64) {
      *mode = m;
      *grid = g;
      found = true;  // the last matching line wins
    }
  }
  std::fclose(f);
  return found;
}

void cache_store(const char *path, const std::string &key, uint32_t mode, uint32_t grid,
                 float ms) {
  if (!path) return;
  FILE *f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f, "%s\t%u %u %.6f\n", key.c_str(), mode, grid, ms);
  std::fclose(f);
}

// Runs one warm-up cycle, then times `cycles` cycles (ms per cycle).
template <class Cycle>
int32_t time_cycles(hipStream_t s, uint32_t cycles, Cycle cycle, float *ms) {
  int32_t rc = cycle();
  if (rc) return rc;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIP_TRY(hipEventCreate(&e0));
  hipError_t e = hipEventCreate(&e1);
  if (e != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(SOMA_E_HIP, "hipEventCreate: %s", hipGetErrorString(e));
  }
  e = hipEventRecord(e0, s);
  for (uint32_t i = 0; i < cycles && !rc && e == hipSuccess; ++i) rc = cycle();
  if (!rc && e == hipSuccess) e = hipEventRecord(e1, s);
  if (!rc && e == hipSuccess) e = hipEventSynchronize(e1);
  float t = 0.f;
  if (!rc && e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return rc;
  if (e != hipSuccess) return fail(SOMA_E_HIP, "timing: %s", hipGetErrorString(e));
  *ms = t / (float)(cycles ? cycles : 1);
  return SOMA_OK;
}

struct Shape {
  uint32_t mode, grid;
};

// Tries each shape (apply, then time cycles), keeps the fastest.
template <class Apply, class Cycle>
int32_t tune(const Shape *shapes, uint32_t n_shapes, uint32_t cycles, const char *cache_path,
             const std::string &key, hipStream_t s, Apply apply, Cycle cycle, soma_tune *out) {
  std::memset(out, 0, sizeof *out);
  uint32_t mode = 0, grid = 0;
  if (cache_lookup(cache_path, key, &mode, &grid)) {
    apply(mode, grid);
    out->mode = mode;
    out->grid_blocks = grid;
    out->from_cache = 1;
    return SOMA_OK;
  }
  float best = 0.f;
  uint32_t best_i = 0;
  for (uint32_t i = 0; i < n_shapes; ++i) {
    apply(shapes[i].mode, shapes[i].grid);
    float ms = 0.f;
    const int32_t rc = time_cycles(s, cycles, cycle, &ms);
    if (rc) return rc;
    out->cycles_run += 1 + cycles;
    out->candidates += 1;
    if (i == 0 || ms < best) {
      best = ms;
      best_i = i;
    }
  }
  apply(shapes[best_i].mode, shapes[best_i].grid);
  out->mode = shapes[best_i].mode;
  out->grid_blocks = shapes[best_i].grid;
  out->ms_per_cycle = best;
  cache_store(cache_path, key, out->mode, out->grid_blocks, best);
  return SOMA_OK;
}

}  // namespace

extern "C" {

int32_t soma_autotune(soma_system *sys, uint32_t cycles, uint32_t move_kind,
                      const char *cache_path, void *stream, soma_tune *out) {
  if (!sys || !out) return fail(SOMA_E_INVAL, "system or out is NULL");
  if (cycles == 0) return fail(SOMA_E_INVAL, "cycles must be positive");
  const int32_t rc = check_kind(sys, move_kind);
  if (rc) return rc;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  // SET order: mode = histogram mode (bit 0) | block size / 64 - 1 (bits 1..3);
  // grid: one tile per wave (0), or the persistent grid of exactly the blocks
  // the device holds at once, whose waves draw their tiles from per-XCD
  // counters.  Molecule order: grid caps small enough to keep its chains in L2.
  std::vector<Shape> shapes;
  const bool mol = sys->scheme == SOMA_SCHEME_MOLECULE;
  if (mol) {
    for (uint32_t g : {0u, 256u, 512u, 1024u, 2048u}) shapes.push_back({0u, g});
  } else {
    const uint32_t n_hist = sys->d.bins_ok ? 2u : 1u;
    const bool fixed_block = move_kind == SOMA_MOVE_MIXED;
    for (uint32_t h = 0; h < n_hist; ++h)
      for (uint32_t t : {256u, 128u, 512u}) {
        if (fixed_block && t != 256u) continue;
        for (uint32_t resident : {0u, 1u}) {
          uint32_t g = 0u;
          if (resident) {
            g = resident_blocks(move_kind, sys->cfg.count_width == 32, h != 0u, t);
            if (g == 0u) g = 2048u;
          }
          shapes.push_back({h | ((t / 64u - 1u) << 1), g});
        }
      }
  }
  char kind_s[24];
  std::snprintf(kind_s, sizeof kind_s, "sys/k%u/s%u/", move_kind, sys->scheme);
  auto apply = [&](uint32_t mode, uint32_t grid) {
    sys->sweep_blocks = grid;
    if (!mol) {
      sys->hist_mode = (mode & 1u) ? soma::kHistBinned : soma::kHistDirect;
      sys->sweep_threads = 64u * (((mode >> 1) & 7u) + 1u);
    }
  };
  const int32_t r = tune(shapes.data(), (uint32_t)shapes.size(), cycles, cache_path,
                         kind_s + system_key(sys), s, apply,
                         [&]() -> int32_t { return soma_cycle(sys, 1, move_kind, stream); }, out);
  if (!r) {
    out->mode = 0;   // the item order exists for batches only
    out->hist_mode = sys->hist_mode == soma::kHistBinned ? SOMA_HIST_BINNED : SOMA_HIST_DIRECT;
    out->block_threads = mol ? 256u : sys->sweep_threads;
  }
  return r;
}

int32_t soma_choose_scheme(soma_system *sys, uint32_t cycles, void *stream, uint32_t *chosen,
                           float *ms) {
  if (!sys || !chosen) return fail(SOMA_E_INVAL, "system or chosen is NULL");
  if (cycles == 0) return fail(SOMA_E_INVAL, "cycles must be positive");
  const uint32_t keep = sys->scheme;
  sys->scheme = SOMA_SCHEME_SET;
  int32_t rc = check_kind(sys, SOMA_MOVE_LOCAL);
  if (rc) {
    sys->scheme = keep;
    return rc;
  }
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  float t[2] = {0.f, 0.f};
  for (uint32_t k = 0; k < 2 && !rc; ++k) {
    sys->scheme = k;
    rc = time_cycles(s, cycles, [&]() -> int32_t { return soma_cycle(sys, 1, SOMA_MOVE_LOCAL, stream); },
                     &t[k]);
  }
  if (rc) {
    sys->scheme = keep;
    return rc;
  }
  sys->scheme = t[1] < t[0] ? SOMA_SCHEME_MOLECULE : SOMA_SCHEME_SET;
  *chosen = sys->scheme;
  if (ms) {
    ms[0] = t[0];
    ms[1] = t[1];
  }
  return SOMA_OK;
}

int32_t soma_batch_autotune(soma_batch *b, uint32_t cycles, uint32_t move_kind,
                            const char *cache_path, void *stream, soma_tune *out) {
  if (!b || !out) return fail(SOMA_E_INVAL, "batch or out is NULL");
  if (cycles == 0) return fail(SOMA_E_INVAL, "cycles must be positive");
  const int32_t rc = batch_check_kind(b, move_kind);
  if (rc) return rc;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  // mode: item order (bit 0) | binned count updates (bit 1)
  std::vector<Shape> shapes;
  for (uint32_t h = 0; h < (b->bins_ok ? 2u : 1u); ++h)
    for (uint32_t g : {0u, 2048u, 8192u})
      for (uint32_t order : {0u, 1u}) shapes.push_back({order | (h << 1), g});
  char kind_s[16];
  std::snprintf(kind_s, sizeof kind_s, "batch/k%u", move_kind);
  std::string key = kind_s;
  for (soma_system *x : b->sys) key += "/" + system_key(x);
  const int32_t r = tune(shapes.data(), (uint32_t)shapes.size(), cycles, cache_path, key, s,
                         [&](uint32_t mode, uint32_t grid) {
                           b->mode = mode & 1u;
                           b->hist = (mode >> 1) ? soma::kHistBinned : soma::kHistDirect;
                           b->grid_blocks = grid;
                         },
                         [&]() -> int32_t { return soma_batch_cycle(b, 1, move_kind, stream); },
                         out);
  if (!r) {
    out->mode = b->mode;
    out->hist_mode = b->hist == soma::kHistBinned ? SOMA_HIST_BINNED : SOMA_HIST_DIRECT;
    out->block_threads = 256u;
  }
  return r;
}

void soma_batch_destroy(soma_batch *b) { delete b; }

void soma_destroy(soma_system *sys) { delete sys; }

}  // extern "C"
