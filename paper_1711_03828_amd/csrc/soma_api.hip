// soma_api.hip -- the C ABI declared in include/soma.h: configuration checks,
// workspace layout, kernel launches and the SCMF cycle bookkeeping.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>

#include "soma.h"
#include "soma_device.hpp"
#include "soma_grid.hpp"
#include "soma_obs.hpp"
#include "soma_sweep.hpp"
#include "soma_train.hpp"

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
           off_opart = 0;
  uint64_t ws_bytes = 0;
};

int32_t derive(const soma_config *c, Derived *d) {
  if (!c) return fail(SOMA_E_INVAL, "config is NULL");
  if (c->nx == 0 || c->ny == 0 || c->nz == 0)
    return fail(SOMA_E_INVAL, "grid dimensions must be positive");
  const uint64_t n_cells = (uint64_t)c->nx * c->ny * c->nz;
  if (n_cells >= (1ull << 31)) return fail(SOMA_E_UNSUPPORTED, "more than 2^31 - 1 cells");
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
  d->off_att = align_up(d->off_acc + 3ull * soma::kAccSlots * 8ull);
  d->off_net = align_up(d->off_att + soma::kAccSlots * 8ull);
  d->off_fpart = align_up(d->off_net + sizeof(soma::NetDev));
  d->off_totals = align_up(d->off_fpart + soma::kFieldBlocks * sizeof(soma::FieldPartial));
  d->off_opart = align_up(d->off_totals + sizeof(soma::Totals));
  d->ws_bytes = align_up(d->off_opart + (d->obs_blocks ? d->obs_blocks : 1) * sizeof(soma::ObsPartial));
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

float inv_rho_f(const Derived &d) { return (float)((double)d.n_cells / (double)d.n_beads); }

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

int32_t launch_hist(const soma_config *c, const Derived &d, const float *pos, void *counts,
                    hipStream_t s) {
  int32_t rc = launch_zero(counts, d.counts_bytes, s);
  if (rc) return rc;
  const soma::Grid g = make_grid(c, d.n_cells);
  for (uint32_t sp = 0; sp < c->n_species; ++sp) {
    const soma_species &S = c->species[sp];
    const uint64_t nb = (uint64_t)S.n_chains * S.n;
    if (!nb) continue;
    const uint64_t blocks = (nb + 255) / 256;
    const float *p = pos + 3 * d.bead_off[sp];
    if (c->count_width == 32)
      hipLaunchKernelGGL(soma::density_hist_kernel<true>, dim3((uint32_t)blocks), dim3(256), 0, s,
                         p, nb, S.n, S.n_a, g, counts);
    else
      hipLaunchKernelGGL(soma::density_hist_kernel<false>, dim3((uint32_t)blocks), dim3(256), 0,
                         s, p, nb, S.n, S.n_a, g, counts);
    LAUNCH_TRY();
  }
  return SOMA_OK;
}

int32_t launch_field(const soma_config *c, const Derived &d, void *counts, float *omega,
                     soma::FieldPartial *partials, int clear, hipStream_t s) {
  soma::FieldArgs a;
  a.counts = counts;
  a.omega = omega;
  a.n_cells = (uint32_t)d.n_cells;
  a.inv_rho = inv_rho_f(d);
  a.chi_n = c->chi_n;
  a.kappa_n = c->kappa_n;
  a.inv_rho_d = (double)d.n_cells / (double)d.n_beads;
  a.chi_n_d = (double)c->chi_n;
  a.kappa_n_d = (double)c->kappa_n;
  a.partials = partials;
  a.clear = clear;
  const uint32_t blocks = soma::kFieldBlocks;
  if (c->count_width == 32)
    hipLaunchKernelGGL(soma::field_update_kernel<true>, dim3(blocks), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(soma::field_update_kernel<false>, dim3(blocks), dim3(256), 0, s, a);
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

struct soma_system {
  soma_config cfg;
  soma_buffers buf;
  Derived d;
  soma::Grid grid;
  uint64_t sweep = 0;
  uint64_t attempted[2] = {0, 0};
  uint32_t sweep_blocks = 0;  // local-move grid: 0 = one tile per wave, else persistent blocks
  uint64_t mixed_moves = 0;   // bead moves made by mixed sweeps (local or learned)
  bool has_net = false;
  unsigned char *ws = nullptr;
  uint32_t *err() { return reinterpret_cast<uint32_t *>(ws + d.off_err); }
  unsigned long long *acc() { return reinterpret_cast<unsigned long long *>(ws + d.off_acc); }
  soma::FieldPartial *fpart() { return reinterpret_cast<soma::FieldPartial *>(ws + d.off_fpart); }
  soma::Totals *totals() { return reinterpret_cast<soma::Totals *>(ws + d.off_totals); }
  soma::ObsPartial *opart() { return reinterpret_cast<soma::ObsPartial *>(ws + d.off_opart); }
  unsigned long long *att() { return reinterpret_cast<unsigned long long *>(ws + d.off_att); }
  soma::NetDev *net() { return reinterpret_cast<soma::NetDev *>(ws + d.off_net); }
};

namespace {

template <bool C64, bool V2>
void launch_sweep_t(uint32_t kind, dim3 grid, hipStream_t s, const soma::SweepArgs &a,
                    const soma::MixArgs &mx, uint32_t *err) {
  if (kind == SOMA_MOVE_MIXED)
    hipLaunchKernelGGL((soma::mc_sweep_mixed_kernel<C64, V2>), grid, dim3(256), 0, s, a, mx, err);
  else if (kind == SOMA_MOVE_SMC)
    hipLaunchKernelGGL((soma::mc_sweep_smc_kernel<C64, V2>), grid, dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL((soma::mc_sweep_local_kernel<C64, V2>), grid, dim3(256), 0, s, a);
}

int32_t launch_sweep(soma_system *sys, uint32_t kind, hipStream_t s) {
  const soma_config *c = &sys->cfg;
  for (uint32_t sp = 0; sp < c->n_species; ++sp) {
    const soma_species &S = c->species[sp];
    if (!S.n_chains) continue;
    soma::SweepArgs a;
    a.pos = sys->buf.pos + 3 * sys->d.bead_off[sp];
    a.omega = sys->buf.omega;
    a.counts = sys->buf.counts;
    a.acc_slots = sys->acc() + (kind == SOMA_MOVE_SMC ? soma::kAccSlots : 0u);
    soma::MixArgs mx;
    mx.net = sys->net();
    mx.head.m_max = c->mu_max;
    mx.head.lo = c->log_sigma_min;
    mx.head.hi = c->log_sigma_max;
    mx.p_learn = c->p_learn;
    mx.att_slots = sys->att();
    a.grid = sys->grid;
    a.n_chains = S.n_chains;
    a.n = S.n;
    a.n_a = S.n_a;
    a.lanes_per_chain = (S.n + 1) / 2;
    a.chains_per_wave = 64u / a.lanes_per_chain;
    a.chain_base = (uint32_t)sys->d.chain_off[sp];
    a.k0 = S.k0;
    a.half_k0 = 0.5f * S.k0;
    a.step = kind == SOMA_MOVE_SMC ? c->smc_a : c->local_a;  // mixed: local half-width
    a.sqrt_2a = (float)std::sqrt(2.0 * (double)c->smc_a);
    a.inv_4a = c->smc_a > 0.f ? (float)(1.0 / (4.0 * (double)c->smc_a)) : 0.f;
    a.inv_nref = (float)(1.0 / (double)c->n_ref);
    a.seed_lo = (uint32_t)c->seed;
    a.seed_hi = (uint32_t)(c->seed >> 32);
    a.sweep = (uint32_t)sys->sweep;
    a.replica = c->replica;
    a.set_order = c->set_order;
    const uint64_t chains_per_block = 4ull * a.chains_per_wave;
    uint64_t blocks = (S.n_chains + chains_per_block - 1) / chains_per_block;
    if (kind == SOMA_MOVE_LOCAL && sys->sweep_blocks && sys->sweep_blocks < blocks)
      blocks = sys->sweep_blocks;
    const bool v2 = (S.n % 2 == 0) && (sys->d.bead_off[sp] % 2 == 0) && aligned(a.pos, 8);
    const bool c64 = c->count_width == 32;
    const dim3 grid((uint32_t)blocks);
    if (c64) {
      if (v2) launch_sweep_t<true, true>(kind, grid, s, a, mx, sys->err());
      else launch_sweep_t<true, false>(kind, grid, s, a, mx, sys->err());
    } else {
      if (v2) launch_sweep_t<false, true>(kind, grid, s, a, mx, sys->err());
      else launch_sweep_t<false, false>(kind, grid, s, a, mx, sys->err());
    }
    LAUNCH_TRY();
  }
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
  if (!rc) rc = launch_hist(cfg, d, buf->pos, buf->counts, s);
  if (!rc) rc = launch_field(cfg, d, buf->counts, buf->omega, sys->fpart(), 0, s);
  if (rc) {
    delete sys;
    return rc;
  }
  *out = sys;
  return SOMA_OK;
}

int32_t soma_mc_sweep(soma_system *sys, uint32_t n_sweeps, uint32_t move_kind, void *stream) {
  if (!sys) return fail(SOMA_E_INVAL, "system is NULL");
  if (move_kind != SOMA_MOVE_LOCAL && move_kind != SOMA_MOVE_SMC && move_kind != SOMA_MOVE_MIXED)
    return fail(SOMA_E_UNSUPPORTED, "move kind %u", move_kind);
  if (move_kind == SOMA_MOVE_MIXED && !sys->has_net && sys->cfg.p_learn > 0.f)
    return fail(SOMA_E_INVAL, "mixed moves need a network (soma_set_proposal)");
  if (move_kind == SOMA_MOVE_SMC && !(sys->cfg.smc_a > 0.f))
    return fail(SOMA_E_INVAL, "smart-MC moves need smc_a > 0");
  if (move_kind != SOMA_MOVE_SMC && !(sys->cfg.local_a < 1.f))
    return fail(SOMA_E_UNSUPPORTED, "local moves need a half-width below one cell");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  for (uint32_t i = 0; i < n_sweeps; ++i) {
    const int32_t rc = launch_sweep(sys, move_kind, s);
    if (rc) return rc;
    sys->sweep += 1;
  }
  if (move_kind == SOMA_MOVE_MIXED) sys->mixed_moves += (uint64_t)n_sweeps * sys->d.n_beads;
  else sys->attempted[move_kind] += (uint64_t)n_sweeps * sys->d.n_beads;
  return SOMA_OK;
}

int32_t soma_set_sweep_blocks(soma_system *sys, uint32_t blocks) {
  if (!sys) return fail(SOMA_E_INVAL, "system is NULL");
  sys->sweep_blocks = blocks;
  return SOMA_OK;
}

int32_t soma_rebuild_histogram(soma_system *sys, void *stream) {
  if (!sys) return fail(SOMA_E_INVAL, "system is NULL");
  return launch_hist(&sys->cfg, sys->d, sys->buf.pos, sys->buf.counts,
                     reinterpret_cast<hipStream_t>(stream));
}

int32_t soma_update_fields(soma_system *sys, void *stream) {
  if (!sys) return fail(SOMA_E_INVAL, "system is NULL");
  return launch_field(&sys->cfg, sys->d, sys->buf.counts, sys->buf.omega, sys->fpart(), 0,
                      reinterpret_cast<hipStream_t>(stream));
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
    a.half_k0 = 0.5 * (double)S.k0;
    a.inv_nref = 1.0 / (double)c->n_ref;
    a.grid = sys->grid;
    a.partials = sys->opart() + sys->d.obs_block_off[sp];
    a.err = sys->err();
    hipLaunchKernelGGL(soma::chain_obs_kernel, dim3((S.n_chains + 255) / 256), dim3(256), 0, s, a);
    LAUNCH_TRY();
  }
  hipLaunchKernelGGL(soma::reduce_totals_kernel, dim3(1), dim3(256), 0, s, sys->opart(),
                     (uint32_t)sys->d.obs_blocks, sys->fpart(), soma::kFieldBlocks, sys->acc(),
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
  for (int k = 0; k < 3; ++k) out->accepted[k] = t.accepted[k];
  out->attempted[0] = sys->attempted[0] + (sys->mixed_moves - t.attempted_learned);
  out->attempted[1] = sys->attempted[1];
  out->attempted[2] = t.attempted_learned;
  out->re2_sum = t.re2;
  out->rg2_sum = t.rg2;
  out->b2_sum = t.b2;
  out->e_bond = t.e_bond;
  out->e_field = t.e_field;
  out->h_nb = t.h_nb / ((double)sys->d.n_cells / (double)sys->d.n_beads * (double)c->n_ref);
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

int32_t soma_set_sweep(soma_system *sys, uint64_t sweep) {
  if (!sys) return fail(SOMA_E_INVAL, "system is NULL");
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
  return launch_field(cfg, d, const_cast<void *>(counts), omega, nullptr, 0,
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
  hipLaunchKernelGGL(soma::net_prepare_kernel, dim3(1), dim3(256), 0,
                     reinterpret_cast<hipStream_t>(stream), params,
                     reinterpret_cast<soma::NetDev *>(net));
  LAUNCH_TRY();
  return SOMA_OK;
}

int32_t soma_set_proposal(soma_system *sys, const float *params, void *stream) {
  if (!sys) return fail(SOMA_E_INVAL, "system is NULL");
  const int32_t rc = soma_prepare_net(params, sys->net(), stream);
  if (rc) return rc;
  sys->has_net = true;
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

int32_t soma_features(soma_system *sys, const uint32_t *chains, const uint32_t *beads,
                      uint32_t n, float *out, void *stream) {
  if (!sys || !chains || !beads || !out) return fail(SOMA_E_INVAL, "NULL argument");
  if (n == 0) return SOMA_OK;
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
  hipLaunchKernelGGL(soma::features_kernel, dim3((n + 255) / 256), dim3(256), 0,
                     reinterpret_cast<hipStream_t>(stream), sys->buf.pos, sys->buf.omega,
                     sys->grid, st, chains, beads, n, out);
  LAUNCH_TRY();
  return SOMA_OK;
}

uint64_t soma_train_workspace_bytes(uint32_t max_waves) {
  if (max_waves == 0) max_waves = 1;
  return align_up(sizeof(soma::NetDev)) + align_up((uint64_t)max_waves * soma::kPSize * 4ull) +
         align_up((uint64_t)max_waves * 4ull);
}

int32_t soma_train_step(const float *features, const float *targets, uint32_t n, float *params,
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
  hipLaunchKernelGGL(soma::net_prepare_kernel, dim3(1), dim3(256), 0, s, params, net);
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
  hipLaunchKernelGGL(soma::mlp_adam_kernel, dim3((soma::kPSize + 255) / 256), dim3(256), 0, s, aa);
  LAUNCH_TRY();
  return SOMA_OK;
}

void soma_destroy(soma_system *sys) { delete sys; }

}  // extern "C"
