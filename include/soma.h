/*
 * soma.h -- C ABI of the MI355X (gfx950) SCMF hot path.
 *
 * The library advances soft, coarse-grained polymer melts with the
 * single-chain-in-mean-field (SCMF) Monte Carlo method of
 *   L. Schneider, M. Mueller, "Multi-Architecture Monte-Carlo (MC) Simulation
 *   of Soft Coarse-Grained Polymeric Materials: SOMA", arXiv:1711.03828.
 * One SCMF cycle (Sec. 2.2) is: MC moves of every bead with the fields held
 * fixed (stage 2), then the per-type occupation histogram of the grid cells
 * (Eq. (4)) and the quasi-instantaneous fields computed from it (Eq. (12),
 * K^1 form of Eq. (8); stage 1).
 *
 * Conventions shared by every call
 *   - Lengths are in grid units (cell side Delta L = 1).  The box has
 *     nx*ny*nz cells and is periodic; a cell is the half-open unit cube and a
 *     position x belongs to cell floor(x) mod n along each axis.  The linear
 *     cell index is (z*ny + y)*nx + x.
 *   - Two bead types, A (0) and B (1).  A species is a linear chain of n beads
 *     whose first n_a beads are A; bead i is bonded to i-1 and i+1 (Eqs. (1),
 *     (2), harmonic springs of constant k0).
 *   - Positions: FP32 [n_beads][3], unwrapped, chain-major; species follow
 *     each other in the order of soma_config.species.
 *   - Counts: per cell one packed word holding both types: with
 *     count_width 16 a uint32 (A in bits 0-15, B in bits 16-31); with
 *     count_width 32 a uint64 (A in bits 0-31, B in bits 32-63).
 *   - Fields omega: FP32 planes [2][n_cells] (A plane, then B plane), in
 *     units of kT per chain; a bead of type t in cell c has energy
 *     omega_t(c) / n_ref (Eq. (13)).
 *   - Random numbers: Philox4x32-10 (Salmon et al., SC'11), key = seed,
 *     counter = (global chain index, bead | purpose << 16, sweep, replica).
 *     Results therefore depend only on the configuration, the seed and the
 *     sweep index -- not on launch geometry.
 *
 * Memory ownership: the caller owns every device buffer (positions, counts,
 * omega, workspace) and keeps it alive for the life of the handle.  The
 * library never allocates or frees device memory.  The handle owns only host
 * memory.
 *
 * Streams: every call takes a HIP stream (hipStream_t passed as void*; NULL is
 * the default stream) and only enqueues work on it, except where a call is
 * marked BLOCKING.
 *
 * Errors: every call returns a soma_status; on failure soma_last_error()
 * returns a message for the calling thread.  No call aborts or throws.  A
 * handle must not be used from two threads at once.
 */
#ifndef SOMA_H
#define SOMA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum soma_status {
  SOMA_OK = 0,
  SOMA_E_INVAL = -1,        /* invalid argument or configuration */
  SOMA_E_HIP = -2,          /* a HIP runtime call or kernel launch failed */
  SOMA_E_SIZE = -3,         /* a caller buffer is smaller than required */
  SOMA_E_UNSUPPORTED = -4,  /* valid request the library does not support */
  SOMA_E_DEVICE_FLAG = -5   /* a kernel raised the device error word */
} soma_status;

/* Move kinds (Sec. 2.2). */
#define SOMA_MOVE_LOCAL 0u /* uniform trial displacement in [-a,a]^3, Metropolis */
#define SOMA_MOVE_SMC 1u   /* force-biased (smart MC) proposal, Metropolis-Hastings */
#define SOMA_MOVE_MIXED 2u /* learned proposal with probability p_learn, else local; MH */
/* bond-Gibbs proposal: a bead's trial position drawn from its law given its
 * bonded neighbours under the bond energy alone (Eqs. (1)-(2)): Gaussian
 * around the mean of the neighbours, variance 1/(n_b k0) per component
 * (n_b = 1 or 2; a bead without bonds steps by N(0, 1/(2 k0))), computed as
 * fma(s, xi, mu) in FP32 with s = 1/sqrt(2 k0) or 1/sqrt(k0) rounded from
 * FP64, xi by Box-Muller from the smart-MC draws.  The bond energy and the
 * proposal densities cancel in the Metropolis-Hastings ratio of Sec. 2.2, so
 * a move is accepted with min(1, exp(-(omega(c') - omega(c))/N)).  Linear
 * chains, SET order (single melts and batches). */
#define SOMA_MOVE_GIBBS 3u

/* Iteration orders of local moves (Sec. 3.1.2). */
#define SOMA_SCHEME_SET 0u      /* per chain, the even and the odd beads as two sets in random
                                   order, each set moved at once (default) */
#define SOMA_SCHEME_MOLECULE 1u /* one thread per chain making N attempts one after another,
                                   each on a bead picked at random */

/* How the SET sweeps keep the occupation histogram (Eq. (4), Sec. 3.1.1)
 * current; see soma_set_histogram. */
#define SOMA_HIST_DIRECT 0u /* one memory-side atomic per +-1 count update (default) */
#define SOMA_HIST_BINNED 1u /* updates binned by brick of 16x16x8 cells, then applied
                               brick by brick in LDS */

/* Device error word bits (returned by soma_check / soma_observables). */
#define SOMA_FLAG_POSITION 1u /* soma_observables found a position non-finite or |x| >= 2^22 */
#define SOMA_FLAG_NETWORK 2u  /* a learned move met a non-finite network output (rejected) */

#define SOMA_MAX_SPECIES 8
#define SOMA_MAX_BEADS_PER_CHAIN 128

typedef struct soma_species {
  uint32_t n_chains; /* chains of this species */
  uint32_t n;        /* beads per chain, 1..SOMA_MAX_BEADS_PER_CHAIN */
  uint32_t n_a;      /* leading beads of type A, 0..n */
  float k0;          /* harmonic bond constant, kT per cell^2 (Eq. (2)) */
} soma_species;

typedef struct soma_config {
  uint32_t nx, ny, nz;   /* cells per axis */
  uint32_t n_species;    /* 1..SOMA_MAX_SPECIES */
  soma_species species[SOMA_MAX_SPECIES];
  uint32_t n_ref;        /* reference chain length N of omega/N, chiN, kappaN */
  float chi_n;           /* chi_AB N (Eq. (8)) */
  float kappa_n;         /* kappa N (Eq. (6)) */
  float local_a;         /* half-width a of the local move, cells; local moves need a < 1 */
  float smc_a;           /* step A of the smart-MC move, cells^2: r' = r + A F + sqrt(2A) xi */
  uint64_t seed;         /* Philox key */
  uint32_t replica;      /* fourth Philox counter word */
  uint32_t count_width;  /* 16 or 32 (bits per type per cell) */
  uint32_t set_order;    /* 0: random even/odd order per chain and sweep; 1: even first */
  uint32_t origin_mode;  /* initial origins: 0 i.i.d. uniform, 1 stratified in bricked order */
  /* learned proposal (SOMA_MOVE_MIXED): probability of the learned move per
   * bead, and the bounds of its Gaussian head: mu = mu_max tanh(z/mu_max),
   * log sigma = log_sigma_min + (log_sigma_max - log_sigma_min) sigmoid(z) */
  float p_learn;
  float mu_max;
  float log_sigma_min, log_sigma_max;
} soma_config;

typedef struct soma_buffers {
  float *pos;          uint64_t pos_bytes;       /* >= 12 * n_beads */
  void *counts;        uint64_t counts_bytes;    /* >= (4 or 8) * n_cells */
  float *omega;        uint64_t omega_bytes;     /* >= 8 * n_cells */
  void *workspace;     uint64_t workspace_bytes; /* >= soma_workspace_size() */
} soma_buffers;

typedef struct soma_obs {
  uint64_t sweeps;        /* sweeps done since init (the next sweep index) */
  uint64_t n_beads, n_chains;
  uint64_t count_a;       /* sum of A counts of the last field update */
  uint64_t count_b;       /* sum of B counts of the last field update */
  uint64_t accepted[4];   /* accepted moves since init: local, smart-MC, learned, bond-Gibbs */
  uint64_t attempted[4];  /* attempted moves since init: local, smart-MC, learned, bond-Gibbs */
  double re2_sum;         /* sum over chains of |r_{N-1} - r_0|^2 */
  double rg2_sum;         /* sum over chains of (1/N) sum_i |r_i - r_cm|^2 */
  double b2_sum;          /* sum over bonds of |r_{i+1} - r_i|^2 */
  double e_bond;          /* H_b / kT, Eqs. (1)-(2) */
  double e_field;         /* sum_j omega_type(j)(c_j) / n_ref at the current fields, Eq. (13) */
  double h_nb;            /* H_nb / kT of the last field update, Eqs. (5), (6), (8) */
  uint32_t error_flags;   /* device error word (SOMA_FLAG_*) */
  uint32_t counts_conserved; /* 1 if count_a/count_b equal the bead totals per type */
} soma_obs;

typedef struct soma_system soma_system;

/* Sizes in bytes of the caller buffers for a configuration.
 * Returns SOMA_E_INVAL for an invalid configuration.  Any output may be NULL. */
int32_t soma_buffer_sizes(const soma_config *cfg, uint64_t *pos_bytes,
                          uint64_t *counts_bytes, uint64_t *omega_bytes,
                          uint64_t *workspace_bytes);

/* Workspace bytes (acceptance slots, reduction partials, error word). */
int32_t soma_workspace_size(const soma_config *cfg, uint64_t *bytes);

/* Creates a handle for the configuration and the caller buffers.
 * If init_positions != 0, fills buf->pos with Gaussian-walk chains: bonds
 * N(0, 1/k0) per component (the ideal chain of Eq. (2), b0^2 = 3/k0, Sec. 2.1)
 * from origins placed per origin_mode; otherwise buf->pos must already hold
 * positions.  Then builds the occupation histogram (Eq. (4)) into buf->counts
 * and the fields from it (stage 1 of Sec. 2.2).  From then on the library keeps
 * buf->counts equal to the histogram of the current positions.
 * Asynchronous on `stream` except for argument validation.  On success *out
 * receives the handle. */
int32_t soma_init_system(const soma_config *cfg, const soma_buffers *buf,
                         uint32_t init_positions, void *stream,
                         soma_system **out);

/* Performs n_sweeps MC sweeps (stage 2 of Sec. 2.2) with the fields held
 * fixed: each sweep attempts one move of every bead, the even and the odd
 * beads of a chain forming the two independent sets of Sec. 3.1.2, moved set
 * after set in a random order per chain and sweep.  move_kind is
 * SOMA_MOVE_LOCAL, SOMA_MOVE_SMC, SOMA_MOVE_MIXED or SOMA_MOVE_GIBBS.  The histogram in buf->counts is updated
 * in the same pass (a bead that changes cell is moved from its old to its new
 * cell), so after the call it equals the histogram of the final positions,
 * bit for bit.  Asynchronous. */
int32_t soma_mc_sweep(soma_system *sys, uint32_t n_sweeps, uint32_t move_kind,
                      void *stream);

/* Stage 1 of Sec. 2.2: omega from the current histogram (Eq. (12)); the count
 * sums and H_nb of this histogram are kept for soma_observables.  The counts
 * are left unchanged.  Asynchronous. */
int32_t soma_update_fields(soma_system *sys, void *stream);

/* After the caller has written buf->omega directly (for example a frozen
 * external field), rebuilds the copies the sweeps read besides it: the
 * learned proposal's halo copy (kept when p_learn > 0) and the gradient field
 * (if kept).  Field refreshes by the library keep them current by themselves.
 * Asynchronous. */
int32_t soma_sync_fields(soma_system *sys, void *stream);

/* Optional gradient field for smart-MC moves: `grad` (device, caller-owned,
 * 16-byte aligned, >= 32 * n_cells bytes) receives, for each type t and cell
 * c, the float4 (omega_t(c), and the central differences along x, y, z,
 * 0.5 (omega_t(c + e) - omega_t(c - e)) over the periodic neighbours) at every
 * field refresh, starting now.  Smart-MC sweeps then read the field and its
 * gradient at a cell with one 16-byte gather instead of seven; results are
 * bit-identical either way.  grad = NULL detaches it.  Attach before creating
 * a batch that holds the system.  Asynchronous. */
int32_t soma_set_grad_field(soma_system *sys, void *grad, uint64_t grad_bytes, void *stream);

/* Interaction term of the grid Hamiltonian, Eq. (6) read over unordered pairs
 * of types: form 1 (default) chiN phi_A phi_B, with the fields of Eq. (12)'s
 * second form, omega_A = kappaN (phi_A + phi_B - 1) + chiN phi_B; form 0
 * -chiN/4 (phi_A - phi_B)^2, with omega_A = kappaN (phi_A + phi_B - 1)
 * - chiN/2 (phi_A - phi_B) and omega_B = ... + chiN/2 (phi_A - phi_B) (FP32:
 * fma(-+chiN/2, phi_A - phi_B, kappaN s)).  H_nb follows.  The fields are
 * recomputed from the current counts (asynchronous).  Set before creating a
 * batch that holds the system; capture graphs again afterwards.
 * SOMA_E_INVAL for another form. */
int32_t soma_set_hamiltonian(soma_system *sys, uint32_t form, void *stream);

/* External fields (Sec. 4).  ext (device, caller-owned, FP32 [2][n_cells], or
 * NULL): per type and cell an energy in the units of the fields, added to the
 * interaction field at every refresh (a bead of type t in cell c then carries
 * (omega_t(c) + ext_t(c)) / N) -- a linear attraction or repulsion, e.g. of one
 * type by a substrate.  forbid (device, caller-owned, ceil(n_cells/32) words,
 * or NULL): bit c % 32 of word c / 32 marks cell c impenetrable; every move
 * whose trial position lies in an impenetrable cell other than the bead's own
 * is rejected (geometric confinement, e.g. the walls of a film), and so is
 * every trial more than one cell away along any axis (floor(x') - floor(x)
 * outside {-1, 0, 1} on the unwrapped coordinates), so that no smart-MC,
 * bond-Gibbs or learned step jumps over a wall plane; the condition is
 * symmetric in (x, x'), so detailed balance holds.  Impenetrable cells get the field
 * 0 and are left out of H_nb, and the reference density counts free cells
 * only.  Positions must start outside impenetrable cells (not checked).  The
 * fields are recomputed from the current counts before the call returns.
 * Capture graphs again afterwards; attach before creating a batch that holds
 * the system.  NULL, NULL detaches both.  BLOCKING.  SOMA_E_SIZE for short
 * buffers, SOMA_E_INVAL if every cell is impenetrable. */
int32_t soma_set_external(soma_system *sys, const float *ext, uint64_t ext_bytes,
                          const uint32_t *forbid, uint64_t forbid_bytes, void *stream);

/* General molecular architecture of one species (Sec. 3.2.1), in place of the
 * linear chain A_{n_a} B_{N - n_a}.  words (host memory, n_words entries):
 * word 0 = N (must equal the species' n); word 1 + i = monomer i's type
 * code (0 = A, 1 = B; up to n_types - 1 after soma_set_types) in the top
 * byte and, in the low 24 bits, the index in the
 * array of its bond list (0: no bonds); a bond word holds partner - i as a
 * signed 27-bit integer in its low bits, the bond type in bits 27-30 (0,
 * harmonic with the species' k0, is the only kind) and, in bit 31, the flag
 * that ends the list.  Every bond must be listed at both ends; N <= 128,
 * <= 2048 list entries, <= 16 independent sets.  The sets are found greedily
 * in index order (monomer i joins the lowest set holding none of its bonded
 * partners of lower index; a linear chain gives the even and the odd
 * monomers) and swept as in SOMA_SCHEME_SET: with two sets, set 1 first iff
 * bit 0 of word 0 of monomer 0's move draw is set; with more, a Fisher-Yates
 * shuffle (step t = k-1 .. 1 swaps t with floor(w (t+1) / 2^32), w = word
 * (k-1-t) mod 4 of the block (chain, floor((k-1-t)/4) | 8 << 16, sweep,
 * replica)); set_order = 1: numerical order.  A linear chain given this way
 * moves bit for bit as without it.  Positions are kept: they must be
 * conformations of the architecture (the library's Gaussian-walk init
 * follows index order).  The histogram and the fields are rebuilt.  Species
 * with an architecture take SOMA_MOVE_LOCAL in the SET order only; they are
 * not batched and give no training data (SOMA_E_UNSUPPORTED).  The bond
 * observables sum over the bonds; Re^2 stays |r_{N-1} - r_0|^2.  words = NULL
 * restores the linear chain.  Capture graphs again afterwards.  BLOCKING;
 * SOMA_E_INVAL for a malformed array. */
int32_t soma_set_architecture(soma_system *sys, uint32_t species, const uint32_t *words,
                              uint32_t n_words, void *stream);

/* n_t bead types (Sec. 2.1) with a symmetric matrix chi_ij N, the fields of
 * Eq. (12) in the form chosen by soma_set_hamiltonian:
 *   K^1: omega_i = kappaN (sum_k phi_k - 1) + sum_{k != i} chi_ik N phi_k,
 *   K^0: omega_i = kappaN (sum_k phi_k - 1) - sum_{k != i} chi_ik N/2 (phi_i - phi_k),
 * in FP32 as s = (((phi_0 + phi_1) + phi_2) + ...) - 1, t = kappaN s, then
 * t = fma(chi_ik, phi_k, t) or fma(-chi_ik/2, phi_i - phi_k, t) for k = 0, 1,
 * ... (k != i); H_nb sums chi_ij N phi_i phi_j (or -chi_ij N/4 (phi_i -
 * phi_j)^2) over pairs i < j.  n_types in 2..8; chi_n (host) holds
 * n_types x n_types floats, row-major, symmetric (the diagonal is ignored);
 * with n_types = 2 it replaces the config's chi_n.  counts and omega (device,
 * caller-owned, 16-byte aligned) replace the buffers given at init: counts
 * holds ceil(n_types/2) planes of n_cells packed words of the config's count
 * width, plane p carrying types 2p (low half) and 2p + 1 (high half); omega
 * holds n_types planes of n_cells floats, plane t the field of type t.  Types
 * come from architectures (soma_set_architecture; call this first for codes
 * above 1); linear species keep types 0 and 1.  With more than two types:
 * SOMA_MOVE_LOCAL only, no external fields or walls, no gradient field, no
 * training data, no batching (SOMA_E_UNSUPPORTED); soma_obs's count_a is the
 * type-0 total and count_b that of all other types; the structure factor is
 * that of phi_0 - phi_1.  The histogram is rebuilt from the positions and the
 * fields recomputed; capture graphs again afterwards, and call before
 * creating a batch that holds the system.  BLOCKING.  SOMA_E_INVAL for a
 * non-symmetric or non-finite matrix or an architecture with a type code
 * >= n_types, SOMA_E_SIZE for short buffers, SOMA_E_UNSUPPORTED if the planes
 * exceed 32-bit byte offsets. */
int32_t soma_set_types(soma_system *sys, uint32_t n_types, const float *chi_n, void *counts,
                       uint64_t counts_bytes, float *omega, uint64_t omega_bytes, void *stream);

/* Total count of each bead type in the kept histogram (out[0 .. n_types-1],
 * host; n_out >= the number of types).  BLOCKING.  SOMA_E_SIZE if n_out is
 * too small. */
int32_t soma_type_counts(soma_system *sys, uint64_t *out, uint32_t n_out, void *stream);

/* Launch shape of the SET sweeps (local, smart-MC, bond-Gibbs and mixed
 * moves): 0 (default) runs one wave per tile of chains; blocks > 0, when
 * fewer than the tile groups, runs that many persistent blocks whose waves
 * draw their tiles from per-XCD counters in the workspace (zeroed by a small
 * kernel before each launch, a graph node).  Results are identical for every
 * value (they depend only on seed, sweep and chain).  A multiple of 8 keeps
 * each XCD on one contiguous range of chains.  Capture graphs again after a
 * change. */
int32_t soma_set_sweep_blocks(soma_system *sys, uint32_t blocks);

/* Threads per block (64, 128, ..., 512; default 256) of the local, smart-MC
 * and bond-Gibbs sweeps in the SET order: each wave of 64 lanes holds the
 * same chains whatever the block size, so results are identical for every
 * value.  SOMA_E_INVAL for other values.  Capture graphs again after a change. */
int32_t soma_set_sweep_threads(soma_system *sys, uint32_t threads);

/* Count updates of the SET-order sweeps (local, smart-MC, bond-Gibbs and
 * mixed moves of linear chains; the histogram of Eq. (4), Sec. 3.1.1).
 * SOMA_HIST_DIRECT: a bead that changes cell adds -1 and +1 to the packed
 * counts with two device atomics.  SOMA_HIST_BINNED: the grid is cut into
 * bricks of 16 x 16 x 8 cells (x fastest; partial bricks at the faces); each
 * wave groups its updates by brick, reserves room in the brick's bin in the
 * workspace with one atomic per (wave, brick) and stores them there; after
 * the sweep one workgroup per brick adds its bin to the counts in LDS (a bin
 * that is full takes further updates as direct atomics).  soma_mc_sweep,
 * soma_cycle and captured cycles run that step themselves, so the counts are
 * current whenever a call returns its stream to the caller.  Both modes give
 * the same counts bit for bit (integer additions in any order); molecule-order,
 * architecture and batched sweeps always use direct atomics.  Capture graphs
 * again after a change.  SOMA_E_INVAL for an unknown mode, SOMA_E_UNSUPPORTED
 * for SOMA_HIST_BINNED on a grid of 2^21 bricks or more. */
int32_t soma_set_histogram(soma_system *sys, uint32_t mode);

/* Iteration order of SOMA_MOVE_LOCAL sweeps (Sec. 3.1.2, schemes 2 and 1).
 * SOMA_SCHEME_SET (default): every bead is attempted once per sweep, the two
 * independent sets of a chain in a random order per chain and sweep.
 * SOMA_SCHEME_MOLECULE: each chain makes N attempts in sequence, attempt s on
 * bead floor(w N / 2^32), w = word s mod 4 of the chain's Philox block
 * (chain, floor(s/4) | 7 << 16, sweep, replica); the attempt draws from the
 * block (chain, s | 6 << 16, sweep, replica).  Both orders sample the same
 * distribution along different trajectories.  With SOMA_SCHEME_MOLECULE,
 * smart-MC and mixed sweeps and batched sweeps return SOMA_E_UNSUPPORTED;
 * soma_set_sweep_blocks then caps the grid of the molecule-order kernel
 * (lanes loop over chains), which keeps fewer chains in flight.  Capture
 * graphs again after a change.  Returns SOMA_E_INVAL for an unknown scheme. */
int32_t soma_set_scheme(soma_system *sys, uint32_t scheme);

/* Times `cycles` local-move SCMF cycles (after one warm-up cycle) with each
 * order, SET first, and keeps the faster one (*chosen; ms, if not NULL,
 * receives {SET, MOLECULE} milliseconds per cycle).  The system advances by
 * 2 (1 + cycles) cycles, so the trajectory differs from an untimed run; the
 * sampled distribution does not.  BLOCKING. */
int32_t soma_choose_scheme(soma_system *sys, uint32_t cycles, void *stream, uint32_t *chosen,
                           float *ms);

/* Single-bead energy of cell-changing moves.  The quasi-instantaneous field
 * of Sec. 2.2 charges a move of a bead of type t from cell c to c'
 * (omega_t(c') - omega_t(c))/N, with the bead itself still counted in c.
 * The grid Hamiltonian (Eqs. (5), (6), (8)) is quadratic in the counts, and
 * the exact change adds the second difference kappaN/(N rho) (K^1 form;
 * (kappaN - chiN/2)/(N rho) for K^0).  on = 1 adds it to every move that
 * changes cell (local, smart-MC, bond-Gibbs and learned moves of linear
 * chains of two types, SET order, single melts and batches created after the
 * call); on = 0 (default) is the paper's SCMF.  With the fields frozen the
 * term is not the energy difference of any fixed distribution: it is meant
 * for SCMF cycles, where it removes the bias that moves changing cell more
 * often (larger moves) would otherwise carry.  SOMA_E_UNSUPPORTED for other
 * systems.  Capture graphs again after a change. */
int32_t soma_set_self_term(soma_system *sys, uint32_t on);

/* Measurement only (the roofline of the histogram updates): n_updates
 * scattered 32-bit updates of the device array words[n_words] on `stream`,
 * one thread each, addresses from an integer hash of the thread index and
 * `seed`.  mode 0: atomicAdd(+1) at a uniformly random word; mode 1:
 * atomicAdd(+1) at a random word of a 4096-word window that moves with the
 * thread index (the locality of a sweep's count updates); mode 2: a plain
 * store at a uniformly random word.  Time it with events on `stream`.
 * SOMA_E_INVAL for an empty or misaligned array or an unknown mode.
 * Asynchronous. */
int32_t soma_probe_atomics(uint32_t *words, uint64_t n_words, uint64_t n_updates,
                           uint32_t mode, uint32_t seed, void *stream);

/* Recounts buf->counts from buf->pos (cleared first).  Needed only after the
 * caller has changed positions outside the library.  Asynchronous. */
int32_t soma_rebuild_histogram(soma_system *sys, void *stream);

/* BLOCKING.  Chain observables in FP64 (Re^2, Rg^2, bond lengths, bond and
 * field energies), acceptance counters, the count sums and H_nb of the last
 * field update, and the device error word.  Synchronizes `stream`.
 * Returns SOMA_E_DEVICE_FLAG (with *out filled) if the error word is set. */
int32_t soma_observables(soma_system *sys, soma_obs *out, void *stream);

/* BLOCKING.  Reads the device error word; SOMA_E_DEVICE_FLAG if set. */
int32_t soma_check(soma_system *sys, uint32_t *flags, void *stream);

/* Sweep index of the next sweep (Philox counter word 2); set it to resume a
 * run from saved positions bit-exactly.  The index lives in the workspace
 * (a device counter that every sweep call, graph replay or batch advances),
 * so setting it is a tiny kernel on `stream` (asynchronous). */
int32_t soma_get_sweep(const soma_system *sys, uint64_t *sweep);
int32_t soma_set_sweep(soma_system *sys, uint64_t sweep, void *stream);

/* ---- SCMF cycles -----------------------------------------------------------
 * soma_cycle runs n_cycles SCMF cycles: the MC sweep of move_kind and the
 * field refresh of stage 1 (Sec. 2.2).  With soma_set_substeps(sys, k), k > 1,
 * a cycle sweeps the chains in k interleaved subsets (chains j, j + k, ...)
 * and refreshes the fields after each subset: every bead still makes one move
 * per cycle, with the draws of an ordinary sweep, but fewer beads move between
 * two field refreshes.  Large moves (the learned proposal) make the
 * quasi-instantaneous field approximation coarser; sub-steps restore it at the
 * cost of k field refreshes per cycle.  k = 1 (default) is the plain cycle.
 * Asynchronous.  SOMA_E_INVAL for k outside 1..4096. */
int32_t soma_set_substeps(soma_system *sys, uint32_t k);
int32_t soma_cycle(soma_system *sys, uint32_t n_cycles, uint32_t move_kind, void *stream);

/* ---- Captured SCMF cycles ----------------------------------------------
 * soma_capture_cycle records `cycles` SCMF cycles of the system (as soma_cycle,
 * with the system's sub-steps), followed by the
 * advance of the device sweep counter, into a HIP graph; soma_run_cycle
 * replays it n_launches times on `stream` (asynchronous).  A replay gives the
 * same bits as the same cycles called one by one.  The graph holds the launch
 * shape and buffers of capture time: capture again after
 * soma_set_sweep_blocks or soma_set_scheme.  The graph contains kernel nodes only. */
int32_t soma_capture_cycle(soma_system *sys, uint32_t cycles, uint32_t move_kind);
int32_t soma_run_cycle(soma_system *sys, uint32_t n_launches, void *stream);

/* ---- Autotuning ----------------------------------------------------------
 * Times candidate launch shapes over real SCMF cycles and keeps the fastest,
 * as the run-time tuner of Sec. 3.2.2 does for every critical parallel loop.
 * Launch shapes never change results, so the trajectory is bit-identical to
 * running the same number of cycles untuned: each candidate runs 1 + cycles
 * SCMF cycles of move_kind (out->cycles_run in total; the sweep index and the
 * acceptance counters advance accordingly).  With a cache file (may be NULL)
 * a stored choice for the same sizes and move kind is applied without running
 * anything (out->from_cache = 1); a new choice is appended to the file (text,
 * one line per key; an unwritable file is ignored).  BLOCKING. */
typedef struct soma_tune {
  uint32_t mode;          /* batches: 0 XCD ranges, 1 round-robin items */
  uint32_t grid_blocks;   /* 0: one block per tile group; else persistent blocks */
  float ms_per_cycle;     /* measured time of the chosen shape (0 on a cache hit) */
  uint32_t candidates;    /* shapes timed */
  uint32_t cycles_run;    /* SCMF cycles run while tuning */
  uint32_t from_cache;
  uint32_t hist_mode;     /* single systems: SOMA_HIST_DIRECT or SOMA_HIST_BINNED */
  uint32_t block_threads; /* single systems: threads per block of the sweep */
} soma_tune;
/* Single systems, SET order: the search space is the histogram mode
 * (SOMA_HIST_DIRECT, and SOMA_HIST_BINNED where the grid allows it) x the
 * block size of the local, smart-MC and bond-Gibbs sweeps (128, 256, 512
 * threads; the mixed sweep always runs 256) x the grid (one block per tile
 * group, or the persistent grid of as many blocks as the device holds at
 * once for that kernel and block size, from the runtime's occupancy query;
 * 2048 if it gives none): up to 12 candidates (4 for mixed moves).
 * Molecule order: the grid caps {none, 256, 512, 1024, 2048}.  Batches: the
 * histogram mode (direct, and binned where every system allows it; hist_mode)
 * x the item order (XCD ranges or round-robin; mode) x the grid {one block per
 * item, 2048, 8192}: up to 12 candidates. */
int32_t soma_autotune(soma_system *sys, uint32_t cycles, uint32_t move_kind,
                      const char *cache_path, void *stream, soma_tune *out);

/* ---- Batches of systems ----------------------------------------------------
 * Several systems (replicas of different sizes, chain lengths, interaction
 * parameters; each created by soma_init_system with its own buffers) swept by
 * one kernel launch per sweep and refreshed by one launch per field update,
 * so that small systems together fill the GPU (Secs. 5.1-5.2).  Chain tiles of all
 * systems form one work list, largest system first, cut into one contiguous
 * range per XCD.  Every bead draws the Philox numbers of its own system, so a
 * batched sweep equals the unbatched sweeps of the systems bit for bit.
 * All systems need the same count_width.  The batch keeps pointers to the
 * systems (they must outlive it) and its tables in a caller workspace of
 * soma_batch_workspace_size bytes (256-byte aligned, device memory).
 * soma_batch_create copies the tables and waits for the copy (blocking). */
typedef struct soma_batch soma_batch;
int32_t soma_batch_workspace_size(soma_system *const *systems, uint32_t n, uint64_t *bytes);
int32_t soma_batch_create(soma_system *const *systems, uint32_t n, void *workspace,
                          uint64_t workspace_bytes, void *stream, soma_batch **out);
/* Launch shape: mode 0 (XCD ranges, default) or 1 (round-robin items);
 * grid_blocks 0 (one block per item, default) or a persistent grid. */
int32_t soma_batch_set_launch(soma_batch *b, uint32_t mode, uint32_t grid_blocks);
/* Count updates of batched sweeps (Eq. (4), Sec. 3.1.1), as soma_set_histogram
 * for one system: SOMA_HIST_DIRECT (default) or SOMA_HIST_BINNED, where each
 * sweep appends to the bins of every system's own workspace and one more launch
 * applies all of them brick by brick (mixed sweeps of a batch keep direct
 * atomics).  Counts, fields and trajectories are the same bits either way.  SOMA_E_UNSUPPORTED for SOMA_HIST_BINNED unless every
 * system has bins (see soma_set_histogram) and at most two bead types. */
int32_t soma_batch_set_histogram(soma_batch *b, uint32_t mode);
/* n_sweeps sweeps of every system with fields fixed (asynchronous). */
int32_t soma_batch_sweep(soma_batch *b, uint32_t n_sweeps, uint32_t move_kind, void *stream);
/* Field refresh of every system (asynchronous). */
int32_t soma_batch_update_fields(soma_batch *b, void *stream);
/* Cycles of the whole batch (as soma_cycle), with k chain subsets per cycle
 * (soma_batch_set_substeps copies the re-cut work list: blocking). */
int32_t soma_batch_set_substeps(soma_batch *b, uint32_t k, void *stream);
int32_t soma_batch_cycle(soma_batch *b, uint32_t n_cycles, uint32_t move_kind, void *stream);
/* Captured cycles of the whole batch, as soma_capture_cycle / soma_run_cycle. */
int32_t soma_batch_capture_cycle(soma_batch *b, uint32_t cycles, uint32_t move_kind);
int32_t soma_batch_run_cycle(soma_batch *b, uint32_t n_launches, void *stream);
/* Autotuning of the batch's launch shape, as soma_autotune. */
int32_t soma_batch_autotune(soma_batch *b, uint32_t cycles, uint32_t move_kind,
                            const char *cache_path, void *stream, soma_tune *out);
/* Releases the batch (host memory; the graph), after its queued work has
 * completed.  The systems stay valid. */
void soma_batch_destroy(soma_batch *b);

/* Stand-alone occupation histogram (Eq. (4)) of `pos` into `counts`
 * (cleared first), in the packed layout of cfg->count_width.  Both are device
 * pointers sized as by soma_buffer_sizes.  Asynchronous. */
int32_t soma_density_hist(const soma_config *cfg, const float *pos,
                           void *counts, void *stream);

/* Stand-alone fields (Eq. (12)) from packed `counts` into `omega` without
 * clearing the counts.  inv_rho = n_cells / n_beads.  Asynchronous. */
int32_t soma_field_from_counts(const soma_config *cfg, const void *counts,
                               float *omega, void *stream);

/* Stand-alone initial positions as in soma_init_system.  Asynchronous. */
int32_t soma_init_positions(const soma_config *cfg, float *pos, void *stream);

/* ---- Learned proposal --------------------------------------------------
 * Network parameters are an FP32 blob (device memory, caller-owned) of 8576
 * floats: shift[60] scale[60] (feature standardisation (f - shift) * scale),
 * W1[64][60] b1[64] W2[64][64] b2[64] W3[6][64] b3[6] (row-major, [out][in]).
 * Features of a bead: its own type's field at the 27 cells around its cell
 * ((dz,dy,dx) in -1..1, dz slowest), the other type's field at the same cells,
 * then the bond vectors r_{i-1} - r and r_{i+1} - r (zero where absent).
 * Network: ReLU, 60 -> 64 -> 64 -> 6, evaluated with BF16 inputs and weights
 * and FP32 accumulation on the matrix cores. */

/* Bytes of a prepared network (see soma_prepare_net). */
uint64_t soma_net_bytes(void);

/* Converts an FP32 parameter blob into the device layout the kernels use
 * (`net`: soma_net_bytes() bytes of device memory, 16-byte aligned).
 * Asynchronous. */
int32_t soma_prepare_net(const float *params, void *net, void *stream);

/* Installs the network of the mixed move for one species (or for every species
 * with species = SOMA_ALL_SPECIES) into the handle's workspace; a copy:
 * `params` may be freed or changed afterwards.  Mixed sweeps with p_learn > 0
 * need a network for every species that has chains.  Asynchronous.
 * SOMA_E_INVAL for a species index out of range. */
#define SOMA_ALL_SPECIES 0xFFFFFFFFu
int32_t soma_set_proposal(soma_system *sys, uint32_t species, const float *params,
                          void *stream);

/* Network outputs z [n][6] (FP32) for raw features [n][60] (FP32), both device
 * memory, with a prepared network.  Asynchronous. */
int32_t soma_mlp_forward(const void *net, const float *features, uint32_t n,
                         float *z, void *stream);

/* Raw features [n][60] (FP32, device) of bead beads[s] of global chain
 * chains[s] at the current positions and fields (training data).
 * Asynchronous. */
int32_t soma_features(soma_system *sys, const uint32_t *chains,
                      const uint32_t *beads, uint32_t n, float *out, void *stream);

/* Training samples from the running melt (plain-sampler trajectories).
 * Sample s (0 <= s < n) of round `round` is bead i of global chain c with
 * c = c0 + floor(w0 * nc / 2^32), i = floor(w1 * N / 2^32), where (w0, w1, ...)
 * is the Philox4x32-10 block of counter (s, 5 << 16, round, replica) and the
 * system's key, [c0, c0 + nc) the chains of `species` (all chains for
 * SOMA_ALL_SPECIES) and N the beads per chain of c's species.
 *   phase 0: writes r0 [n][3] = its position, features [n][60] (if not NULL)
 *            and picked [n][2] = (c, i) (if not NULL);
 *   phase 1: writes dr [n][3] = position now - r0 (same samples: same round).
 * Call phase 0, run K SCMF cycles, call phase 1: (features, dr) is one batch
 * of (input, target) pairs for soma_train_step.  All buffers device memory,
 * caller-owned.  Asynchronous. */
int32_t soma_collect_training(soma_system *sys, uint32_t species, uint32_t n, uint32_t round,
                              uint32_t phase, float *features, float *r0, float *dr,
                              uint32_t *picked, void *stream);

/* Options of one training step of the network. */
typedef struct soma_train_opts {
  float lr, beta1, beta2, eps;  /* Adam */
  float mu_max, log_sigma_min, log_sigma_max;  /* head bounds (as in soma_config) */
  uint32_t apply;               /* 0: gradient and loss only; 1: also the Adam update */
  uint32_t max_waves;           /* parallel partial gradients (0: one per 64 samples) */
} soma_train_opts;

/* ---- Structure factor (Sec. 5.6) ---------------------------------------
 * S(q) = N^2 rho0 / (4 V) |F[phi_A - phi_B](q)|^2, F the grid Fourier
 * transform dL^3 sum_c (.) exp(-i q.r_c), on every reciprocal-lattice vector
 * q = 2 pi (mx/nx, my/ny, mz/nz) (grid units); with phi = n/(rho0 dL^3) this
 * is N^2 |G(q)|^2 / (4 n_beads), G the transform of the count difference
 * n_A - n_B, N = n_ref.  Computed from the current counts in FP64 (three 1-D
 * transforms) into sq [n_cells] (device, cell order: index (mz*ny + my)*nx
 * + mx, m the non-negative lattice index).  Workspace (device, 256-byte
 * aligned): soma_sq_workspace_bytes(sys).  Asynchronous. */
uint64_t soma_sq_workspace_bytes(const soma_system *sys);
int32_t soma_structure_factor(soma_system *sys, void *workspace, uint64_t workspace_bytes,
                              double *sq, void *stream);

/* Host-side shell average of S(q) (host array `sq` as above): shell
 * k = round(|q| / dq), dq = 2 pi / min(nx, ny, nz), for k < n_shells;
 * s_avg[k] the mean over the shell, count[k] its size, q_mid[k] = k dq (may
 * be NULL); *peak (may be NULL) the shell k >= 1 of largest mean (first on
 * ties).  Runs on the calling thread. */
int32_t soma_sq_shells(const double *sq, uint32_t nx, uint32_t ny, uint32_t nz,
                       uint32_t n_shells, double *q_mid, double *s_avg, uint64_t *count,
                       uint32_t *peak);

/* The in-plane structure factor of a film (Sec. 5.6: S(q_par)), shell-averaged
 * over |q_par|: the first nx * ny entries of soma_structure_factor's output
 * (the m_z = 0 plane, i.e. the transform of the composition summed over z),
 * shell width 2 pi / min(nx, ny); otherwise as soma_sq_shells. */
int32_t soma_sq_plane_shells(const double *sq, uint32_t nx, uint32_t ny, uint32_t n_shells,
                             double *q_mid, double *s_avg, uint64_t *count, uint32_t *peak);

/* Device workspace bytes of soma_train_step for up to max_waves partials. */
uint64_t soma_train_workspace_bytes(uint32_t max_waves);

/* One training step on a batch of n samples (device memory): features
 * [n][60] raw features at time t, targets [n][3] the displacements of the
 * same beads between t and a later time.  Loss: mean Gaussian negative
 * log-likelihood of the targets under the head, without the constant.
 * Computes the mean gradient with BF16 MFMA forward and back-propagation (FP32
 * accumulation); with opts->apply, updates params (FP32 master blob, in
 * place) by Adam with moments adam_m, adam_v ([8576] FP32, zero before the
 * first step) at step `step` (1-based).  grad_out ([8576]) and loss_out (one
 * float) may be NULL.  workspace: soma_train_workspace_bytes(waves) bytes,
 * 256-byte aligned.  Asynchronous. */
int32_t soma_train_step(const float *features, const float *targets, uint32_t n,
                        float *params, float *adam_m, float *adam_v, uint32_t step,
                        const soma_train_opts *opts, void *workspace,
                        uint64_t workspace_bytes, float *grad_out, float *loss_out,
                        void *stream);

/* soma_train_step for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same step, arguments and results, without a workspace argument.  Its
 * scratch (the prepared network and up to SOMA_NOALLOC_TRAIN_WAVES partial
 * gradients, about 4.4 MB) is a fixed device array of the library, one per
 * GPU, held until the process ends; the call allocates nothing.  The number
 * of partial gradients is that of soma_train_step (opts->max_waves, or one
 * per 64 samples if 0); SOMA_E_SIZE if it exceeds SOMA_NOALLOC_TRAIN_WAVES
 * (larger batches: set opts->max_waves <= SOMA_NOALLOC_TRAIN_WAVES).  Every
 * scratch byte a step reads is written by the same step first.  All calls on
 * one GPU share the array: calls that overlap on one GPU (concurrent streams
 * or threads) race and must be serialised by the caller.  Asynchronous. */
#define SOMA_NOALLOC_TRAIN_WAVES 128u
int32_t soma_train_step_noalloc(const float *features, const float *targets, uint32_t n,
                                float *params, float *adam_m, float *adam_v, uint32_t step,
                                const soma_train_opts *opts, float *grad_out, float *loss_out,
                                void *stream);

/* Releases the handle (host memory and a captured graph).  Call it after the
 * work queued through the handle has completed. */
void soma_destroy(soma_system *sys);

/* Message of the last failed call on this thread ("" if none). */
const char *soma_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SOMA_H */
