"""Plain CPU oracle for the SCMF hot path -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product library never loads it, and
it imports nothing from the product package: the two sides implement the same
written specification independently and share only the seeded input generators
in ``synth``.

Contents
  * ``soma_oracle.c`` -- the method step by step in plain C (FP64 energies on
    the FP32 state), wrapped here with ctypes;
  * ``philox_py``     -- a second, independent Philox4x32-10 in Python integers;
  * ``references``    -- closed forms and brute-force references that pin the
    oracle (ideal-chain acceptance, 3-bead Boltzmann marginals, ...).

Paper: arXiv:1711.03828 (SCMF simulation of soft coarse-grained polymers).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "soma_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

MOVE_LOCAL = 0
MOVE_SMC = 1
MOVE_GIBBS = 3


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (no fast-math, no FP contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=gnu11", "-ffp-contract=off", "-fno-fast-math",
               "-fopenmp", "-fPIC", "-shared", _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        u32, u64, f32, f64, i32 = (ctypes.c_uint32, ctypes.c_uint64, ctypes.c_float,
                                   ctypes.c_double, ctypes.c_int)
        L.orc_philox_batch.argtypes = [u64, P, P, P]
        L.orc_u01.argtypes = [u32]
        L.orc_u01.restype = f32
        L.orc_v11.argtypes = [u32]
        L.orc_v11.restype = f32
        L.orc_density_hist.argtypes = [P, u32, P, P, P, u32, u32, u32, P]
        L.orc_field_f64.argtypes = [P, u64, f64, f64, f64, u32, P, P, P]
        L.orc_field_f32.argtypes = [P, u64, f32, f32, f32, u32, P, P, P]
        L.orc_h_nb.argtypes = [P, u64, f64, f64, f64, u32, u32, P]
        L.orc_set_forbidden.argtypes = [P]
        L.orc_set_self_term.argtypes = [ctypes.c_double]
        L.orc_h_nb.restype = f64
        L.orc_mc_sweep.argtypes = [P, u32, u32, u32, f32, u32, P, u32, u32, u32, u32,
                                   f32, u64, u32, u32, u32, u32, P, i32]
        L.orc_mc_sweep.restype = u64
        L.orc_mc_sweep_molecule.argtypes = [P, u32, u32, u32, f32, u32, P, u32, u32, u32, f32,
                                            u64, u32, u32, u32, P, P, ctypes.c_int]
        L.orc_mc_sweep_molecule.restype = u64
        L.orc_mc_sweep_arch.argtypes = [P, u32, P, u32, f32, u32, P, u32, u32, u32, f32, u64,
                                        u32, u32, u32, u32, P, ctypes.c_int]
        L.orc_mc_sweep_arch.restype = u64
        L.orc_arch_sets.argtypes = [P, u32, P]
        L.orc_arch_sets.restype = ctypes.c_int
        L.orc_density_hist_arch.argtypes = [P, u32, P, u32, u32, u32, u32, u32, P]
        L.orc_field_multi_f64.argtypes = [P, u64, u32, f64, P, f64, u32, P]
        L.orc_field_multi_f32.argtypes = [P, u64, u32, f32, P, f32, u32, P]
        L.orc_h_nb_multi.argtypes = [P, u64, u32, f64, P, f64, u32, u32]
        L.orc_h_nb_multi.restype = f64
        L.orc_density_hist_arch.restype = ctypes.c_int
        L.orc_pick_bead.argtypes = [u32, u32]
        L.orc_pick_bead.restype = u32
        L.orc_brick_cell_batch.argtypes = [u64, P, u32, u32, u32, P]
        L.orc_init_chains.argtypes = [P, u32, u32, f32, u32, u32, u32, u64, u32, u32,
                                      u32, u32]
        L.orc_chain_observables.argtypes = [P, u32, u32, P, P, P]
        L.orc_field_energy.argtypes = [P, u32, u32, u32, P, u32, u32, u32, u32]
        L.orc_field_energy.restype = f64
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


# --------------------------------------------------------------------------
# Thin wrappers (argument marshalling only; all arithmetic is in the C file)
# --------------------------------------------------------------------------
def philox(ctr: np.ndarray, key: np.ndarray) -> np.ndarray:
    ctr = _c(ctr, np.uint32).reshape(-1, 4)
    key = _c(np.broadcast_to(key, (ctr.shape[0], 2)), np.uint32)
    out = np.empty_like(ctr)
    lib().orc_philox_batch(ctr.shape[0], _ptr(ctr), _ptr(key), _ptr(out))
    return out


def u01(x: int) -> float:
    return lib().orc_u01(int(x))


def v11(x: int) -> float:
    return lib().orc_v11(int(x))


@dataclass
class Species:
    n_chains: int
    n: int          # beads per chain
    n_a: int        # leading A beads


def density_hist(pos: np.ndarray, species: list[Species], grid) -> np.ndarray:
    """Counts as uint32 array [2, n_cells] (type A plane, type B plane)."""
    nx, ny, nz = grid
    pos = _c(pos, np.float32)
    counts = np.zeros((2, nx * ny * nz), np.uint32)
    nc = _c([s.n_chains for s in species], np.uint32)
    nn = _c([s.n for s in species], np.uint32)
    na = _c([s.n_a for s in species], np.uint32)
    lib().orc_density_hist(_ptr(pos), len(species), _ptr(nc), _ptr(nn), _ptr(na),
                           nx, ny, nz, _ptr(counts))
    return counts


def _opt(a, dtype):
    return None if a is None else _c(a, dtype)


def field_f64(counts: np.ndarray, inv_rho: float, chi_n: float, kappa_n: float, ext=None,
              forbid=None, form=1) -> np.ndarray:
    """ext: optional float32 [2, n_cells] external field; forbid: optional packed
    bit mask (uint32, bit c % 32 of word c // 32) of impenetrable cells."""
    counts = _c(counts, np.uint32)
    n_cells = counts.shape[-1]
    ext, forbid = _opt(ext, np.float32), _opt(forbid, np.uint32)
    om = np.empty((2, n_cells), np.float64)
    lib().orc_field_f64(_ptr(counts), n_cells, inv_rho, chi_n, kappa_n, form,
                        _ptr(ext) if ext is not None else None,
                        _ptr(forbid) if forbid is not None else None, _ptr(om))
    return om


def field_f32(counts: np.ndarray, inv_rho, chi_n, kappa_n, ext=None, forbid=None,
              form=1) -> np.ndarray:
    counts = _c(counts, np.uint32)
    n_cells = counts.shape[-1]
    ext, forbid = _opt(ext, np.float32), _opt(forbid, np.uint32)
    om = np.empty((2, n_cells), np.float32)
    lib().orc_field_f32(_ptr(counts), n_cells, float(np.float32(inv_rho)),
                        float(np.float32(chi_n)), float(np.float32(kappa_n)), form,
                        _ptr(ext) if ext is not None else None,
                        _ptr(forbid) if forbid is not None else None, _ptr(om))
    return om


def h_nb(counts, inv_rho, chi_n, kappa_n, n_ref, forbid=None, form=1) -> float:
    """form 1: the K^1 interaction term, 0: K^0 (Eq. (6))."""
    counts = _c(counts, np.uint32)
    forbid = _opt(forbid, np.uint32)
    return lib().orc_h_nb(_ptr(counts), counts.shape[-1], inv_rho, chi_n, kappa_n, n_ref, form,
                          _ptr(forbid) if forbid is not None else None)


def _chi_matrix(chi, n_t, dtype):
    chi = np.ascontiguousarray(np.asarray(chi, dtype=dtype).reshape(n_t, n_t))
    if not np.array_equal(chi, chi.T):
        raise ValueError("chi matrix must be symmetric")
    return chi


def field_multi_f64(counts, inv_rho, chi, kappa_n, form=1) -> np.ndarray:
    """Fields of n_t types (counts [n_t, n_cells], chi [n_t, n_t] of chi_ij N)."""
    counts = _c(counts, np.uint32)
    n_t, n_cells = counts.shape
    chi = _chi_matrix(chi, n_t, np.float64)
    om = np.empty((n_t, n_cells), np.float64)
    lib().orc_field_multi_f64(_ptr(counts), n_cells, n_t, inv_rho, _ptr(chi), kappa_n, form,
                              _ptr(om))
    return om


def field_multi_f32(counts, inv_rho, chi, kappa_n, form=1) -> np.ndarray:
    counts = _c(counts, np.uint32)
    n_t, n_cells = counts.shape
    chi = _chi_matrix(chi, n_t, np.float32)
    om = np.empty((n_t, n_cells), np.float32)
    lib().orc_field_multi_f32(_ptr(counts), n_cells, n_t, float(np.float32(inv_rho)), _ptr(chi),
                              float(np.float32(kappa_n)), form, _ptr(om))
    return om


def h_nb_multi(counts, inv_rho, chi, kappa_n, n_ref, form=1) -> float:
    counts = _c(counts, np.uint32)
    n_t, n_cells = counts.shape
    chi = _chi_matrix(chi, n_t, np.float64)
    return lib().orc_h_nb_multi(_ptr(counts), n_cells, n_t, inv_rho, _ptr(chi), kappa_n, n_ref,
                                form)


class _walls:
    """Sets the oracle's impenetrable-cell mask for the duration of one sweep."""

    def __init__(self, forbid):
        self.mask = _opt(forbid, np.uint32)

    def __enter__(self):
        lib().orc_set_forbidden(_ptr(self.mask) if self.mask is not None else None)

    def __exit__(self, *exc):
        lib().orc_set_forbidden(None)


class _self_term:
    """Sets the energy of cell-changing moves (orc_set_self_term) for one call."""

    def __init__(self, s):
        self.s = float(s)

    def __enter__(self):
        lib().orc_set_self_term(self.s)

    def __exit__(self, *exc):
        lib().orc_set_self_term(0.0)


def self_energy(kappa_n, chi_n, inv_rho, n_ref, form=1) -> np.float32:
    """Second difference of the grid Hamiltonian per bead, kT (FP32 as the
    device rounds it): kappaN/(N rho) for the K^1 form, (kappaN - chiN/2)/(N rho)
    for K^0."""
    k = float(kappa_n) - (0.5 * float(chi_n) if form == 0 else 0.0)
    return np.float32(k * float(inv_rho) / float(n_ref))


def mc_sweep(pos: np.ndarray, sp: Species, omega: np.ndarray, grid, *, k0, n_ref,
             move_kind=MOVE_LOCAL, step, seed, sweep, replica=0, chain_base=0,
             set_order=0, want_flags=False, threads=1, forbid=None, self_term=0.0):
    """In-place sweep of one species' chains (pos is that species' slice).
    self_term: energy added to every move that changes cell (0: none).

    Returns (n_accepted, flags or None)."""
    assert pos.dtype == np.float32 and pos.flags.c_contiguous
    assert pos.size == sp.n_chains * sp.n * 3
    nx, ny, nz = grid
    omega = _c(omega, np.float32)
    assert omega.size == 2 * nx * ny * nz
    flags = np.zeros(sp.n_chains * sp.n, np.uint8) if want_flags else None
    with _walls(forbid), _self_term(self_term):
        acc = lib().orc_mc_sweep(_ptr(pos), sp.n_chains, sp.n, sp.n_a, float(np.float32(k0)),
                                 n_ref, _ptr(omega), nx, ny, nz, move_kind,
                                 float(np.float32(step)), seed, sweep, replica, chain_base,
                                 set_order, _ptr(flags) if flags is not None else None,
                                 threads)
    return acc, flags


def mc_sweep_molecule(pos: np.ndarray, sp: Species, omega: np.ndarray, grid, *, k0, n_ref,
                      step, seed, sweep, replica=0, chain_base=0, want_flags=False,
                      threads=1, forbid=None):
    """In-place local-move sweep in the molecule-parallel order (N attempts per
    chain on randomly picked beads).  Returns (n_accepted, accept flags or None,
    picked beads or None), the last two per attempt [n_chains * N]."""
    assert pos.dtype == np.float32 and pos.flags.c_contiguous
    assert pos.size == sp.n_chains * sp.n * 3
    nx, ny, nz = grid
    omega = _c(omega, np.float32)
    assert omega.size == 2 * nx * ny * nz
    flags = np.zeros(sp.n_chains * sp.n, np.uint8) if want_flags else None
    picked = np.zeros(sp.n_chains * sp.n, np.uint32) if want_flags else None
    with _walls(forbid):
        acc = lib().orc_mc_sweep_molecule(_ptr(pos), sp.n_chains, sp.n, sp.n_a,
                                          float(np.float32(k0)), n_ref, _ptr(omega), nx, ny, nz,
                                          float(np.float32(step)), seed, sweep, replica, chain_base,
                                          _ptr(flags) if flags is not None else None,
                                          _ptr(picked) if picked is not None else None, threads)
    return acc, flags, picked


def arch_sets(words: np.ndarray):
    """(number of independent sets, set of every monomer) of an architecture, or
    (-1, None) if the words are malformed."""
    words = _c(words, np.uint32)
    n = int(words[0]) if words.size else 0
    out = np.zeros(max(n, 1), np.uint32)
    k = lib().orc_arch_sets(_ptr(words), words.size, _ptr(out))
    return (k, out[:n]) if k > 0 else (-1, None)


def mc_sweep_arch(pos: np.ndarray, n_chains: int, words: np.ndarray, omega: np.ndarray, grid, *,
                  k0, n_ref, step, seed, sweep, replica=0, chain_base=0, set_order=0,
                  want_flags=False, threads=1, forbid=None):
    """In-place local-move sweep (SET order) of chains of one architecture.
    Returns (n_accepted, flags or None)."""
    words = _c(words, np.uint32)
    n = int(words[0])
    assert pos.dtype == np.float32 and pos.flags.c_contiguous and pos.size == n_chains * n * 3
    nx, ny, nz = grid
    omega = _c(omega, np.float32)
    n_cells = nx * ny * nz
    types = words[1:1 + n] >> 24
    assert omega.size % n_cells == 0 and omega.size // n_cells > int(types.max()), \
        "omega needs a plane for every type of the architecture"
    flags = np.zeros(n_chains * n, np.uint8) if want_flags else None
    with _walls(forbid):
        acc = lib().orc_mc_sweep_arch(_ptr(pos), n_chains, _ptr(words), words.size,
                                      float(np.float32(k0)), n_ref, _ptr(omega), nx, ny, nz,
                                      float(np.float32(step)), seed, sweep, replica, chain_base,
                                      set_order, _ptr(flags) if flags is not None else None,
                                      threads)
    if acc == 2 ** 64 - 1:
        raise ValueError("malformed architecture")
    return acc, flags


def density_hist_arch(pos: np.ndarray, n_chains: int, words: np.ndarray, grid,
                      n_types: int = 2) -> np.ndarray:
    """Counts [n_types, n_cells] of chains of one architecture."""
    words = _c(words, np.uint32)
    pos = _c(pos, np.float32)
    nx, ny, nz = grid
    out = np.empty((n_types, nx * ny * nz), np.uint32)
    if lib().orc_density_hist_arch(_ptr(pos), n_chains, _ptr(words), words.size, nx, ny, nz,
                                   n_types, _ptr(out)):
        raise ValueError("malformed architecture")
    return out


def pick_bead(word: int, n: int) -> int:
    return lib().orc_pick_bead(int(word), int(n))


def brick_cell(k: np.ndarray, grid) -> np.ndarray:
    k = _c(k, np.uint64)
    out = np.empty((k.size, 3), np.uint64)
    lib().orc_brick_cell_batch(k.size, _ptr(k), *grid, _ptr(out))
    return out


def init_chains(sp: Species, grid, *, bond_sigma, seed, replica=0, chain_base=0,
                total_chains=None, origin_mode=1) -> np.ndarray:
    pos = np.empty((sp.n_chains * sp.n, 3), np.float32)
    total = sp.n_chains if total_chains is None else total_chains
    lib().orc_init_chains(_ptr(pos), sp.n_chains, sp.n, float(np.float32(bond_sigma)),
                          *grid, seed, replica, chain_base, total, origin_mode)
    return pos


def chain_observables(pos: np.ndarray, n_chains: int, n: int):
    pos = _c(pos, np.float32)
    re2 = np.empty(n_chains)
    rg2 = np.empty(n_chains)
    b2 = np.empty(n_chains)
    lib().orc_chain_observables(_ptr(pos), n_chains, n, _ptr(re2), _ptr(rg2), _ptr(b2))
    return re2, rg2, b2


def field_energy(pos, sp: Species, omega, grid, n_ref) -> float:
    pos = _c(pos, np.float32)
    omega = _c(omega, np.float32)
    return lib().orc_field_energy(_ptr(pos), sp.n_chains, sp.n, sp.n_a, _ptr(omega),
                                  *grid, n_ref)


# --------------------------------------------------------------------------
# Learned proposal (network, loss, features, mixed sweep)
# --------------------------------------------------------------------------
MOVE_MIXED = 2
NF, NH, NO = 60, 64, 6


def _lib_mlp():
    L = lib()
    if getattr(L, "_mlp_ready", False):
        return L
    P = ctypes.c_void_p
    u32, u64, f32, f64, i32 = (ctypes.c_uint32, ctypes.c_uint64, ctypes.c_float,
                               ctypes.c_double, ctypes.c_int)
    L.orc_param_layout.argtypes = [u32]
    L.orc_param_layout.restype = u32
    L.orc_bf16.argtypes = [f32]
    L.orc_bf16.restype = f32
    L.orc_mlp_forward.argtypes = [P, P, i32, P, P]
    L.orc_fold_params.argtypes = [P, P]
    L.orc_mlp_backward.argtypes = [P, P, P, i32, P]
    L.orc_nll.argtypes = [P, P, f64, f64, f64, P]
    L.orc_nll.restype = f64
    L.orc_nll_batch.argtypes = [P, u64, P, P, f64, f64, f64, i32, P, P]
    L.orc_nll_batch.restype = f64
    L.orc_features_batch.argtypes = [P, u32, u32, u32, P, P, u32, u32, u32, P]
    L.orc_mc_sweep_mixed.argtypes = [P, u32, u32, u32, f32, u32, P, u32, u32, u32, f32, f32,
                                     P, f32, f32, f32, i32, u64, u32, u32, u32, u32, P, P, P,
                                     P, P, P, i32]
    L.orc_bf16_boundary.argtypes = [f64, P]
    L.orc_bf16_boundary.restype = f64
    L.orc_set_envelope.argtypes = [f64]
    L.orc_set_acc_f32.argtypes = [i32]
    L.orc_nll_batch_envelope.argtypes = [P, u64, P, P, f64, f64, f64, P, P, P, P]
    L.orc_nll_batch_envelope.restype = f64
    L.orc_mlp_forward_envelope.argtypes = [P, u64, P, P, P]
    L.orc_mlp_forward_envelope.restype = u64
    L.orc_mc_sweep_mixed.restype = u64
    L._mlp_ready = True
    return L


def param_layout():
    L = _lib_mlp()
    names = ["shift", "scale", "w1", "b1", "w2", "b2", "w3", "b3", "size"]
    return {n: int(L.orc_param_layout(i)) for i, n in enumerate(names)}


def bf16(x: float) -> float:
    return _lib_mlp().orc_bf16(float(x))


def fold_params(params: np.ndarray) -> np.ndarray:
    """The network with its input standardisation folded into the first layer
    (the form the learned move evaluates; see orc_fold_params)."""
    p = _c(params, np.float32)
    q = np.empty_like(p)
    _lib_mlp().orc_fold_params(_ptr(p), _ptr(q))
    return q


def mlp_forward(params: np.ndarray, features: np.ndarray, bf16_mode=False):
    """z [n, 6] for features [n, 60]."""
    L = _lib_mlp()
    params = _c(params, np.float32)
    f = _c(features, np.float64).reshape(-1, NF)
    z = np.empty((f.shape[0], NO))
    for s in range(f.shape[0]):
        zs = np.empty(NO)
        L.orc_mlp_forward(_ptr(params), _ptr(f[s]), int(bf16_mode), _ptr(zs), None)
        z[s] = zs
    return z


def nll(z, dr, *, m_max, lo, hi):
    """(NLL of one displacement dr [3] under the head of z [6], dL/dz [6])."""
    L = _lib_mlp()
    z = _c(z, np.float64).reshape(NO)
    dr = _c(dr, np.float64).reshape(3)
    dz = np.empty(NO)
    loss = L.orc_nll(_ptr(z), _ptr(dr), m_max, lo, hi, _ptr(dz))
    return loss, dz


def nll_batch(params, features, targets, *, m_max, lo, hi, bf16_mode=False):
    """(mean NLL, gradient [P], z [n, 6])."""
    L = _lib_mlp()
    params = _c(params, np.float32)
    f = _c(features, np.float64).reshape(-1, NF)
    t = _c(targets, np.float64).reshape(-1, 3)
    grad = np.zeros(param_layout()["size"])
    z = np.empty((f.shape[0], NO))
    loss = L.orc_nll_batch(_ptr(params), f.shape[0], _ptr(f), _ptr(t), m_max, lo, hi,
                           int(bf16_mode), _ptr(grad), _ptr(z))
    return loss, grad, z


def bf16_boundary(v: float):
    """(distance of v from the nearest BF16 rounding boundary, the BF16 value
    on the other side of it)."""
    other = ctypes.c_double()
    d = _lib_mlp().orc_bf16_boundary(float(v), ctypes.byref(other))
    return d, other.value


class fp32_sums:
    """Context manager: the BF16 forward sums in FP32 in index order (another
    order of FP32 additions a device may take) instead of FP64."""

    def __enter__(self):
        _lib_mlp().orc_set_acc_f32(1)

    def __exit__(self, *exc):
        _lib_mlp().orc_set_acc_f32(0)


class envelope_scale:
    """Context manager scaling the rounding windows of the envelope."""

    def __init__(self, scale):
        self.scale = float(scale)

    def __enter__(self):
        _lib_mlp().orc_set_envelope(self.scale)

    def __exit__(self, *exc):
        _lib_mlp().orc_set_envelope(1.0)


def mlp_forward_envelope(params, features):
    """(z [n, 6] with the device's rounding points, bound [n, 6], ambiguous
    roundings): the device's outputs satisfy |z_dev - z| <= bound where every
    FP32 sum of the device lies within the error bound of its terms."""
    L = _lib_mlp()
    params = _c(params, np.float32)
    f = _c(features, np.float64).reshape(-1, NF)
    z = np.empty((f.shape[0], NO))
    bound = np.empty((f.shape[0], NO))
    na = L.orc_mlp_forward_envelope(_ptr(params), f.shape[0], _ptr(f), _ptr(z), _ptr(bound))
    return z, bound, int(na)


def nll_batch_envelope(params, features, targets, *, m_max, lo, hi):
    """Training gradient with the device's rounding points and its envelope:
    (mean loss, gradient [P], bound [P], ambiguous roundings, samples with
    one).  The device's gradient g satisfies |g - gradient| <= bound where
    every sum of the device lies within the FP32 error bound of its terms."""
    L = _lib_mlp()
    params = _c(params, np.float32)
    f = _c(features, np.float64).reshape(-1, NF)
    t = _c(targets, np.float64).reshape(-1, 3)
    size = param_layout()["size"]
    grad = np.zeros(size)
    bound = np.zeros(size)
    n_amb = ctypes.c_uint64()
    n_flag = ctypes.c_uint64()
    loss = L.orc_nll_batch_envelope(_ptr(params), f.shape[0], _ptr(f), _ptr(t), m_max, lo, hi,
                                    _ptr(grad), _ptr(bound), ctypes.byref(n_amb),
                                    ctypes.byref(n_flag))
    return loss, grad, bound, n_amb.value, n_flag.value


def features(pos, sp: Species, beads, omega, grid):
    """Features of bead beads[c] of chain c, [n_chains, 60]."""
    L = _lib_mlp()
    pos = _c(pos, np.float32)
    b = _c(beads, np.uint32)
    omega = _c(omega, np.float32)
    out = np.empty((sp.n_chains, NF))
    L.orc_features_batch(_ptr(pos), sp.n_chains, sp.n, sp.n_a, _ptr(b), _ptr(omega), *grid,
                         _ptr(out))
    return out


def mc_sweep_mixed(pos, sp: Species, omega, grid, *, k0, n_ref, local_a, p_learn, params,
                   m_max, lo, hi, bf16_mode=True, seed, sweep, replica=0, chain_base=0,
                   set_order=0, want_flags=False, threads=1, forbid=None, ambiguous=None,
                   pos_env=None, self_term=0.0):
    """In-place mixed (local / learned) sweep.  Returns (accepted, accepted_learned,
    bad_net, kind_flags, accept_flags).  With `ambiguous` (a uint8 array of
    n_chains * n, BF16 mode only) each move's entry is set to 1 where rounding
    alone may let the device decide it otherwise, and `pos_env` (float32, same
    size, optional) to how far the device's new position of an accepted move
    may lie from the oracle's through rounding (see ``nll_batch_envelope``)."""
    L = _lib_mlp()
    assert pos.dtype == np.float32 and pos.flags.c_contiguous
    params = _c(params, np.float32)
    omega = _c(omega, np.float32)
    kf = np.zeros(sp.n_chains * sp.n, np.uint8) if want_flags else None
    af = np.zeros(sp.n_chains * sp.n, np.uint8) if want_flags else None
    acc_l = ctypes.c_uint64()
    bad = ctypes.c_uint32()
    if ambiguous is not None:
        assert ambiguous.dtype == np.uint8 and ambiguous.size == sp.n_chains * sp.n
        assert ambiguous.flags.c_contiguous
        if pos_env is None:
            pos_env = np.zeros(sp.n_chains * sp.n, np.float32)
        assert pos_env.dtype == np.float32 and pos_env.size == ambiguous.size
        assert pos_env.flags.c_contiguous
        pos_env[:] = 0.0
    walls = _opt(forbid, np.uint32)
    lib().orc_set_forbidden(_ptr(walls) if walls is not None else None)
    lib().orc_set_self_term(float(self_term))
    try:
        acc = L.orc_mc_sweep_mixed(_ptr(pos), sp.n_chains, sp.n, sp.n_a, float(np.float32(k0)), n_ref,
                                   _ptr(omega), *grid, float(np.float32(local_a)),
                                   float(np.float32(p_learn)), _ptr(params), float(np.float32(m_max)),
                                   float(np.float32(lo)), float(np.float32(hi)), int(bf16_mode), seed,
                                   sweep, replica, chain_base, set_order,
                                   _ptr(kf) if kf is not None else None,
                                   _ptr(af) if af is not None else None,
                                   _ptr(ambiguous) if ambiguous is not None else None,
                                   _ptr(pos_env) if ambiguous is not None else None,
                                   ctypes.byref(acc_l), ctypes.byref(bad), threads)
    finally:
        lib().orc_set_forbidden(None)
        lib().orc_set_self_term(0.0)
    return acc, acc_l.value, bad.value, kf, af
