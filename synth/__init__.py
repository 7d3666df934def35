"""Seeded synthetic inputs shared by the device path's tests and the oracle.

This module draws random inputs and describes workloads; it holds none of the
method's arithmetic (no energies, fields, moves or histograms).  Both sides of
a parity test start from the arrays made here.

Workloads follow the melts of arXiv:1711.03828 (Secs. 5.1-5.6): linear AB
diblock chains, grid spacing Re0/6, bonds Gaussian with the ideal-chain
statistics of the harmonic model.  No dataset is involved anywhere.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

MASTER_SEED = 20171110


@dataclass(frozen=True)
class SpeciesSpec:
    n_chains: int
    n: int        # beads per chain
    n_a: int      # leading A beads


@dataclass(frozen=True)
class Workload:
    """A melt: box in grid cells, Re0 in cells, interaction strengths, moves."""
    name: str
    grid: tuple            # (nx, ny, nz) cells
    species: tuple         # SpeciesSpec, ...
    re_cells: float        # Re0 in grid units
    n_ref: int             # reference chain length N of chiN, kappaN
    chi_n: float
    kappa_n: float
    count_width: int       # 16 or 32 bit per-type occupation counts
    a_frac: float = 0.1    # local move half-width in units of b0 = Re0/sqrt(Nref-1)
    smc_frac: float = 0.05 # smart-MC step A in units of Re0^2 / Nref
    sweeps: int = 100
    seed: int = MASTER_SEED

    @property
    def n_cells(self):
        nx, ny, nz = self.grid
        return nx * ny * nz

    @property
    def n_beads(self):
        return sum(s.n_chains * s.n for s in self.species)

    @property
    def n_chains(self):
        return sum(s.n_chains for s in self.species)


# Plain SCMF, AB diblock melt: 1024 A16B16 chains, 4x4x4 Re0 box, 24^3 grid.
C1_SMALL = Workload("diblock_1k_N32_grid24", (24, 24, 24),
                    (SpeciesSpec(1024, 32, 16),), 6.0, 32, 30.0, 50.0, 16, sweeps=100)
# Plain SCMF at scale: 4,194,304 A16B16 chains (134M beads), 64x64x32 Re0 box,
# 384x384x192 grid, u32 counts, local plus force-biased moves, 1000 sweeps.
C2_LARGE = Workload("diblock_4M_N32_grid384x384x192", (384, 384, 192),
                    (SpeciesSpec(4194304, 32, 16),), 6.0, 32, 20.0, 50.0, 32, sweeps=1000)
# Single melt of the learned-proposal study: 262,144 A16B16 chains, 96^3 grid.
C4_MEDIUM = Workload("diblock_256k_N32_grid96", (96, 96, 96),
                     (SpeciesSpec(262144, 32, 16),), 6.0, 32, 25.0, 50.0, 16, sweeps=100)

WORKLOADS = {w.name: w for w in (C1_SMALL, C2_LARGE, C4_MEDIUM)}


def scaled(w: Workload, n_chains: int, grid) -> Workload:
    """Same chemistry, different size (for tests)."""
    sp = tuple(SpeciesSpec(n_chains, s.n, s.n_a) for s in w.species)
    return Workload(w.name + f"_scaled{n_chains}", tuple(grid), sp, w.re_cells, w.n_ref,
                    w.chi_n, w.kappa_n, w.count_width, w.a_frac, w.smc_frac, w.sweeps,
                    w.seed)


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def gaussian_walks(seed: int, n_chains: int, n: int, grid, bond_sigma: float,
                   origin_spread=None) -> np.ndarray:
    """Chains as random walks with N(0, bond_sigma^2) bond components and origins
    uniform in the box (or in [0, origin_spread) per axis); float32 [n_chains*n, 3],
    chain-major, unwrapped."""
    g = rng(seed)
    box = np.asarray(grid if origin_spread is None else origin_spread, np.float64)
    origin = g.random((n_chains, 1, 3)) * box
    bonds = g.standard_normal((n_chains, n - 1, 3)) * bond_sigma
    walk = np.concatenate([np.zeros((n_chains, 1, 3)), np.cumsum(bonds, axis=1)], axis=1)
    return (origin + walk).astype(np.float32).reshape(-1, 3)


def pack_mask(cells: np.ndarray) -> np.ndarray:
    """Boolean per-cell array (cell order) -> packed uint32 words, bit c % 32 of
    word c // 32 set for a True cell (the interface format of impenetrable cells)."""
    cells = np.asarray(cells, bool).ravel()
    n_words = (cells.size + 31) // 32
    padded = np.zeros(n_words * 32, bool)
    padded[:cells.size] = cells
    bits = padded.reshape(n_words, 32).astype(np.uint64) << np.arange(32, dtype=np.uint64)
    return bits.sum(axis=1).astype(np.uint32)


def wall_cells(grid, z_planes) -> np.ndarray:
    """Boolean [n_cells] (cell order (z*ny + y)*nx + x) marking whole z planes."""
    nx, ny, nz = grid
    m = np.zeros((nz, ny, nx), bool)
    m[list(z_planes)] = True
    return m.ravel()


def film_walks(seed: int, n_chains: int, n: int, grid, bond_sigma: float, z_lo: float,
               z_hi: float) -> np.ndarray:
    """Random walks as gaussian_walks, with origins uniform in the slab
    z_lo <= z < z_hi and every z coordinate folded back into the slab by
    reflection at its faces (an initial state inside a film; float32)."""
    g = rng(seed)
    nx, ny, _ = grid
    width = z_hi - z_lo
    origin = g.random((n_chains, 1, 3)) * np.array([nx, ny, width]) + np.array([0, 0, z_lo])
    bonds = g.standard_normal((n_chains, n - 1, 3)) * bond_sigma
    walk = np.concatenate([np.zeros((n_chains, 1, 3)), np.cumsum(bonds, axis=1)], axis=1)
    pos = origin + walk
    t = np.mod(pos[..., 2] - z_lo, 2 * width)
    pos[..., 2] = z_lo + np.where(t < width, t, 2 * width - t)
    pos = pos.astype(np.float32)
    # float32 rounding may land on the upper face: keep it inside
    pos[..., 2] = np.minimum(pos[..., 2], np.nextafter(np.float32(z_hi), np.float32(0)))
    pos[..., 2] = np.maximum(pos[..., 2], np.float32(z_lo))
    return pos.reshape(-1, 3)


def encode_architecture(n: int, types, bonds) -> np.ndarray:
    """Molecular architecture in the 32-bit array format (interface format):
    word 0 = N; word 1+i = type_i << 24 | index of monomer i's bond list (0: no
    bonds); a bond word = (partner - i) in the low 27 bits (two's complement),
    bond type 0 in bits 27-30, bit 31 set on the last bond of a list.  Each
    bond (i, j) is listed at both ends, partners in ascending order."""
    nbrs = [[] for _ in range(n)]
    for i, j in bonds:
        nbrs[i].append(j)
        nbrs[j].append(i)
    words = [n] + [0] * n
    for i in range(n):
        lst = sorted(nbrs[i])
        start = len(words) if lst else 0
        words[1 + i] = (int(types[i]) << 24) | start
        for q, j in enumerate(lst):
            words.append(((j - i) & 0x7FFFFFF) | ((1 << 31) if q == len(lst) - 1 else 0))
    return np.asarray(words, np.uint32)


def linear_architecture(n: int, n_a: int) -> np.ndarray:
    return encode_architecture(n, [0 if i < n_a else 1 for i in range(n)],
                               [(i, i + 1) for i in range(n - 1)])


def star_bonds(arms: int, arm_len: int):
    """Star of `arms` arms of `arm_len` monomers around a core (monomer 0),
    numbered arm by arm outward: (n, bonds)."""
    bonds = []
    for a in range(arms):
        first = 1 + a * arm_len
        bonds.append((0, first))
        bonds += [(first + k, first + k + 1) for k in range(arm_len - 1)]
    return 1 + arms * arm_len, bonds


def ring_bonds(n: int):
    return n, [(i, (i + 1) % n) for i in range(n)]


def tree_walks(seed: int, n_chains: int, n: int, bonds, grid, bond_sigma: float) -> np.ndarray:
    """Ideal conformations of a tree molecule: monomer 0 uniform in the box, every
    other monomer its lower-numbered bonded partner plus an N(0, bond_sigma^2)
    vector per component (every monomer must have one; float32)."""
    parent = [-1] * n
    for i, j in bonds:
        lo, hi = min(i, j), max(i, j)
        if parent[hi] < 0:
            parent[hi] = lo
    assert all(p >= 0 for p in parent[1:])
    g = rng(seed)
    pos = np.zeros((n_chains, n, 3))
    pos[:, 0] = g.random((n_chains, 3)) * np.asarray(grid, np.float64)
    steps = g.standard_normal((n_chains, n, 3)) * bond_sigma
    for i in range(1, n):
        pos[:, i] = pos[:, parent[i]] + steps[:, i]
    return pos.astype(np.float32).reshape(-1, 3)


def ring_walks(seed: int, n_chains: int, n: int, grid, bond_sigma: float) -> np.ndarray:
    """Ideal ring conformations: a Gaussian walk of n steps with its end-to-end
    vector spread back over the steps (the walk conditioned to close); float32."""
    g = rng(seed)
    steps = g.standard_normal((n_chains, n, 3)) * bond_sigma
    walk = np.cumsum(steps, axis=1)
    frac = (np.arange(1, n + 1) / n)[None, :, None]
    bridge = walk - frac * walk[:, -1:, :]
    origin = g.random((n_chains, 1, 3)) * np.asarray(grid, np.float64)
    pos = origin + np.concatenate([np.zeros((n_chains, 1, 3)), bridge[:, :-1]], axis=1)
    return pos.astype(np.float32).reshape(-1, 3)


def uniform_field(seed: int, n_cells: int, lo: float, hi: float) -> np.ndarray:
    """Random per-type fields, float32 [2, n_cells]."""
    return rng(seed).uniform(lo, hi, size=(2, n_cells)).astype(np.float32)


def boundary_positions(grid) -> np.ndarray:
    """Hand-picked positions on and near cell faces, box faces and negative
    coordinates (float32 [k, 3])."""
    nx, ny, nz = grid
    eps = np.float32(1e-6)
    vals_x = [0.0, 0.5, 1.0, -0.0, -0.5, -1.0, nx, nx - eps, nx + 0.25, -nx, -nx - 0.5,
              2.0 * nx + 1.0, 3.999999, 1e4 + 0.5, -1e4 - 0.25]
    out = []
    for i, x in enumerate(vals_x):
        out.append([x, (x * 0.5 + i) % (2 * ny) - ny / 2, -x + 0.25 * i])
    return np.asarray(out, np.float32)


# Parameter blob of the learned proposal's network (FP32, flat).  This is an
# interface format shared by every consumer: per-feature standardisation
# (shift[60], scale[60]), then W1[64][60], b1[64], W2[64][64], b2[64],
# W3[6][64], b3[6], padded to 8576 floats.
MLP_LAYOUT = {"shift": 0, "scale": 60, "w1": 120, "b1": 3960, "w2": 4024, "b2": 8120,
              "w3": 8184, "b3": 8568, "size": 8576}


def mlp_params(seed: int, *, shift=None, scale=None, weight_gain=1.0, out_gain=0.1) -> np.ndarray:
    """Random network weights (He-like scaling), standardisation constants given
    or identity; output layer scaled by out_gain."""
    g = rng(seed)
    L = MLP_LAYOUT
    p = np.zeros(L["size"], np.float32)
    p[L["shift"]:L["shift"] + 60] = 0.0 if shift is None else shift
    p[L["scale"]:L["scale"] + 60] = 1.0 if scale is None else scale
    p[L["w1"]:L["w1"] + 3840] = g.standard_normal(3840) * weight_gain / np.sqrt(60)
    p[L["b1"]:L["b1"] + 64] = g.standard_normal(64) * 0.1
    p[L["w2"]:L["w2"] + 4096] = g.standard_normal(4096) * weight_gain / np.sqrt(64)
    p[L["b2"]:L["b2"] + 64] = g.standard_normal(64) * 0.1
    p[L["w3"]:L["w3"] + 384] = g.standard_normal(384) * out_gain / np.sqrt(64)
    p[L["b3"]:L["b3"] + 6] = g.standard_normal(6) * out_gain
    return p


def splitmix64(x: int) -> int:
    """SplitMix64 output for state x (Steele, Lea, Flood 2014): per-replica seeds."""
    z = (x + 0x9E3779B97F4A7C15) & 0xFFFFFFFFFFFFFFFF
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & 0xFFFFFFFFFFFFFFFF
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & 0xFFFFFFFFFFFFFFFF
    return z ^ (z >> 31)


def _cube_side(volume_re3: float, re_cells: float) -> int:
    return max(2, int(round(re_cells * volume_re3 ** (1.0 / 3.0))))


def c3_replicas(n_rep: int = 64, master: int = MASTER_SEED, scale: float = 1.0):
    """Replica ensemble of the batched study: chains log-uniform on [2048, 262144]
    (times `scale`), N in {16, 32, 64}, A fraction in {0.3, 0.5}, chiN from 10 to 40
    over the replicas, kappaN 50; volume 4 Re0^3 per 1024 chains, a cube at grid
    spacing Re0/6.  Replica r has seed SplitMix64(master + r)."""
    g = rng(master + 3)
    out = []
    for r in range(n_rep):
        n_chains = max(1, int(round(np.exp(g.uniform(np.log(2048), np.log(262144))) * scale)))
        n = int(g.choice([16, 32, 64]))
        f = float(g.choice([0.3, 0.5]))
        chi = 10.0 + 30.0 * r / max(1, n_rep - 1)
        side = _cube_side(4.0 * n_chains / 1024.0, 6.0)
        out.append(Workload(f"c3_r{r}", (side, side, side),
                            (SpeciesSpec(n_chains, n, int(round(f * n))),), 6.0, n, chi, 50.0,
                            16, seed=splitmix64(master + r)))
    return out


def c5_replicas(n_rep: int = 32, master: int = MASTER_SEED, scale: float = 1.0):
    """Blend replicas: chains log-uniform on [16384, 131072] (times `scale`), beads
    70% A16B16 diblocks, 15% A16 and 15% B16 homopolymers (chains 1 : 0.4286 :
    0.4286), chiN from 15 to 35 over the replicas, kappaN 50, reference N 32,
    the bead density of a 1024-chain N=32 melt in 4 Re0^3."""
    g = rng(master + 5)
    out = []
    for r in range(n_rep):
        n_total = np.exp(g.uniform(np.log(16384), np.log(131072))) * scale
        n_d = max(1, int(round(n_total / (1.0 + 2 * 0.15 / 0.70 * 2))))
        n_h = max(1, int(round(n_d * 0.15 / 0.70 * 2)))
        beads = 32 * n_d + 16 * 2 * n_h
        side = _cube_side(beads / (1024.0 * 32 / 4.0), 6.0)
        chi = 15.0 + 20.0 * r / max(1, n_rep - 1)
        sp = (SpeciesSpec(n_d, 32, 16), SpeciesSpec(n_h, 16, 16), SpeciesSpec(n_h, 16, 0))
        out.append(Workload(f"c5_r{r}", (side, side, side), sp, 6.0, 32, chi, 50.0, 16,
                            seed=splitmix64(master + 1000 + r)))
    return out


# ----------------------------------------------------------------------------
# Statistical parity of observables: protocols run by both sides with their
# own seeds (the two samples are independent), compared at equal cycles.
# ----------------------------------------------------------------------------
# A melt at the bead density of the 256k-chain study (256/27 per cell):
# 256 A16B16 chains on 12 x 9 x 8 cells, chiN 25, kappaN 50.
C4_DENSITY_SUB = Workload("diblock_256_N32_grid12x9x8", (12, 9, 8),
                          (SpeciesSpec(256, 32, 16),), 6.0, 32, 25.0, 50.0, 16, sweeps=100)


@dataclass(frozen=True)
class ObsProtocol:
    """Init from the seed (Philox init, stratified origins), `cycles` SCMF
    cycles of `move`; samples of Re^2 and Rg^2 after cycles first, first +
    every, ..., cycles; acceptance over cycles first+1 .. cycles; S(q) shells
    after the last cycle."""
    name: str
    workload: Workload
    move: str            # "local", "smc", "gibbs" or "learned" (p_learn = 1)
    cycles: int
    first: int
    every: int
    n_shells: int = 8


OBS_PROTOCOLS = (
    ObsProtocol("c1_local", C1_SMALL, "local", 300, 100, 10),
    ObsProtocol("c1_smc", C1_SMALL, "smc", 300, 100, 10),
    ObsProtocol("c1_gibbs", C1_SMALL, "gibbs", 300, 100, 10),
    ObsProtocol("c4dens_local", C4_DENSITY_SUB, "local", 100, 40, 5),
    ObsProtocol("c4dens_learned", C4_DENSITY_SUB, "learned", 100, 40, 5),
)
OBS_SEEDS_ORACLE = tuple(1001 + i for i in range(12))
OBS_SEEDS_DEVICE = tuple(2001 + i for i in range(12))


def designed_net_params(seed: int = 1, c: float = 0.1, sigma_bias: float = 0.36,
                        noise: float = 0.01) -> np.ndarray:
    """Network weights (interface layout) for a proposal that drifts a bead by
    about c (b_prev + b_next) -- towards its bonded neighbours: ReLU pairs carry
    the six bond features through both hidden layers; every other weight is
    small noise, so the fields still enter.  The log-sigma outputs get the bias
    sigma_bias (0.36: a width of about 0.2 cells with log-sigma bounds
    log 0.02 .. 0)."""
    L = MLP_LAYOUT
    g = rng(seed)
    p = np.zeros(L["size"], np.float32)
    p[L["scale"]:L["scale"] + 60] = 1.0
    w1 = g.standard_normal((64, 60)) * noise
    for j in range(6):
        w1[j, 54 + j] = 1.0
        w1[6 + j, 54 + j] = -1.0
    w2 = g.standard_normal((64, 64)) * noise
    for u in range(12):
        w2[u, u] = 1.0
    w3 = g.standard_normal((6, 64)) * noise
    for d in range(3):
        w3[d, d] += c
        w3[d, 6 + d] -= c
        w3[d, 3 + d] += c
        w3[d, 9 + d] -= c
    p[L["w1"]:L["w1"] + 3840] = w1.ravel()
    p[L["w2"]:L["w2"] + 4096] = w2.ravel()
    p[L["w3"]:L["w3"] + 384] = w3.ravel()
    p[L["b3"] + 3:L["b3"] + 6] = sigma_bias
    return p
