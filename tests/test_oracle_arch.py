"""Pins of the oracle's general-architecture sweep (Sec. 3.2.1 encoding,
Sec. 3.1.2 independent sets).

* decoding: malformed arrays are rejected; greedy sets are independent and
  give even/odd for a linear chain, two sets for a star, three for an odd ring;
* a linear chain given as an architecture sweeps bit for bit like the linear
  oracle (positions and accept flags, random and fixed set order, with walls);
* ideal star (f arms): attempts on monomers of degree g are accepted at the
  closed-form rate of a local move with bond stiffness g k0 / 2 (middle-bead
  form), and <|r_i - r_j|^2> = 3 d(i, j) / k0 stays at its Gaussian value;
* ideal ring of odd N (three sets, shuffled order): <|r_i - r_j|^2> =
  3 d (N - d) / (N k0) stays at its closed form.
"""
import math

import numpy as np
import pytest

import synth
from oracle import Species, references

RE = 6.0


def test_malformed_architectures_rejected(orc):
    good = synth.linear_architecture(4, 2)
    assert orc.arch_sets(good)[0] == 2
    # bond listed on one side only: drop monomer 3's list
    w = good.copy()
    w[4] = w[4] & 0xFF000000
    assert orc.arch_sets(w)[0] == -1
    # partner out of range
    w = good.copy()
    w[int(w[4] & 0xFFFFFF)] = (3 & 0x7FFFFFF) | (1 << 31)
    assert orc.arch_sets(w)[0] == -1
    # non-harmonic bond type
    w = good.copy()
    w[int(w[1] & 0xFFFFFF)] |= 1 << 27
    assert orc.arch_sets(w)[0] == -1
    # type code 8 (at most 8 types)
    w = good.copy()
    w[2] = (8 << 24) | (w[2] & 0xFFFFFF)
    assert orc.arch_sets(w)[0] == -1
    # list running off the array
    assert orc.arch_sets(good[:-1])[0] == -1


@pytest.mark.parametrize("kind", ["linear", "star", "ring7", "ring8", "comb"])
def test_sets_are_independent(orc, kind):
    if kind == "linear":
        n, bonds = 9, [(i, i + 1) for i in range(8)]
    elif kind == "star":
        n, bonds = synth.star_bonds(5, 4)
    elif kind == "comb":
        n, bonds = 16, [(i, i + 1) for i in range(7)] + [(i, 8 + i) for i in range(8)]
    else:
        n, bonds = synth.ring_bonds(int(kind[4:]))
    k, sets = orc.arch_sets(synth.encode_architecture(n, [0] * n, bonds))
    for i, j in bonds:
        assert sets[i] != sets[j]
    exp = {"linear": 2, "star": 2, "comb": 2, "ring7": 3, "ring8": 2}[kind]
    assert k == exp
    if kind == "linear":
        assert (sets == np.arange(n) % 2).all()


@pytest.mark.parametrize("set_order", [0, 1])
def test_linear_architecture_equals_linear_oracle(orc, set_order):
    n, n_chains = 32, 500
    grid = (24, 24, 12)
    omega = synth.uniform_field(7, 24 * 24 * 12, -3, 3)
    base = synth.film_walks(8, n_chains, n, grid, 0.6, 1.0, 11.0)
    mask = synth.pack_mask(synth.wall_cells(grid, [0, 11]))
    words = synth.linear_architecture(n, 12)
    p1, p2 = base.copy(), base.copy()
    for sweep in range(3):
        a1, f1 = orc.mc_sweep(p1, Species(n_chains, n, 12), omega, grid, k0=2.58, n_ref=32,
                              step=0.5, seed=17, sweep=sweep, set_order=set_order, chain_base=9,
                              want_flags=True, forbid=mask, threads=4)
        a2, f2 = orc.mc_sweep_arch(p2, n_chains, words, omega, grid, k0=2.58, n_ref=32,
                                   step=0.5, seed=17, sweep=sweep, set_order=set_order,
                                   chain_base=9, want_flags=True, forbid=mask, threads=4)
        assert a1 == a2
        np.testing.assert_array_equal(f1, f2)
    np.testing.assert_array_equal(p1, p2)
    np.testing.assert_array_equal(orc.density_hist_arch(p2, n_chains, words, grid),
                                  orc.density_hist(p1, [Species(n_chains, n, 12)], grid))


def _graph_distance(n, bonds):
    adj = [[] for _ in range(n)]
    for i, j in bonds:
        adj[i].append(j)
        adj[j].append(i)
    d = np.full((n, n), -1)
    for s in range(n):
        d[s, s] = 0
        q = [s]
        while q:
            u = q.pop(0)
            for v in adj[u]:
                if d[s, v] < 0:
                    d[s, v] = d[s, u] + 1
                    q.append(v)
    return d


def test_ideal_star_acceptance_and_distances(orc):
    arms, arm_len = 6, 5
    n, bonds = synth.star_bonds(arms, arm_len)
    words = synth.encode_architecture(n, [0] * n, bonds)
    k0 = np.float32(3.0 * 31 / RE ** 2)
    n_chains = 6000
    grid = (24, 24, 24)
    pos = synth.tree_walks(41, n_chains, n, bonds, grid, 1 / math.sqrt(float(k0)))
    omega = np.zeros((2, 24 ** 3), np.float32)
    a = np.float32(0.1 * RE / math.sqrt(31))
    flags = []
    for sweep in range(4):
        _, f = orc.mc_sweep_arch(pos, n_chains, words, omega, grid, k0=k0, n_ref=32, step=a,
                                 seed=43, sweep=sweep, want_flags=True, threads=8)
        flags.append(f.reshape(n_chains, n))
    f = np.concatenate(flags).astype(np.float64)
    deg = np.zeros(n, int)
    for i, j in bonds:
        deg[i] += 1
        deg[j] += 1
    for g in sorted(set(deg)):
        sel = deg == g
        exp = references.ideal_local_acceptance(g * float(k0) / 2, float(a))[0]
        obs = f[:, sel].mean()
        sd = math.sqrt(exp * (1 - exp) / f[:, sel].size)
        assert abs(obs - exp) < 4 * sd, (g, obs, exp)
    for sweep in range(4, 30):
        orc.mc_sweep_arch(pos, n_chains, words, omega, grid, k0=k0, n_ref=32, step=a, seed=43,
                          sweep=sweep, threads=8)
    d = _graph_distance(n, bonds)
    p = pos.reshape(n_chains, n, 3).astype(np.float64)
    for i, j in [(0, arm_len), (1, 1 + arm_len), (arm_len, 2 * arm_len), (0, 3)]:
        r2 = ((p[:, i] - p[:, j]) ** 2).sum(axis=1)
        exp = 3 * d[i, j] / float(k0)
        assert abs(r2.mean() - exp) < 4 * r2.std() / math.sqrt(n_chains), (i, j, r2.mean(), exp)


def test_ideal_ring_distances(orc):
    n = 15
    _, bonds = synth.ring_bonds(n)
    words = synth.encode_architecture(n, [0] * 8 + [1] * 7, bonds)
    assert orc.arch_sets(words)[0] == 3
    k0 = np.float32(2.0)
    n_chains = 8000
    grid = (24, 24, 24)
    pos = synth.ring_walks(51, n_chains, n, grid, 1 / math.sqrt(float(k0)))
    omega = np.zeros((2, 24 ** 3), np.float32)
    for sweep in range(150):
        orc.mc_sweep_arch(pos, n_chains, words, omega, grid, k0=k0, n_ref=32, step=0.4, seed=53,
                          sweep=sweep, threads=8)
    p = pos.reshape(n_chains, n, 3).astype(np.float64)
    for dd in (1, 3, 7):
        r2 = ((p[:, 0] - p[:, dd]) ** 2).sum(axis=1)
        exp = 3 * dd * (n - dd) / (n * float(k0))
        assert abs(r2.mean() - exp) < 4 * r2.std() / math.sqrt(n_chains), (dd, r2.mean(), exp)
