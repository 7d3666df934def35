"""Pins of the oracle's molecule-parallel sweep (Sec. 3.1.2, scheme 1: every
chain makes N attempts one after another, each on a bead picked uniformly at
random independently of the configuration).

* the picked beads: for N a power of two the pick is the top log2(N) bits of
  its word; they are uniform (chi-square) and follow the Philox words of the
  independent Python generator (purpose 7, word s mod 4 of block floor(s/4));
* ideal chain (chiN = kappaN = 0, zero field): attempts on middle and end
  beads are accepted at the closed-form Metropolis rates of a local move, and
  <b^2>, <Re^2>, <Rg^2> keep their Gaussian-chain values;
* 3-bead chain in a frozen random field: per-bead cell marginals and the
  end-bead joint match the exact Boltzmann distribution;
* results do not depend on the number of threads.
"""
import math

import numpy as np
import pytest

import synth
from oracle import Species, philox_py, references

RE = 6.0


@pytest.mark.parametrize("n", [1, 2, 8, 32, 64, 1024])
def test_pick_power_of_two_is_top_bits(orc, n):
    rng = np.random.default_rng(n)
    bits = n.bit_length() - 1
    for w in rng.integers(0, 1 << 32, 2000, dtype=np.uint64).tolist() + [0, (1 << 32) - 1]:
        assert orc.pick_bead(w, n) == (w >> (32 - bits) if bits else 0)


@pytest.mark.parametrize("n", [3, 5, 32, 33, 100])
def test_pick_bounds_and_uniformity(orc, n):
    rng = np.random.default_rng(7 + n)
    words = rng.integers(0, 1 << 32, 60000, dtype=np.uint64)
    picks = np.array([orc.pick_bead(int(w), n) for w in words])
    assert picks.min() >= 0 and picks.max() < n
    obs = np.bincount(picks, minlength=n)
    pval, _, _ = references.chi2_pvalue(obs, np.full(n, 1.0 / n))
    assert pval > 1e-4
    # the largest word picks the last bead, the smallest the first
    assert orc.pick_bead((1 << 32) - 1, n) == n - 1 and orc.pick_bead(0, n) == 0


def test_picks_follow_philox_words(orc):
    n, n_chains = 12, 20
    grid = (24, 24, 24)
    omega = synth.uniform_field(3, 24 ** 3, -3, 3)
    pos = synth.gaussian_walks(4, n_chains, n, grid, 0.6)
    seed, sweep, base = 987654321987, 5, 40
    _, flags, picked = orc.mc_sweep_molecule(pos, Species(n_chains, n, 6), omega, grid, k0=2.58,
                                             n_ref=32, step=0.6, seed=seed, sweep=sweep,
                                             chain_base=base, replica=3, want_flags=True)
    key = [seed & 0xFFFFFFFF, seed >> 32]
    picked = picked.reshape(n_chains, n)
    for c in range(n_chains):
        for s in range(n):
            w = philox_py.philox4x32_10([base + c, (s // 4) | (7 << 16), sweep, 3], key)[s % 4]
            assert picked[c, s] == (w * n) >> 32


def _ideal_system(n_chains, n, seed):
    k0 = np.float32(3.0 * (n - 1) / RE**2)
    grid = (24, 24, 24)
    pos = synth.gaussian_walks(seed, n_chains, n, grid, 1.0 / math.sqrt(float(k0)))
    omega = np.zeros((2, 24 ** 3), np.float32)
    return k0, grid, pos, omega


def test_ideal_acceptance_closed_form(orc):
    n, n_chains = 32, 12000
    k0, grid, pos, omega = _ideal_system(n_chains, n, 31)
    a = np.float32(0.1 * RE / math.sqrt(n - 1))
    fl, pk = [], []
    for sweep in range(3):
        _, f, p = orc.mc_sweep_molecule(pos, Species(n_chains, n, 16), omega, grid, k0=k0,
                                        n_ref=n, step=a, seed=41, sweep=sweep, want_flags=True,
                                        threads=4)
        fl.append(f)
        pk.append(p)
    f = np.concatenate(fl).astype(np.float64)
    p = np.concatenate(pk)
    end = (p == 0) | (p == n - 1)
    mid_exp, end_exp = references.ideal_local_acceptance(float(k0), float(a))
    for sel, exp in ((~end, mid_exp), (end, end_exp)):
        k = sel.sum()
        assert abs(f[sel].mean() - exp) < 4 * math.sqrt(exp * (1 - exp) / k)
    # one attempt per bead and sweep on average
    assert abs(end.mean() - 2 / n) < 4 * math.sqrt((2 / n) * (1 - 2 / n) / end.size)


def test_ideal_chain_moments_stationary(orc):
    n, n_chains = 32, 6000
    k0, grid, pos, omega = _ideal_system(n_chains, n, 32)
    a = np.float32(0.1 * RE / math.sqrt(n - 1))
    for sweep in range(20):
        orc.mc_sweep_molecule(pos, Species(n_chains, n, 16), omega, grid, k0=k0, n_ref=n, step=a,
                              seed=6, sweep=sweep, threads=4)
    re2, rg2, b2 = orc.chain_observables(pos, n_chains, n)
    b2_exp, re2_exp, rg2_exp = references.ideal_chain_moments(n, float(k0))
    for vals, exp in ((b2 / (n - 1), b2_exp), (re2, re2_exp), (rg2, rg2_exp)):
        sigma = vals.std() / math.sqrt(n_chains)
        assert abs(vals.mean() - exp) < 4 * sigma, (vals.mean(), exp, sigma)


def test_three_bead_boltzmann_marginals(orc):
    L, k0 = 4, np.float32(3.0)
    grid = (L, L, L)
    n_chains = 65536
    omega = synth.uniform_field(21, L ** 3, -2.0, 2.0)
    pos = synth.gaussian_walks(23, n_chains, 3, grid, 1.0 / math.sqrt(3.0))
    for sweep in range(300):
        orc.mc_sweep_molecule(pos, Species(n_chains, 3, 2), omega, grid, k0=k0, n_ref=1,
                              step=np.float32(0.7), seed=78, sweep=sweep, threads=8)
    cells = np.floor(pos.astype(np.float64)).astype(np.int64) % L
    lin = ((cells[:, 2] * L + cells[:, 1]) * L + cells[:, 0]).reshape(n_chains, 3)
    p = references.three_bead_cell_distribution(omega[0], omega[1], float(k0), L)
    marg = [p.sum(axis=(1, 2)), p.sum(axis=(0, 2)), p.sum(axis=(0, 1))]
    for b in range(3):
        obs = np.bincount(lin[:, b], minlength=L ** 3)
        pval, stat, dof = references.chi2_pvalue(obs, marg[b])
        assert pval > 1e-4, (b, stat, dof)
    obs = np.bincount(lin[:, 0] * L ** 3 + lin[:, 2], minlength=L ** 6)
    pval, stat, dof = references.chi2_pvalue(obs, p.sum(axis=1).ravel())
    assert pval > 1e-4, (stat, dof)


def test_threads_do_not_change_results(orc):
    n, n_chains = 32, 300
    grid = (24, 24, 24)
    omega = synth.uniform_field(3, 24 ** 3, -3, 3)
    base = synth.gaussian_walks(4, n_chains, n, grid, 0.6)
    outs = []
    for th in (1, 5):
        pos = base.copy()
        orc.mc_sweep_molecule(pos, Species(n_chains, n, 16), omega, grid, k0=2.58, n_ref=32,
                              step=0.1, seed=8, sweep=3, threads=th)
        outs.append(pos)
    np.testing.assert_array_equal(outs[0], outs[1])
