"""Pins of the oracle's MC sweep (Sec. 2.2 moves, Sec. 3.1.2 set order).

* ideal chain (chiN = kappaN = 0, zero field): the Metropolis acceptance of a
  local move has the closed form erfc(sqrt(mu)/2) averaged over the trial
  displacement (middle and end beads separately);
* ideal chain: <b^2>, <Re^2>, <Rg^2> keep their Gaussian-chain values under
  local and under force-biased moves (the walk starts in equilibrium);
* 3-bead chain in a frozen random field: per-bead cell marginals match the
  exact Boltzmann distribution (brute force over 4^9 cell states);
* results do not depend on the number of threads; the set order follows its
  Philox bit.
"""
import math

import numpy as np
import pytest
from scipy.stats import norm

import synth
from oracle import MOVE_LOCAL, MOVE_SMC, Species, philox_py, references

RE = 6.0


def _ideal_system(n_chains, n, seed):
    k0 = np.float32(3.0 * (n - 1) / RE**2)
    grid = (24, 24, 24)
    pos = synth.gaussian_walks(seed, n_chains, n, grid, 1.0 / math.sqrt(float(k0)))
    omega = np.zeros((2, 24 ** 3), np.float32)
    return k0, grid, pos, omega


def test_ideal_local_acceptance_closed_form(orc):
    n, n_chains = 32, 12000
    k0, grid, pos, omega = _ideal_system(n_chains, n, 11)
    a = np.float32(0.1 * RE / math.sqrt(n - 1))
    flags = []
    for sweep in range(3):
        _, f = orc.mc_sweep(pos, Species(n_chains, n, 16), omega, grid, k0=k0, n_ref=n,
                            step=a, seed=99, sweep=sweep, want_flags=True, threads=4)
        flags.append(f.reshape(n_chains, n))
    f = np.concatenate(flags)
    mid_exp, end_exp = references.ideal_local_acceptance(float(k0), float(a))
    mid = f[:, 1:-1].mean()
    end = f[:, [0, -1]].mean()
    n_mid, n_end = f[:, 1:-1].size, f[:, [0, -1]].size
    assert abs(mid - mid_exp) < 4 * math.sqrt(mid_exp * (1 - mid_exp) / n_mid)
    assert abs(end - end_exp) < 4 * math.sqrt(end_exp * (1 - end_exp) / n_end)
    # the values quoted for k0 a^2 = 0.03
    assert mid_exp == pytest.approx(0.906399, abs=2e-6)
    assert end_exp == pytest.approx(0.933719, abs=2e-6)


@pytest.mark.parametrize("kind", [MOVE_LOCAL, MOVE_SMC])
def test_ideal_chain_moments_stationary(orc, kind):
    n, n_chains = 32, 6000
    k0, grid, pos, omega = _ideal_system(n_chains, n, 12)
    step = np.float32(0.1 * RE / math.sqrt(n - 1)) if kind == MOVE_LOCAL else np.float32(
        0.05 * RE**2 / n)
    total = 0
    for sweep in range(20):
        acc, _ = orc.mc_sweep(pos, Species(n_chains, n, 16), omega, grid, k0=k0, n_ref=n,
                              move_kind=kind, step=step, seed=5, sweep=sweep, threads=4)
        total += acc
    assert 0.3 < total / (20 * n_chains * n) < 1.0
    re2, rg2, b2 = orc.chain_observables(pos, n_chains, n)
    b2_exp, re2_exp, rg2_exp = references.ideal_chain_moments(n, float(k0))
    for vals, exp in ((b2 / (n - 1), b2_exp), (re2, re2_exp), (rg2, rg2_exp)):
        sigma = vals.std() / math.sqrt(n_chains)
        assert abs(vals.mean() - exp) < 4 * sigma, (vals.mean(), exp, sigma)


def _three_bead_run(orc, kind, step, n_chains=65536, sweeps=300):
    L, k0 = 4, np.float32(3.0)
    grid = (L, L, L)
    omega = synth.uniform_field(21, L ** 3, -2.0, 2.0)
    pos = synth.gaussian_walks(22, n_chains, 3, grid, 1.0 / math.sqrt(3.0))
    for sweep in range(sweeps):
        orc.mc_sweep(pos, Species(n_chains, 3, 2), omega, grid, k0=k0, n_ref=1,
                     move_kind=kind, step=step, seed=77, sweep=sweep, threads=8)
    cells = np.floor(pos.astype(np.float64)).astype(np.int64) % L
    lin = (cells[:, 2] * L + cells[:, 1]) * L + cells[:, 0]
    return lin.reshape(n_chains, 3), omega, k0, L


@pytest.mark.parametrize("kind,step", [(MOVE_LOCAL, 0.7), (MOVE_SMC, 0.12)])
def test_three_bead_boltzmann_marginals(orc, kind, step):
    lin, omega, k0, L = _three_bead_run(orc, kind, np.float32(step))
    p = references.three_bead_cell_distribution(omega[0], omega[1], float(k0), L)
    marg = [p.sum(axis=(1, 2)), p.sum(axis=(0, 2)), p.sum(axis=(0, 1))]
    for b in range(3):
        obs = np.bincount(lin[:, b], minlength=L ** 3)
        pval, stat, dof = references.chi2_pvalue(obs, marg[b])
        assert pval > 1e-4, (b, stat, dof)
    # joint of the end beads (4096 bins) catches a wrong bond coupling
    obs = np.bincount(lin[:, 0] * L ** 3 + lin[:, 2], minlength=L ** 6)
    pval, stat, dof = references.chi2_pvalue(obs, p.sum(axis=1).ravel())
    assert pval > 1e-4, (stat, dof)


def test_three_bead_detects_planted_sign_error(orc):
    # the same comparison rejects the distribution of the flipped field
    lin, omega, k0, L = _three_bead_run(orc, MOVE_LOCAL, np.float32(0.7), 32768, 200)
    p_wrong = references.three_bead_cell_distribution(-omega[0], -omega[1], float(k0), L)
    obs = np.bincount(lin[:, 1], minlength=L ** 3)
    pval, _, _ = references.chi2_pvalue(obs, p_wrong.sum(axis=(0, 2)))
    assert pval < 1e-10


def test_threads_do_not_change_results(orc):
    n, n_chains = 32, 300
    grid = (24, 24, 24)
    omega = synth.uniform_field(3, 24 ** 3, -3, 3)
    base = synth.gaussian_walks(4, n_chains, n, grid, 0.6)
    outs = []
    for th in (1, 5):
        for kind, step in ((MOVE_LOCAL, 0.1), (MOVE_SMC, 0.05)):
            pos = base.copy()
            orc.mc_sweep(pos, Species(n_chains, n, 16), omega, grid, k0=2.58, n_ref=32,
                         move_kind=kind, step=step, seed=8, sweep=3, threads=th)
            outs.append(pos)
    np.testing.assert_array_equal(outs[0], outs[2])
    np.testing.assert_array_equal(outs[1], outs[3])


def test_set_order_follows_philox_bit(orc):
    n, n_chains = 8, 64
    grid = (24, 24, 24)
    omega = synth.uniform_field(3, 24 ** 3, -3, 3)
    base = synth.gaussian_walks(4, n_chains, n, grid, 0.6)
    seed, sweep = 1234567890123, 9
    runs = {}
    for order in (0, 1):
        pos = base.copy()
        orc.mc_sweep(pos, Species(n_chains, n, 4), omega, grid, k0=2.58, n_ref=32,
                     step=0.6, seed=seed, sweep=sweep, chain_base=100, set_order=order)
        runs[order] = pos.reshape(n_chains, n, 3)
    key = [seed & 0xFFFFFFFF, seed >> 32]
    for c in range(n_chains):
        bit = philox_py.philox4x32_10([100 + c, 0, sweep, 0], key)[0] & 1
        same = np.array_equal(runs[0][c], runs[1][c])
        if bit == 0:
            assert same
    assert any(not np.array_equal(runs[0][c], runs[1][c]) for c in range(n_chains))
