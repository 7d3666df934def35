"""Pins of the oracle's bond-Gibbs move: the trial position of a bead is drawn
from its distribution given its bonded neighbours under the bond energy of
Eqs. (1)-(2) (a Gaussian around the neighbours' mean, variance 1/(n_b k0)),
accepted by the Metropolis-Hastings ratio of Sec. 2.2 evaluated term by term.

* ideal chain (zero field): every move is accepted (the proposal is the exact
  conditional distribution), and the moved middle bead's offset from its
  neighbours' midpoint is N(0, 1/(2 k0)) per component, an end bead's from its
  neighbour N(0, 1/k0) (KS tests);
* ideal chain: <b^2>, <Re^2>, <Rg^2> keep their Gaussian-chain values;
* 3-bead chain in a frozen random field: cell marginals and the end-bead joint
  match the exact Boltzmann distribution; a single bead (no bonds) keeps the
  field's Boltzmann weights.
"""
import math

import numpy as np
import pytest
from scipy.stats import kstest

import synth
from oracle import MOVE_GIBBS, Species, references

RE = 6.0


def test_ideal_chain_all_accepted_and_conditional_law(orc):
    n, n_chains = 32, 4000
    k0 = np.float32(3.0 * (n - 1) / RE ** 2)
    grid = (24, 24, 24)
    pos = synth.gaussian_walks(31, n_chains, n, grid, 1.0 / math.sqrt(float(k0)))
    omega = np.zeros((2, 24 ** 3), np.float32)
    acc, flags = orc.mc_sweep(pos, Species(n_chains, n, 16), omega, grid, k0=k0, n_ref=n,
                              move_kind=MOVE_GIBBS, step=np.float32(0.0), seed=3, sweep=0,
                              set_order=1, want_flags=True, threads=8)
    assert acc == n_chains * n and flags.all()
    p = pos.reshape(n_chains, n, 3).astype(np.float64)
    # with set_order 1 the odd beads move last: their neighbours are final
    mid = (p[:, 3, :] - 0.5 * (p[:, 2, :] + p[:, 4, :])).ravel()
    assert kstest(mid * math.sqrt(2 * float(k0)), "norm").pvalue > 1e-3
    end = (p[:, n - 1, :] - p[:, n - 2, :]).ravel()      # bead 31 is odd: moved last
    assert kstest(end * math.sqrt(float(k0)), "norm").pvalue > 1e-3
    # a planted variance error (1/k0 for a middle bead) is rejected
    assert kstest(mid * math.sqrt(float(k0)), "norm").pvalue < 1e-6


def test_ideal_chain_moments_stationary(orc):
    n, n_chains = 32, 6000
    k0 = np.float32(3.0 * (n - 1) / RE ** 2)
    grid = (24, 24, 24)
    pos = synth.gaussian_walks(32, n_chains, n, grid, 1.0 / math.sqrt(float(k0)))
    omega = np.zeros((2, 24 ** 3), np.float32)
    for sweep in range(20):
        orc.mc_sweep(pos, Species(n_chains, n, 16), omega, grid, k0=k0, n_ref=n,
                     move_kind=MOVE_GIBBS, step=np.float32(0.0), seed=6, sweep=sweep, threads=8)
    re2, rg2, b2 = orc.chain_observables(pos, n_chains, n)
    b2_exp, re2_exp, rg2_exp = references.ideal_chain_moments(n, float(k0))
    for vals, exp in ((b2 / (n - 1), b2_exp), (re2, re2_exp), (rg2, rg2_exp)):
        sigma = vals.std() / math.sqrt(n_chains)
        assert abs(vals.mean() - exp) < 4 * sigma, (vals.mean(), exp, sigma)


def test_three_bead_boltzmann(orc):
    L, k0 = 4, np.float32(3.0)
    grid = (L, L, L)
    n_chains = 65536
    omega = synth.uniform_field(23, L ** 3, -2.0, 2.0)
    pos = synth.gaussian_walks(24, n_chains, 3, grid, 1.0 / math.sqrt(3.0))
    for sweep in range(200):
        orc.mc_sweep(pos, Species(n_chains, 3, 2), omega, grid, k0=k0, n_ref=1,
                     move_kind=MOVE_GIBBS, step=np.float32(0.0), seed=78, sweep=sweep, threads=8)
    cells = np.floor(pos.astype(np.float64)).astype(np.int64) % L
    lin = ((cells[:, 2] * L + cells[:, 1]) * L + cells[:, 0]).reshape(n_chains, 3)
    p = references.three_bead_cell_distribution(omega[0], omega[1], float(k0), L)
    marg = [p.sum(axis=(1, 2)), p.sum(axis=(0, 2)), p.sum(axis=(0, 1))]
    for b in range(3):
        pval, stat, dof = references.chi2_pvalue(np.bincount(lin[:, b], minlength=L ** 3),
                                                 marg[b])
        assert pval > 1e-4, (b, stat, dof)
    obs = np.bincount(lin[:, 0] * L ** 3 + lin[:, 2], minlength=L ** 6)
    pval, stat, dof = references.chi2_pvalue(obs, p.sum(axis=1).ravel())
    assert pval > 1e-4, (stat, dof)


def test_single_bead_samples_the_field(orc):
    L = 4
    grid = (L, L, L)
    n_chains = 100000
    omega = synth.uniform_field(25, L ** 3, -1.5, 1.5)
    pos = synth.gaussian_walks(26, n_chains, 1, grid, 1.0)
    for sweep in range(60):
        orc.mc_sweep(pos, Species(n_chains, 1, 1), omega, grid, k0=np.float32(3.0), n_ref=1,
                     move_kind=MOVE_GIBBS, step=np.float32(0.0), seed=79, sweep=sweep, threads=8)
    cells = np.floor(pos.astype(np.float64)).astype(np.int64) % L
    lin = (cells[:, 2] * L + cells[:, 1]) * L + cells[:, 0]
    w = np.exp(-omega[0].astype(np.float64))
    pval, stat, dof = references.chi2_pvalue(np.bincount(lin, minlength=L ** 3), w / w.sum())
    assert pval > 1e-4, (stat, dof)
