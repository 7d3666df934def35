"""Pins of the oracle's learned proposal (network, loss, features, mixed move).

* back-propagation equals central finite differences of the FP64 loss
  (relative error < 1e-6 on every parameter group);
* the loss itself: closed values at the head's mean (sum of log sigma, plus 1/2
  one sigma away), equality with scipy's normal log-density, the mean over
  targets drawn from the head's Gaussian (sum log sigma + 3/2), and dL/dz
  against finite differences of the loss;
* bfloat16 rounding equals the library converter (torch, round to nearest even);
* BF16-emulating forward stays close to FP64 (rounding only);
* features: hand-checked own/other field blocks, cell order and bond vectors;
* exactness of Metropolis-Hastings: 3-bead chain in a frozen random field with
  random (untrained) network weights, pure learned and 50/50 mixed moves,
  matches the exact Boltzmann distribution (MH exactness does not depend on
  training).
"""
import math

import numpy as np
import pytest
import torch

import synth
from oracle import Species, references

HEAD = dict(m_max=1.0, lo=math.log(0.02), hi=math.log(1.0))


def _batch(n, seed):
    g = np.random.default_rng(seed)
    f = g.standard_normal((n, 60))
    t = g.standard_normal((n, 3)) * 0.3
    return f, t


def test_gradient_matches_finite_differences(orc):
    p = synth.mlp_params(3, weight_gain=1.3, out_gain=0.8).astype(np.float64)
    f, t = _batch(16, 4)
    loss, grad, _ = orc.nll_batch(p.astype(np.float32), f, t, **HEAD)
    L = synth.MLP_LAYOUT
    g = np.random.default_rng(5)
    # parameters are stored as float32, so perturb by a step that float32 holds; a small
    # step keeps every pre-activation on one side of the ReLU kink (no crossing in this batch)
    for name, size in (("w1", 3840), ("b1", 64), ("w2", 4096), ("b2", 64), ("w3", 384),
                       ("b3", 6)):
        for idx in g.choice(size, min(size, 6), replace=False):
            k = L[name] + int(idx)
            h = 2.0 ** -20
            pp = p.copy(); pp[k] += h
            pm = p.copy(); pm[k] -= h
            lp, _, _ = orc.nll_batch(pp.astype(np.float32), f, t, **HEAD)
            lm, _, _ = orc.nll_batch(pm.astype(np.float32), f, t, **HEAD)
            fd = (lp - lm) / (2 * h)
            assert abs(fd - grad[k]) <= 1e-6 * max(1.0, abs(grad[k])) + 2e-7, (name, idx, fd, grad[k])
    assert np.all(grad[:120] == 0.0)        # no gradient for the standardisation constants


def test_bf16_rounding_matches_library(orc):
    g = np.random.default_rng(6)
    xs = np.concatenate([g.standard_normal(3000) * 10.0 ** g.integers(-8, 8, 3000),
                         [0.0, -0.0, 1.0, 1.00390625, 1.005859375, 3.4e38, 1e-40]]).astype(np.float32)
    lib = torch.from_numpy(xs).to(torch.bfloat16).to(torch.float32).numpy()
    ours = np.array([orc.bf16(float(x)) for x in xs], np.float32)
    np.testing.assert_array_equal(ours, lib)


def test_bf16_forward_close_to_fp64(orc):
    p = synth.mlp_params(7)
    f, _ = _batch(50, 8)
    z64 = orc.mlp_forward(p, f, bf16_mode=False)
    z16 = orc.mlp_forward(p, f, bf16_mode=True)
    assert np.abs(z16 - z64).max() < 0.05 * (1 + np.abs(z64).max())


def test_features_hand_checked(orc):
    grid = (5, 4, 3)
    n_cells = 60
    omega = np.zeros((2, n_cells), np.float32)
    omega[0] = np.arange(n_cells)            # A field: cell index
    omega[1] = 1000 + np.arange(n_cells)     # B field: 1000 + cell index
    # one chain of 3 beads, types A B B (n_a = 1)
    pos = np.array([[0.5, 0.5, 0.5], [1.25, 3.5, 2.75], [2.0, 0.25, 2.5]], np.float32)
    sp = Species(1, 3, 1)
    fa = orc.features(pos, sp, [0], omega, grid)[0]
    fb = orc.features(pos, sp, [1], omega, grid)[0]
    # bead 0 is A in cell (0,0,0): own block = A field; (dz,dy,dx)=(-1,-1,-1) ->
    # cell (4, 3, 2) -> index (2*4+3)*5+4 = 59; centre = cell 0
    assert fa[0] == 59 and fa[13] == 0 and fa[27 + 13] == 1000
    np.testing.assert_array_equal(fa[54:57], 0.0)                     # no previous bead
    np.testing.assert_allclose(fa[57:60], pos[1] - pos[0])
    # bead 1 is B in cell (1,3,2) -> centre index (2*4+3)*5+1 = 56; own block = B field
    assert fb[13] == 1056 and fb[27 + 13] == 56
    # (dz,dy,dx) = (+1,+1,+1) wraps to cell (2,0,0) -> index 2
    assert fb[26] == 1002
    np.testing.assert_allclose(fb[54:57], pos[0] - pos[1])
    np.testing.assert_allclose(fb[57:60], pos[2] - pos[1])


def _three_bead_mixed(orc, p_learn, params, n_chains=8192, equil=150, sweeps=200):
    """Equilibrate with local moves, then continue with the mixed move: exact
    Metropolis-Hastings keeps the Boltzmann distribution stationary."""
    L, k0 = 4, np.float32(3.0)
    grid = (L, L, L)
    omega = synth.uniform_field(21, L ** 3, -2.0, 2.0)
    pos = synth.gaussian_walks(24, n_chains, 3, grid, 1.0 / math.sqrt(3.0))
    acc_l = 0
    for sweep in range(equil + sweeps):
        pl = 0.0 if sweep < equil else p_learn
        _, al, bad, _, _ = orc.mc_sweep_mixed(pos, Species(n_chains, 3, 2), omega, grid, k0=k0,
                                              n_ref=1, local_a=0.7, p_learn=pl,
                                              params=params, **HEAD, seed=5, sweep=sweep,
                                              threads=8)
        acc_l += al
        assert bad == 0
    cells = np.floor(pos.astype(np.float64)).astype(np.int64) % L
    lin = ((cells[:, 2] * L + cells[:, 1]) * L + cells[:, 0]).reshape(n_chains, 3)
    return lin, omega, acc_l


def drifting_params(seed):
    """Random weights with a position-dependent drift of ~0.1 cell and sigma
    ~0.5 cell: far from a symmetric proposal, so the proposal ratio matters."""
    params = synth.mlp_params(seed, out_gain=0.1)
    b3 = synth.MLP_LAYOUT["b3"]
    params[b3 + 3:b3 + 6] = 1.5
    return params


@pytest.mark.parametrize("p_learn", [1.0, 0.5])
def test_mixed_move_is_exact_with_random_weights(orc, p_learn):
    # random weights give a position-dependent drift of about 0.1 cell: the
    # proposal is far from symmetric, so a wrong proposal ratio would bias the
    # sampled distribution
    params = drifting_params(9)
    lin, omega, acc_l = _three_bead_mixed(orc, p_learn, params)
    assert acc_l > 0
    p = references.three_bead_cell_distribution(omega[0], omega[1], 3.0, 4)
    marg = [p.sum(axis=(1, 2)), p.sum(axis=(0, 2)), p.sum(axis=(0, 1))]
    for b in range(3):
        pval, stat, dof = references.chi2_pvalue(np.bincount(lin[:, b], minlength=64), marg[b])
        assert pval > 1e-4, (b, stat, dof)
    obs = np.bincount(lin[:, 0] * 64 + lin[:, 2], minlength=4096)
    pval, stat, dof = references.chi2_pvalue(obs, p.sum(axis=1).ravel())
    assert pval > 1e-4, (stat, dof)


# ----------------------------------------------------------------------------
# The loss itself (Gaussian negative log-likelihood without its constant), pinned
# by closed values and by the normal density of scipy, independently of the
# finite-difference check above (which ties only the gradient to the loss).
# ----------------------------------------------------------------------------
def test_nll_closed_value_at_the_mean(orc):
    lo, hi = HEAD["lo"], HEAD["hi"]
    # z = 0: mu = 0, sigmoid = 1/2, log sigma = (lo + hi)/2 on every axis; dr = mu
    loss, dz = orc.nll(np.zeros(6), np.zeros(3), **HEAD)
    assert loss == pytest.approx(3 * 0.5 * (lo + hi), rel=1e-14)
    # dL/dmu = 0 at the mean; dL/dlog sigma = 1, times d log sigma/dz = (hi - lo)/4
    np.testing.assert_allclose(dz[:3], 0.0, atol=1e-15)
    np.testing.assert_allclose(dz[3:], (hi - lo) * 0.25, rtol=1e-14)
    # any z, dr = mu(z): the loss is the sum of log sigma
    z = np.array([0.3, -1.7, 0.05, 2.0, -0.4, 0.9])
    mu = np.tanh(z[:3])                                   # m_max = 1
    lsig = lo + (hi - lo) / (1 + np.exp(-z[3:]))
    loss, dz = orc.nll(z, mu, **HEAD)
    assert loss == pytest.approx(lsig.sum(), rel=1e-13)
    np.testing.assert_allclose(dz[:3], 0.0, atol=1e-15)
    # one sigma away on the first axis: + 1/2
    dr = mu.copy()
    dr[0] += np.exp(lsig[0])
    loss1, _ = orc.nll(z, dr, **HEAD)
    assert loss1 == pytest.approx(lsig.sum() + 0.5, rel=1e-13)


def test_nll_equals_normal_log_density(orc):
    from scipy.stats import norm
    g = np.random.default_rng(17)
    for _ in range(50):
        z = g.standard_normal(6) * 2.0
        dr = g.standard_normal(3) * 0.7
        mu = HEAD["m_max"] * np.tanh(z[:3] / HEAD["m_max"])
        sig = np.exp(HEAD["lo"] + (HEAD["hi"] - HEAD["lo"]) / (1 + np.exp(-z[3:])))
        exp = -norm.logpdf(dr, loc=mu, scale=sig).sum() - 1.5 * math.log(2 * math.pi)
        loss, _ = orc.nll(z, dr, **HEAD)
        assert loss == pytest.approx(exp, rel=1e-12, abs=1e-12)


def test_nll_mean_over_gaussian_targets(orc):
    """Targets drawn from the head's own Gaussian: E[loss] = sum log sigma + 3/2
    (each axis contributes log sigma + E[xi^2]/2)."""
    g = np.random.default_rng(23)
    z = np.array([0.4, -0.2, 1.1, -0.5, 0.7, 0.0])
    mu = np.tanh(z[:3])
    lsig = HEAD["lo"] + (HEAD["hi"] - HEAD["lo"]) / (1 + np.exp(-z[3:]))
    n = 20000
    dr = mu + np.exp(lsig) * g.standard_normal((n, 3))
    losses = np.array([orc.nll(z, d, **HEAD)[0] for d in dr])
    se = losses.std() / math.sqrt(n)
    assert abs(losses.mean() - (lsig.sum() + 1.5)) < 4 * se


def test_nll_gradient_in_z_matches_finite_differences(orc):
    g = np.random.default_rng(29)
    for _ in range(20):
        z = g.standard_normal(6)
        dr = g.standard_normal(3) * 0.5
        _, dz = orc.nll(z, dr, **HEAD)
        for k in range(6):
            h = 1e-6
            zp = z.copy(); zp[k] += h
            zm = z.copy(); zm[k] -= h
            fd = (orc.nll(zp, dr, **HEAD)[0] - orc.nll(zm, dr, **HEAD)[0]) / (2 * h)
            assert fd == pytest.approx(dz[k], rel=1e-6, abs=1e-8)


def test_fold_params_is_the_same_network(orc):
    """The folded form of the learned move's network (standardisation inside the
    first layer): identity for shift 0 and scale 1 (bit for bit), a hand-worked
    unit, and in FP64 the same outputs as the standardised network up to the
    FP32 rounding of W1' and b1' (a planted wrong sign of the shift term is
    caught by the same comparison)."""
    L = synth.MLP_LAYOUT
    p0 = synth.mlp_params(5, shift=np.zeros(60, np.float32), scale=np.ones(60, np.float32))
    np.testing.assert_array_equal(orc.fold_params(p0), p0)
    # hand case: unit 0 sees only feature 0 with weight 2, shift 5, scale 3
    p = np.zeros(8576, np.float32)
    p[L["scale"]:L["scale"] + 60] = 1.0
    p[L["w1"]] = 2.0
    p[L["scale"]] = 3.0
    p[L["shift"]] = 5.0
    p[L["b1"]] = 0.25
    q = orc.fold_params(p)
    assert q[L["w1"]] == 6.0 and q[L["b1"]] == np.float32(0.25 - 30.0)
    assert np.all(q[L["shift"]:L["shift"] + 60] == 0.0) and np.all(q[L["scale"]:L["scale"] + 60] == 1.0)
    # random networks with real standardisation constants
    g = np.random.default_rng(12)
    f = g.standard_normal((200, 60)) * 8.0 + 20.0
    p = synth.mlp_params(9, weight_gain=1.1, out_gain=0.5, shift=(20 + g.standard_normal(60)).astype(np.float32),
                         scale=(0.1 + 0.2 * g.random(60)).astype(np.float32))
    z = orc.mlp_forward(p, f, bf16_mode=False)
    zf = orc.mlp_forward(orc.fold_params(p), f, bf16_mode=False)
    assert np.abs(zf - z).max() < 1e-4 * (1.0 + np.abs(z).max())
    bad = orc.fold_params(p)
    bad[L["b1"]:L["b1"] + 64] = p[L["b1"]:L["b1"] + 64] + (p[L["b1"]:L["b1"] + 64] - bad[L["b1"]:L["b1"] + 64])
    assert np.abs(orc.mlp_forward(bad, f, bf16_mode=False) - z).max() > 1e-2
