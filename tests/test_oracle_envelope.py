"""The oracle's rounding envelope of the BF16 network against what rounding can
do.

The device evaluates the learned proposal's network (and its training
gradient) with BF16 operands summed in FP32 on the matrix cores, in an order of
the hardware's.  The oracle lists every rounding that such sums may take the
other way and bounds the effect; the parity tests of the device then require
every difference to lie inside that envelope.  Pinned here:

* the BF16 rounding boundary and the value across it, against torch's own
  round-to-nearest-even conversion of FP32 to bfloat16;
* the training-gradient envelope against an independent FP32 model of the
  device (numpy, float32 sums in random orders, torch's BF16 rounding at the
  device's rounding points): every simulated gradient lies inside the bound,
  and one with a planted mistake in the back-propagation does not;
* the move flags of the mixed sweep against the oracle run with FP32 sums in
  index order (another legal order): every chain that ends differently holds a
  flagged move, and flagged chains are a small minority.
"""
import math

import numpy as np
import pytest
import torch

import synth
from oracle import Species

HEAD = dict(m_max=1.0, lo=math.log(0.02), hi=math.log(1.0))


def _bf16(a):
    t = torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32))
    return t.to(torch.bfloat16).to(torch.float32).numpy()


def test_bf16_boundary_against_torch_rounding(orc):
    g = np.random.default_rng(1)
    vals = np.concatenate([
        g.standard_normal(3000) * np.exp(g.uniform(-20, 20, 3000)),
        _bf16(g.standard_normal(300)),                       # exact BF16 values
        _bf16(g.standard_normal(300)) * (1 + 2.0 ** -8),     # near midpoints
    ])
    for v in vals:
        v = float(np.float32(v))
        d, other = orc.bf16_boundary(v)
        q = float(_bf16(np.float32(v))[0])
        assert other != q and d >= 0.0
        # the boundary lies halfway between q and the other value, at distance d from v
        mid = 0.5 * (q + other)
        assert abs(abs(v - mid) - d) <= 1e-12 * max(abs(v), 1e-30)
        # points short of the boundary round to q, points beyond it to the other value
        step = abs(other - q)
        for frac in (0.25, 0.75):
            inner = mid - (1 if other > q else -1) * frac * (step / 2) * 0.999
            outer = mid + (1 if other > q else -1) * frac * (step / 2) * 0.999
            assert float(_bf16(np.float32(inner))[0]) == q
            assert float(_bf16(np.float32(outer))[0]) == other


# ---------------------------------------------------------------------------
# An FP32 model of the device's training pass, written for this test: float32
# sums of the exact BF16 products in a random order per call, BF16 rounding
# (torch) of activations and back-propagated errors where the device rounds.
# ---------------------------------------------------------------------------
def _sum_f32(terms, rng):
    """Sum over the last axis in float32, in a random order."""
    acc = np.zeros(terms.shape[:-1], np.float32)
    for k in rng.permutation(terms.shape[-1]):
        acc = acc + terms[..., k].astype(np.float32)
    return acc


def _device_model(params, feats, targets, rng, plant=False):
    L = synth.MLP_LAYOUT
    p = params.astype(np.float32)
    w1 = _bf16(p[L["w1"]:L["w1"] + 3840]).reshape(64, 60)
    w2 = _bf16(p[L["w2"]:L["w2"] + 4096]).reshape(64, 64)
    w3 = _bf16(p[L["w3"]:L["w3"] + 384]).reshape(6, 64)
    b1, b2, b3 = p[L["b1"]:L["b1"] + 64], p[L["b2"]:L["b2"] + 64], p[L["b3"]:L["b3"] + 6]
    x = _bf16((feats.astype(np.float32) - p[L["shift"]:L["shift"] + 60]) * p[L["scale"]:L["scale"] + 60])
    a1 = _sum_f32(w1[None] * x[:, None, :], rng) + b1
    h1 = _bf16(np.maximum(a1, 0))
    a2 = _sum_f32(w2[None] * h1[:, None, :], rng) + b2
    h2 = _bf16(np.maximum(a2, 0))
    z = _sum_f32(w3[None] * h2[:, None, :], rng) + b3
    m, lo, hi = (np.float32(HEAD[k]) for k in ("m_max", "lo", "hi"))
    t = targets.astype(np.float32)
    mu = m * np.tanh(z[:, :3] / m)
    sg = np.float32(1) / (np.float32(1) + np.exp(-z[:, 3:]))
    ls = lo + (hi - lo) * sg
    inv_var = np.exp(np.float32(-2) * ls)
    e = t - mu
    dz = np.concatenate([-e * inv_var * (1 - (mu / m) ** 2),
                         (1 - e * e * inv_var) * (hi - lo) * sg * (1 - sg)], axis=1).astype(np.float32)
    dzb = _bf16(dz)
    d2 = _sum_f32(w3.T[None] * dzb[:, None, :], rng) * (a2 > 0)
    d2b = _bf16(d2)
    w2t = w2.T.copy()
    if plant:   # a wrong row of W2^T in the back-propagation
        w2t[5] = w2t[6]
    d1 = _sum_f32(w2t[None] * d2b[:, None, :], rng) * (a1 > 0)
    d1b = _bf16(d1)
    n = feats.shape[0]
    grad = np.zeros(L["size"], np.float32)
    for name, val in (("w1", d1b[:, :, None] * x[:, None, :]), ("w2", d2b[:, :, None] * h1[:, None, :]),
                      ("w3", dzb[:, :, None] * h2[:, None, :]), ("b1", d1), ("b2", d2), ("b3", dz)):
        flat = val.reshape(n, -1).astype(np.float32)
        grad[L[name]:L[name] + flat.shape[1]] = _sum_f32(flat.T, rng) / np.float32(n)
    return grad


def _net_and_batch(seed, n):
    g = np.random.default_rng(seed)
    params = synth.mlp_params(31, weight_gain=1.2, out_gain=0.5,
                              shift=g.standard_normal(60) * 0.1, scale=1 + 0.2 * g.random(60))
    f = (g.standard_normal((n, 60)) * 1.5).astype(np.float32)
    t = (g.standard_normal((n, 3)) * 0.3).astype(np.float32)
    return params, f, t


def test_gradient_envelope_covers_fp32_orders(orc):
    params, f, t = _net_and_batch(7, 300)
    loss, grad, bound, n_amb, n_flag = orc.nll_batch_envelope(params, f, t, **HEAD)
    loss_o, _, _ = orc.nll_batch(params, f, t, **HEAD, bf16_mode=True)
    assert loss == pytest.approx(loss_o, rel=1e-12)     # same forward as the BF16 oracle
    assert n_amb > 0 and n_flag > 0
    rng = np.random.default_rng(3)
    for trial in range(4):
        g = _device_model(params, f, t, rng).astype(np.float64)
        excess = np.abs(g - grad) - bound
        assert excess.max() <= 0.0, (trial, int(excess.argmax()), excess.max())
    # the bound is far below the gradient itself: it still sees a wrong row
    g = _device_model(params, f, t, rng, plant=True).astype(np.float64)
    assert (np.abs(g - grad) > bound).sum() >= 30


def test_gradient_envelope_no_window_is_not_enough(orc):
    """With the windows scaled to zero the FP32 orders fall outside: the
    envelope's windows are what covers them."""
    params, f, t = _net_and_batch(8, 300)
    with orc.envelope_scale(0.0):
        _, grad, bound, n_amb, _ = orc.nll_batch_envelope(params, f, t, **HEAD)
    assert n_amb < 20           # exact ties only
    g = _device_model(params, f, t, np.random.default_rng(4)).astype(np.float64)
    assert (np.abs(g - grad) > bound).any()


def _melt(orc, n_chains=1024):
    w = synth.scaled(synth.C4_MEDIUM, n_chains, (18, 18, 18))
    k0 = np.float32(3.0 * (w.n_ref - 1) / w.re_cells ** 2)
    a = np.float32(w.a_frac * w.re_cells / math.sqrt(w.n_ref - 1))
    inv_rho = np.float32(w.n_cells / w.n_beads)
    pos = synth.gaussian_walks(13, n_chains, 32, w.grid, 1 / math.sqrt(float(k0)))
    sp = Species(n_chains, 32, 16)
    omega = orc.field_f32(orc.density_hist(pos, [sp], w.grid), inv_rho, np.float32(w.chi_n),
                          np.float32(w.kappa_n))
    return w, k0, a, pos, sp, omega


@pytest.mark.parametrize("p_learn", [1.0, 0.5])
def test_move_flags_explain_fp32_orders(orc, p_learn):
    """The oracle with FP32 sums in index order stands in for a device: every
    chain whose moves it decides otherwise, or whose new positions it places
    outside the position envelope, holds a flagged move."""
    from tests.gpu_helpers import explain_mismatches, proposal_test_params
    w, k0, a, pos, sp, omega = _melt(orc)
    params = proposal_test_params(orc, pos, sp, omega, w.grid, seed=12)
    kw = dict(k0=k0, n_ref=w.n_ref, local_a=a, p_learn=p_learn, params=params, **HEAD,
              bf16_mode=True, seed=w.seed, sweep=0, want_flags=True, threads=8)
    ref = pos.copy()
    amb = np.zeros(sp.n_chains * sp.n, np.uint8)
    env = np.zeros(sp.n_chains * sp.n, np.float32)
    acc, _, _, _, acc_flags = orc.mc_sweep_mixed(ref, sp, omega, w.grid, ambiguous=amb, pos_env=env,
                                                 **kw)
    alt = pos.copy()
    with orc.fp32_sums():
        orc.mc_sweep_mixed(alt, sp, omega, w.grid, **kw)
    differ = np.abs(alt.astype(np.float64) - ref).reshape(sp.n_chains, -1).max(axis=1) > 6e-5
    bad, unexplained, flagged, dec = explain_mismatches(alt, pos, ref, acc_flags, amb, env, sp.n)
    print("accepted", acc / pos.shape[0], "chains differing", differ.sum(), "mismatched", bad,
          "unexplained", unexplained, "flagged", flagged, "decisions", dec,
          "envelope max", env.max())
    assert acc > 0.3 * pos.shape[0]           # a proposal that moves beads
    assert differ.sum() >= 1                  # the orders do change positions ...
    assert unexplained == 0                   # ... and every mismatch is explained
    assert flagged < 0.08 * sp.n_chains
    # a stand-in that is not the device's arithmetic (the network in FP64,
    # no BF16 rounding) falls outside the envelope in chains nothing flags
    far = pos.copy()
    kw64 = dict(kw, bf16_mode=False)
    orc.mc_sweep_mixed(far, sp, omega, w.grid, **kw64)
    bad, unexplained, _, _ = explain_mismatches(far, pos, ref, acc_flags, amb, env, sp.n)
    print("FP64 network: mismatched", bad, "unexplained", unexplained)
    assert unexplained > 10
