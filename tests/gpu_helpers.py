"""Shared set-up for the GPU parity tests: configurations on both sides.

The device side gets a ``soma_config`` through the package; the oracle side
gets the same numbers as plain arguments.  Model constants are derived once
here from the workload description (they are configuration, not method).
"""
from __future__ import annotations

import math
import sys

import numpy as np

import synth


def flush(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def constants(w):
    k0 = np.float32(3.0 * (w.n_ref - 1) / w.re_cells ** 2)
    a = np.float32(w.a_frac * w.re_cells / math.sqrt(w.n_ref - 1))
    A = np.float32(w.smc_frac * w.re_cells ** 2 / w.n_ref)
    inv_rho = np.float32(w.n_cells / w.n_beads)
    return k0, a, A, inv_rho


def device_config(w, **kw):
    from paper_1711_03828_amd.melt import make_config
    return make_config(w, **kw)


def custom_config(grid, species, *, k0, n_ref, chi_n=0.0, kappa_n=0.0, local_a=0.1,
                  smc_a=0.05, seed=1, count_width=16, set_order=0, origin_mode=1, replica=0,
                  p_learn=0.0, mu_max=1.0, sigma_min=0.02, sigma_max=1.0):
    from paper_1711_03828_amd import soma as C
    cfg = C.soma_config()
    cfg.nx, cfg.ny, cfg.nz = grid
    cfg.n_species = len(species)
    for i, s in enumerate(species):
        cfg.species[i].n_chains = s.n_chains
        cfg.species[i].n = s.n
        cfg.species[i].n_a = s.n_a
        cfg.species[i].k0 = float(np.float32(k0))
    cfg.n_ref = n_ref
    cfg.chi_n = chi_n
    cfg.kappa_n = kappa_n
    cfg.local_a = float(np.float32(local_a))
    cfg.smc_a = float(np.float32(smc_a))
    cfg.seed = seed
    cfg.replica = replica
    cfg.count_width = count_width
    cfg.set_order = set_order
    cfg.origin_mode = origin_mode
    cfg.p_learn = p_learn
    cfg.mu_max = mu_max
    cfg.log_sigma_min = math.log(sigma_min)
    cfg.log_sigma_max = math.log(sigma_max)
    return cfg


def walks_for(w, seed):
    k0 = constants(w)[0]
    parts = [synth.gaussian_walks(seed + i, s.n_chains, s.n, w.grid, 1.0 / math.sqrt(float(k0)))
             for i, s in enumerate(w.species)]
    return np.concatenate(parts) if parts else np.zeros((0, 3), np.float32)


def unpack_counts(c: np.ndarray, width: int) -> np.ndarray:
    if width == 16:
        u = c.view(np.uint32)
        return np.stack([u & 0xFFFF, u >> 16]).astype(np.uint32)
    u = c.view(np.uint64)
    return np.stack([u & 0xFFFFFFFF, u >> 32]).astype(np.uint32)


def stepwise_cycles(melt, orc, sp, grid, n_cycles, oracle_sweep, field_of, *, n_per_chain,
                    tol=0.0):
    """SCMF cycles checked one by one from the device's own state.

    Before each cycle the device's positions, histogram and fields are read;
    the histogram must equal the oracle's count of those positions and the
    fields the oracle's fields of that histogram (bit for bit).  The device
    then runs one cycle and the oracle one sweep from the same positions and
    fields (``oracle_sweep(pos, omega, cycle)``, in place).  Per cycle the
    chains whose positions differ by more than ``tol`` must number at most
    ceil(1e-6 x moves), and the histogram the device kept must equal the
    oracle's count of the device's new positions.  Every cycle is compared in
    full, whether or not an earlier one had a mismatch.  Returns the number of
    mismatched chains per cycle."""
    import torch
    n_beads = sum(s.n_chains * s.n for s in sp)
    allowed = math.ceil(1e-6 * n_beads)
    per_cycle = []
    for cyc in range(n_cycles):
        torch.cuda.synchronize()
        pos = melt.pos.cpu().numpy()
        omega = melt.omega.cpu().numpy()
        counts = orc.density_hist(pos, sp, grid)
        np.testing.assert_array_equal(melt.counts_planes(), counts)
        np.testing.assert_array_equal(omega, field_of(counts))
        melt.cycle(1)
        ref = pos.copy()
        oracle_sweep(ref, omega, cyc)
        torch.cuda.synchronize()
        got = melt.pos.cpu().numpy()
        bad = int((np.abs(got.astype(np.float64) - ref.astype(np.float64)).reshape(-1, n_per_chain * 3)
                   .max(axis=1) > tol).sum())
        per_cycle.append(bad)
        assert bad <= allowed, (cyc, bad, allowed)
        np.testing.assert_array_equal(melt.counts_planes(), orc.density_hist(got, sp, grid))
        if bad == 0 and tol == 0.0:
            np.testing.assert_array_equal(melt.counts_planes(), orc.density_hist(ref, sp, grid))
    torch.cuda.synchronize()
    pos = melt.pos.cpu().numpy()
    np.testing.assert_array_equal(melt.omega.cpu().numpy(), field_of(orc.density_hist(pos, sp, grid)))
    flush("mismatched chains per cycle:", per_cycle, "allowed per cycle:", allowed)
    return per_cycle


def proposal_test_params(orc, pos, sp, omega, grid, *, seed, mu_gain=0.2, out_gain=0.3,
                         n_std=2048, sigma_bias=0.0):
    """A random network for the parity tests of the learned move that moves
    beads: inputs standardised with the mean and standard deviation of the
    oracle's features of up to n_std chains (beads 0, 7, N/2, N-1), the rows of
    the mean damped by mu_gain (a random drift makes the reverse move unlikely
    and nearly every move rejected), sigma's bias set to sigma_bias."""
    n_ch = min(sp.n_chains, n_std)
    sub = Species_like(sp, n_ch)
    beads = sorted({0, min(7, sp.n - 1), sp.n // 2, sp.n - 1})
    feats = np.concatenate([orc.features(pos[:n_ch * sp.n], sub, np.full(n_ch, b, np.uint32),
                                         omega, grid) for b in beads])
    shift = feats.mean(axis=0)
    sd = feats.std(axis=0)
    scale = np.where(sd > 1e-6, 1.0 / np.maximum(sd, 1e-6), 1.0)
    params = synth.mlp_params(seed, out_gain=out_gain, shift=shift.astype(np.float32),
                              scale=scale.astype(np.float32))
    L = synth.MLP_LAYOUT
    params[L["w3"]:L["w3"] + 192] *= np.float32(mu_gain)
    params[L["b3"]:L["b3"] + 3] = 0.0
    params[L["b3"] + 3:L["b3"] + 6] = sigma_bias
    return params


def Species_like(sp, n_chains):
    from oracle import Species
    return Species(n_chains, sp.n, sp.n_a)


def explain_mismatches(got, init, ref, accepted, amb, pos_env, n_per_chain, *, tol=6e-5):
    """Per-move comparison of a mixed sweep with the oracle's (one sweep from
    positions `init`; `ref`, `accepted`, `amb`, `pos_env` from the oracle).

    The device accepted a move iff the bead moved.  A move is a mismatch if
    the decisions differ, or, both accepting, if the new positions differ by
    more than tol + the move's rounding envelope (plus a quarter of its bonded
    neighbours'), or, both rejecting, if the bead is not where it started.  A
    mismatched chain is explained if the oracle flags one of its moves as
    decidable otherwise by rounding.  Returns (mismatched chains, unexplained
    chains, flagged chains, decision mismatches)."""
    nc = got.shape[0] // n_per_chain
    g = got.astype(np.float64).reshape(nc, n_per_chain, 3)
    r = ref.astype(np.float64).reshape(nc, n_per_chain, 3)
    i0 = init.astype(np.float64).reshape(nc, n_per_chain, 3)
    acc_o = accepted.reshape(nc, n_per_chain).astype(bool)
    moved = np.abs(g - i0).max(axis=2) > 0
    env = pos_env.reshape(nc, n_per_chain).astype(np.float64)
    nb = np.zeros_like(env)
    nb[:, 1:] += env[:, :-1]
    nb[:, :-1] += env[:, 1:]
    tol_b = tol + env + 0.25 * nb
    dec = moved != acc_o
    pos_bad = np.abs(g - r).max(axis=2) > tol_b
    bad = (dec | pos_bad).any(axis=1)
    flagged = amb.reshape(nc, n_per_chain).astype(bool).any(axis=1)
    return int(bad.sum()), int((bad & ~flagged).sum()), int(flagged.sum()), int(dec.sum())
