"""Statistical parity of the device sampler with what the model fixes.

* ideal chain (chiN = kappaN = 0): Metropolis acceptance of local moves equals
  the closed form, bond-Gibbs moves are all accepted; <b^2>, <Re^2>, <Rg^2>
  keep their Gaussian-chain values under local, smart-MC and bond-Gibbs moves
  (the walk starts in equilibrium);
* 3-bead chain in a frozen random field: per-bead cell marginals and the joint
  of the two end beads match the exact Boltzmann distribution (chi-square,
  fixed p-threshold 1e-4), for local, smart-MC and bond-Gibbs moves;
* the 1024-chain melt after 100 SCMF cycles: <Re^2> and the acceptance rate of
  the device and of an independent oracle run agree within 4 sigma.
"""
import math

import numpy as np
import pytest

import synth
from oracle import MOVE_LOCAL, MOVE_SMC, Species, references
from tests.gpu_helpers import constants, custom_config, device_config, flush

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]
RE = 6.0


def test_ideal_chain_acceptance_and_moments():
    from paper_1711_03828_amd import soma as C
    from paper_1711_03828_amd.melt import Melt
    n, n_chains = 32, 65536
    w = synth.Workload("ideal", (48, 48, 48), (synth.SpeciesSpec(n_chains, n, 16),), RE, n,
                       0.0, 0.0, 32)
    k0 = float(constants(w)[0])
    for kind in (C.SOMA_MOVE_LOCAL, C.SOMA_MOVE_SMC, C.SOMA_MOVE_GIBBS):
        m = Melt(device_config(w, seed=11 + kind))
        m.omega.zero_()                       # chiN = kappaN = 0: zero field
        m.sweep(20, kind)
        obs = m.observables()
        rate = obs.accepted[kind] / obs.attempted[kind]
        if kind == C.SOMA_MOVE_LOCAL:
            a = float(np.float32(0.1 * RE / math.sqrt(n - 1)))
            exp = references.ideal_local_acceptance_chain(n, k0, a)
            sigma = math.sqrt(exp * (1 - exp) / obs.attempted[kind])
            flush("acceptance", rate, "closed form", exp)
            assert abs(rate - exp) < 6 * sigma + 1e-4   # moves within a sweep are correlated
        if kind == C.SOMA_MOVE_GIBBS:   # the exact conditional law of the bonds: all accepted
            assert obs.accepted[kind] == obs.attempted[kind] == 20 * n * n_chains
        re2_exp = 3 * (n - 1) / k0
        rg2_exp = (3 / k0) * (n * n - 1) / (6 * n)
        b2_exp = 3 / k0 * (n - 1)
        # per-chain std of Re^2 for a Gaussian chain is sqrt(2/3) <Re^2>
        for val, e, rel_sd in ((obs.re2_sum / n_chains, re2_exp, math.sqrt(2 / 3)),
                               (obs.b2_sum / n_chains, b2_exp, math.sqrt(2 / 3 / (n - 1))),
                               (obs.rg2_sum / n_chains, rg2_exp, 0.5)):
            assert abs(val - e) < 5 * rel_sd * e / math.sqrt(n_chains), (kind, val, e)
        m.close()


@pytest.mark.parametrize("kind,step", [(0, 0.7), (1, 0.12), (3, 0.0)])
def test_three_bead_boltzmann_on_device(kind, step):
    from paper_1711_03828_amd.melt import Melt
    L, n_chains = 4, 65536
    grid = (L, L, L)
    omega = synth.uniform_field(21, L ** 3, -2.0, 2.0)
    pos = synth.gaussian_walks(23, n_chains, 3, grid, 1.0 / math.sqrt(3.0))
    cfg = custom_config(grid, [Species(n_chains, 3, 2)], k0=3.0, n_ref=1, local_a=step,
                        smc_a=step, seed=99, count_width=32)
    m = Melt(cfg, positions=torch.from_numpy(pos))
    m.omega.copy_(torch.from_numpy(omega))      # frozen field: no field updates
    m.sync_fields()
    m.sweep(300, kind)
    torch.cuda.synchronize()
    p = m.pos.cpu().numpy().astype(np.float64)
    cells = np.floor(p).astype(np.int64) % L
    lin = ((cells[:, 2] * L + cells[:, 1]) * L + cells[:, 0]).reshape(n_chains, 3)
    dist = references.three_bead_cell_distribution(omega[0], omega[1], 3.0, L)
    marg = [dist.sum(axis=(1, 2)), dist.sum(axis=(0, 2)), dist.sum(axis=(0, 1))]
    for b in range(3):
        pval, stat, dof = references.chi2_pvalue(np.bincount(lin[:, b], minlength=L ** 3), marg[b])
        assert pval > 1e-4, (b, stat, dof)
    obs = np.bincount(lin[:, 0] * L ** 3 + lin[:, 2], minlength=L ** 6)
    pval, stat, dof = references.chi2_pvalue(obs, dist.sum(axis=1).ravel())
    assert pval > 1e-4, (stat, dof)
    m.close()


def test_melt_100_cycles_matches_oracle_statistics(orc):
    from paper_1711_03828_amd.melt import Melt
    w = synth.C1_SMALL
    k0, a, A, inv_rho = constants(w)
    pos0 = synth.gaussian_walks(51, 1024, 32, w.grid, 1 / math.sqrt(float(k0)))
    sp = Species(1024, 32, 16)
    # oracle run
    pos = pos0.copy()
    omega = orc.field_f32(orc.density_hist(pos, [sp], w.grid), inv_rho, np.float32(w.chi_n),
                          np.float32(w.kappa_n))
    acc_o = 0
    for s in range(100):
        acc, _ = orc.mc_sweep(pos, sp, omega, w.grid, k0=k0, n_ref=w.n_ref, step=a,
                              seed=w.seed + 1, sweep=s, threads=8)
        acc_o += acc
        omega = orc.field_f32(orc.density_hist(pos, [sp], w.grid), inv_rho,
                              np.float32(w.chi_n), np.float32(w.kappa_n))
    re2_o, _, _ = orc.chain_observables(pos, 1024, 32)
    # device run (different seed: statistically independent trajectory)
    m = Melt(device_config(w), positions=torch.from_numpy(pos0))
    m.cycle(100)
    obs = m.observables()
    re2_d = obs.re2_sum / 1024
    sd = re2_o.std() / math.sqrt(1024)
    flush("Re2 oracle", re2_o.mean(), "device", re2_d, "sd", sd)
    assert abs(re2_d - re2_o.mean()) < 4 * math.sqrt(2) * sd
    rate_o = acc_o / (100 * w.n_beads)
    rate_d = obs.accepted[0] / obs.attempted[0]
    assert abs(rate_d - rate_o) < 2e-3
    assert obs.counts_conserved == 1
    m.close()
