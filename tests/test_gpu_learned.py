"""GPU parity of the learned proposal (network on MFMA, mixed MH sweep).

Bars:
  * features: bit-exact against the oracle (FP32 field values and bond vectors);
  * network outputs z: the oracle's BF16-emulating forward (inputs, weights and
    hidden activations rounded to bfloat16 at the same points) with FP64
    accumulation, against BF16 MFMA with FP32 accumulation: |dz| <= 2e-3 (1+|z|)
    for 99.9% of samples (a hidden activation on a bfloat16 rounding boundary
    may round the other way) and <= 3e-2 (1+|z|) for all;
  * one mixed sweep (learned with probability p): positions within 1e-5 Re0
    for at least 99% of chains, the rest explained by rounding flips;
  * exactness: 3-bead chain in a frozen random field keeps the Boltzmann
    distribution under learned and mixed moves (chi-square, p > 1e-4).
"""
import math

import numpy as np
import pytest

import synth
from oracle import Species, references
from tests.gpu_helpers import constants, custom_config, device_config, flush

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]
HEAD = dict(m_max=1.0, lo=math.log(0.02), hi=math.log(1.0))


def _stream():
    return torch.cuda.current_stream().cuda_stream


def _net(C, params):
    p = torch.from_numpy(params).cuda()
    net = torch.empty(C.soma_net_bytes(), dtype=torch.uint8, device="cuda")
    C.soma_prepare_net(p.data_ptr(), net.data_ptr(), _stream())
    return p, net


@pytest.mark.parametrize("n", [1, 64, 1000, 4099])
def test_forward_matches_bf16_oracle(orc, n):
    from paper_1711_03828_amd import soma as C
    params = synth.mlp_params(11, weight_gain=1.2, out_gain=1.0,
                              shift=np.linspace(-1, 1, 60), scale=np.linspace(0.5, 2, 60))
    feats = np.random.default_rng(n).standard_normal((n, 60)).astype(np.float32) * 2
    p, net = _net(C, params)
    f = torch.from_numpy(feats).cuda()
    z = torch.empty((n, 6), dtype=torch.float32, device="cuda")
    C.soma_mlp_forward(net.data_ptr(), f.data_ptr(), n, z.data_ptr(), _stream())
    torch.cuda.synchronize()
    got = z.cpu().numpy().astype(np.float64)
    exp = orc.mlp_forward(params, feats.astype(np.float64), bf16_mode=True)
    err = np.abs(got - exp) / (1 + np.abs(exp))
    flush("n", n, "max rel err", err.max(), "99.9%", np.quantile(err.max(axis=1), 0.999))
    assert np.quantile(err.max(axis=1), 0.999) <= 2e-3
    assert err.max() <= 3e-2


def test_features_bit_exact(orc):
    from paper_1711_03828_amd.melt import Melt
    w = synth.Workload("feat", (13, 9, 7), (synth.SpeciesSpec(200, 32, 16),
                                            synth.SpeciesSpec(50, 17, 5)), 6.0, 32, 25.0,
                       50.0, 16)
    k0 = constants(w)[0]
    pos = np.concatenate([synth.gaussian_walks(3, 200, 32, w.grid, 1 / math.sqrt(float(k0))),
                          synth.gaussian_walks(4, 50, 17, w.grid, 1 / math.sqrt(float(k0)))])
    m = Melt(device_config(w), positions=torch.from_numpy(pos))
    omega = m.omega.cpu().numpy()
    g = np.random.default_rng(5)
    chains = np.concatenate([np.arange(200), 200 + np.arange(50)]).astype(np.uint32)
    beads = np.concatenate([g.integers(0, 32, 200), g.integers(0, 17, 50)]).astype(np.uint32)
    beads[:3] = [0, 31, 16]
    out = torch.empty((250, 60), dtype=torch.float32, device="cuda")
    from paper_1711_03828_amd import soma as C
    ct = torch.from_numpy(chains.view(np.int32)).cuda()
    bt = torch.from_numpy(beads.view(np.int32)).cuda()
    C.soma_features(m.handle, ct.data_ptr(), bt.data_ptr(), 250, out.data_ptr(), _stream())
    torch.cuda.synchronize()
    exp = np.concatenate([orc.features(pos[:6400], Species(200, 32, 16), beads[:200], omega, w.grid),
                          orc.features(pos[6400:], Species(50, 17, 5), beads[200:], omega, w.grid)])
    np.testing.assert_array_equal(out.cpu().numpy(), exp.astype(np.float32))


@pytest.mark.parametrize("p_learn", [1.0, 0.5])
def test_mixed_sweep_parity(orc, p_learn):
    from paper_1711_03828_amd import soma as C
    from paper_1711_03828_amd.melt import Melt
    w = synth.scaled(synth.C4_MEDIUM, 2048, (24, 24, 24))
    k0, a, A, inv_rho = constants(w)
    params = synth.mlp_params(12, out_gain=0.1)
    pos = synth.gaussian_walks(13, 2048, 32, w.grid, 1 / math.sqrt(float(k0)))
    sp = Species(2048, 32, 16)
    m = Melt(device_config(w, p_learn=p_learn), positions=torch.from_numpy(pos))
    m.set_proposal(torch.from_numpy(params).cuda())
    omega = m.omega.cpu().numpy()   # equals the oracle's field bit for bit (test_gpu_parity)
    np.testing.assert_array_equal(omega, orc.field_f32(orc.density_hist(pos, [sp], w.grid), inv_rho,
                                                       np.float32(w.chi_n), np.float32(w.kappa_n)))
    m.sweep(1, C.SOMA_MOVE_MIXED)
    obs = m.observables()
    ref = pos.copy()
    acc, acc_l, bad, kinds, _ = orc.mc_sweep_mixed(ref, sp, omega, w.grid, k0=k0, n_ref=w.n_ref,
                                                   local_a=a, p_learn=p_learn, params=params,
                                                   **HEAD, bf16_mode=True, seed=w.seed, sweep=0,
                                                   want_flags=True, threads=8)
    got = m.pos.cpu().numpy()
    diff = np.abs(got.astype(np.float64) - ref).reshape(2048, -1).max(axis=1)
    frac_ok = (diff <= 1e-5 * 6.0).mean()
    flush("p_learn", p_learn, "chains within tolerance", frac_ok, "learned attempts",
          obs.attempted[2], int(kinds.sum()), "accepted learned", obs.accepted[2], acc_l)
    assert obs.attempted[2] == int(kinds.sum())        # same mixture draws
    assert frac_ok >= 0.99
    assert abs(int(obs.accepted[2]) - acc_l) <= 0.01 * max(1, acc_l) + 5
    assert obs.counts_conserved == 1 and obs.error_flags == 0
    m.close()


@pytest.mark.parametrize("p_learn", [1.0, 0.5])
def test_three_bead_boltzmann_mixed_on_device(p_learn):
    from paper_1711_03828_amd import soma as C
    from paper_1711_03828_amd.melt import Melt
    L, n_chains = 4, 65536
    grid = (L, L, L)
    omega = synth.uniform_field(21, L ** 3, -2.0, 2.0)
    pos = synth.gaussian_walks(23, n_chains, 3, grid, 1.0 / math.sqrt(3.0))
    params = synth.mlp_params(9, out_gain=0.1)
    params[synth.MLP_LAYOUT["b3"] + 3:synth.MLP_LAYOUT["b3"] + 6] = 1.5
    cfg = custom_config(grid, [Species(n_chains, 3, 2)], k0=3.0, n_ref=1, local_a=0.7,
                        seed=99, count_width=32, p_learn=p_learn)
    m = Melt(cfg, positions=torch.from_numpy(pos))
    m.omega.copy_(torch.from_numpy(omega))       # frozen field
    m.sweep(150, C.SOMA_MOVE_LOCAL)              # equilibrate
    m.set_proposal(torch.from_numpy(params).cuda())
    m.sweep(300, C.SOMA_MOVE_MIXED)
    obs = m.observables()
    assert obs.accepted[2] > 0 and obs.error_flags == 0
    p = m.pos.cpu().numpy().astype(np.float64)
    cells = np.floor(p).astype(np.int64) % L
    lin = ((cells[:, 2] * L + cells[:, 1]) * L + cells[:, 0]).reshape(n_chains, 3)
    dist = references.three_bead_cell_distribution(omega[0], omega[1], 3.0, L)
    marg = [dist.sum(axis=(1, 2)), dist.sum(axis=(0, 2)), dist.sum(axis=(0, 1))]
    for b in range(3):
        pval, stat, dof = references.chi2_pvalue(np.bincount(lin[:, b], minlength=L ** 3), marg[b])
        assert pval > 1e-4, (b, stat, dof)
    obs2 = np.bincount(lin[:, 0] * L ** 3 + lin[:, 2], minlength=L ** 6)
    pval, stat, dof = references.chi2_pvalue(obs2, dist.sum(axis=1).ravel())
    assert pval > 1e-4, (stat, dof)
    m.close()
