"""GPU parity of the learned proposal (network on MFMA, mixed MH sweep).

Bars:
  * features: bit-exact against the oracle (FP32 field values and bond vectors);
  * network outputs z: the oracle's BF16-emulating forward (inputs, weights and
    hidden activations rounded to bfloat16 at the same points) with FP64
    accumulation, against BF16 MFMA with FP32 accumulation: every output
    within the oracle's rounding envelope (the FP32 error bound of its own sum
    plus the effect of every hidden rounding that such sums may take the other
    way);
  * one mixed sweep (learned with probability p): move by move, decisions equal
    and accepted positions within 1e-5 Re0 plus the move's rounding envelope;
    every chain that breaks this holds a move the oracle flags as decidable
    otherwise by rounding (unexplained chains at most ceil(1e-6 x moves));
  * exactness: 3-bead chain in a frozen random field keeps the Boltzmann
    distribution under learned and mixed moves (chi-square, p > 1e-4).
"""
import math

import numpy as np
import pytest

import synth
from oracle import Species, references
from tests.gpu_helpers import (constants, custom_config, device_config, explain_mismatches, flush,
                               proposal_test_params)

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
    exp, bound, n_amb = orc.mlp_forward_envelope(params, feats.astype(np.float64))
    # the device evaluates the network with the standardisation folded into the
    # first layer; the envelope's centre is the oracle's BF16 forward of that form
    np.testing.assert_array_equal(exp, orc.mlp_forward(orc.fold_params(params),
                                                       feats.astype(np.float64), bf16_mode=True))
    excess = np.abs(got - exp) - bound
    flush("n", n, "ambiguous roundings", n_amb, "max |dz|", np.abs(got - exp).max(),
          "max |dz| / bound", (np.abs(got - exp) / bound).max(), "max excess", excess.max())
    assert excess.max() <= 0.0


def test_features_bit_exact(orc):
    from paper_1711_03828_amd.melt import Melt
    w = synth.Workload("feat", (13, 9, 7), (synth.SpeciesSpec(200, 32, 16),
                                            synth.SpeciesSpec(50, 17, 5)), 6.0, 32, 25.0,
                       50.0, 16)
    k0 = constants(w)[0]
    pos = np.concatenate([synth.gaussian_walks(3, 200, 32, w.grid, 1 / math.sqrt(float(k0))),
                          synth.gaussian_walks(4, 50, 17, w.grid, 1 / math.sqrt(float(k0)))])
    m = Melt(device_config(w), positions=torch.from_numpy(pos))
    omega = _oracle_field(orc, w, pos)
    np.testing.assert_array_equal(m.omega.cpu().numpy(), omega)
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


def _oracle_field(orc, w, pos):
    sps = [Species(s.n_chains, s.n, s.n_a) for s in w.species]
    inv_rho = np.float32(w.n_cells / w.n_beads)
    return orc.field_f32(orc.density_hist(pos, sps, w.grid), inv_rho, np.float32(w.chi_n),
                         np.float32(w.kappa_n))


def test_collect_training(orc):
    """Sample choice from the Philox block (s, 5<<16, round, replica); features
    bit-exact against the oracle; r0 the bead's position; dr = r(later) - r0."""
    from paper_1711_03828_amd import soma as C
    from paper_1711_03828_amd.melt import Melt
    w = synth.Workload("collect", (13, 9, 7), (synth.SpeciesSpec(200, 32, 16),
                                               synth.SpeciesSpec(50, 17, 5)), 6.0, 32, 25.0,
                       50.0, 16)
    k0 = constants(w)[0]
    pos = np.concatenate([synth.gaussian_walks(6, 200, 32, w.grid, 1 / math.sqrt(float(k0))),
                          synth.gaussian_walks(7, 50, 17, w.grid, 1 / math.sqrt(float(k0)))])
    seed, replica, rnd, n = 0x1234_5678_9ABC_DEF1, 3, 9, 3001
    m = Melt(device_config(w, seed=seed, replica=replica), positions=torch.from_numpy(pos))
    omega = _oracle_field(orc, w, pos)
    np.testing.assert_array_equal(m.omega.cpu().numpy(), omega)
    feats = torch.empty((n, 60), dtype=torch.float32, device="cuda")
    r0 = torch.empty((n, 3), dtype=torch.float32, device="cuda")
    dr = torch.empty((n, 3), dtype=torch.float32, device="cuda")
    picked = torch.empty((n, 2), dtype=torch.int32, device="cuda")
    C.soma_collect_training(m.handle, n, rnd, 0, feats.data_ptr(), r0.data_ptr(), 0,
                            picked.data_ptr(), _stream())
    torch.cuda.synchronize()
    ctr = np.zeros((n, 4), np.uint32)
    ctr[:, 0] = np.arange(n)
    ctr[:, 1] = 5 << 16
    ctr[:, 2] = rnd
    ctr[:, 3] = replica
    key = np.array([seed & 0xFFFFFFFF, seed >> 32], np.uint32)
    blk = orc.philox(ctr, key).astype(np.uint64)
    chain = (blk[:, 0] * 250) >> 32
    n_of = np.where(chain < 200, 32, 17).astype(np.uint64)
    bead = (blk[:, 1] * n_of) >> 32
    got = picked.cpu().numpy().view(np.uint32)
    np.testing.assert_array_equal(got[:, 0], chain)
    np.testing.assert_array_equal(got[:, 1], bead)
    idx = np.where(chain < 200, chain * 32 + bead, 6400 + (chain - 200) * 17 + bead).astype(np.int64)
    np.testing.assert_array_equal(r0.cpu().numpy(), pos[idx])
    exp = np.empty((n, 60))
    for sp_i, (lo, sp) in enumerate([(0, Species(200, 32, 16)), (200, Species(50, 17, 5))]):
        sel = (chain >= lo) & (chain < lo + sp.n_chains)
        base = 0 if sp_i == 0 else 6400
        for b in np.unique(bead[sel]):
            rows = orc.features(pos[base:base + sp.n_chains * sp.n], sp,
                                np.full(sp.n_chains, b, np.uint32), omega, w.grid)
            k = sel & (bead == b)
            exp[k] = rows[(chain[k] - lo).astype(np.int64)]
    np.testing.assert_array_equal(feats.cpu().numpy(), exp.astype(np.float32))
    m.cycle(3)
    C.soma_collect_training(m.handle, n, rnd, 1, 0, r0.data_ptr(), dr.data_ptr(), 0, _stream())
    torch.cuda.synchronize()
    now = m.pos.cpu().numpy()[idx]
    np.testing.assert_array_equal(dr.cpu().numpy(), now - pos[idx])
    assert np.abs(dr.cpu().numpy()).max() > 0
    # one species only: chains 200 + floor(w0 * 50 / 2^32)
    C.soma_collect_training(m.handle, n, rnd, 0, 0, r0.data_ptr(), 0, picked.data_ptr(),
                            _stream(), species=1)
    torch.cuda.synchronize()
    got = picked.cpu().numpy().view(np.uint32)
    np.testing.assert_array_equal(got[:, 0], 200 + ((blk[:, 0] * 50) >> 32))
    np.testing.assert_array_equal(got[:, 1], (blk[:, 1] * 17) >> 32)
    with pytest.raises(C.SomaError):
        C.soma_collect_training(m.handle, n, rnd, 0, 0, r0.data_ptr(), 0, 0, _stream(), species=2)


@pytest.mark.parametrize("p_learn,self_term", [(1.0, False), (0.5, False), (1.0, True)])
def test_mixed_sweep_parity(orc, p_learn, self_term):
    """One mixed sweep on the device against the oracle's BF16-emulating sweep
    from the same positions and fields, move by move: the device accepted a
    move iff the bead moved; decisions must agree, and accepted positions agree
    within 1e-5 Re0 plus the move's rounding envelope (how far BF16 roundings
    that FP32 sums may take either way can shift the trial).  Every chain that
    breaks this must hold a move the oracle flags as decidable otherwise by
    rounding; unexplained chains at most ceil(1e-6 x moves).  The network moves
    beads (standardised inputs, damped mean), so most moves are accepted."""
    from paper_1711_03828_amd import soma as C
    from paper_1711_03828_amd.melt import Melt
    w = synth.scaled(synth.C4_MEDIUM, 2048, (24, 24, 24))
    k0, a, A, inv_rho = constants(w)
    pos = synth.gaussian_walks(13, 2048, 32, w.grid, 1 / math.sqrt(float(k0)))
    sp = Species(2048, 32, 16)
    m = Melt(device_config(w, p_learn=p_learn), positions=torch.from_numpy(pos))
    omega = m.omega.cpu().numpy()   # equals the oracle's field bit for bit (test_gpu_parity)
    np.testing.assert_array_equal(omega, orc.field_f32(orc.density_hist(pos, [sp], w.grid), inv_rho,
                                                       np.float32(w.chi_n), np.float32(w.kappa_n)))
    params = proposal_test_params(orc, pos, sp, omega, w.grid, seed=12)
    m.set_proposal(torch.from_numpy(params).cuda())
    s_term = 0.0
    if self_term:   # the bead's own share of a cell-changing move on both sides
        C.soma_set_self_term(m.handle, 1)
        s_term = orc.self_energy(np.float32(w.kappa_n), np.float32(w.chi_n),
                                 w.n_cells / w.n_beads, w.n_ref)
    m.sweep(1, C.SOMA_MOVE_MIXED)
    obs = m.observables()
    ref = pos.copy()
    amb = np.zeros(2048 * 32, np.uint8)
    env = np.zeros(2048 * 32, np.float32)
    acc, acc_l, bad, kinds, acc_flags = orc.mc_sweep_mixed(
        ref, sp, omega, w.grid, k0=k0, n_ref=w.n_ref, local_a=a, p_learn=p_learn, params=params,
        **HEAD, bf16_mode=True, seed=w.seed, sweep=0, want_flags=True, threads=8, ambiguous=amb,
        pos_env=env, self_term=s_term)
    got = m.pos.cpu().numpy()
    n_bad, unexplained, flagged, dec = explain_mismatches(got, pos, ref, acc_flags, amb, env, 32)
    allowed = math.ceil(1e-6 * pos.shape[0])
    flush("p_learn", p_learn, "accepted", acc / pos.shape[0], "mismatched chains", n_bad,
          "unexplained", unexplained, "allowed", allowed, "flagged chains", flagged,
          "decision mismatches", dec, "learned attempts", obs.attempted[2], int(kinds.sum()),
          "accepted learned", obs.accepted[2], acc_l)
    assert obs.attempted[2] == int(kinds.sum())        # same mixture draws
    assert acc > 0.3 * pos.shape[0]
    assert unexplained <= allowed
    assert flagged <= 0.08 * 2048
    assert abs(int(obs.accepted[2]) - acc_l) <= int(amb[kinds == 1].sum())
    assert obs.counts_conserved == 1 and obs.error_flags == 0
    m.close()


@pytest.mark.parametrize("p_learn,trained", [(1.0, False), (0.5, False), (1.0, True)])
def test_three_bead_boltzmann_mixed_on_device(p_learn, trained):
    """Random (drifting) weights, and weights trained on this system's own plain
    trajectories: the Boltzmann distribution holds either way."""
    from paper_1711_03828_amd import learned, soma as C
    from paper_1711_03828_amd.melt import Melt
    L, n_chains = 4, 65536
    grid = (L, L, L)
    omega = synth.uniform_field(21, L ** 3, -2.0, 2.0)
    pos = synth.gaussian_walks(23, n_chains, 3, grid, 1.0 / math.sqrt(3.0))
    cfg = custom_config(grid, [Species(n_chains, 3, 2)], k0=3.0, n_ref=1, local_a=0.7,
                        seed=99, count_width=32, p_learn=p_learn)
    m = Melt(cfg, positions=torch.from_numpy(pos))
    m.omega.copy_(torch.from_numpy(omega))       # frozen field
    m.sync_fields()
    m.sweep(150, C.SOMA_MOVE_LOCAL)              # equilibrate
    if trained:
        F, D = learned.collect(m, 65536, 10, 4, frozen_field=True)
        pt = learned.init_params(F, seed=2)
        losses = learned.train(pt, F, D, steps=600, batch=4096, lr=3e-3, loss_every=100)
        flush("3-bead training loss", losses)
        assert losses[-1] < losses[0]
        m.set_proposal(pt)
    else:
        params = synth.mlp_params(9, out_gain=0.1)
        params[synth.MLP_LAYOUT["b3"] + 3:synth.MLP_LAYOUT["b3"] + 6] = 1.5
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


def _re_vectors(m, n):
    x = m.pos.view(-1, n, 3)
    return (x[:, -1] - x[:, 0]).double()


def test_learned_proposal_gain():
    """Train on plain trajectories of a melt at the density of the 256k-chain
    study (9.48 beads per cell, chiN 25), then compare: bead mean-square
    displacement per sweep and the end-to-end autocorrelation after 1000 SCMF
    cycles, plain local move against the trained proposal."""
    from paper_1711_03828_amd import learned, soma as C
    from paper_1711_03828_amd.melt import Melt
    w = synth.scaled(synth.C4_MEDIUM, 4096, (24, 24, 24))
    m = Melt(device_config(w, p_learn=1.0))
    m.cycle(200)
    F, D = learned.collect(m, 65536, 128, 8)
    params = learned.init_params(F, seed=1)
    losses = learned.train(params, F, D, steps=2000, batch=4096, lr=3e-3, loss_every=200)
    flush("training loss", losses)
    assert losses[-1] < losses[0] - 5.0
    m.set_proposal(params)
    res = {}
    for kind in (C.SOMA_MOVE_LOCAL, C.SOMA_MOVE_MIXED):
        o0 = m.observables()
        r0 = m.pos.clone()
        e0 = _re_vectors(m, 32)
        m.cycle(1, kind)
        msd = float((m.pos - r0).double().pow(2).sum(1).mean())
        m.cycle(999, kind)
        o1 = m.observables()
        e1 = _re_vectors(m, 32)
        corr = float((e0 * e1).sum(1).mean() / (e0 * e0).sum(1).mean())
        k = 0 if kind == C.SOMA_MOVE_LOCAL else 2
        acc = (o1.accepted[k] - o0.accepted[k]) / (o1.attempted[k] - o0.attempted[k])
        res[kind] = (msd, corr, acc)
        flush("move", kind, "msd/sweep", msd, "C_Re(1000)", corr, "acceptance", acc)
        assert o1.error_flags == 0 and o1.counts_conserved == 1
    (msd_p, c_p, _), (msd_l, c_l, acc_l) = res[C.SOMA_MOVE_LOCAL], res[C.SOMA_MOVE_MIXED]
    assert acc_l > 0.3
    assert msd_l > 10 * msd_p
    assert c_p > 0.75 and c_l < c_p - 0.3
    m.close()
