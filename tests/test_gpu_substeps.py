"""SCMF cycles with chain sub-steps (field refresh after each chain subset), GPU.

Bars: with fields identically zero (chiN = kappaN = 0) a cycle of k subsets
equals a plain cycle bit for bit (every chain moves once with its own draws);
with fields, the device cycle equals the oracle's cycle done subset by subset
(local moves: positions bit-identical up to threshold mismatches, as for one
sweep); a batch with k subsets equals its melts with k subsets, bit for bit.
"""
import math

import numpy as np
import pytest

import synth
from oracle import Species
from tests.gpu_helpers import constants, device_config, flush, walks_for

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]


def _w(chi, kappa):
    return synth.Workload("sub", (13, 11, 9), (synth.SpeciesSpec(301, 32, 16),
                                               synth.SpeciesSpec(57, 17, 5)),
                          6.0, 32, chi, kappa, 16)


@pytest.mark.parametrize("k", [3, 7])
@pytest.mark.parametrize("kind", ["local", "smc"])
def test_substeps_equal_plain_cycles_without_fields(k, kind):
    from paper_1711_03828_amd import soma as C
    from paper_1711_03828_amd.melt import Melt
    move = C.SOMA_MOVE_LOCAL if kind == "local" else C.SOMA_MOVE_SMC
    w = _w(0.0, 0.0)
    pos = walks_for(w, 5)
    a = Melt(device_config(w), positions=torch.from_numpy(pos))
    b = Melt(device_config(w), positions=torch.from_numpy(pos))
    b.set_substeps(k)
    a.cycle(4, move)
    b.cycle(4, move)
    torch.cuda.synchronize()
    assert np.abs(a.omega.cpu().numpy()).max() == 0.0
    np.testing.assert_array_equal(a.pos.cpu().numpy(), b.pos.cpu().numpy())
    np.testing.assert_array_equal(a.counts.cpu().numpy(), b.counts.cpu().numpy())
    assert tuple(a.observables().accepted) == tuple(b.observables().accepted)


def test_substep_cycle_matches_oracle(orc):
    from paper_1711_03828_amd.melt import Melt
    w = _w(25.0, 50.0)
    k0, a, A, inv_rho = constants(w)
    pos = walks_for(w, 6)
    sps = [Species(s.n_chains, s.n, s.n_a) for s in w.species]
    m = Melt(device_config(w), positions=torch.from_numpy(pos))
    m.set_substeps(3)
    m.cycle(2)
    torch.cuda.synchronize()
    ref = pos.copy()
    omega = orc.field_f32(orc.density_hist(ref, sps, w.grid), inv_rho, np.float32(w.chi_n),
                          np.float32(w.kappa_n))
    for cyc in range(2):
        for j in range(3):
            off, base = 0, 0
            for s in sps:
                for c in range(j, s.n_chains, 3):
                    seg = ref[off + c * s.n: off + (c + 1) * s.n]
                    orc.mc_sweep(seg, Species(1, s.n, s.n_a), omega, w.grid, k0=k0,
                                 n_ref=w.n_ref, step=a, seed=w.seed, sweep=cyc,
                                 chain_base=base + c)
                off += s.n_chains * s.n
                base += s.n_chains
            omega = orc.field_f32(orc.density_hist(ref, sps, w.grid), inv_rho,
                                  np.float32(w.chi_n), np.float32(w.kappa_n))
    got = m.pos.cpu().numpy()
    bad = 0
    off = 0
    for s in sps:
        g = got[off:off + s.n_chains * s.n].reshape(s.n_chains, -1)
        e = ref[off:off + s.n_chains * s.n].reshape(s.n_chains, -1)
        bad += int((g != e).any(axis=1).sum())
        off += s.n_chains * s.n
    flush("chains differing after 2 sub-stepped cycles:", bad)
    assert bad <= 2      # a threshold decision (FP32 vs FP64 energy) moves at most a chain or two
    np.testing.assert_array_equal(m.counts_planes(), orc.density_hist(got, sps, w.grid))


@pytest.mark.parametrize("kind", ["local", "mixed"])
def test_batch_substeps_equal_single(kind):
    from paper_1711_03828_amd import soma as C
    from paper_1711_03828_amd.melt import Batch, Melt
    move = C.SOMA_MOVE_LOCAL if kind == "local" else C.SOMA_MOVE_MIXED
    reps = synth.c3_replicas(n_rep=4, scale=0.02) + synth.c5_replicas(n_rep=1, scale=0.05)
    p_learn = 0.5 if kind == "mixed" else 0.0

    def make():
        ms = [Melt(device_config(w, replica=i, p_learn=p_learn)) for i, w in enumerate(reps)]
        if kind == "mixed":
            for m in ms:
                m.set_proposal(torch.from_numpy(synth.mlp_params(8, out_gain=0.1)).cuda())
        return ms
    ma, mb = make(), make()
    batch = Batch(ma)
    batch.set_substeps(5)
    for m in mb:
        m.set_substeps(5)
    batch.cycle(3, move)
    for m in mb:
        m.cycle(3, move)
    torch.cuda.synchronize()
    for x, y in zip(ma, mb):
        np.testing.assert_array_equal(x.pos.cpu().numpy(), y.pos.cpu().numpy())
        np.testing.assert_array_equal(x.counts.cpu().numpy(), y.counts.cpu().numpy())
        np.testing.assert_array_equal(x.omega.cpu().numpy(), y.omega.cpu().numpy())
    batch.capture_cycle(2, move)
    batch.run_cycle(1)
    for m in mb:
        m.cycle(2, move)
    torch.cuda.synchronize()
    for x, y in zip(ma, mb):
        np.testing.assert_array_equal(x.pos.cpu().numpy(), y.pos.cpu().numpy())
    batch.close()
