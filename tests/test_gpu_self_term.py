"""The self term of cell-changing moves (soma_set_self_term) on the device
against the oracle with the same term.

Bars as in test_gpu_parity: one sweep from identical state and fields, local
moves bit-identical per chain, smart-MC and bond-Gibbs moves within 1e-5 Re0
per coordinate, mismatched chains at most ceil(1e-6 x moves); histogram
bit-exact.  Batched sweeps with the term equal single ones bit for bit, and
the term refuses systems it does not cover.
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

RE = 6.0


def _chain_bad(got, exp, n, tol):
    g = got.reshape(-1, n, 3).astype(np.float64)
    e = exp.reshape(-1, n, 3).astype(np.float64)
    return int((np.abs(g - e).reshape(g.shape[0], -1).max(axis=1) > tol).sum())


@pytest.mark.parametrize("kind", ["local", "smc", "gibbs"])
def test_one_sweep_parity_with_self_term(orc, kind):
    from paper_1711_03828_amd import soma as C
    from paper_1711_03828_amd.melt import Melt
    w = synth.Workload("ragged_self", (17, 23, 9),
                       (synth.SpeciesSpec(301, 32, 16), synth.SpeciesSpec(77, 16, 16),
                        synth.SpeciesSpec(45, 17, 4)), 6.0, 32, 25.0, 50.0, 32)
    k0, a, A, inv_rho = constants(w)
    pos = walks_for(w, 52)
    melt = Melt(device_config(w), positions=torch.from_numpy(pos))
    C.soma_set_self_term(melt.handle, 1)
    sp = [Species(s.n_chains, s.n, s.n_a) for s in w.species]
    omega = orc.field_f32(orc.density_hist(pos, sp, w.grid), inv_rho, np.float32(w.chi_n),
                          np.float32(w.kappa_n))
    s_term = orc.self_energy(np.float32(w.kappa_n), np.float32(w.chi_n),
                                 w.n_cells / w.n_beads, w.n_ref)
    move = {"local": C.SOMA_MOVE_LOCAL, "smc": C.SOMA_MOVE_SMC, "gibbs": C.SOMA_MOVE_GIBBS}[kind]
    melt.sweep(1, move)
    torch.cuda.synchronize()
    got = melt.pos.cpu().numpy()
    ref = pos.copy()
    off, base, bad = 0, 0, 0
    for s in sp:
        seg = ref[off:off + s.n_chains * s.n]
        orc.mc_sweep(seg, s, omega, w.grid, k0=k0, n_ref=w.n_ref,
                     move_kind={"local": 0, "smc": 1, "gibbs": 3}[kind],
                     step=a if kind == "local" else A, seed=w.seed, sweep=0, chain_base=base,
                     threads=8, self_term=s_term)
        bad += _chain_bad(got[off:off + s.n_chains * s.n], seg, s.n,
                          0.0 if kind == "local" else 1e-5 * RE)
        off += s.n_chains * s.n
        base += s.n_chains
    allowed = math.ceil(1e-6 * w.n_beads)
    flush(kind, "self term", float(s_term), "mismatched chains", bad, "allowed", allowed)
    assert bad <= allowed
    if bad == 0:
        np.testing.assert_array_equal(melt.counts_planes(), orc.density_hist(ref, sp, w.grid))
    # the term changes the outcome: without it the oracle accepts more cell changes
    plain = pos.copy()
    off, base = 0, 0
    for s in sp:
        orc.mc_sweep(plain[off:off + s.n_chains * s.n], s, omega, w.grid, k0=k0, n_ref=w.n_ref,
                     move_kind={"local": 0, "smc": 1, "gibbs": 3}[kind],
                     step=a if kind == "local" else A, seed=w.seed, sweep=0, chain_base=base,
                     threads=8)
        off += s.n_chains * s.n
        base += s.n_chains
    assert _chain_bad(plain, ref, 1, 0.0) > 0
    melt.close()


def test_batched_cycles_with_self_term_equal_single():
    from paper_1711_03828_amd import soma as C
    from paper_1711_03828_amd.melt import Batch, Melt
    reps = [synth.scaled(synth.C4_MEDIUM, n, g) for n, g in ((512, (12, 12, 12)),
                                                           (2048, (20, 18, 16)))]
    ma = [Melt(device_config(w, replica=i)) for i, w in enumerate(reps)]
    mb = [Melt(device_config(w, replica=i)) for i, w in enumerate(reps)]
    for m in ma + mb:
        C.soma_set_self_term(m.handle, 1)
    batch = Batch(ma)
    for kind in (C.SOMA_MOVE_LOCAL, C.SOMA_MOVE_GIBBS, C.SOMA_MOVE_SMC):
        batch.cycle(3, kind)
        for m in mb:
            m.cycle(3, kind)
        torch.cuda.synchronize()
        for x, y in zip(ma, mb):
            assert torch.equal(x.pos, y.pos), kind
            assert torch.equal(x.counts, y.counts), kind
    batch.close()
    for m in ma + mb:
        m.close()


def test_self_term_refusals():
    from paper_1711_03828_amd import soma as C
    from paper_1711_03828_amd.melt import Melt
    w = synth.scaled(synth.C1_SMALL, 64, (8, 8, 8))
    m = Melt(device_config(w))
    with pytest.raises(C.SomaError):
        C.soma_set_self_term(m.handle, 2)
    m.set_scheme(C.SOMA_SCHEME_MOLECULE)
    with pytest.raises(C.SomaError):
        C.soma_set_self_term(m.handle, 1)
    m.set_scheme(C.SOMA_SCHEME_SET)
    C.soma_set_self_term(m.handle, 1)
    m.set_scheme(C.SOMA_SCHEME_MOLECULE)
    with pytest.raises(C.SomaError):      # the molecule order refuses to sweep with it
        m.sweep(1, C.SOMA_MOVE_LOCAL)
    m.close()
