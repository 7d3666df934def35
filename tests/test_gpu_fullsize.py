"""Parity at the benchmark's full size: 4,194,304 A16B16 chains (134,217,728 beads),
384x384x192 cells, 32-bit counts, chiN = 20, kappaN = 50, in the launch
configuration bench.py times.

The oracle histograms and fields the whole melt (bit-exact comparison on all
28.3 M cells) and sweeps a sample of chains spread over the whole range one by
one; the device sweeps the whole melt.  Bars as in test_gpu_parity.
"""
import math

import numpy as np
import pytest

import synth
from oracle import Species
from tests.gpu_helpers import (constants, device_config, explain_mismatches, flush,
                               proposal_test_params)

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]


@pytest.fixture(scope="module")
def big():
    w = synth.C2_LARGE
    k0 = constants(w)[0]
    flush("generating", w.n_beads, "beads")
    pos = synth.gaussian_walks(77, w.n_chains, 32, w.grid, 1 / math.sqrt(float(k0)))
    return w, pos


@pytest.fixture(scope="module")
def big_fields(orc, big):
    """The oracle's histogram and fields of the full-size initial positions."""
    w, pos = big
    inv_rho = constants(w)[3]
    flush("oracle histogram + fields")
    counts = orc.density_hist(pos, [Species(w.n_chains, 32, 16)], w.grid)
    omega = orc.field_f32(counts, inv_rho, np.float32(w.chi_n), np.float32(w.kappa_n))
    return counts, omega


def test_fullsize_histogram_fields_and_sampled_sweep(orc, big, big_fields):
    from paper_1711_03828_amd import soma as C
    from paper_1711_03828_amd.melt import Melt
    w, pos = big
    k0, a, A, inv_rho = constants(w)
    sp = Species(w.n_chains, 32, 16)
    counts, omega = big_fields
    flush("device init")
    melt = Melt(device_config(w), positions=torch.from_numpy(pos))
    torch.cuda.synchronize()
    np.testing.assert_array_equal(melt.counts_planes(), counts)
    np.testing.assert_array_equal(melt.omega.cpu().numpy(), omega)

    # the launch shape the bench's autotuner picks at this size (binned count
    # updates, 512-thread blocks, one tile per wave; positions streamed with the
    # non-temporal hint)
    melt.set_histogram(C.SOMA_HIST_BINNED)
    C.soma_set_sweep_threads(melt.handle, 512)
    flush("device sweep")
    melt.sweep(1, C.SOMA_MOVE_LOCAL)
    torch.cuda.synchronize()
    got = melt.pos.cpu().numpy().reshape(w.n_chains, 32, 3)
    sample = np.unique(np.linspace(0, w.n_chains - 1, 4096).astype(np.int64))
    bad = 0
    for c in sample:
        ref = pos.reshape(w.n_chains, 32, 3)[c].copy()
        orc.mc_sweep(ref.reshape(-1, 3), Species(1, 32, 16), omega, w.grid, k0=k0,
                     n_ref=w.n_ref, step=a, seed=w.seed, sweep=0, chain_base=int(c))
        bad += int(not np.array_equal(ref, got[c]))
    allowed = math.ceil(1e-6 * w.n_beads)
    flush("sampled chains", sample.size, "mismatched", bad, "allowed", allowed)
    assert bad <= allowed
    # properties at full size: exact conservation and the kept histogram equals
    # a from-scratch recount of the device positions
    obs = melt.observables()
    assert obs.counts_conserved == 1
    recount = torch.zeros_like(melt.counts)
    C.soma_density_hist(melt.cfg, melt.pos.data_ptr(), recount.data_ptr(),
                        torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    assert torch.equal(recount, melt.counts)
    melt.close()


def test_fullsize_smc_sweep_sampled(orc, big, big_fields):
    """One smart-MC sweep of the whole 134M-bead melt on the device (field
    gradient from the neighbour gathers); the oracle sweeps 4096 chains spread
    over the whole range one by one from the same positions and fields.
    Positions within 1e-5 Re0 per coordinate; chains beyond it at most
    ceil(1e-6 x moves)."""
    from paper_1711_03828_amd import soma as C
    from paper_1711_03828_amd.melt import Melt
    w, pos = big
    k0, a, A, inv_rho = constants(w)
    _, omega = big_fields
    melt = Melt(device_config(w), positions=torch.from_numpy(pos))
    melt.set_histogram(C.SOMA_HIST_BINNED)   # as the bench's smart-MC leg
    C.soma_set_sweep_threads(melt.handle, 512)
    flush("device smart-MC sweep")
    melt.sweep(1, C.SOMA_MOVE_SMC)
    torch.cuda.synchronize()
    got = melt.pos.cpu().numpy().reshape(w.n_chains, 32, 3)
    sample = np.unique(np.linspace(0, w.n_chains - 1, 4096).astype(np.int64))
    tol = 1e-5 * w.re_cells
    bad = 0
    for c in sample:
        ref = pos.reshape(w.n_chains, 32, 3)[c].copy()
        orc.mc_sweep(ref.reshape(-1, 3), Species(1, 32, 16), omega, w.grid, k0=k0,
                     n_ref=w.n_ref, move_kind=orc.MOVE_SMC, step=A, seed=w.seed, sweep=0,
                     chain_base=int(c))
        bad += int(np.abs(ref.astype(np.float64) - got[c].astype(np.float64)).max() > tol)
    allowed = math.ceil(1e-6 * w.n_beads)
    flush("smart-MC sampled chains", sample.size, "beyond 1e-5 Re0", bad, "allowed", allowed)
    assert bad <= allowed
    obs = melt.observables()
    assert obs.counts_conserved == 1 and obs.error_flags == 0
    recount = torch.zeros_like(melt.counts)
    C.soma_density_hist(melt.cfg, melt.pos.data_ptr(), recount.data_ptr(),
                        torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    assert torch.equal(recount, melt.counts)
    melt.close()


def test_fullsize_learned_sweep_sampled(orc):
    """The 262,144-chain melt of the learned-proposal study (96^3 cells) at full
    size: one mixed sweep with learned moves only on the device (a random
    network with standardised inputs that moves beads); the oracle's
    BF16-emulating sweep of 2048 sampled chains from the same positions and
    fields, compared move by move as in the learned parity test: decisions
    equal, accepted positions within 1e-5 Re0 plus the move's rounding
    envelope, every other chain explained by a move the oracle flags
    (unexplained at most ceil(1e-6 x sampled moves)); the kept histogram
    equals the recount of the device positions."""
    from paper_1711_03828_amd import soma as C
    from paper_1711_03828_amd.melt import Melt
    w = synth.C4_MEDIUM
    k0, a, A, inv_rho = constants(w)
    pos = synth.gaussian_walks(78, w.n_chains, 32, w.grid, 1 / math.sqrt(float(k0)))
    melt = Melt(device_config(w, p_learn=1.0), positions=torch.from_numpy(pos))
    omega = melt.omega.cpu().numpy()
    params = proposal_test_params(orc, pos, Species(w.n_chains, 32, 16), omega, w.grid, seed=31)
    melt.set_proposal(torch.from_numpy(params).cuda())
    flush("device mixed sweep at full size")
    melt.sweep(1, C.SOMA_MOVE_MIXED)
    torch.cuda.synchronize()
    got = melt.pos.cpu().numpy().reshape(w.n_chains, 32, 3)
    head = dict(m_max=1.0, lo=math.log(0.02), hi=math.log(1.0))
    sample = np.unique(np.linspace(0, w.n_chains - 64, 32).astype(np.int64))
    tot = dict(bad=0, unexplained=0, flagged=0, dec=0, acc=0)
    for c0 in sample:   # 32 blocks of 64 consecutive chains spread over the melt
        init = pos.reshape(w.n_chains, 32, 3)[c0:c0 + 64].copy().reshape(-1, 3)
        ref = init.copy()
        amb = np.zeros(64 * 32, np.uint8)
        env = np.zeros(64 * 32, np.float32)
        acc, _, _, _, acc_flags = orc.mc_sweep_mixed(
            ref, Species(64, 32, 16), omega, w.grid, k0=k0, n_ref=w.n_ref, local_a=a, p_learn=1.0,
            params=params, **head, bf16_mode=True, seed=w.seed, sweep=0, chain_base=int(c0),
            want_flags=True, threads=8, ambiguous=amb, pos_env=env)
        b, u, fl, d = explain_mismatches(got[c0:c0 + 64].reshape(-1, 3), init, ref, acc_flags, amb,
                                         env, 32)
        for k, v in zip(("bad", "unexplained", "flagged", "dec", "acc"), (b, u, fl, d, acc)):
            tot[k] += v
    n_moves = 32 * 64 * len(sample)
    allowed = math.ceil(1e-6 * n_moves)
    flush("sampled chains", 64 * len(sample), "accepted", tot["acc"] / n_moves, tot, "allowed", allowed)
    assert tot["acc"] > 0.3 * n_moves
    assert tot["unexplained"] <= allowed
    assert tot["flagged"] <= 0.08 * 64 * len(sample)
    obs = melt.observables()
    assert obs.counts_conserved == 1 and obs.error_flags == 0
    recount = torch.zeros_like(melt.counts)
    C.soma_density_hist(melt.cfg, melt.pos.data_ptr(), recount.data_ptr(),
                        torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    assert torch.equal(recount, melt.counts)
    melt.close()


def test_fullsize_batch_equals_single():
    """The 64-replica ensemble at full size (1.9e8 beads), in the launch shape
    the autotuner picks: two batched SCMF cycles give the bits of the same
    cycles run melt by melt (whose parity with the oracle the other tests pin)."""
    from paper_1711_03828_amd import soma as C
    from paper_1711_03828_amd.melt import Batch, Melt, make_config
    reps = synth.c3_replicas()
    runs = []
    for batched in (True, False):
        melts = [Melt(make_config(w, replica=i)) for i, w in enumerate(reps)]
        if batched:
            b = Batch(melts)
            tune = b.autotune(1, C.SOMA_MOVE_LOCAL)
            flush("tuned", tune.mode, tune.grid_blocks)
            # the tuning ran cycles: bring the unbatched run to the same sweep index
            b.cycle(2, C.SOMA_MOVE_LOCAL)
            b.close()
            n_tuned = tune.cycles_run
        else:
            for m in melts:
                m.cycle(n_tuned + 2)
        torch.cuda.synchronize()
        runs.append([(m.pos.cpu().numpy(), m.omega.cpu().numpy()) for m in melts])
        for m in melts:
            m.close()
    for (p0, o0), (p1, o1) in zip(runs[0], runs[1]):
        np.testing.assert_array_equal(p0, p1)
        np.testing.assert_array_equal(o0, o1)
