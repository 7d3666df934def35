"""Batched sweeps over many melts, captured cycles and the autotuner (GPU).

Bars (all bit-exact -- launch shapes and batching never change results):
  * one batched local sweep of several uneven melts equals the oracle's sweep
    of each melt, position for position;
  * batched cycles (sweep + field refresh, every move kind) equal the same
    cycles of each melt alone: positions, counts, fields, acceptance counters
    and the FP64 field energy -- with direct and with binned count updates;
  * replays of a captured graph equal the same cycles called one by one,
    checked after every replay with eager work in between;
  * an autotuned run equals an untuned run of the same number of cycles, and
    a cache hit runs nothing.
"""
import math
import os

import numpy as np
import pytest

import synth
from oracle import Species
from tests.gpu_helpers import constants, device_config, flush, walks_for

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]


def _replicas():
    """Small uneven melts: chain lengths 16/32/64 (ragged tiles), a blend with
    three species, different grids and chiN."""
    reps = synth.c3_replicas(n_rep=5, scale=0.02)
    reps += synth.c5_replicas(n_rep=2, scale=0.05)
    return reps


def _melts(reps, p_learn=0.0, positions=None):
    from paper_1711_03828_amd.melt import Melt
    out = []
    for i, w in enumerate(reps):
        cfg = device_config(w, p_learn=p_learn, replica=i)
        if positions is None:
            out.append(Melt(cfg))
        else:
            out.append(Melt(cfg, positions=torch.from_numpy(positions[i])))
    return out


def _state(m):
    o = m.observables()
    return (m.pos.cpu().numpy(), m.counts.cpu().numpy(), m.omega.cpu().numpy(),
            tuple(o.accepted), tuple(o.attempted), o.h_nb, o.sweeps)


def _assert_same(ma, mb, what):
    for i, (a, b) in enumerate(zip(ma, mb)):
        sa, sb = _state(a), _state(b)
        for k, name in enumerate(["pos", "counts", "omega"]):
            assert np.array_equal(sa[k], sb[k]), (what, i, name)
        assert sa[3:] == sb[3:], (what, i, sa[3:], sb[3:])


def test_batched_local_sweep_matches_oracle(orc):
    from paper_1711_03828_amd import soma as C
    from paper_1711_03828_amd.melt import Batch
    reps = _replicas()
    pos = [walks_for(w, 100 + i) for i, w in enumerate(reps)]
    melts = _melts(reps, positions=pos)
    batch = Batch(melts)
    flush("items", [w.n_chains for w in reps])
    batch.sweep(1, C.SOMA_MOVE_LOCAL)
    torch.cuda.synchronize()
    for i, (w, m) in enumerate(zip(reps, melts)):
        k0, a, A, inv_rho = constants(w)
        sp = [Species(s.n_chains, s.n, s.n_a) for s in w.species]
        omega = orc.field_f32(orc.density_hist(pos[i], sp, w.grid), inv_rho,
                              np.float32(w.chi_n), np.float32(w.kappa_n))
        exp = pos[i].copy()
        off, base = 0, 0
        for s in sp:
            seg = exp[off:off + s.n_chains * s.n]
            orc.mc_sweep(seg, s, omega, w.grid, k0=k0, n_ref=w.n_ref, step=a, seed=w.seed,
                         sweep=0, replica=i, chain_base=base, threads=8)
            exp[off:off + s.n_chains * s.n] = seg
            off += s.n_chains * s.n
            base += s.n_chains
        np.testing.assert_array_equal(m.pos.cpu().numpy(), exp, err_msg=f"replica {i}")
        np.testing.assert_array_equal(m.counts_planes(), orc.density_hist(exp, sp, w.grid))
    batch.close()


@pytest.mark.parametrize("kind", ["local", "smc", "mixed", "gibbs"])
def test_batched_cycles_equal_single(kind):
    from paper_1711_03828_amd import soma as C
    from paper_1711_03828_amd.melt import Batch
    move = {"local": C.SOMA_MOVE_LOCAL, "smc": C.SOMA_MOVE_SMC, "mixed": C.SOMA_MOVE_MIXED,
            "gibbs": C.SOMA_MOVE_GIBBS}[kind]
    reps = _replicas()
    p_learn = 0.5 if kind == "mixed" else 0.0
    ma, mb = _melts(reps, p_learn), _melts(reps, p_learn)
    if kind == "mixed":   # a different network per species
        for mset in (ma, mb):
            for m in mset:
                for sp in range(m.cfg.n_species):
                    params = synth.mlp_params(50 + sp, out_gain=0.1)
                    m.set_proposal(torch.from_numpy(params).cuda(), species=sp)
    batch = Batch(ma)
    for rep_ in range(2):
        batch.cycle(3, move)
        for m in mb:
            m.cycle(3, move)
        torch.cuda.synchronize()
        _assert_same(ma, mb, f"{kind} round {rep_}")
    flush(kind, "accepted", [tuple(m.observables().accepted) for m in ma][:3])
    batch.close()


@pytest.mark.parametrize("kind", ["local", "smc", "mixed", "gibbs"])
def test_batched_binned_cycles_equal_single(kind):
    """Binned batched sweeps (every melt's own bins, one apply launch for all
    bricks of the batch) against each melt alone with direct atomics, in two
    launch shapes (one block per item, and a persistent round-robin grid)."""
    from paper_1711_03828_amd import soma as C
    from paper_1711_03828_amd.melt import Batch
    move = {"local": C.SOMA_MOVE_LOCAL, "smc": C.SOMA_MOVE_SMC, "mixed": C.SOMA_MOVE_MIXED,
            "gibbs": C.SOMA_MOVE_GIBBS}[kind]
    reps = _replicas()
    p_learn = 0.5 if kind == "mixed" else 0.0
    ma, mb = _melts(reps, p_learn), _melts(reps, p_learn)
    if kind == "mixed":
        for mset in (ma, mb):
            for m in mset:
                for sp in range(m.cfg.n_species):
                    params = synth.mlp_params(50 + sp, out_gain=0.1)
                    m.set_proposal(torch.from_numpy(params).cuda(), species=sp)
    batch = Batch(ma)
    batch.set_histogram(C.SOMA_HIST_BINNED)
    flush("binned batch", kind)
    for rep_, (mode, grid) in enumerate([(0, 0), (1, 24)]):
        batch.set_launch(mode, grid)
        batch.cycle(3, move)
        for m in mb:
            m.cycle(3, move)
        torch.cuda.synchronize()
        _assert_same(ma, mb, f"binned {kind} shape {mode} {grid}")
    batch.close()


def test_batch_histogram_refusals():
    from paper_1711_03828_amd import soma as C
    from paper_1711_03828_amd.melt import Batch
    reps = _replicas()[:2]
    batch = Batch(_melts(reps))
    with pytest.raises(C.SomaError):
        batch.set_histogram(7)
    batch.set_histogram(C.SOMA_HIST_BINNED)
    batch.set_histogram(C.SOMA_HIST_DIRECT)
    batch.close()


def test_graph_replays_equal_eager_cycles():
    from paper_1711_03828_amd import soma as C
    from paper_1711_03828_amd.melt import Batch, Melt
    w = synth.scaled(synth.C1_SMALL, 3000, (28, 28, 28))
    a, b = Melt(device_config(w)), Melt(device_config(w))
    a.capture_cycle(4, C.SOMA_MOVE_LOCAL)
    for r in range(3):
        a.run_cycle(1)
        b.cycle(4, C.SOMA_MOVE_LOCAL)
        torch.cuda.synchronize()
        _assert_same([a], [b], f"single replay {r}")
        a.observables()          # eager work between replays
    reps = _replicas()
    ma, mb = _melts(reps), _melts(reps)
    batch = Batch(ma)
    batch.capture_cycle(3, C.SOMA_MOVE_SMC)
    for r in range(3):
        batch.run_cycle(1)
        for m in mb:
            m.cycle(3, C.SOMA_MOVE_SMC)
        torch.cuda.synchronize()
        _assert_same(ma, mb, f"batch replay {r}")
    batch.run_cycle(2)
    for m in mb:
        m.cycle(6, C.SOMA_MOVE_SMC)
    _assert_same(ma, mb, "batch double replay")
    batch.close()


def test_autotune_keeps_results(tmp_path):
    from paper_1711_03828_amd import soma as C
    from paper_1711_03828_amd.melt import Batch, Melt
    cache = str(tmp_path / "tune.txt")
    w = synth.scaled(synth.C4_MEDIUM, 8192, (36, 36, 36))
    a, b = Melt(device_config(w)), Melt(device_config(w))
    t = a.autotune(2, C.SOMA_MOVE_LOCAL, cache)
    flush("single tune", t.mode, t.grid_blocks, t.ms_per_cycle, t.candidates, t.cycles_run)
    # histogram mode {direct, binned} x block size {256, 128, 512} x grid {0, 2048}
    assert t.candidates == 12 and t.cycles_run == 36 and t.from_cache == 0
    b.cycle(t.cycles_run)
    a.cycle(5)
    b.cycle(5)
    _assert_same([a], [b], "tuned single")
    t2 = a.autotune(2, C.SOMA_MOVE_LOCAL, cache)
    assert t2.from_cache == 1 and t2.cycles_run == 0
    assert (t2.mode, t2.grid_blocks, t2.hist_mode, t2.block_threads) == \
        (t.mode, t.grid_blocks, t.hist_mode, t.block_threads)
    reps = _replicas()
    ma, mb = _melts(reps), _melts(reps)
    batch = Batch(ma)
    tb = batch.autotune(2, C.SOMA_MOVE_LOCAL, cache)
    flush("batch tune", tb.mode, tb.grid_blocks, tb.ms_per_cycle, tb.candidates, tb.cycles_run)
    # histogram {direct, binned} x item order {XCD ranges, round-robin} x grid
    # {one block per item, 2048, 8192}
    assert tb.candidates == 12 and tb.cycles_run == 36
    for m in mb:
        m.cycle(tb.cycles_run)
    batch.cycle(3)
    for m in mb:
        m.cycle(3)
    _assert_same(ma, mb, "tuned batch")
    assert open(cache).read().count("\n") == 2
    batch.close()


@pytest.mark.parametrize("mode,grid", [(0, 16), (1, 24), (0, 0), (1, 0)])
def test_batch_launch_shapes(mode, grid):
    """Persistent and round-robin shapes (every block loops over items)."""
    from paper_1711_03828_amd import soma as C
    from paper_1711_03828_amd.melt import Batch
    reps = _replicas()
    ma, mb = _melts(reps), _melts(reps)
    batch = Batch(ma)
    batch.set_launch(mode, grid)
    batch.cycle(2, C.SOMA_MOVE_LOCAL)
    batch.cycle(1, C.SOMA_MOVE_SMC)
    for m in mb:
        m.cycle(2, C.SOMA_MOVE_LOCAL)
        m.cycle(1, C.SOMA_MOVE_SMC)
    _assert_same(ma, mb, f"shape {mode} {grid}")
    batch.close()
