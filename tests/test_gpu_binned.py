"""Binned count updates (SOMA_HIST_BINNED) against direct atomics and the oracle.

Integer counts are order-independent, so the bar is bit-exact everywhere:
  * the same sweeps from the same state with either histogram mode give
    bit-identical positions (the moves do not depend on the mode) and
    bit-identical counts, equal to the oracle's count of the device positions;
  * with more updates than a bin holds (a dense melt and bond-Gibbs moves,
    which move most beads to another cell) the overflow goes to direct
    atomics and the counts are still exact;
  * captured cycles with binned updates replay like eager cycles;
  * at the benchmark's full size (134M beads) the binned sweep equals the
    direct one, and the kept histogram equals a recount.
"""
import math

import numpy as np
import pytest

import synth
from oracle import Species
from tests.gpu_helpers import constants, custom_config, device_config, flush

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]


def _stream():
    return torch.cuda.current_stream().cuda_stream


def _pair(cfg, pos, params=None):
    from paper_1711_03828_amd import soma as C
    from paper_1711_03828_amd.melt import Melt
    melts = []
    for mode in (C.SOMA_HIST_DIRECT, C.SOMA_HIST_BINNED):
        m = Melt(cfg, positions=torch.from_numpy(pos))
        m.set_histogram(mode)
        if params is not None:
            m.set_proposal(torch.from_numpy(params).cuda())
        melts.append(m)
    return melts


def _recount(orc, melt, sp, grid):
    torch.cuda.synchronize()
    return orc.density_hist(melt.pos.cpu().numpy(), sp, grid)


def _compare(orc, direct, binned, sp, grid, what):
    torch.cuda.synchronize()
    assert torch.equal(direct.pos, binned.pos), f"{what}: positions differ between modes"
    assert torch.equal(direct.counts, binned.counts), f"{what}: counts differ between modes"
    np.testing.assert_array_equal(binned.counts_planes(), _recount(orc, binned, sp, grid),
                                  err_msg=f"{what}: kept counts differ from a recount")


KINDS = ["local", "smc", "gibbs", "mixed"]


@pytest.mark.parametrize("width", [16, 32])
@pytest.mark.parametrize("kind", KINDS)
def test_binned_equals_direct(orc, kind, width):
    from paper_1711_03828_amd import soma as C
    move = {"local": C.SOMA_MOVE_LOCAL, "smc": C.SOMA_MOVE_SMC, "gibbs": C.SOMA_MOVE_GIBBS,
            "mixed": C.SOMA_MOVE_MIXED}[kind]
    # ragged grid (partial bricks on every face) and ragged species
    grid = (37, 21, 19)
    sp = [Species(301, 32, 16), Species(45, 17, 5), Species(60, 16, 16)]
    k0 = np.float32(3.0 * 31 / 36.0)
    pos = np.concatenate([synth.gaussian_walks(11 + i, s.n_chains, s.n, grid,
                                               1 / math.sqrt(float(k0))) for i, s in enumerate(sp)])
    cfg = custom_config(grid, sp, k0=k0, n_ref=32, chi_n=25.0, kappa_n=50.0, local_a=0.107763,
                        smc_a=0.05625, count_width=width, seed=5,
                        p_learn=0.5 if kind == "mixed" else 0.0)
    params = synth.mlp_params(3, out_gain=0.3) if kind == "mixed" else None
    direct, binned = _pair(cfg, pos, params)
    flush("case", kind, width)
    for m in (direct, binned):
        m.sweep(3, move)       # frozen fields: the counts accumulate three sweeps
    _compare(orc, direct, binned, sp, grid, "three sweeps")
    for m in (direct, binned):
        m.cycle(4, move)
    _compare(orc, direct, binned, sp, grid, "four cycles")
    for m in (direct, binned):
        obs = m.observables()
        assert obs.counts_conserved == 1 and obs.error_flags == 0
    direct.close()
    binned.close()


@pytest.mark.parametrize("width", [16, 32])
def test_binned_overflow_goes_direct(orc, width):
    """81,920 beads on 3,960 cells (about 21 per cell) and bond-Gibbs moves: a
    sweep moves about two thirds of the beads to another cell, more updates
    than a bin holds; the overflow takes the direct path."""
    from paper_1711_03828_amd import soma as C
    grid = (20, 18, 11)
    sp = [Species(2560, 32, 16)]
    k0 = np.float32(3.0 * 31 / 36.0)
    pos = synth.gaussian_walks(21, 2560, 32, grid, 1 / math.sqrt(float(k0)))
    cfg = custom_config(grid, sp, k0=k0, n_ref=32, chi_n=10.0, kappa_n=20.0, local_a=0.107763,
                        smc_a=0.5, count_width=width, seed=9)
    direct, binned = _pair(cfg, pos)
    for kind in (C.SOMA_MOVE_GIBBS, C.SOMA_MOVE_SMC, C.SOMA_MOVE_LOCAL):
        flush("kind", kind)
        for m in (direct, binned):
            m.sweep(2, kind)
        _compare(orc, direct, binned, sp, grid, f"kind {kind}")
        for m in (direct, binned):
            m.cycle(2, kind)
        _compare(orc, direct, binned, sp, grid, f"kind {kind} cycles")
    direct.close()
    binned.close()


def test_binned_graph_replays_equal_eager_cycles(orc):
    """Captured cycles (binned) replayed several times, eager work and
    synchronisations in between, against the same cycles run eagerly."""
    from paper_1711_03828_amd import soma as C
    w = synth.C1_SMALL
    sp = [Species(1024, 32, 16)]
    k0 = constants(w)[0]
    pos = synth.gaussian_walks(31, 1024, 32, w.grid, 1 / math.sqrt(float(k0)))
    cfg = device_config(w)
    eager, graph = _pair(cfg, pos)
    eager.set_histogram(C.SOMA_HIST_BINNED)
    graph.capture_cycle(3, C.SOMA_MOVE_LOCAL)
    for rep in range(4):
        eager.cycle(3, C.SOMA_MOVE_LOCAL)
        graph.run_cycle(1)
        torch.cuda.synchronize()
        _ = eager.observables()
        assert torch.equal(eager.pos, graph.pos), rep
        assert torch.equal(eager.counts, graph.counts), rep
        assert torch.equal(eager.omega, graph.omega), rep
        np.testing.assert_array_equal(graph.counts_planes(), _recount(orc, graph, sp, w.grid))
    eager.close()
    graph.close()


def test_binned_fullsize_equals_direct():
    """134,217,728 beads on 384x384x192 cells, 32-bit counts: one local sweep
    and one smart-MC sweep in each mode from the same state; positions and
    counts bit-identical, the kept counts equal a device recount."""
    from paper_1711_03828_amd import soma as C
    from paper_1711_03828_amd.melt import Melt
    w = synth.C2_LARGE
    cfg = device_config(w)
    flush("full size: device init (Philox walks)")
    direct = Melt(cfg)   # positions initialised on the device from the seed
    binned = Melt(cfg)
    binned.set_histogram(C.SOMA_HIST_BINNED)
    torch.cuda.synchronize()
    assert torch.equal(direct.pos, binned.pos)
    for kind in (C.SOMA_MOVE_LOCAL, C.SOMA_MOVE_SMC):
        flush("full size: kind", kind)
        direct.cycle(1, kind)
        binned.cycle(1, kind)
        torch.cuda.synchronize()
        assert torch.equal(direct.pos, binned.pos)
        assert torch.equal(direct.counts, binned.counts)
        assert torch.equal(direct.omega, binned.omega)
    recount = torch.zeros_like(binned.counts)
    C.soma_density_hist(binned.cfg, binned.pos.data_ptr(), recount.data_ptr(), _stream())
    torch.cuda.synchronize()
    assert torch.equal(recount, binned.counts)
    obs = binned.observables()
    assert obs.counts_conserved == 1 and obs.error_flags == 0
    direct.close()
    binned.close()
