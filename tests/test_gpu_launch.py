"""Launch shapes never change results: block sizes of the SET sweeps and the
autotuner's search space (histogram mode x block size x grid).

Bar: bit-identical positions, counts and fields (integer counts and per-bead
Philox draws do not depend on how waves are grouped into blocks).
"""
import math

import numpy as np
import pytest

import synth
from oracle import Species
from tests.gpu_helpers import custom_config, flush

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]


def _setup(width=32, p_learn=0.0):
    grid = (29, 23, 17)
    sp = [Species(250, 32, 16), Species(33, 17, 8)]
    k0 = np.float32(3.0 * 31 / 36.0)
    pos = np.concatenate([synth.gaussian_walks(61 + i, s.n_chains, s.n, grid,
                                               1 / math.sqrt(float(k0))) for i, s in enumerate(sp)])
    cfg = custom_config(grid, sp, k0=k0, n_ref=32, chi_n=20.0, kappa_n=40.0, local_a=0.107763,
                        smc_a=0.05625, count_width=width, seed=3, p_learn=p_learn)
    return cfg, pos


@pytest.mark.parametrize("threads", [64, 128, 512])
def test_block_sizes_equal_default(threads):
    from paper_1711_03828_amd import soma as C
    from paper_1711_03828_amd.melt import Melt
    cfg, pos = _setup()
    ref = Melt(cfg, positions=torch.from_numpy(pos))
    got = Melt(cfg, positions=torch.from_numpy(pos))
    C.soma_set_sweep_threads(got.handle, threads)
    for kind in (C.SOMA_MOVE_LOCAL, C.SOMA_MOVE_SMC, C.SOMA_MOVE_GIBBS):
        for m in (ref, got):
            m.cycle(3, kind)
        torch.cuda.synchronize()
        assert torch.equal(ref.pos, got.pos), (threads, kind)
        assert torch.equal(ref.counts, got.counts), (threads, kind)
        assert torch.equal(ref.omega, got.omega), (threads, kind)
    o_ref, o_got = ref.observables(), got.observables()
    assert list(o_ref.accepted) == list(o_got.accepted)
    ref.close()
    got.close()


def _random_params(seed):
    """A network blob with identity standardisation and small random weights."""
    g = np.random.default_rng(seed)
    p = np.zeros(8576, np.float32)
    p[60:120] = 1.0                                        # scale
    p[120:3960] = g.normal(0, 0.15, 3840)                  # W1 [64][60]
    p[4024:8120] = g.normal(0, 0.15, 4096)                 # W2 [64][64]
    p[8184:8568] = g.normal(0, 0.1, 384)                   # W3 [6][64]
    return torch.from_numpy(p).cuda()


@pytest.mark.parametrize("hist", [0, 1])
@pytest.mark.parametrize("blocks", [5, 8, 24])
@pytest.mark.parametrize("kind_name", ["local", "smc", "gibbs", "mixed"])
def test_persistent_grids_equal_default(hist, blocks, kind_name):
    """Persistent SET sweeps (fewer blocks than tile groups) draw their tiles
    from per-part counters; any grid gives the default trajectory bit for bit
    (5 blocks: one part; 8 and 24: eight parts), for every move kind."""
    from paper_1711_03828_amd import soma as C
    from paper_1711_03828_amd.melt import Melt
    kind = {"local": C.SOMA_MOVE_LOCAL, "smc": C.SOMA_MOVE_SMC, "gibbs": C.SOMA_MOVE_GIBBS,
            "mixed": C.SOMA_MOVE_MIXED}[kind_name]
    cfg, pos = _setup(p_learn=0.5 if kind_name == "mixed" else 0.0)
    ref = Melt(cfg, positions=torch.from_numpy(pos))
    got = Melt(cfg, positions=torch.from_numpy(pos))
    for m in (ref, got):
        m.set_histogram(C.SOMA_HIST_BINNED if hist else C.SOMA_HIST_DIRECT)
        if kind_name == "mixed":
            m.set_proposal(_random_params(7))
    if kind_name != "mixed":
        C.soma_set_sweep_threads(got.handle, 128)
    C.soma_set_sweep_blocks(got.handle, blocks)
    for m in (ref, got):
        m.cycle(4, kind)
    got.capture_cycle(3, kind)     # the counters' reset is a graph node too
    got.run_cycle(2)
    ref.cycle(6, kind)
    torch.cuda.synchronize()
    assert torch.equal(ref.pos, got.pos)
    assert torch.equal(ref.counts, got.counts)
    assert torch.equal(ref.omega, got.omega)
    assert list(ref.observables().accepted) == list(got.observables().accepted)
    ref.close()
    got.close()


def test_sweep_threads_refused():
    from paper_1711_03828_amd import soma as C
    from paper_1711_03828_amd.melt import Melt
    cfg, pos = _setup()
    m = Melt(cfg, positions=torch.from_numpy(pos))
    for bad in (0, 32, 96, 1024):
        with pytest.raises(C.SomaError):
            C.soma_set_sweep_threads(m.handle, bad)
    m.close()


@pytest.mark.parametrize("kind_name,n_expected", [("local", 12), ("smc", 12), ("gibbs", 12)])
def test_autotune_search_space_keeps_results(tmp_path, kind_name, n_expected):
    """Every candidate (histogram mode x block size x grid) runs real cycles;
    the tuned system's trajectory equals an untuned one advanced by the same
    number of cycles, bit for bit; a second call reads the cache."""
    from paper_1711_03828_amd import soma as C
    from paper_1711_03828_amd.melt import Melt
    kind = {"local": C.SOMA_MOVE_LOCAL, "smc": C.SOMA_MOVE_SMC,
            "gibbs": C.SOMA_MOVE_GIBBS}[kind_name]
    cfg, pos = _setup()
    tuned = Melt(cfg, positions=torch.from_numpy(pos))
    plain = Melt(cfg, positions=torch.from_numpy(pos))
    cache = str(tmp_path / "tune.txt")
    t = tuned.autotune(2, kind, cache)
    flush(kind_name, "chosen hist", t.hist_mode, "threads", t.block_threads, "grid",
          t.grid_blocks, "candidates", t.candidates, "ms", t.ms_per_cycle)
    assert t.candidates == n_expected and t.cycles_run == 3 * n_expected
    assert t.hist_mode in (C.SOMA_HIST_DIRECT, C.SOMA_HIST_BINNED)
    assert t.block_threads in (128, 256, 512)
    plain.cycle(t.cycles_run, kind)
    for m in (tuned, plain):
        m.cycle(4, kind)
    torch.cuda.synchronize()
    assert torch.equal(tuned.pos, plain.pos)
    assert torch.equal(tuned.counts, plain.counts)
    assert torch.equal(tuned.omega, plain.omega)
    t2 = tuned.autotune(2, kind, cache)
    assert t2.from_cache == 1 and t2.hist_mode == t.hist_mode and t2.block_threads == t.block_threads
    tuned.close()
    plain.close()


@pytest.mark.parametrize("mode", [0, 1])
def test_probe_atomics_adds_every_update(mode):
    """The throughput probe's atomic modes add exactly one per update."""
    from paper_1711_03828_amd import soma as C
    words = torch.zeros(100003, dtype=torch.int32, device="cuda")
    C.soma_probe_atomics(words.data_ptr(), words.numel(), 1234567, mode, 9,
                         torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    assert int(words.sum().item()) == 1234567
    with pytest.raises(C.SomaError):
        C.soma_probe_atomics(words.data_ptr(), words.numel(), 10, 3, 9,
                             torch.cuda.current_stream().cuda_stream)
