"""The seeded input generators (CPU): SplitMix64 known answers, and the replica
ensembles follow their recipe (counts, ranges, densities, species ratios)."""
import math

import numpy as np

import synth


def test_splitmix64_known_answers():
    # the first outputs of the SplitMix64 sequence seeded with 0 (state advanced
    # by the golden gamma before each output)
    assert synth.splitmix64(0) == 0xE220A8397B1DCDAF
    assert synth.splitmix64(0x9E3779B97F4A7C15) == 0x6E789E6AA1B965F4
    assert synth.splitmix64(2 * 0x9E3779B97F4A7C15 & 0xFFFFFFFFFFFFFFFF) == 0x06C45D188009454F


def test_c3_ensemble_recipe():
    reps = synth.c3_replicas()
    assert len(reps) == 64
    chains = np.array([w.species[0].n_chains for w in reps])
    assert chains.min() >= 2048 and chains.max() <= 262144
    assert {w.species[0].n for w in reps} <= {16, 32, 64}
    for r, w in enumerate(reps):
        s = w.species[0]
        assert s.n_a in (round(0.3 * s.n), round(0.5 * s.n))
        assert math.isclose(w.chi_n, 10 + 30 * r / 63)
        side = w.grid[0]
        assert w.grid == (side, side, side)
        assert side == round(6 * (4 * s.n_chains / 1024) ** (1 / 3))
        assert w.seed == synth.splitmix64(synth.MASTER_SEED + r)
    assert len({w.seed for w in reps}) == 64


def test_c5_ensemble_recipe():
    reps = synth.c5_replicas()
    assert len(reps) == 32
    for r, w in enumerate(reps):
        d, ha, hb = w.species
        assert (d.n, d.n_a, ha.n, ha.n_a, hb.n, hb.n_a) == (32, 16, 16, 16, 16, 0)
        beads = 32 * d.n_chains + 16 * (ha.n_chains + hb.n_chains)
        assert abs(32 * d.n_chains / beads - 0.70) < 0.01
        assert ha.n_chains == hb.n_chains
        assert math.isclose(w.chi_n, 15 + 20 * r / 31)
        assert 16384 * 0.9 <= d.n_chains + ha.n_chains + hb.n_chains <= 131072 * 1.1
        rho = beads / w.n_cells            # 8192 beads per Re0^3 at 6 cells per Re0
        assert abs(rho / (8192 / 216) - 1) < 0.25
