"""Structure factor on the device against the oracle (GPU).

Bar: S(q) elementwise within 1e-10 of the largest value (FP64 direct
transforms against numpy's FFT of the same counts), the same shell peak; a
two-slab composition pattern puts the peak at its period.
"""
import math

import numpy as np
import pytest

import synth
from oracle import Species
from oracle import analysis as A
from tests.gpu_helpers import constants, device_config, flush, walks_for

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]


def _device_sq(m):
    from paper_1711_03828_amd import soma as C
    ws_b = C.soma_sq_workspace_bytes(m.handle)
    ws = torch.empty(ws_b, dtype=torch.uint8, device="cuda")
    sq = torch.empty(m.n_cells, dtype=torch.float64, device="cuda")
    C.soma_structure_factor(m.handle, ws.data_ptr(), ws_b, sq.data_ptr(),
                            torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    return sq.cpu().numpy()


@pytest.mark.parametrize("wname", ["c1", "ragged32"])
def test_structure_factor_matches_oracle(orc, wname):
    from paper_1711_03828_amd import soma as C
    from paper_1711_03828_amd.melt import Melt
    if wname == "c1":
        w = synth.C1_SMALL
    else:
        w = synth.Workload("ragged32", (13, 10, 7), (synth.SpeciesSpec(300, 17, 9),), 6.0, 17,
                           20.0, 50.0, 32)
    pos = walks_for(w, 61)
    m = Melt(device_config(w), positions=torch.from_numpy(pos))
    sp = [Species(s.n_chains, s.n, s.n_a) for s in w.species]
    counts = orc.density_hist(pos, sp, w.grid)
    np.testing.assert_array_equal(m.counts_planes(), counts)
    got = _device_sq(m)
    exp = A.structure_factor(counts, w.grid, w.n_ref, w.n_beads)
    err = np.abs(got - exp).max() / exp.max()
    flush(wname, "max rel err", err)
    assert err <= 1e-10
    _, m1, c1, p1 = C.soma_sq_shells(got, w.grid, 20)
    _, m2, c2, p2 = A.sq_shells(exp, w.grid, 20)
    assert p1 == p2
    np.testing.assert_allclose(m1, m2, rtol=1e-9)


def test_slab_pattern_peak():
    """A beads in two slabs along z (period L/2): peak shell 2."""
    from paper_1711_03828_amd import soma as C
    from paper_1711_03828_amd.melt import Melt
    w = synth.scaled(synth.C1_SMALL, 2048, (24, 24, 24))
    pos = walks_for(w, 62).reshape(2048, 32, 3)
    L = 24.0
    z = np.mod(pos[:, :, 2], L)
    a = np.arange(32) < 16
    slab = np.floor(z / 6.0)            # four slabs of 6 cells
    want_a = (slab % 2 == 0)
    # move every bead into a slab of its own type (shift by 6 cells where needed)
    shift = np.where(a[None, :] != want_a, 6.0, 0.0)
    pos[:, :, 2] = pos[:, :, 2] + shift
    pos = pos.reshape(-1, 3).astype(np.float32)
    m = Melt(device_config(w), positions=torch.from_numpy(pos))
    sq = _device_sq(m)
    _, mean, cnt, peak = C.soma_sq_shells(sq, w.grid, 12)
    flush("slab shells", np.round(mean[:6], 1), "peak", peak)
    assert peak == 2
