"""GPU parity of the K^0 interaction term (Eq. (6), first form; fields of Eq.
(12), first form) against the oracle: fields bit-exact in the FP32 order for
both count widths and a ragged grid, H_nb within 1e-9 relative, and eight SCMF
cycles of local moves chain-for-chain identical (a decision mismatch spreads
through the fields; at most 8 chains may differ); switching back restores the
K^1 fields."""
import numpy as np
import pytest

import synth
from oracle import Species
from tests.gpu_helpers import constants, device_config, flush, stepwise_cycles, walks_for

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]


@pytest.mark.parametrize("grid,width", [((24, 24, 24), 16), ((17, 23, 9), 32)])
def test_k0_fields_and_h_nb(orc, grid, width):
    from paper_1711_03828_amd.melt import Melt
    w = synth.Workload("k0", grid, (synth.SpeciesSpec(900, 32, 16), synth.SpeciesSpec(41, 17, 5)),
                       6.0, 32, 30.0, 50.0, width)
    pos = walks_for(w, 91)
    m = Melt(device_config(w), positions=torch.from_numpy(pos))
    m.set_hamiltonian(0)
    sp = [Species(s.n_chains, s.n, s.n_a) for s in w.species]
    counts = orc.density_hist(pos, sp, w.grid)
    inv_rho = constants(w)[3]
    exp = orc.field_f32(counts, inv_rho, np.float32(w.chi_n), np.float32(w.kappa_n), form=0)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(m.omega.cpu().numpy(), exp)
    obs = m.observables()
    h = orc.h_nb(counts, w.n_cells / w.n_beads, w.chi_n, w.kappa_n, w.n_ref, form=0)
    assert obs.h_nb == pytest.approx(h, rel=1e-9)
    m.set_hamiltonian(1)
    exp1 = orc.field_f32(counts, inv_rho, np.float32(w.chi_n), np.float32(w.kappa_n))
    torch.cuda.synchronize()
    np.testing.assert_array_equal(m.omega.cpu().numpy(), exp1)
    with pytest.raises(RuntimeError):
        m.set_hamiltonian(2)
    m.close()


def test_k0_cycles_parity(orc):
    """Eight SCMF cycles with the K0 Hamiltonian, each compared in full from the
    device's own state (histogram and K0 fields bit-exact, positions
    bit-identical per chain up to ceil(1e-6 x moves) threshold mismatches)."""
    from paper_1711_03828_amd.melt import Melt
    w = synth.C1_SMALL
    k0, a, A, inv_rho = constants(w)
    pos = walks_for(w, 92)
    m = Melt(device_config(w), positions=torch.from_numpy(pos))
    m.set_hamiltonian(0)
    sp = [Species(1024, 32, 16)]

    def sweep(p, om, cyc):
        orc.mc_sweep(p, sp[0], om, w.grid, k0=k0, n_ref=w.n_ref, step=a, seed=w.seed,
                     sweep=cyc, threads=8)

    def field_of(counts):
        return orc.field_f32(counts, inv_rho, np.float32(w.chi_n), np.float32(w.kappa_n), form=0)

    stepwise_cycles(m, orc, sp, w.grid, 8, sweep, field_of, n_per_chain=32)
    m.close()
