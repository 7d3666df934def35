"""GPU parity of n_t bead types (Sec. 2.1; Eqs. (6), (8), (12)) against the
oracle.

Bars: the kept histogram planes equal the oracle's recount bit for bit; the
fields equal the oracle's FP32 order bit for bit (both interaction forms, 16-
and 32-bit counts); H_nb within 1e-12; a sweep of an ABC triblock (three
types, next to a linear AB diblock species), of a four-type miktoarm star and
of a chain cycling through all eight types (four count planes, an odd number
of cells) matches the oracle's sweep bit for bit per molecule, with at most 1e-6 of the
moves in molecules with an accept-decision mismatch (rounded up); per-type
totals and the conservation flag hold; two types set this way equal the
two-type path bit for bit; unsupported combinations are refused.
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

CHI3 = [[0.0, 20.0, 35.0], [20.0, 0.0, 12.5], [35.0, 12.5, 0.0]]
CHI4 = [[0.0, 20.0, 30.0, 10.0], [20.0, 0.0, 15.0, 25.0],
        [30.0, 15.0, 0.0, 40.0], [10.0, 25.0, 40.0, 0.0]]


@pytest.fixture(scope="module")
def C():
    from paper_1711_03828_amd import soma
    return soma


def _system(kind):
    """(species tuples, architecture words of species 0, its bonds, its types, chi)."""
    if kind == "abc":   # A10 B12 C10 triblock next to linear A16 B16 chains
        n = 32
        types = [0] * 10 + [1] * 12 + [2] * 10
        bonds = [(i, i + 1) for i in range(n - 1)]
        return [(900, n, 0), (500, 32, 16)], synth.encode_architecture(n, types, bonds), \
            bonds, types, CHI3
    if kind == "octa":   # eight types (four count planes), a linear 24-mer cycling through them
        n = 24
        types = [i % 8 for i in range(n)]
        bonds = [(i, i + 1) for i in range(n - 1)]
        chi = np.random.default_rng(8).uniform(0.0, 40.0, (8, 8)).astype(np.float32)
        chi = np.triu(chi, 1) + np.triu(chi, 1).T
        return [(1500, n, 0)], synth.encode_architecture(n, types, bonds), bonds, types, \
            chi.tolist()
    n, bonds = synth.star_bonds(4, 6)   # core + four arms of six, arm k of type k
    types = [0] + [k for k in range(4) for _ in range(6)]
    return [(1200, n, 0)], synth.encode_architecture(n, types, bonds), bonds, types, CHI4


def _positions(species, bonds, grid, k0):
    sig = 1 / math.sqrt(float(k0))
    parts = [synth.tree_walks(71, species[0][0], species[0][1], bonds, grid, sig)]
    for i, (n_c, n, _) in enumerate(species[1:]):
        parts.append(synth.gaussian_walks(72 + i, n_c, n, grid, sig))
    return np.concatenate(parts).astype(np.float32)


def _oracle_hist(orc, pos, species, words, grid, n_t):
    n0 = species[0][0] * species[0][1]
    h = orc.density_hist_arch(pos[:n0], species[0][0], words, grid, n_types=n_t)
    if len(species) > 1:
        h[:2] += orc.density_hist(pos[n0:], [Species(*s) for s in species[1:]], grid)
    return h


def _oracle_sweep(orc, pos, species, words, omega, grid, k0, sweep):
    n0 = species[0][0] * species[0][1]
    ref = pos.copy()
    a0 = ref[:n0]
    acc, _ = orc.mc_sweep_arch(a0, species[0][0], words, omega, grid, k0=k0, n_ref=32,
                               step=np.float32(0.3), seed=321, sweep=sweep, threads=8)
    ref[:n0] = a0
    if len(species) > 1:
        n_c, n, n_a = species[1]
        a1 = np.ascontiguousarray(ref[n0:])
        acc1, _ = orc.mc_sweep(a1, Species(n_c, n, n_a), np.ascontiguousarray(omega[:2]), grid,
                               k0=k0, n_ref=32, step=np.float32(0.3), seed=321, sweep=sweep,
                               chain_base=species[0][0], threads=8)
        ref[n0:] = a1
        acc += acc1
    return ref, acc


@pytest.mark.parametrize("kind,width,form", [("abc", 16, 1), ("abc", 32, 0), ("mikto4", 16, 0),
                                             ("mikto4", 32, 1), ("octa", 32, 1), ("octa", 16, 0)])
def test_types_sweep_and_fields_match_oracle(C, orc, kind, width, form):
    from paper_1711_03828_amd.melt import Melt
    species, words, bonds, types, chi = _system(kind)
    n_t = len(chi)
    grid = (23, 19, 13) if kind == "octa" else (26, 22, 18)   # octa: n_cells odd
    k0 = np.float32(2.0)
    pos = _positions(species, bonds, grid, k0)
    cfg = custom_config(grid, [Species(*s) for s in species], k0=k0, n_ref=32, chi_n=20.0,
                        kappa_n=40.0, local_a=0.3, count_width=width, seed=321)
    m = Melt(cfg, positions=torch.from_numpy(pos))
    m.set_hamiltonian(form)
    m.set_types(chi)                         # before the architecture: codes up to n_t - 1
    m.set_architecture(words, 0)
    n_beads = len(pos)
    inv_rho = np.float32(np.prod(grid) / n_beads)
    total = np.bincount(np.concatenate([np.tile(types, species[0][0])] +
                                       [np.tile([0] * s[2] + [1] * (s[1] - s[2]), s[0])
                                        for s in species[1:]]), minlength=n_t)
    cur = pos
    for sweep in range(2):
        counts = _oracle_hist(orc, cur, species, words, grid, n_t)
        np.testing.assert_array_equal(m.counts_planes(), counts)
        omega = orc.field_multi_f32(counts, inv_rho, chi, np.float32(40.0), form=form)
        np.testing.assert_array_equal(m.omega.cpu().numpy(), omega)
        obs = m.observables()
        h = orc.h_nb_multi(counts, np.prod(grid) / n_beads, chi, 40.0, 32, form=form)
        assert obs.h_nb == pytest.approx(h, rel=1e-12, abs=1e-9)
        assert obs.counts_conserved == 1
        assert obs.count_a == total[0] and obs.count_b == total[1:].sum()
        assert m.type_counts() == [int(x) for x in total]
        m.sweep(1, C.SOMA_MOVE_LOCAL)
        torch.cuda.synchronize()
        got = m.pos.cpu().numpy()
        ref, _ = _oracle_sweep(orc, cur, species, words, omega, grid, k0, sweep)
        n0 = species[0][0] * species[0][1]
        bad0 = (got[:n0].reshape(species[0][0], -1) != ref[:n0].reshape(species[0][0], -1)).any(1)
        bad = int(bad0.sum())
        if len(species) > 1:
            bad += int((got[n0:].reshape(species[1][0], -1)
                        != ref[n0:].reshape(species[1][0], -1)).any(1).sum())
        allowed = math.ceil(1e-6 * n_beads)
        flush(kind, width, form, "sweep", sweep, "mismatched molecules", bad, "allowed", allowed)
        assert bad <= allowed
        m.update_fields()
        cur = got
    np.testing.assert_array_equal(m.counts_planes(),
                                  _oracle_hist(orc, cur, species, words, grid, n_t))
    m.close()


def test_two_types_set_explicitly_equal_the_two_type_path(C):
    from paper_1711_03828_amd.melt import Melt
    grid = (24, 20, 16)
    species = [Species(700, 32, 12), Species(300, 16, 16)]
    pos = np.concatenate([synth.gaussian_walks(81 + i, s.n_chains, s.n, grid, 0.6)
                          for i, s in enumerate(species)])
    runs = []
    for explicit in (False, True):
        cfg = custom_config(grid, species, k0=2.0, n_ref=32, chi_n=25.0 if not explicit else 0.0,
                            kappa_n=40.0, local_a=0.3, count_width=32, seed=5)
        m = Melt(cfg, positions=torch.from_numpy(pos))
        if explicit:
            m.set_types([[0.0, 25.0], [25.0, 0.0]])
        m.cycle(3)
        torch.cuda.synchronize()
        obs = m.observables()
        runs.append((m.pos.cpu().numpy(), m.counts_planes(), m.omega.cpu().numpy(), obs.h_nb))
        m.close()
    for x, y in zip(runs[0][:3], runs[1][:3]):
        np.testing.assert_array_equal(x, y)
    assert runs[0][3] == runs[1][3]


def test_types_refusals(C):
    from paper_1711_03828_amd.melt import Melt
    grid = (12, 12, 12)
    n, bonds = synth.star_bonds(3, 4)
    types3 = [0] + [k for k in range(3) for _ in range(4)]
    cfg = custom_config(grid, [Species(200, n, 0)], k0=2.0, n_ref=32, chi_n=20.0, kappa_n=40.0,
                        local_a=0.3, count_width=16, seed=9)
    pos = synth.tree_walks(91, 200, n, bonds, grid, 0.7)
    m = Melt(cfg, positions=torch.from_numpy(pos))
    words = synth.encode_architecture(n, types3, bonds)
    with pytest.raises(C.SomaError):          # type code 2 needs three types first
        m.set_architecture(words)
    with pytest.raises(C.SomaError):          # not symmetric
        m.set_types([[0, 1, 2], [1, 0, 3], [2, 4, 0]])
    with pytest.raises(C.SomaError):          # more than eight types
        m.set_types(np.zeros((9, 9)))
    m.set_types(CHI3)
    m.set_architecture(words)
    with pytest.raises(C.SomaError):          # smart-MC with three types
        m.sweep(1, C.SOMA_MOVE_SMC)
    mask = torch.zeros((12 ** 3 + 31) // 32, dtype=torch.int32, device="cuda")
    with pytest.raises(C.SomaError):          # walls with three types
        m.set_external(None, mask)
    with pytest.raises(C.SomaError):          # a type code without a plane
        m.set_types([[0, 1], [1, 0]])
    m.sweep(2, C.SOMA_MOVE_LOCAL)
    assert m.observables().counts_conserved == 1
    m.close()
