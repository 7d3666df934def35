"""GPU parity of the external fields (Sec. 4): a per-type external energy added
to the fields and impenetrable cells (film walls), against the oracle.

Bars: fields bit-exact against the oracle's FP32 order (with the reference
density of the free cells); H_nb within 1e-9 relative; one sweep of local and
molecule-order moves bit-identical per chain without a decision mismatch
(mismatches at most 1e-6 of the moves, rounded up), smart-MC and mixed moves to
the bars of their own parity tests; no bead ever enters an impenetrable cell;
the 3-bead chain samples the Boltzmann distribution restricted to the free
cells; batched cycles equal the cycles melt by melt bit for bit.
"""
import math

import numpy as np
import pytest

import synth
from oracle import Species, references
from tests.gpu_helpers import (constants, custom_config, device_config, explain_mismatches, flush,
                               proposal_test_params)

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

HEAD = dict(m_max=1.0, lo=math.log(0.02), hi=math.log(1.0))


@pytest.fixture(scope="module")
def C():
    from paper_1711_03828_amd import soma
    return soma


def _film(grid, species, width=16, name="film"):
    return synth.Workload(name, grid, species, 6.0, 32, 25.0, 50.0, width)


def _setup(C, w, seed, ext_scale=1.5, **cfg_kw):
    """Device melt with walls at z = 0 and z = nz-1 and a random external field,
    and the oracle's view of the same state."""
    from paper_1711_03828_amd.melt import Melt
    nz = w.grid[2]
    k0 = constants(w)[0]
    parts = [synth.film_walks(seed + i, s.n_chains, s.n, w.grid, 1 / math.sqrt(float(k0)), 1.0,
                              nz - 1.0) for i, s in enumerate(w.species)]
    pos = np.concatenate(parts)
    walls = synth.wall_cells(w.grid, [0, nz - 1])
    mask = synth.pack_mask(walls)
    ext = synth.uniform_field(seed + 50, w.n_cells, -ext_scale, ext_scale)
    m = Melt(device_config(w, **cfg_kw), positions=torch.from_numpy(pos))
    m.set_external(torch.from_numpy(ext).cuda(), torch.from_numpy(mask.view(np.int32)).cuda())
    sp = [Species(s.n_chains, s.n, s.n_a) for s in w.species]
    n_free = int((~walls).sum())
    inv_rho = np.float32(n_free / w.n_beads)
    return m, pos, sp, walls, mask, ext, inv_rho


@pytest.mark.parametrize("grid,width", [((24, 24, 10), 16), ((17, 23, 9), 32)])
def test_fields_and_h_nb_with_external(C, orc, grid, width):
    w = _film(grid, (synth.SpeciesSpec(600, 32, 16), synth.SpeciesSpec(50, 17, 5)), width)
    m, pos, sp, walls, mask, ext, inv_rho = _setup(C, w, 71)
    counts = orc.density_hist(pos, sp, w.grid)
    exp = orc.field_f32(counts, inv_rho, np.float32(w.chi_n), np.float32(w.kappa_n), ext, mask)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(m.omega.cpu().numpy(), exp)
    obs = m.observables()
    n_free = int((~walls).sum())
    h = orc.h_nb(counts, n_free / w.n_beads, w.chi_n, w.kappa_n, w.n_ref, mask)
    assert obs.h_nb == pytest.approx(h, rel=1e-9)
    # detaching restores the plain fields of all cells
    m.set_external(None, None)
    plain = orc.field_f32(counts, np.float32(w.n_cells / w.n_beads), np.float32(w.chi_n),
                          np.float32(w.kappa_n))
    np.testing.assert_array_equal(m.omega.cpu().numpy(), plain)
    m.close()


def _bad_chains(got, exp, n, tol):
    g = got.reshape(-1, n, 3).astype(np.float64)
    e = exp.reshape(-1, n, 3).astype(np.float64)
    return np.abs(g - e).reshape(g.shape[0], -1).max(axis=1) > tol


@pytest.mark.parametrize("order", ["local", "molecule", "smc"])
def test_one_sweep_parity_with_walls(C, orc, order):
    w = _film((32, 32, 8), (synth.SpeciesSpec(3000, 32, 16), synth.SpeciesSpec(77, 16, 16)), 32)
    m, pos, sp, walls, mask, ext, inv_rho = _setup(C, w, 72)
    k0, a, A, _ = constants(w)
    omega = m.omega.cpu().numpy()
    np.testing.assert_array_equal(omega, orc.field_f32(orc.density_hist(pos, sp, w.grid), inv_rho,
                                                       np.float32(w.chi_n),
                                                       np.float32(w.kappa_n), ext, mask))
    if order == "molecule":
        m.set_scheme(C.SOMA_SCHEME_MOLECULE)
    m.sweep(1, C.SOMA_MOVE_SMC if order == "smc" else C.SOMA_MOVE_LOCAL)
    torch.cuda.synchronize()
    got = m.pos.cpu().numpy()
    off = base = bad = 0
    for s in sp:
        seg = pos[off:off + s.n_chains * s.n]
        if order == "molecule":
            orc.mc_sweep_molecule(seg, s, omega, w.grid, k0=k0, n_ref=w.n_ref, step=a,
                                  seed=w.seed, sweep=0, chain_base=base, forbid=mask, threads=8)
        else:
            orc.mc_sweep(seg, s, omega, w.grid, k0=k0, n_ref=w.n_ref,
                         move_kind=1 if order == "smc" else 0, step=A if order == "smc" else a,
                         seed=w.seed, sweep=0, chain_base=base, forbid=mask, threads=8)
        tol = 1e-5 * 6.0 if order == "smc" else 0.0
        bad += int(_bad_chains(got[off:off + s.n_chains * s.n], seg, s.n, tol).sum())
        off += s.n_chains * s.n
        base += s.n_chains
    allowed = math.ceil(1e-6 * w.n_beads)
    flush(order, "mismatched chains", bad, "allowed", allowed)
    assert bad <= allowed
    z = np.floor(got[:, 2].astype(np.float64)).astype(np.int64) % w.grid[2]
    assert ((z >= 1) & (z <= w.grid[2] - 2)).all()
    hist = m.counts_planes()
    np.testing.assert_array_equal(hist, orc.density_hist(got, sp, w.grid))
    m.close()


def test_mixed_sweep_parity_with_walls(C, orc):
    """One mixed sweep in a film with wall planes, learned moves of sigma ~ 0.6
    cells (walls matter), compared move by move with the oracle as in the
    learned parity test; no bead ends in a wall plane."""
    w = _film((24, 24, 8), (synth.SpeciesSpec(2048, 32, 16),), 16)
    m, pos, sp, walls, mask, ext, inv_rho = _setup(C, w, 73, p_learn=0.5)
    k0, a, A, _ = constants(w)
    omega = m.omega.cpu().numpy()
    params = proposal_test_params(orc, pos, sp[0], omega, w.grid, seed=14, sigma_bias=0.5)
    m.set_proposal(torch.from_numpy(params).cuda())
    m.sweep(1, C.SOMA_MOVE_MIXED)
    obs = m.observables()
    ref = pos.copy()
    amb = np.zeros(pos.shape[0], np.uint8)
    env = np.zeros(pos.shape[0], np.float32)
    acc, acc_l, bad, kinds, acc_flags = orc.mc_sweep_mixed(
        ref, sp[0], omega, w.grid, k0=k0, n_ref=w.n_ref, local_a=a, p_learn=0.5, params=params,
        **HEAD, bf16_mode=True, seed=w.seed, sweep=0, want_flags=True, threads=8, forbid=mask,
        ambiguous=amb, pos_env=env)
    got = m.pos.cpu().numpy()
    n_bad, unexplained, flagged, dec = explain_mismatches(got, pos, ref, acc_flags, amb, env, 32)
    allowed = math.ceil(1e-6 * pos.shape[0])
    flush("mixed with walls: accepted", acc / pos.shape[0], "mismatched", n_bad, "unexplained",
          unexplained, "allowed", allowed, "flagged", flagged, "accepted learned", obs.accepted[2],
          acc_l)
    assert obs.attempted[2] == int(kinds.sum())
    assert acc > 0.3 * pos.shape[0]
    assert unexplained <= allowed
    assert flagged <= 0.08 * sp[0].n_chains
    assert abs(int(obs.accepted[2]) - acc_l) <= int(amb[kinds == 1].sum())
    z = np.floor(got[:, 2].astype(np.float64)).astype(np.int64) % w.grid[2]
    assert ((z >= 1) & (z <= w.grid[2] - 2)).all()
    m.close()


def test_three_bead_boltzmann_with_walls_on_device(C):
    from paper_1711_03828_amd.melt import Melt
    L, n_chains = 4, 65536
    grid = (L, L, L)
    walls = synth.wall_cells(grid, [0])
    mask = synth.pack_mask(walls)
    omega = synth.uniform_field(31, L ** 3, -2.0, 2.0)
    pos = synth.film_walks(33, n_chains, 3, grid, 0.3, 1.0, 4.0)
    cfg = custom_config(grid, [Species(n_chains, 3, 2)], k0=3.0, n_ref=1, local_a=0.7, seed=97,
                        count_width=32)
    m = Melt(cfg, positions=torch.from_numpy(pos))
    m.set_external(None, torch.from_numpy(mask.view(np.int32)).cuda())
    m.omega.copy_(torch.from_numpy(omega))      # frozen field
    m.sync_fields()
    m.sweep(300, C.SOMA_MOVE_LOCAL)
    torch.cuda.synchronize()
    p = m.pos.cpu().numpy().astype(np.float64)
    cells = np.floor(p).astype(np.int64) % L
    lin = ((cells[:, 2] * L + cells[:, 1]) * L + cells[:, 0]).reshape(n_chains, 3)
    dist = references.three_bead_cell_distribution(omega[0], omega[1], 3.0, L)
    free = (~walls).astype(np.float64)
    dist = dist * free[:, None, None] * free[None, :, None] * free[None, None, :]
    dist /= dist.sum()
    marg = [dist.sum(axis=(1, 2)), dist.sum(axis=(0, 2)), dist.sum(axis=(0, 1))]
    for b in range(3):
        obs = np.bincount(lin[:, b], minlength=L ** 3)
        assert obs[walls].sum() == 0
        pval, stat, dof = references.chi2_pvalue(obs[~walls], marg[b][~walls])
        assert pval > 1e-4, (b, stat, dof)
    m.close()


def test_batched_cycles_equal_single_with_walls(C, orc):
    from paper_1711_03828_amd.melt import Batch
    ws = [_film((20, 20, 8), (synth.SpeciesSpec(900, 32, 16),), 16, "f0"),
          _film((28, 16, 10), (synth.SpeciesSpec(1100, 16, 8),), 16, "f1")]
    runs = []
    for batched in (False, True):
        melts, keep = [], []
        for i, w in enumerate(ws):
            m, *_ = _setup(C, w, 80 + i)
            melts.append(m)
        if batched:
            b = Batch(melts)
            b.cycle(4, C.SOMA_MOVE_LOCAL)
            b.close()
        else:
            for m in melts:
                m.cycle(4)
        torch.cuda.synchronize()
        runs.append([(m.pos.cpu().numpy(), m.omega.cpu().numpy()) for m in melts])
        for m in melts:
            m.close()
    for (p0, o0), (p1, o1) in zip(runs[0], runs[1]):
        np.testing.assert_array_equal(p0, p1)
        np.testing.assert_array_equal(o0, o1)


def test_small_film_cycles_and_in_plane_structure_factor(C, orc):
    """A lamella-forming film (N = 32 here, 8 x 8 Re0, thickness 1.2 Re0 between
    two wall planes), 200 SCMF cycles: no bead enters a wall, the kept
    histogram equals the recount of the positions, the fields equal the
    oracle's fields of those counts, and the in-plane S(q_par) from the device
    equals the oracle's transform of the same counts (its shell average too)."""
    from oracle import analysis as A
    w = _film((48, 48, 9), (synth.SpeciesSpec(4000, 32, 16),), 16, "small_film")
    m, pos, sp, walls, mask, ext, inv_rho = _setup(C, w, 90, ext_scale=0.0)
    m.set_external(None, torch.from_numpy(mask.view(np.int32)).cuda())
    m.cycle(200)
    torch.cuda.synchronize()
    got = m.pos.cpu().numpy()
    z = np.floor(got[:, 2].astype(np.float64)).astype(np.int64) % w.grid[2]
    assert ((z >= 1) & (z <= w.grid[2] - 2)).all()
    counts = orc.density_hist(got, sp, w.grid)
    np.testing.assert_array_equal(m.counts_planes(), counts)
    omega = orc.field_f32(counts, inv_rho, np.float32(w.chi_n), np.float32(w.kappa_n), None, mask)
    np.testing.assert_array_equal(m.omega.cpu().numpy(), omega)
    ws = torch.empty(C.soma_sq_workspace_bytes(m.handle), dtype=torch.uint8, device="cuda")
    sq = torch.empty(w.n_cells, dtype=torch.float64, device="cuda")
    C.soma_structure_factor(m.handle, ws.data_ptr(), ws.numel(), sq.data_ptr(),
                            torch.cuda.current_stream().cuda_stream)
    sq = sq.cpu().numpy()
    ref = A.structure_factor(counts, w.grid, w.n_ref, w.n_beads)
    np.testing.assert_allclose(sq[:48 * 48], ref[:48 * 48], rtol=1e-9, atol=1e-9 * ref.max())
    q1, m1, c1, p1 = C.soma_sq_plane_shells(sq, w.grid, 24)
    q2, m2, c2, p2 = A.sq_plane_shells(ref, w.grid, 24)
    np.testing.assert_array_equal(c1, c2)
    np.testing.assert_allclose(m1, m2, rtol=1e-8)
    assert p1 == p2
    flush("small film: S(q_par) peak shell", p1)
    m.close()
