"""Pins of the oracle's external fields (Sec. 4): a per-type external energy
added to the interaction field, and impenetrable cells.

* fields: closed values with the external term (an empty cell -kappaN + e, a
  balanced cell at the reference density chiN/2 + e) in FP64 and in the FP32
  order; impenetrable cells carry the field 0;
* H_nb leaves impenetrable cells out: a film of balanced cells at the
  reference density of its free cells has H_nb = rho0 dL^3/N * n_free chiN/4;
* moves: with impenetrable planes, no bead starting outside them ever enters
  them (local, smart-MC and molecule-order moves), and the 3-bead chain in a
  frozen random field samples the exact Boltzmann distribution restricted to
  the free cells (the unrestricted distribution is rejected);
* no smart-MC, bond-Gibbs or learned step jumps over a wall of one cell plane
  (with walls set, trials more than one cell away along an axis are rejected),
  while the same moves without walls do make such steps.
"""
import math

import numpy as np
import pytest

import synth
from oracle import MOVE_GIBBS, MOVE_LOCAL, MOVE_SMC, Species, references


def test_field_closed_values_with_external_term(orc):
    n_cells = 6
    counts = np.zeros((2, n_cells), np.uint32)
    counts[:, 1] = [5, 5]                 # balanced at rho = 10 per cell
    counts[:, 2] = [10, 0]                # pure A
    counts[:, 3] = [0, 10]                # pure B
    counts[:, 4] = [5, 5]                 # balanced, but impenetrable
    inv_rho, chi, kap = 0.1, 20.0, 50.0
    ext = np.array([[0.5, -1.25, 2.0, 0.0, 7.0, 3.0], [-0.5, 0.75, 0.0, -2.0, 7.0, 3.0]],
                   np.float32)
    forbid = synth.pack_mask(np.array([0, 0, 0, 0, 1, 0], bool))
    exp = np.array([[-kap + 0.5, chi / 2 - 1.25, 0.0 + 2.0, chi + 0.0, 0.0, -kap + 3.0],
                    [-kap - 0.5, chi / 2 + 0.75, chi + 0.0, 0.0 - 2.0, 0.0, -kap + 3.0]])
    np.testing.assert_allclose(orc.field_f64(counts, inv_rho, chi, kap, ext, forbid), exp,
                               rtol=0, atol=1e-12)
    np.testing.assert_allclose(orc.field_f32(counts, np.float32(inv_rho), chi, kap, ext, forbid),
                               exp, rtol=0, atol=1e-5)
    # without the extras the same counts give the plain closed values
    plain = orc.field_f64(counts, inv_rho, chi, kap)
    assert plain[0, 0] == -kap and plain[0, 4] == pytest.approx(chi / 2)


def test_h_nb_skips_impenetrable_cells(orc):
    nx = ny = 4
    nz = 5
    n_cells = nx * ny * nz
    walls = synth.wall_cells((nx, ny, nz), [0])
    n_free = int((~walls).sum())
    counts = np.zeros((2, n_cells), np.uint32)
    counts[:, ~walls] = 3                 # balanced free cells at rho = 6
    n_beads = int(counts.sum())
    inv_rho = n_free / n_beads
    chi, kap, n_ref = 10.0, 40.0, 32
    h = orc.h_nb(counts, inv_rho, chi, kap, n_ref, synth.pack_mask(walls))
    rho = n_beads / n_free
    assert h == pytest.approx(rho / n_ref * n_free * chi / 4, rel=1e-12)
    # counting the walls as empty cells would add kappaN/2 per wall cell
    h_all = orc.h_nb(counts, inv_rho, chi, kap, n_ref)
    assert h_all == pytest.approx(h + rho / n_ref * (n_cells - n_free) * kap / 2, rel=1e-12)


@pytest.mark.parametrize("order", ["local", "smc", "molecule"])
def test_no_bead_enters_impenetrable_cells(orc, order):
    grid = (12, 12, 8)
    n, n_chains = 16, 400
    walls = synth.wall_cells(grid, [0, 7])
    mask = synth.pack_mask(walls)
    pos = synth.film_walks(5, n_chains, n, grid, 0.6, 1.0, 7.0)
    omega = synth.uniform_field(6, 12 * 12 * 8, -2, 2)
    sp = Species(n_chains, n, 8)
    for sweep in range(30):
        if order == "molecule":
            orc.mc_sweep_molecule(pos, sp, omega, grid, k0=2.0, n_ref=16, step=0.9, seed=3,
                                  sweep=sweep, forbid=mask, threads=4)
        else:
            orc.mc_sweep(pos, sp, omega, grid, k0=2.0, n_ref=16,
                         move_kind=MOVE_LOCAL if order == "local" else MOVE_SMC,
                         step=0.9 if order == "local" else 0.3, seed=3, sweep=sweep,
                         forbid=mask, threads=4)
    z = np.floor(pos[:, 2].astype(np.float64)).astype(np.int64) % 8
    assert ((z >= 1) & (z <= 6)).all()
    # and without the mask the same run does enter them
    pos2 = synth.film_walks(5, n_chains, n, grid, 0.6, 1.0, 7.0)
    for sweep in range(30):
        orc.mc_sweep(pos2, sp, omega, grid, k0=2.0, n_ref=16, step=0.9, seed=3, sweep=sweep,
                     threads=4)
    z2 = np.floor(pos2[:, 2].astype(np.float64)).astype(np.int64) % 8
    assert ((z2 == 0) | (z2 == 7)).any()


@pytest.mark.parametrize("order,step", [("local", 0.7), ("smc", 0.12), ("molecule", 0.7)])
def test_three_bead_boltzmann_with_walls(orc, order, step):
    L, k0 = 4, np.float32(3.0)
    grid = (L, L, L)
    n_chains = 65536
    walls = synth.wall_cells(grid, [0])
    mask = synth.pack_mask(walls)
    omega = synth.uniform_field(31, L ** 3, -2.0, 2.0)
    pos = synth.film_walks(32, n_chains, 3, grid, 0.3, 1.0, 4.0)
    sp = Species(n_chains, 3, 2)
    for sweep in range(300):
        if order == "molecule":
            orc.mc_sweep_molecule(pos, sp, omega, grid, k0=k0, n_ref=1, step=np.float32(step),
                                  seed=79, sweep=sweep, forbid=mask, threads=8)
        else:
            orc.mc_sweep(pos, sp, omega, grid, k0=k0, n_ref=1,
                         move_kind=MOVE_LOCAL if order != "smc" else MOVE_SMC,
                         step=np.float32(step), seed=79, sweep=sweep, forbid=mask, threads=8)
    cells = np.floor(pos.astype(np.float64)).astype(np.int64) % L
    lin = ((cells[:, 2] * L + cells[:, 1]) * L + cells[:, 0]).reshape(n_chains, 3)
    p = references.three_bead_cell_distribution(omega[0], omega[1], float(k0), L)
    free = (~walls).astype(np.float64)
    p_w = p * free[:, None, None] * free[None, :, None] * free[None, None, :]
    p_w /= p_w.sum()
    marg = [p_w.sum(axis=(1, 2)), p_w.sum(axis=(0, 2)), p_w.sum(axis=(0, 1))]
    for b in range(3):
        obs = np.bincount(lin[:, b], minlength=L ** 3)
        assert obs[walls].sum() == 0
        keep = ~walls
        pval, stat, dof = references.chi2_pvalue(obs[keep], marg[b][keep])
        assert pval > 1e-4, (b, stat, dof)
    obs = np.bincount(lin[:, 0] * L ** 3 + lin[:, 2], minlength=L ** 6)
    joint = p_w.sum(axis=1).ravel()
    keep = joint > 0
    pval, stat, dof = references.chi2_pvalue(obs[keep], joint[keep])
    assert pval > 1e-4, (stat, dof)
    # the unrestricted distribution (renormalised on the free cells of bead 1) is rejected
    m_free = p.sum(axis=(0, 2)) * free
    m_free /= m_free.sum()
    obs1 = np.bincount(lin[:, 1], minlength=L ** 3)
    pval, _, _ = references.chi2_pvalue(obs1[~walls], m_free[~walls])
    assert pval < 1e-6


def _big_step_params():
    """Network weights whose proposal width is about 1.6 cells (log sigma near
    0.46 with the head used below): far enough to jump a one-plane wall."""
    params = synth.mlp_params(9, out_gain=0.1)
    b3 = synth.MLP_LAYOUT["b3"]
    params[b3 + 3:b3 + 6] = 3.0
    return params


WIDE_HEAD = dict(m_max=1.0, lo=math.log(0.02), hi=math.log(2.0))


def _sweep_kind(orc, kind, pos, sp, omega, grid, sweep, mask):
    if kind == "mixed":
        orc.mc_sweep_mixed(pos, sp, omega, grid, k0=0.5, n_ref=16, local_a=0.5, p_learn=1.0,
                           params=_big_step_params(), **WIDE_HEAD, seed=4, sweep=sweep,
                           forbid=mask, threads=4)
    else:
        orc.mc_sweep(pos, sp, omega, grid, k0=0.5, n_ref=16,
                     move_kind=MOVE_SMC if kind == "smc" else MOVE_GIBBS, step=0.5, seed=4,
                     sweep=sweep, forbid=mask, threads=4)


@pytest.mark.parametrize("kind", ["smc", "gibbs", "mixed"])
def test_no_move_jumps_a_wall(orc, kind):
    """Smart-MC (A = 0.5), bond-Gibbs (k0 = 0.5: width 1 cell) and learned moves
    (width about 1.6 cells) next to a wall of a single cell plane (z = 0, nz = 6,
    periodic): with the walls set, no trial more than one cell away along an axis
    is taken, so every unwrapped z stays inside the free slab [1, 6).  Without
    the walls the same moves do make such steps (the test has power)."""
    grid = (10, 10, 6)
    n, n_chains = 8, 300
    walls = synth.wall_cells(grid, [0])
    mask = synth.pack_mask(walls)
    omega = synth.uniform_field(6, 10 * 10 * 6, -1, 1)
    sp = Species(n_chains, n, 4)
    pos = synth.film_walks(8, n_chains, n, grid, 0.5, 1.0, 6.0)
    assert ((pos[:, 2] >= 1.0) & (pos[:, 2] < 6.0)).all()
    for sweep in range(20):
        _sweep_kind(orc, kind, pos, sp, omega, grid, sweep, mask)
        z = pos[:, 2].astype(np.float64)
        assert ((z >= 1.0) & (z < 6.0)).all(), sweep
    free = pos.copy()
    jumps = 0
    for sweep in range(5):
        before = np.floor(free.astype(np.float64))
        _sweep_kind(orc, kind, free, sp, omega, grid, sweep, None)
        jumps += int((np.abs(np.floor(free.astype(np.float64)) - before) > 1).any(axis=1).sum())
    assert jumps > 0
