"""Pins of the oracle's density histogram (Eq. (4)) and field (Eq. (12), K^1 form).

* cell assignment: hand-computed cells for points on and around cell faces,
  box faces and negative, unwrapped coordinates;
* exact bead-count conservation and independence of the bead order;
* fields: closed values for an empty cell, a pure cell and a balanced cell,
  and omega = N * dH_nb/dn, i.e. the field is the derivative of the grid
  Hamiltonian of Eqs. (5), (6), (8) (a central difference, exact for a
  quadratic), which ties two independently written oracle functions together;
* field energy of the beads (Eq. (13) divided by N): a hand-worked case (cells
  worked out by hand, including wrapped coordinates; the other field plane and
  another type boundary give other values), constant fields (n_A alpha +
  n_B beta)/N, and agreement with the histogram times the field.
"""
import numpy as np
import pytest

import synth
from oracle import Species

# (coordinate, cells along the axis, expected cell index) -- worked by hand
AXIS_CASES = [
    (0.0, 24, 0), (0.5, 24, 0), (1.0, 24, 1), (-0.0, 24, 0), (-0.5, 24, 23),
    (-1.0, 24, 23), (-1.0000001, 24, 22), (24.0, 24, 0), (23.999998, 24, 23),
    (24.25, 24, 0), (-24.0, 24, 0), (-24.5, 24, 23), (49.0, 24, 1), (7.0, 7, 0),
    (-7.5, 7, 6), (13.9, 7, 6), (1000.5, 7, 6), (-1000.5, 7, 0), (3.0, 1, 0), (-3.5, 1, 0),
]


def _single_bead_cell(orc, r, grid):
    pos = np.asarray([r], np.float32)
    counts = orc.density_hist(pos, [Species(1, 1, 1)], grid)
    assert counts.sum() == 1 and counts[1].sum() == 0
    return int(np.flatnonzero(counts[0])[0])


@pytest.mark.parametrize("x,n,cell", AXIS_CASES)
def test_cell_assignment_each_axis(orc, x, n, cell):
    for axis in range(3):
        grid = [5, 6, 3]
        grid[axis] = n
        r = [0.25, 0.25, 0.25]
        r[axis] = x
        lin = _single_bead_cell(orc, r, tuple(grid))
        nx, ny, _ = grid
        got = [lin % nx, (lin // nx) % ny, lin // (nx * ny)][axis]
        assert got == cell, (axis, x, n)


def test_linear_index_order(orc):
    grid = (5, 6, 3)
    # x fastest, then y, then z
    assert _single_bead_cell(orc, (1.5, 0.5, 0.5), grid) == 1
    assert _single_bead_cell(orc, (0.5, 1.5, 0.5), grid) == 5
    assert _single_bead_cell(orc, (0.5, 0.5, 1.5), grid) == 30
    assert _single_bead_cell(orc, (4.5, 5.5, 2.5), grid) == 89


def test_conservation_and_order_independence(orc):
    grid = (11, 7, 9)
    sp = [Species(37, 32, 16), Species(5, 16, 16), Species(3, 17, 0)]
    n_beads = sum(s.n_chains * s.n for s in sp)
    pos = synth.gaussian_walks(5, 1, n_beads, grid, 1.1).reshape(-1, 3)  # one long walk, cut
    counts = orc.density_hist(pos, sp, grid)
    n_a = sum(s.n_chains * s.n_a for s in sp)
    assert int(counts[0].sum()) == n_a and int(counts[1].sum()) == n_beads - n_a
    # any permutation of whole chains of one species leaves the histogram unchanged
    first = pos[:37 * 32].reshape(37, 32, 3)[np.random.default_rng(0).permutation(37)]
    pos2 = np.concatenate([first.reshape(-1, 3), pos[37 * 32:]])
    np.testing.assert_array_equal(orc.density_hist(pos2, sp, grid), counts)


def test_boundary_positions_conserved(orc):
    grid = (24, 10, 7)
    pos = synth.boundary_positions(grid)
    counts = orc.density_hist(pos, [Species(pos.shape[0], 1, 1)], grid)
    assert int(counts.sum()) == pos.shape[0]


def test_field_closed_values(orc):
    chi, kappa = 30.0, 50.0
    inv_rho = 27.0 / 64.0            # rho0 dL^3 = 64/27 beads per cell
    counts = np.zeros((2, 4), np.uint32)
    # cell 0 empty; cell 1 pure A at phi_A = 1 (n = rho = 64/27 is not an integer,
    # so take inv_rho = 1/2 in a second call for it); cell 2 balanced n_A = n_B
    counts[:, 2] = [3, 3]
    counts[:, 3] = [7, 0]
    om = orc.field_f64(counts, inv_rho, chi, kappa)
    assert om[0, 0] == -kappa and om[1, 0] == -kappa
    phi = 3 * inv_rho
    assert om[0, 2] == pytest.approx(kappa * (2 * phi - 1) + chi * phi, rel=1e-15)
    assert om[0, 2] == om[1, 2]
    om_half = orc.field_f64(np.array([[2, 1], [0, 1]], np.uint32), 0.5, chi, kappa)
    assert om_half[0, 0] == pytest.approx(0.0, abs=1e-12)      # pure A at phi_A = 1
    assert om_half[1, 0] == pytest.approx(chi, rel=1e-15)      # B bead in pure A
    assert om_half[0, 1] == pytest.approx(chi / 2, rel=1e-15)  # balanced at phi = 1
    assert om_half[1, 1] == pytest.approx(chi / 2, rel=1e-15)


def test_field_is_derivative_of_grid_hamiltonian(orc):
    g = np.random.default_rng(7)
    n_cells = 50
    counts = g.integers(1, 12, size=(2, n_cells)).astype(np.uint32)
    inv_rho, chi, kappa, n_ref = 0.21, 17.0, 45.0, 32
    om = orc.field_f64(counts, inv_rho, chi, kappa)
    for t in range(2):
        for c in g.choice(n_cells, 10, replace=False):
            up = counts.copy(); up[t, c] += 1
            dn = counts.copy(); dn[t, c] -= 1
            d = (orc.h_nb(up, inv_rho, chi, kappa, n_ref)
                 - orc.h_nb(dn, inv_rho, chi, kappa, n_ref)) / 2.0
            assert n_ref * d == pytest.approx(om[t, c], rel=1e-9, abs=1e-9)


def test_field_fp32_close_to_fp64(orc):
    g = np.random.default_rng(8)
    counts = g.integers(0, 30, size=(2, 1000)).astype(np.uint32)
    a = orc.field_f64(counts, 27.0 / 128.0, 20.0, 50.0)
    b = orc.field_f32(counts, 27.0 / 128.0, 20.0, 50.0)
    np.testing.assert_allclose(b, a, rtol=0, atol=5e-5 * np.abs(a).max())


def test_k0_field_closed_values(orc):
    """The K^0 interaction (Eq. (6), first form): an empty cell -kappaN, a pure A
    cell at the reference density -chiN/2 for A and +chiN/2 for B, a balanced
    cell 0 for both; FP64 and the FP32 order."""
    counts = np.array([[0, 10, 0, 5], [0, 0, 10, 5]], np.uint32)
    inv_rho, chi, kap = 0.1, 24.0, 50.0
    exp = np.array([[-kap, -chi / 2, chi / 2, 0.0], [-kap, chi / 2, -chi / 2, 0.0]])
    np.testing.assert_allclose(orc.field_f64(counts, inv_rho, chi, kap, form=0), exp, atol=1e-12)
    np.testing.assert_allclose(orc.field_f32(counts, np.float32(inv_rho), chi, kap, form=0), exp,
                               atol=1e-5)


def test_k0_field_is_derivative_of_grid_hamiltonian(orc):
    g = np.random.default_rng(17)
    n_cells = 50
    counts = g.integers(1, 12, size=(2, n_cells)).astype(np.uint32)
    inv_rho, chi, kappa, n_ref = 0.21, 17.0, 45.0, 32
    om = orc.field_f64(counts, inv_rho, chi, kappa, form=0)
    for t in range(2):
        for c in g.choice(n_cells, 10, replace=False):
            up = counts.copy(); up[t, c] += 1
            dn = counts.copy(); dn[t, c] -= 1
            d = (orc.h_nb(up, inv_rho, chi, kappa, n_ref, form=0)
                 - orc.h_nb(dn, inv_rho, chi, kappa, n_ref, form=0)) / 2.0
            assert n_ref * d == pytest.approx(om[t, c], rel=1e-9, abs=1e-9)
    # the two forms differ by -chiN/4 (phi_A + phi_B)^2 per cell (a total-density term)
    h1 = orc.h_nb(counts, inv_rho, chi, kappa, n_ref, form=1)
    h0 = orc.h_nb(counts, inv_rho, chi, kappa, n_ref, form=0)
    tot = (counts.sum(axis=0) * inv_rho) ** 2
    assert h0 - h1 == pytest.approx(-chi / 4 * tot.sum() / (inv_rho * n_ref), rel=1e-9)


# ----------------------------------------------------------------------------
# Field energy of the beads in their cells (the right-hand side of Eq. (13)
# divided by N): closed values.
# ----------------------------------------------------------------------------
def test_field_energy_hand_worked(orc):
    """Six beads in hand-computed cells of a 4 x 3 x 2 grid (x fastest), fields
    omega_A(c) = c + 1/2 and omega_B(c) = 100 + 2c, species A2B1 (types A A B),
    reference N = 4.  Cells, worked by hand (floor, then periodic wrap):
      chain 0: ( 0.5,  0.5,  0.5) -> (0,0,0) = 0,  A:   0.5
               ( 1.5,  2.5,  0.5) -> (1,2,0) = 9,  A:   9.5
               (-0.5,  0.5,  1.5) -> (3,0,1) = 15, B: 130
      chain 1: (4.25,  3.5,  2.5) -> (0,0,0) = 0,  A:   0.5
               (3.75, -0.25,-0.75) -> (3,2,1) = 23, A:  23.5
               ( 2.0,  1.0,  1.0) -> (2,1,1) = 18, B: 136
    sum 300, energy 300 / 4 = 75."""
    grid = (4, 3, 2)
    c = np.arange(24, dtype=np.float32)
    omega = np.stack([c + 0.5, 100 + 2 * c]).astype(np.float32)
    pos = np.array([[0.5, 0.5, 0.5], [1.5, 2.5, 0.5], [-0.5, 0.5, 1.5],
                    [4.25, 3.5, 2.5], [3.75, -0.25, -0.75], [2.0, 1.0, 1.0]], np.float32)
    assert orc.field_energy(pos, Species(2, 3, 2), omega, grid, 4) == 75.0
    # the other plane for every bead: A beads read 100 + 2c, B beads c + 1/2,
    # (100 + 118 + 15.5 + 100 + 146 + 18.5) / 4
    swapped = omega[::-1].copy()
    assert orc.field_energy(pos, Species(2, 3, 2), swapped, grid, 4) == pytest.approx(498.0 / 4)
    # all beads of type A (n_a = 3): the third beads read omega_A (15.5 and 18.5)
    assert orc.field_energy(pos, Species(2, 3, 3), omega, grid, 4) == pytest.approx(
        (0.5 + 9.5 + 15.5 + 0.5 + 23.5 + 18.5) / 4)


def test_field_energy_constant_fields(orc):
    """Constant fields omega_A = alpha, omega_B = beta: the energy is
    (n_A alpha + n_B beta) / N whatever the positions."""
    grid = (7, 5, 6)
    n_cells = 7 * 5 * 6
    sp = Species(37, 32, 11)
    pos = synth.gaussian_walks(12, 37, 32, grid, 1.1)
    omega = np.stack([np.full(n_cells, 1.25), np.full(n_cells, -3.5)]).astype(np.float32)
    e = orc.field_energy(pos, sp, omega, grid, 32)
    assert e == pytest.approx(37 * (11 * 1.25 + 21 * -3.5) / 32, rel=1e-14)


def test_field_energy_equals_counts_times_field(orc):
    """The sum over beads equals sum_c sum_t n_t(c) omega_t(c) / N with the
    (independently pinned) histogram of the same positions."""
    grid = (9, 8, 7)
    sp = Species(50, 17, 6)
    pos = synth.gaussian_walks(13, 50, 17, grid, 1.3)
    omega = synth.uniform_field(14, 9 * 8 * 7, -3.0, 3.0)
    counts = orc.density_hist(pos, [sp], grid).astype(np.float64)
    exp = float((counts * omega.astype(np.float64)).sum()) / 17
    assert orc.field_energy(pos, sp, omega, grid, 17) == pytest.approx(exp, rel=1e-12)
