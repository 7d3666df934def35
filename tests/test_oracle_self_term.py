"""The self term of cell-changing moves, pinned to the grid Hamiltonian.

Moving one bead of type t from cell c to c' changes H_nb (Eqs. (5), (6), (8),
quadratic in the counts) by exactly (omega_t(c') - omega_t(c))/N + s with s
the second difference kappaN/(N rho) (K^1) or (kappaN - chiN/2)/(N rho) (K^0);
H_nb and omega = N dH/dn are pinned in test_oracle_hist_field.  And a lone
bead in a zero field with a local move of half-width a < 1 is accepted with
probability (1 - a/2)^3 + (1 - (1 - a/2)^3) exp(-s): staying in the cell
costs nothing, each axis is crossed with probability a/2.
"""
import math

import numpy as np
import pytest

from oracle import Species


@pytest.mark.parametrize("form", [1, 0])
def test_self_term_is_the_exact_single_bead_change(orc, form):
    g = np.random.default_rng(11 + form)
    n_cells, n_ref, chi_n, kappa_n = 300, 32, 17.0, 45.0
    counts = g.integers(0, 12, size=(2, n_cells)).astype(np.uint32)
    inv_rho = n_cells / float(counts.sum())
    omega = orc.field_f64(counts, inv_rho, chi_n, kappa_n, form=form)
    h0 = orc.h_nb(counts, inv_rho, chi_n, kappa_n, n_ref, form=form)
    s = (kappa_n - (0.5 * chi_n if form == 0 else 0.0)) * inv_rho / n_ref
    assert math.isclose(float(orc.self_energy(kappa_n, chi_n, inv_rho, n_ref, form)), s,
                        rel_tol=1e-7)
    for _ in range(200):
        t = int(g.integers(2))
        c = int(g.choice(np.flatnonzero(counts[t] > 0)))
        c2 = int(g.integers(n_cells))
        moved = counts.copy()
        moved[t, c] -= 1
        moved[t, c2] += 1
        dh = orc.h_nb(moved, inv_rho, chi_n, kappa_n, n_ref, form=form) - h0
        pred = (omega[t, c2] - omega[t, c]) / n_ref + (s if c2 != c else 0.0)
        assert abs(dh - pred) <= 1e-9 * (1.0 + abs(h0)), (t, c, c2, dh, pred)
    # the term is not optional: without it the change is missed by s exactly
    t, c = 0, int(np.flatnonzero(counts[0] > 0)[0])
    c2 = (c + 1) % n_cells
    moved = counts.copy()
    moved[t, c] -= 1
    moved[t, c2] += 1
    dh = orc.h_nb(moved, inv_rho, chi_n, kappa_n, n_ref, form=form) - h0
    assert abs(dh - (omega[t, c2] - omega[t, c]) / n_ref - s) < 1e-9 * (1.0 + abs(h0))
    assert abs(dh - (omega[t, c2] - omega[t, c]) / n_ref) > 0.5 * s


def test_lone_bead_acceptance_with_self_term(orc):
    grid = (8, 8, 8)
    n_chains = 20000
    sp = Species(n_chains, 1, 1)
    g = np.random.default_rng(3)
    a = np.float32(0.8)
    s = 0.7
    omega = np.zeros((2, 512), np.float32)
    acc_total = 0
    for sweep in range(5):
        pos = (g.random((n_chains, 3)) * 8).astype(np.float32)
        acc, _ = orc.mc_sweep(pos, sp, omega, grid, k0=1.0, n_ref=1, step=a, seed=5,
                              sweep=sweep, threads=8, self_term=s)
        acc_total += acc
    p_stay = (1.0 - float(a) / 2.0) ** 3
    expected = p_stay + (1.0 - p_stay) * math.exp(-s)
    n = 5 * n_chains
    rate = acc_total / n
    sigma = math.sqrt(expected * (1 - expected) / n)
    assert abs(rate - expected) < 5 * sigma, (rate, expected, sigma)
    # a planted wrong sign (exp(+s), capped at 1) would accept everything
    assert abs(rate - 1.0) > 20 * sigma
    # without the term every move is accepted
    pos = (g.random((n_chains, 3)) * 8).astype(np.float32)
    acc, _ = orc.mc_sweep(pos, sp, omega, grid, k0=1.0, n_ref=1, step=a, seed=5, sweep=9,
                          threads=8)
    assert acc == n_chains
