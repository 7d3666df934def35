"""Pins of the oracle's n_t bead types (Sec. 2.1; Eqs. (5), (6), (8), (12)).

* two types: the n_t-type fields and H_nb equal the two-type ones (FP32 bit for
  bit, both interaction forms);
* closed values: an empty cell has omega_i = -kappaN for every type; a cell of
  pure type k at the reference density has omega_i = chi_ik N (K^1) or
  chi_ik N / 2 (K^0) for i != k and omega_k = 0 (K^1) or
  -sum_j chi_kj N / 2 (K^0);
* the field is the derivative of the grid Hamiltonian: omega_i(c) equals the
  central difference of H_nb in the count n_i(c) (exact for a quadratic);
* relabelling the types permutes the fields;
* moves: a 3-bead chain of types 0, 1, 2 in a frozen random field of three
  planes samples the exact Boltzmann distribution, and the histogram of an
  architecture fills the plane of each monomer's type.
"""
import numpy as np
import pytest

import synth
from oracle import references

CHI3 = np.array([[0.0, 20.0, 35.0], [20.0, 0.0, 12.5], [35.0, 12.5, 0.0]])


def _counts(n_t, n_cells, seed, hi=12):
    return np.random.default_rng(seed).integers(0, hi, size=(n_t, n_cells)).astype(np.uint32)


@pytest.mark.parametrize("form", [0, 1])
def test_two_types_equal_the_two_type_field(orc, form):
    counts = _counts(2, 500, 3)
    inv_rho, chi, kap = 27 / 128, 20.0, 50.0
    m32 = orc.field_multi_f32(counts, inv_rho, [[0, chi], [chi, 0]], kap, form=form)
    t32 = orc.field_f32(counts, inv_rho, chi, kap, form=form)
    assert np.array_equal(m32.view(np.uint32), t32.view(np.uint32))
    m64 = orc.field_multi_f64(counts, inv_rho, [[0, chi], [chi, 0]], kap, form=form)
    np.testing.assert_allclose(m64, orc.field_f64(counts, inv_rho, chi, kap, form=form),
                               rtol=1e-13, atol=1e-12)
    h_m = orc.h_nb_multi(counts, inv_rho, [[0, chi], [chi, 0]], kap, 32, form=form)
    h_2 = orc.h_nb(counts, inv_rho, chi, kap, 32, form=form)
    assert h_m == pytest.approx(h_2, rel=1e-13)


@pytest.mark.parametrize("form", [0, 1])
def test_closed_values(orc, form):
    n_t, rho, kap = 3, 8, 50.0
    counts = np.zeros((n_t, 4), np.uint32)
    for k in range(n_t):
        counts[k, 1 + k] = rho            # cell 1 + k: pure type k at the reference density
    for fn in (orc.field_multi_f64, orc.field_multi_f32):
        om = np.asarray(fn(counts, 1.0 / rho, CHI3, kap, form=form), np.float64)
        np.testing.assert_allclose(om[:, 0], -kap, rtol=1e-6)
        for k in range(n_t):
            for i in range(n_t):
                if i != k:
                    want = CHI3[i, k] if form == 1 else CHI3[i, k] / 2
                else:
                    want = 0.0 if form == 1 else -CHI3[k].sum() / 2
                assert om[i, 1 + k] == pytest.approx(want, rel=1e-6, abs=1e-5), (fn, i, k)


@pytest.mark.parametrize("form", [0, 1])
def test_field_is_the_derivative_of_h_nb(orc, form):
    n_t, n_ref = 4, 32
    chi = np.random.default_rng(5).uniform(0, 40, (n_t, n_t))
    chi = np.triu(chi, 1) + np.triu(chi, 1).T
    inv_rho, kap = 0.125, 30.0
    counts = _counts(n_t, 40, 7) + 1      # every count >= 1 so that n - 1 exists
    om = orc.field_multi_f64(counts, inv_rho, chi, kap, form=form)
    for c in range(0, 40, 7):
        cell = np.ascontiguousarray(counts[:, c:c + 1])
        for i in range(n_t):
            up, dn = cell.copy(), cell.copy()
            up[i] += 1
            dn[i] -= 1
            d = (orc.h_nb_multi(up, inv_rho, chi, kap, n_ref, form=form)
                 - orc.h_nb_multi(dn, inv_rho, chi, kap, n_ref, form=form)) * n_ref / 2
            assert om[i, c] == pytest.approx(d, rel=1e-10, abs=1e-9), (c, i)


def test_relabelling_permutes_the_fields(orc):
    counts = _counts(3, 300, 9)
    perm = [2, 0, 1]
    for form in (0, 1):
        a = orc.field_multi_f32(counts, 0.2, CHI3, 40.0, form=form)
        b = orc.field_multi_f32(np.ascontiguousarray(counts[perm]), 0.2,
                                np.ascontiguousarray(CHI3[np.ix_(perm, perm)]), 40.0, form=form)
        np.testing.assert_allclose(b, a[perm], rtol=1e-6, atol=1e-5)


def test_histogram_fills_the_type_planes(orc):
    n, bonds = 7, [(i, i + 1) for i in range(6)]
    types = [0, 0, 1, 1, 2, 2, 3]
    words = synth.encode_architecture(n, types, bonds)
    grid = (6, 5, 4)
    pos = synth.tree_walks(3, 50, n, bonds, grid, 0.6)
    h = orc.density_hist_arch(pos, 50, words, grid, n_types=4)
    cells = np.floor(pos.astype(np.float64)).astype(np.int64) % np.array(grid)
    lin = (cells[:, 2] * grid[1] + cells[:, 1]) * grid[0] + cells[:, 0]
    t = np.tile(np.array(types), 50)
    for k in range(4):
        assert np.array_equal(h[k], np.bincount(lin[t == k], minlength=120))
    with pytest.raises(ValueError):       # a type without a plane
        orc.density_hist_arch(pos, 50, words, grid, n_types=3)


def test_three_types_three_bead_boltzmann(orc):
    L, k0 = 4, np.float32(3.0)
    grid = (L, L, L)
    n_chains = 65536
    n, bonds = 3, [(0, 1), (1, 2)]
    words = synth.encode_architecture(n, [0, 1, 2], bonds)
    omega = np.random.default_rng(37).uniform(-2.0, 2.0, (3, L ** 3)).astype(np.float32)
    pos = synth.tree_walks(38, n_chains, n, bonds, grid, 0.6)
    for sweep in range(300):
        orc.mc_sweep_arch(pos, n_chains, words, omega, grid, k0=k0, n_ref=1,
                          step=np.float32(0.7), seed=39, sweep=sweep, threads=8)
    cells = np.floor(pos.astype(np.float64)).astype(np.int64) % L
    lin = ((cells[:, 2] * L + cells[:, 1]) * L + cells[:, 0]).reshape(n_chains, 3)
    p = references.three_bead_cell_distribution(omega[0], omega[1], float(k0), L,
                                                types=(0, 1, 2), omega_c=omega[2])
    marg = [p.sum(axis=(1, 2)), p.sum(axis=(0, 2)), p.sum(axis=(0, 1))]
    for b in range(3):
        pval, stat, dof = references.chi2_pvalue(np.bincount(lin[:, b], minlength=L ** 3),
                                                 marg[b])
        assert pval > 1e-4, (b, stat, dof)
    obs = np.bincount(lin[:, 0] * L ** 3 + lin[:, 2], minlength=L ** 6)
    pval, stat, dof = references.chi2_pvalue(obs, p.sum(axis=1).ravel())
    assert pval > 1e-4, (stat, dof)
    # bead 2 sampled with the type-1 field instead is rejected
    wrong = references.three_bead_cell_distribution(omega[0], omega[1], float(k0), L,
                                                    types=(0, 1, 1))
    pval, _, _ = references.chi2_pvalue(np.bincount(lin[:, 2], minlength=L ** 3),
                                        wrong.sum(axis=(0, 1)))
    assert pval < 1e-6
