"""Pins of the oracle's initial configuration (Gaussian walks, Sec. 2.1).

* the bricked cell order is a bijection of [0, n_cells) onto the grid for
  divisible and ragged grids, and keeps bricks contiguous;
* stratified origins: chain g lands in a cell of rank in
  [floor(g n_cells / G), floor((g+1) n_cells / G)] and inside that cell;
* bond components are N(0, 1/k0) (KS test), origins of the i.i.d. mode are
  uniform (chi-square over cells).
"""
import math

import numpy as np
import pytest
from scipy.stats import kstest

from oracle import Species, references


@pytest.mark.parametrize("grid", [(24, 24, 24), (5, 7, 3), (17, 9, 12), (16, 8, 9), (1, 1, 1),
                                  (40, 3, 8)])
def test_brick_order_is_bijection(orc, grid):
    nx, ny, nz = grid
    n = nx * ny * nz
    cells = orc.brick_cell(np.arange(n, dtype=np.uint64), grid).astype(np.int64)
    assert (cells >= 0).all() and (cells < np.array(grid)).all()
    lin = (cells[:, 2] * ny + cells[:, 1]) * nx + cells[:, 0]
    assert np.array_equal(np.sort(lin), np.arange(n))


def test_brick_order_contiguous_bricks(orc):
    grid = (24, 16, 8)
    cells = orc.brick_cell(np.arange(24 * 16 * 8, dtype=np.uint64), grid).astype(np.int64)
    brick = cells // 8
    bid = (brick[:, 2] * 2 + brick[:, 1]) * 3 + brick[:, 0]
    # every run of 512 ranks is one whole brick, bricks row-major
    assert np.array_equal(bid, np.repeat(np.arange(6), 512))


def test_stratified_origins(orc):
    grid = (20, 12, 9)
    G = 997
    k0 = 3.0 * 31 / 36.0
    pos = orc.init_chains(Species(G, 32, 16), grid, bond_sigma=1 / math.sqrt(k0), seed=5,
                          origin_mode=1).reshape(G, 32, 3)
    n_cells = 20 * 12 * 9
    order = orc.brick_cell(np.arange(n_cells, dtype=np.uint64), grid).astype(np.int64)
    rank_of = np.empty(n_cells, np.int64)
    rank_of[(order[:, 2] * 12 + order[:, 1]) * 20 + order[:, 0]] = np.arange(n_cells)
    o = pos[:, 0, :].astype(np.float64)
    assert (o >= 0).all() and (o < np.array(grid)).all()
    c = np.floor(o).astype(np.int64)
    r = rank_of[(c[:, 2] * 12 + c[:, 1]) * 20 + c[:, 0]]
    g = np.arange(G)
    assert (r >= (g * n_cells) // G).all() and (r <= ((g + 1) * n_cells) // G).all()


def test_bonds_gaussian_and_origins_uniform(orc):
    grid = (6, 6, 6)
    n_chains, n = 20000, 16
    k0 = 2.5
    sigma = 1 / math.sqrt(k0)
    pos = orc.init_chains(Species(n_chains, n, 8), grid, bond_sigma=sigma, seed=6,
                          origin_mode=0).reshape(n_chains, n, 3).astype(np.float64)
    bonds = np.diff(pos, axis=1).reshape(-1, 3)
    for d in range(3):
        assert kstest(bonds[:, d] / sigma, "norm").pvalue > 1e-4
    c = np.floor(pos[:, 0, :]).astype(np.int64)
    lin = (c[:, 2] * 6 + c[:, 1]) * 6 + c[:, 0]
    pval, _, _ = references.chi2_pvalue(np.bincount(lin, minlength=216), np.full(216, 1 / 216))
    assert pval > 1e-4
    # an ideal chain from the start
    re2 = ((pos[:, -1] - pos[:, 0]) ** 2).sum(1)
    assert abs(re2.mean() - 3 * (n - 1) / k0) < 4 * re2.std() / math.sqrt(n_chains)
