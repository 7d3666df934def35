"""Closed forms and brute-force references that pin the oracle.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

None of these reuse the oracle's code; each follows from the model of the
paper (arXiv:1711.03828, Sec. 2) by an independent route:

* ``ideal_chain_*``: with chiN = kappaN = 0 the model is a Gaussian chain with
  harmonic bonds (Eqs. (1)-(2)); bond vectors are i.i.d. N(0, 1/k0) per
  component and b0^2 = 3/k0 (Sec. 2.1, after Eq. (9)).
* ``ideal_local_acceptance``: for a Metropolis move of one bead of an ideal
  chain at equilibrium, the energy change is Gaussian with variance twice its
  mean, mu = k0 |d|^2 (middle bead) or k0 |d|^2 / 2 (end bead); averaging
  min(1, e^-dE) over that Gaussian gives erfc(sqrt(mu)/2), which is then
  averaged over the uniform trial displacement d in [-a,a]^3 by Gauss-Legendre
  quadrature.
* ``three_bead_cell_distribution``: the exact Boltzmann distribution of the
  cells of a 3-bead chain in a frozen periodic field (the stage-2 Hamiltonian
  of Sec. 2.2, Eq. (13), plus Eq. (2)), integrated over positions in closed
  form per Cartesian direction with error functions and Gauss-Legendre.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf, erfc


def ideal_chain_moments(n: int, k0: float):
    """<b^2> per bond, <Re^2>, <Rg^2> of an N-bead Gaussian chain, b0^2 = 3/k0."""
    b2 = 3.0 / k0
    return b2, (n - 1) * b2, b2 * (n * n - 1) / (6.0 * n)


def _gl(npts, lo, hi):
    x, w = np.polynomial.legendre.leggauss(npts)
    return 0.5 * (hi - lo) * x + 0.5 * (hi + lo), 0.5 * (hi - lo) * w


def ideal_local_acceptance(k0: float, a: float, npts: int = 48):
    """(A_middle, A_end) for uniform trial moves in [-a,a]^3 on an ideal chain."""
    x, w = _gl(npts, 0.0, a)          # the integrand is even in every component
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    W = w[:, None, None] * w[None, :, None] * w[None, None, :]
    s = X * X + Y * Y + Z * Z
    vol = a ** 3
    mid = float(np.sum(W * erfc(np.sqrt(k0 * s) / 2.0)) / vol)
    end = float(np.sum(W * erfc(np.sqrt(k0 * s / 8.0))) / vol)
    return mid, end


def ideal_local_acceptance_chain(n: int, k0: float, a: float):
    mid, end = ideal_local_acceptance(k0, a)
    return ((n - 2) * mid + 2 * end) / n


def _bond_cell_kernel(k0: float, L: int, npts: int = 64, images: int = 3):
    """I[i, j, k] = int_{x2 in [j,j+1)} G(i, x2) G(k, x2) dx2, where G(i, x2) is the
    integral of exp(-k0/2 (x1-x2)^2) over x1 in cell i and all its periodic images."""
    c = math.sqrt(k0 / 2.0)
    pref = math.sqrt(math.pi / (2.0 * k0))
    I = np.zeros((L, L, L))
    for j in range(L):
        x2, w2 = _gl(npts, j, j + 1.0)
        G = np.zeros((L, npts))
        for i in range(L):
            for m in range(-images, images + 1):
                lo = i + m * L
                G[i] += pref * (erf(c * (lo + 1 - x2)) - erf(c * (lo - x2)))
        I[:, j, :] = np.einsum("in,kn,n->ik", G, G, w2)
    return I


def three_bead_cell_distribution(omega_a: np.ndarray, omega_b: np.ndarray, k0: float,
                                 L: int, n_ref: int = 1, types=(0, 0, 1), omega_c=None):
    """Exact P(c1, c2, c3) for a 3-bead linear chain in an L^3 periodic box with a
    frozen field, as an array [L^3, L^3, L^3] over linear cell indices
    (z*L + y)*L + x.  omega_* are the fields of types 0, 1 (and 2) (bead energy
    omega/n_ref)."""
    I = _bond_cell_kernel(k0, L)
    idx = np.arange(L ** 3)
    cx, cy, cz = idx % L, (idx // L) % L, idx // (L * L)
    om = [np.asarray(omega_a, float), np.asarray(omega_b, float)]
    if omega_c is not None:
        om.append(np.asarray(omega_c, float))
    # positional weight, separable over x, y, z
    wpos = (I[cx[:, None, None], cx[None, :, None], cx[None, None, :]]
            * I[cy[:, None, None], cy[None, :, None], cy[None, None, :]]
            * I[cz[:, None, None], cz[None, :, None], cz[None, None, :]])
    e = (om[types[0]][:, None, None] + om[types[1]][None, :, None]
         + om[types[2]][None, None, :]) / n_ref
    p = wpos * np.exp(-(e - e.min()))
    return p / p.sum()


def chi2_pvalue(observed: np.ndarray, expected_prob: np.ndarray, min_expected=5.0):
    """Pearson chi-square p-value, pooling bins with small expectation."""
    from scipy.stats import chi2

    obs = np.asarray(observed, float).ravel()
    n = obs.sum()
    exp = np.asarray(expected_prob, float).ravel() * n
    order = np.argsort(exp)
    obs, exp = obs[order], exp[order]
    small = np.cumsum(exp) < min_expected * 4
    o = np.concatenate([[obs[small].sum()], obs[~small]]) if small.any() else obs
    e = np.concatenate([[exp[small].sum()], exp[~small]]) if small.any() else exp
    keep = e > 0
    stat = float(np.sum((o[keep] - e[keep]) ** 2 / e[keep]))
    dof = int(keep.sum()) - 1
    return float(chi2.sf(stat, dof)), stat, dof
