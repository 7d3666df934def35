"""Oracle analysis quantities -- TEST INFRASTRUCTURE ONLY (see ``oracle``).

* Structure factor of the composition field (Sec. 5.6, the equation for
  S(q, t)): S(q) = N^2 rho0 / (4 V) |F[phi_A - phi_B](q)|^2, F the grid Fourier
  transform dL^3 sum_c (.) exp(-i q.r_c) on the reciprocal lattice
  q = 2 pi m / L.  Reading: rho0 is the bead number density (Sec. 2.1, after
  the density-operator equation), N the reference chain length, grid units
  (dL = 1).  Written out with phi = n/(rho0 dL^3):
  S(q) = N^2 |sum_c (n_A - n_B)(c) exp(-i q.r_c)|^2 / (4 n_beads).
  The transform is numpy's FFT (a library primitive).
* Shell average: shell k = round(|q| / dq), dq = 2 pi / L_min; the peak is the
  shell k >= 1 of largest mean (the paper reads the lamellar period off the
  primary peak of the radially averaged S(q)).
* Integrated autocorrelation time by Sokal's automatic window (c = 5).
"""
from __future__ import annotations

import numpy as np


def structure_factor(counts: np.ndarray, grid, n_ref: int, n_beads: int) -> np.ndarray:
    """counts uint [2, n_cells] (cell order (z*ny + y)*nx + x) -> S [n_cells] in the
    same order (index m of the lattice vector per axis)."""
    nx, ny, nz = (int(v) for v in grid)
    psi = (counts[0].astype(np.float64) - counts[1].astype(np.float64)).reshape(nz, ny, nx)
    g = np.fft.fftn(psi)
    return (float(n_ref) ** 2 / (4.0 * n_beads) * np.abs(g) ** 2).reshape(-1)


def lattice_q(grid) -> np.ndarray:
    """|q| of every lattice vector, cell order."""
    nx, ny, nz = (int(v) for v in grid)
    fx = np.fft.fftfreq(nx)
    fy = np.fft.fftfreq(ny)
    fz = np.fft.fftfreq(nz)
    # fftfreq puts the Nyquist index of an even length at -1/2; |q| is the same
    q2 = fz[:, None, None] ** 2 + fy[None, :, None] ** 2 + fx[None, None, :] ** 2
    return (2.0 * np.pi * np.sqrt(q2)).reshape(-1)


def sq_shells(sq: np.ndarray, grid, n_shells: int, l_min=None):
    """(q_mid, mean, count, peak) of the shell average."""
    dq = 2.0 * np.pi / (min(int(v) for v in grid) if l_min is None else l_min)
    k = np.floor(lattice_q(grid) / dq + 0.5).astype(np.int64)
    keep = k < n_shells
    cnt = np.bincount(k[keep], minlength=n_shells)[:n_shells]
    tot = np.bincount(k[keep], weights=sq[keep], minlength=n_shells)[:n_shells]
    mean = np.where(cnt > 0, tot / np.maximum(cnt, 1), 0.0)
    cand = [j for j in range(1, n_shells) if cnt[j] > 0]
    peak = max(cand, key=lambda j: (mean[j], -j)) if cand else 0
    return dq * np.arange(n_shells), mean, cnt, peak


def sq_plane_shells(sq: np.ndarray, grid, n_shells: int):
    """In-plane structure factor of a film (Sec. 5.6, S(q_par)): the m_z = 0 plane
    of the 3-D S(q) (the transform of the composition summed over z), averaged
    over shells of |q_par| of width 2 pi / min(nx, ny).  (q_mid, mean, count, peak)."""
    nx, ny = int(grid[0]), int(grid[1])
    return sq_shells(np.asarray(sq).ravel()[:nx * ny], (nx, ny, 1), n_shells,
                     l_min=min(nx, ny))


def autocorrelation(x: np.ndarray) -> np.ndarray:
    """Normalised autocorrelation rho(t) of a series [T] or of independent
    series [T, m] (averaged over the columns), by direct sums."""
    x = np.asarray(x, np.float64)
    if x.ndim == 1:
        x = x[:, None]
    x = x - x.mean(axis=0)
    T = x.shape[0]
    c = np.array([np.mean(np.sum(x[:T - t] * x[t:], axis=0) / (T - t)) for t in range(T)])
    return c / c[0]


def tau_int(x: np.ndarray, c: float = 5.0):
    """Integrated autocorrelation time tau = 1/2 + sum_{t=1}^{M} rho(t) with the
    smallest window M >= c tau(M) (Sokal).  Returns (tau, M)."""
    rho = autocorrelation(x)
    tau = 0.5
    for m in range(1, len(rho)):
        tau += rho[m]
        if m >= c * tau:
            return tau, m
    return tau, len(rho) - 1
