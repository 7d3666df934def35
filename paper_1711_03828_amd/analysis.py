"""Host-side analysis of measured time series (not part of the sampling path).

``tau_int``: integrated autocorrelation time of a stationary series with
Sokal's automatic window, tau = 1/2 + sum_{t=1}^{M} rho(t), M the smallest
window with M >= c tau(M) (c = 5); the autocorrelation comes from FFTs of
the zero-padded series.  Used to turn sweeps/s into uncorrelated samples/s:
n_chains * sweeps_per_second / (2 tau_int).
"""
from __future__ import annotations

import numpy as np


def autocorrelation(x) -> np.ndarray:
    """rho(t) of a series [T] or of independent series [T, m] (pooled)."""
    x = np.asarray(x, np.float64)
    if x.ndim == 1:
        x = x[:, None]
    T = x.shape[0]
    x = x - x.mean(axis=0)
    n = 1 << int(np.ceil(np.log2(2 * T)))
    f = np.fft.rfft(x, n=n, axis=0)
    acf = np.fft.irfft(f * np.conj(f), n=n, axis=0)[:T].sum(axis=1)
    acf /= np.arange(T, 0, -1)
    return acf / acf[0]


def tau_int(x, c: float = 5.0):
    """(tau_int, window M)."""
    rho = autocorrelation(x)
    csum = 0.5 + np.cumsum(rho[1:])
    for m in range(1, len(rho)):
        if m >= c * csum[m - 1]:
            return float(csum[m - 1]), m
    return float(csum[-1]), len(rho) - 1
