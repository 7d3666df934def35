"""Pins of the oracle's analysis quantities (CPU): structure factor of a pure
composition wave and of uncorrelated beads, Parseval, shell bookkeeping,
tau_int of an AR(1) series; plus the library's host shell average against
the oracle's."""
import math

import numpy as np
import pytest

from oracle import analysis as A


def _wave_counts(grid, m, amp, base):
    nx, ny, nz = grid
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    ph = 2 * np.pi * (m[0] * x / nx + m[1] * y / ny + m[2] * z / nz)
    diff = np.rint(amp * np.cos(ph)).astype(np.int64)
    na = base + np.maximum(diff, 0)
    nb = base + np.maximum(-diff, 0)
    return np.stack([na.reshape(-1), nb.reshape(-1)]).astype(np.uint32)


def test_pure_wave_has_two_peaks():
    grid, m = (12, 10, 8), (3, 0, 2)
    amp = 1000.0        # multiples of the rounding: cos values give integers when rounded
    counts = _wave_counts(grid, m, amp, 2000)
    n_beads = int(counts.sum())
    s = A.structure_factor(counts, grid, 32, n_beads).reshape(8, 10, 12)
    top = np.argsort(s.ravel())[-2:]
    idx = {np.unravel_index(t, s.shape) for t in top}
    assert idx == {(2, 0, 3), (8 - 2, 0, 12 - 3)}
    # the wave's own power dominates what rounding the counts leaves elsewhere
    psi = (counts[0].astype(float) - counts[1]).reshape(8, 10, 12)
    g = abs(np.sum(psi * np.exp(-2j * np.pi * (3 * np.arange(12)[None, None, :] / 12 +
                                              2 * np.arange(8)[:, None, None] / 8))))
    assert s[2, 0, 3] == pytest.approx(32 ** 2 * g ** 2 / (4 * n_beads), rel=1e-12)
    assert g == pytest.approx(amp * 960 / 2, rel=1e-3)


def test_parseval_and_zero_mode():
    rng = np.random.default_rng(1)
    grid = (7, 9, 5)
    counts = rng.integers(0, 40, size=(2, 315)).astype(np.uint32)
    n_beads = int(counts.sum())
    s = A.structure_factor(counts, grid, 16, n_beads)
    psi = counts[0].astype(float) - counts[1]
    g2 = s * 4 * n_beads / 16 ** 2
    assert g2.sum() == pytest.approx(315 * np.sum(psi ** 2), rel=1e-12)
    assert g2[0] == pytest.approx(psi.sum() ** 2, rel=1e-12)


def test_uncorrelated_beads_give_flat_n_squared_over_four():
    """Independent uniform beads with random types: <|G|^2> = n_beads at q != 0, so
    S = N^2/4 on average."""
    rng = np.random.default_rng(2)
    grid = (16, 16, 16)
    nb = 200000
    cells = rng.integers(0, 4096, nb)
    typ = rng.integers(0, 2, nb)
    counts = np.stack([np.bincount(cells[typ == 0], minlength=4096),
                       np.bincount(cells[typ == 1], minlength=4096)]).astype(np.uint32)
    s = A.structure_factor(counts, grid, 32, nb)
    assert s[1:].mean() == pytest.approx(32 ** 2 / 4, rel=0.03)


def test_shell_bookkeeping():
    grid = (8, 8, 6)
    sq = np.ones(384)
    q, mean, cnt, peak = A.sq_shells(sq, grid, 64)
    assert cnt.sum() == 384 and cnt[0] == 1
    assert np.allclose(mean[cnt > 0], 1.0)
    # a spike on one lattice vector lands in its own shell
    sq2 = np.zeros(384)
    sq2[(1 * 8 + 0) * 8 + 2] = 5.0   # m = (2, 0, 1): |q| = 2 pi sqrt(1/16 + 1/36)
    k = int(np.floor(2 * np.pi * math.sqrt(4 / 64 + 1 / 36) / (2 * np.pi / 6) + 0.5))
    _, mean2, cnt2, peak2 = A.sq_shells(sq2, grid, 64)
    assert peak2 == k and mean2[k] == pytest.approx(5.0 / cnt2[k])


def test_tau_int_ar1():
    """AR(1) x_t = phi x_{t-1} + e_t: tau_int = (1 + phi) / (2 (1 - phi))."""
    rng = np.random.default_rng(3)
    phi, T, m = 0.8, 4000, 20
    e = rng.standard_normal((T, m))
    x = np.zeros((T, m))
    for t in range(1, T):
        x[t] = phi * x[t - 1] + e[t]
    tau, M = A.tau_int(x)
    assert tau == pytest.approx((1 + phi) / (2 * (1 - phi)), rel=0.08)
    assert M >= 5 * tau


def test_library_shell_average_matches_oracle():
    import os
    lib = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                       "paper_1711_03828_amd", "libsoma_hip.so")
    if not os.path.exists(lib):
        pytest.skip("library not built")
    from paper_1711_03828_amd import soma as C
    rng = np.random.default_rng(4)
    for grid in [(8, 8, 6), (9, 7, 5), (24, 24, 24)]:
        n = grid[0] * grid[1] * grid[2]
        sq = rng.random(n) * 10
        q1, m1, c1, p1 = C.soma_sq_shells(sq, grid, 40)
        q2, m2, c2, p2 = A.sq_shells(sq, grid, 40)
        np.testing.assert_array_equal(c1, c2)
        np.testing.assert_allclose(m1, m2, rtol=1e-12)
        np.testing.assert_allclose(q1, q2, rtol=1e-15)
        assert p1 == p2


def test_package_tau_int_matches_oracle():
    """The package's FFT-based tau_int against the oracle's direct sums."""
    from paper_1711_03828_amd import analysis as P
    rng = np.random.default_rng(5)
    x = np.zeros((3000, 8))
    for t in range(1, 3000):
        x[t] = 0.9 * x[t - 1] + rng.standard_normal(8)
    np.testing.assert_allclose(P.autocorrelation(x), A.autocorrelation(x), atol=1e-12)
    assert P.tau_int(x) == pytest.approx(A.tau_int(x), rel=1e-12)


def test_plane_structure_factor_of_a_film():
    """A z-invariant stripe pattern n_A - n_B ~ cos(2 pi 3 x / nx) in a film:
    the in-plane S(q_par) is the 2-D transform of the z-summed composition
    (numpy fft2, a separate route from the 3-D transform) and peaks in the
    shell of |q_par| = 2 pi 3 / nx."""
    grid = (24, 18, 5)
    nx, ny, nz = grid
    x = np.arange(nx)
    wave = np.round(4 + 3 * np.cos(2 * np.pi * 3 * x / nx)).astype(np.uint32)
    a = np.broadcast_to(wave[None, None, :], (nz, ny, nx)).ravel()
    b = np.broadcast_to((8 - wave)[None, None, :], (nz, ny, nx)).ravel()
    counts = np.stack([a, b]).astype(np.uint32)
    nb = int(counts.sum())
    s3 = A.structure_factor(counts, grid, 32, nb)
    psi2 = (a.astype(np.float64) - b).reshape(nz, ny, nx).sum(axis=0)
    s2 = 32 ** 2 / (4 * nb) * np.abs(np.fft.fft2(psi2)) ** 2
    np.testing.assert_allclose(s3[:nx * ny], s2.ravel(), rtol=1e-9, atol=1e-9)
    q, mean, cnt, peak = A.sq_plane_shells(s3, grid, 20)
    assert cnt.sum() == nx * ny and cnt[0] == 1
    dq = 2 * np.pi / min(nx, ny)
    assert peak == int(np.floor(2 * np.pi * 3 / nx / dq + 0.5))


def test_library_plane_shells_match_oracle():
    import os
    lib = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                       "paper_1711_03828_amd", "libsoma_hip.so")
    if not os.path.exists(lib):
        pytest.skip("library not built")
    from paper_1711_03828_amd import soma as C
    rng = np.random.default_rng(6)
    for grid in [(8, 8, 3), (9, 7, 5), (30, 24, 4)]:
        n = grid[0] * grid[1] * grid[2]
        sq = rng.random(n) * 10
        q1, m1, c1, p1 = C.soma_sq_plane_shells(sq, grid, 30)
        q2, m2, c2, p2 = A.sq_plane_shells(sq, grid, 30)
        np.testing.assert_array_equal(c1, c2)
        np.testing.assert_allclose(m1, m2, rtol=1e-12)
        np.testing.assert_allclose(q1, q2, rtol=1e-15)
        assert p1 == p2
