"""Pins for the spectral corrections of Section 3.5 (oracle/spectral.py).

Each pin reaches the expected values by a route that shares no arithmetic with the oracle's
multipliers: cell averages by Gauss-Legendre quadrature, sub-cell averages by direct sampling,
finite-difference potentials by the real-space stencils and closed-form plane-wave solutions.
"""

import numpy as np
import pytest

from oracle import spectral, stencil, highorder


def _centres(n, h):
    return (np.arange(n) + 0.5) * h


def _plane(n, h, m, phase=0.3):
    """sin(k . x + phase) at cell centres for integer mode numbers m (periodic box of n cells)."""
    L = n * h
    x = np.meshgrid(*[_centres(n, h)] * 3, indexing="ij")
    k = [2.0 * np.pi * mi / L for mi in m]
    return k, sum(ki * xi for ki, xi in zip(k, x)) + phase


def test_pad_length():
    assert [spectral.pad_length(n) for n in (1, 2, 8, 96, 128, 130)] == [2, 4, 16, 256, 256, 512]


@pytest.mark.parametrize("m", [(1, 0, 0), (3, -2, 5), (7, 7, -7), (8, 1, -3)])
def test_fv_deconvolve_recovers_point_samples_from_cell_averages(m):
    """Section 3.5.1: deconvolving cell averages of a plane wave returns its centre values."""
    n, h = 16, 0.7
    k, theta = _plane(n, h, m)
    # cell averages by 6-point Gauss-Legendre on each axis (exact to rounding for this sine)
    t, w = np.polynomial.legendre.leggauss(6)
    avg = np.zeros_like(theta)
    for ta, wa in zip(t, w):
        for tb, wb in zip(t, w):
            for tc, wc in zip(t, w):
                off = k[0] * ta * h / 2 + k[1] * tb * h / 2 + k[2] * tc * h / 2
                avg += (wa * wb * wc / 8.0) * np.sin(theta + off)
    got = spectral.fv_deconvolve(avg)
    np.testing.assert_allclose(got, np.sin(theta), atol=1e-12)


@pytest.mark.parametrize("m", [(1, 0, 0), (3, -2, 5), (8, 8, 8), (5, 0, -8)])
def test_sg_deconvolve_recovers_point_samples_from_subcell_means(m):
    """Section 3.5.3: deconvolving the mean over the 8 sub-cell centres returns the centre value."""
    n, h = 16, 1.3
    k, theta = _plane(n, h, m)
    mean8 = np.zeros_like(theta)
    for sx in (-0.25, 0.25):
        for sy in (-0.25, 0.25):
            for sz in (-0.25, 0.25):
                mean8 += np.sin(theta + (k[0] * sx + k[1] * sy + k[2] * sz) * h) / 8.0
    np.testing.assert_allclose(spectral.sg_deconvolve(mean8), np.sin(theta), atol=1e-12)


def test_deconvolutions_keep_the_mean_and_are_real_linear():
    rng = np.random.default_rng(5)
    a, b = rng.standard_normal((2, 8, 12, 16))
    for fn in (spectral.fv_deconvolve, spectral.sg_deconvolve):
        np.testing.assert_allclose(np.mean(fn(a)), np.mean(a), atol=1e-14)
        np.testing.assert_allclose(fn(2.0 * a - b), 2.0 * fn(a) - fn(b), atol=1e-12)


def _fd_displacement(f, h, lap_order, grad_order, scale):
    """scale * G phi with L phi = f - mean(f), the potential from the real-space multigrid."""
    if lap_order == 2:
        from oracle import periodic
        phi, _ = periodic.solve_level(f, h, tol=1e-14, max_cycles=60)
    else:
        phi, _ = highorder.solve_level(f, h, lap_order, tol=1e-14, max_cycles=60)
    return np.stack([scale * stencil.grad(phi, h, a, grad_order) for a in range(3)])


@pytest.mark.parametrize("lap_order,grad_order", [(2, 4), (4, 4), (6, 6), (2, 6)])
def test_hybrid_periodic_makes_the_fd_displacement_exact(lap_order, grad_order):
    """Section 3.5.2: FD displacement + correction = the continuum displacement, mode by mode.

    f = sum of plane waves A cos(k.x + p); the continuum solution of lap phi = f has
    d_j phi = A k_j sin(k.x + p) / |k|^2.  The FD side is a real-space multigrid solve and the
    real-space gradient stencil, so the multipliers' algebra (signs, symbols, the Nyquist rule)
    is checked against an independent route.
    """
    n, h, scale = 16, 0.5, -1.7
    waves = [((1, 2, -3), 0.8, 0.1), ((5, -6, 2), 0.3, 1.2), ((7, 0, 4), -0.5, 2.0),
             ((8, 3, 1), 0.4, 0.0)]                      # the last one sits on the x Nyquist plane
    L = n * h
    x = np.meshgrid(*[_centres(n, h)] * 3, indexing="ij")
    f = np.zeros((n, n, n))
    exact = np.zeros((3, n, n, n))
    for m, A, p in waves:
        k = [2 * np.pi * mi / L for mi in m]
        th = sum(ki * xi for ki, xi in zip(k, x)) + p
        f += A * np.cos(th)
        k2 = sum(ki * ki for ki in k)
        for j in range(3):
            if m[j] == n // 2:
                continue       # the sampled Nyquist pattern has zero continuum derivative
            exact[j] += scale * A * k[j] * np.sin(th) / k2
    fd = _fd_displacement(f, h, lap_order, grad_order, scale)
    corr = spectral.hybrid_correction(f, h, lap_order, grad_order, scale, periodic=True)
    np.testing.assert_allclose(fd + corr, exact, atol=1e-11)
    # the correction is not trivially small: the FD result alone is off at these wave numbers
    assert np.max(np.abs(fd - exact)) > 1e-3


def test_exact_displacement_closed_form():
    n, h, scale = 12, 2.0, 0.6
    k, th = _plane(n, h, (2, -1, 3), phase=0.4)
    f = np.cos(th)
    k2 = sum(ki * ki for ki in k)
    want = np.stack([scale * k[j] * np.sin(th) / k2 for j in range(3)])
    np.testing.assert_allclose(spectral.exact_displacement(f, h, scale), want, atol=1e-13)


def test_hybrid_isolated_is_the_zero_padded_periodic_correction():
    """Isolated mode: the periodic correction of f zero-padded to 2n, cut back to the patch."""
    rng = np.random.default_rng(9)
    f = rng.standard_normal((8, 16, 12))
    P = (16, 32, 32)
    g = np.zeros(P)
    g[:8, :16, :12] = f
    want = spectral.hybrid_correction(g, 0.25, 2, 4, 1.0, periodic=True)[:, :8, :16, :12]
    got = spectral.hybrid_correction(f, 0.25, 2, 4, 1.0, periodic=False)
    np.testing.assert_allclose(got, want, atol=1e-13)


def test_hybrid_isolated_boundaries_are_far_enough():
    """A compact source deep inside a patch: 2x padding and 4x padding agree closely (the
    correction's kernel, exact minus FD Green's function gradient, is short-ranged)."""
    n, h = 32, 1.0
    x = np.meshgrid(*[np.arange(n) - n / 2 + 0.5] * 3, indexing="ij")
    f = np.exp(-sum(xi * xi for xi in x) / 4.0)
    c2 = spectral.hybrid_correction(f, h, 2, 4, 1.0, periodic=False)
    big = np.zeros((4 * n,) * 3)
    big[:n, :n, :n] = f
    c4 = spectral.hybrid_correction(big, h, 2, 4, 1.0, periodic=True)[:, :n, :n, :n]
    assert np.max(np.abs(c2 - c4)) < 1e-3 * np.max(np.abs(c4))
    # antisymmetry of a symmetric source: component x is odd about the patch centre
    np.testing.assert_allclose(c2[0], -c2[0][::-1, :, :], atol=1e-5 * np.max(np.abs(c2[0])))


def test_hybrid_zero_on_nyquist_plane_and_mean_free():
    rng = np.random.default_rng(3)
    f = rng.standard_normal((8, 8, 8))
    s = spectral.hybrid_multipliers((8, 8, 8))
    assert np.all(s[0][4, :, :] == 0.0) and np.all(s[1][:, 4, :] == 0.0) and s[2][0, 0, 0] == 0.0
    c = spectral.hybrid_correction(f, 1.0)
    assert np.max(np.abs(np.mean(c, axis=(1, 2, 3)))) < 1e-14
