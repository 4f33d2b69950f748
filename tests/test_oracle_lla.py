"""Pins of the oracle's LLA baryon density (Section 5.3, eq. gasdens: rho / rho_bar = 1 / det(I + dL/dq)).

The closed forms use the symbol of the fourth-order gradient stencil on a sine,
    G4 sin(k x) = g(k) cos(k x),  g(k) = (8 sin(k h) - sin(2 k h)) / (6 h),
derived here from the stencil weights (1, -8, 0, 8, -1) / (12 h), so each case fixes the
determinant of a known Jacobian.  A wrong sign of the cross term, a dropped diagonal term, a
derivative taken along the wrong axis or a wrong stencil scale fails one of them.
"""

import numpy as np
import pytest

from oracle import lpt, zoom

pytestmark = pytest.mark.filterwarnings("error")


def _g(k, h):
    return (8.0 * np.sin(k * h) - np.sin(2.0 * k * h)) / (6.0 * h)


def _coords(N, h):
    x = (np.arange(N) + 0.5) * h
    return np.meshgrid(x, x, x, indexing="ij")


def test_single_plane_wave_closed_form():
    N, h = 16, 0.5
    X, Y, Z = _coords(N, h)
    k = 2 * np.pi * 2 / (N * h)
    A = 0.3 / _g(k, h)
    L = np.stack([A * np.sin(k * X), np.zeros_like(X), np.zeros_like(X)])
    got = lpt.lla_density(L, h, renorm=False)
    want = 1.0 / (1.0 + A * _g(k, h) * np.cos(k * X)) - 1.0
    assert np.max(np.abs(got - want)) <= 1e-13


def test_separable_waves_give_the_product_of_the_diagonal_terms():
    N, h = 16, 0.25
    X, Y, Z = _coords(N, h)
    ks = [2 * np.pi * m / (N * h) for m in (1, 2, 3)]
    amp = [0.2, -0.25, 0.15]
    A = [a / _g(k, h) for a, k in zip(amp, ks)]
    L = np.stack([A[0] * np.sin(ks[0] * X), A[1] * np.sin(ks[1] * Y), A[2] * np.sin(ks[2] * Z)])
    got = lpt.lla_density(L, h, renorm=False)
    det = ((1.0 + A[0] * _g(ks[0], h) * np.cos(ks[0] * X)) * (1.0 + A[1] * _g(ks[1], h) * np.cos(ks[1] * Y))
           * (1.0 + A[2] * _g(ks[2], h) * np.cos(ks[2] * Z)))
    assert np.max(np.abs(got - (1.0 / det - 1.0))) <= 1e-13


def test_cross_shear_closed_form():
    # L_x = C sin(k y), L_y = D sin(k x): J_xy = C g cos(k y), J_yx = D g cos(k x), det = 1 - J_xy J_yx
    N, h = 16, 0.5
    X, Y, Z = _coords(N, h)
    k = 2 * np.pi / (N * h)
    C, D = 0.4 / _g(k, h), 0.5 / _g(k, h)
    L = np.stack([C * np.sin(k * Y), D * np.sin(k * X), np.zeros_like(X)])
    got = lpt.lla_density(L, h, renorm=False)
    det = 1.0 - (C * _g(k, h) * np.cos(k * Y)) * (D * _g(k, h) * np.cos(k * X))
    assert np.max(np.abs(got - (1.0 / det - 1.0))) <= 1e-13


def test_pure_off_diagonal_shear_leaves_the_density_unchanged():
    N, h = 8, 1.0
    X, Y, Z = _coords(N, h)
    k = 2 * np.pi / (N * h)
    L = np.stack([0.7 * np.sin(k * Y), np.zeros_like(X), 0.3 * np.cos(k * Y)])
    assert np.max(np.abs(lpt.lla_density(L, h, renorm=False))) <= 1e-15


def test_renormalisation_conserves_mass():
    rng = np.random.default_rng(5)
    N, h = 12, 1.0
    L = 0.05 * rng.standard_normal((3, N, N, N))
    raw = lpt.lla_density(L, h, renorm=False)
    ren = lpt.lla_density(L, h)
    assert abs(float(np.mean(ren))) <= 1e-16
    assert np.allclose(ren, raw - raw.mean(), rtol=0, atol=1e-15)


def test_linear_limit_is_minus_the_divergence():
    # for L = eps * v, det(I + eps J) = 1 + eps tr J + O(eps^2), so (rho/rho_bar - 1)/eps -> -div v
    rng = np.random.default_rng(7)
    N, h = 12, 0.5
    v = rng.standard_normal((3, N, N, N))
    div = np.zeros((N, N, N))
    for a in range(3):   # the fourth-order gradient written out from the stencil weights
        div += (np.roll(v[a], 2, a) - 8 * np.roll(v[a], 1, a) + 8 * np.roll(v[a], -1, a)
                - np.roll(v[a], -2, a)) / (12 * h)
    errs = []
    for eps in (1e-3, 1e-4):
        d = lpt.lla_density(eps * v, h, renorm=False) / eps
        errs.append(np.max(np.abs(d + div)))
    assert errs[1] < errs[0] / 5 and errs[1] < 1e-2 * np.max(np.abs(div))


def _analytic(X, Y, Z, box):
    k = 2 * np.pi / box
    return np.stack([0.02 * box * np.sin(k * X + 0.3) * np.cos(k * Z),
                     0.015 * box * np.sin(2 * k * Y) + 0.01 * box * np.cos(k * X),
                     0.02 * box * np.cos(k * Z - 0.5) * np.sin(k * Y)])


def _level_coords(H, p):
    n, h = H.n[p], H.h[p]
    org = np.zeros(3)
    for q in range(1, p + 1):
        org = org + np.array(H.off[q]) * H.h[q - 1]
    ax = [org[a] + (np.arange(n[a]) + 0.5) * h for a in range(3)]
    return np.meshgrid(*ax, indexing="ij")


def test_hierarchy_patch_interior_equals_the_fine_periodic_grid():
    # away from its faces a patch sees only its own cells: there it must equal the periodic
    # computation on a uniform grid of the patch's spacing (same values, same stencil)
    N0, h0 = 16, 1.0
    H = zoom.Hierarchy(N0, h0, [((12, 12, 12), (2, 3, 2))])
    box = N0 * h0
    L = [_analytic(*_level_coords(H, p), box) for p in range(H.P + 1)]
    out = zoom.lla_hierarchy(H, L, renorm=False)
    Xf, Yf, Zf = _coords(2 * N0, h0 / 2)
    fine = lpt.lla_density(_analytic(Xf, Yf, Zf, box), h0 / 2, renorm=False)
    o = [2 * v for v in H.off[1]]
    sub = fine[o[0]:o[0] + 12, o[1]:o[1] + 12, o[2]:o[2] + 12]
    assert np.max(np.abs(out[1][2:-2, 2:-2, 2:-2] - sub[2:-2, 2:-2, 2:-2])) <= 1e-14
    # next to the faces the ghosts are interpolated from the parent: close, not equal
    assert np.max(np.abs(out[1] - sub)) <= 0.05 * np.max(np.abs(sub))
    # base cells whose stencils stay 3 or more cells away from the covered box (which holds the
    # restriction of the patch) are the base's own periodic computation
    base = lpt.lla_density(L[0], h0, renorm=False)
    m = np.ones(H.n[0], dtype=bool)
    m[tuple(slice(H.off[1][a] - 2, H.off[1][a] + H.n[1][a] // 2 + 2) for a in range(3))] = False
    assert np.max(np.abs(out[0][m] - base[m])) <= 1e-15
    assert np.max(np.abs(out[0][~m] - base[~m])) > 1e-6   # the restricted box does reach the others


def test_hierarchy_renormalisation_has_zero_composite_mean():
    N0, h0 = 8, 1.0
    H = zoom.Hierarchy(N0, h0, [((12, 12, 12), (1, 1, 1)), ((8, 8, 8), (4, 4, 4))])
    L = [_analytic(*_level_coords(H, p), N0 * h0) for p in range(H.P + 1)]
    out = zoom.lla_hierarchy(H, L)
    scale = sum(float(np.sum(np.abs(a))) * H.h[p] ** 3 for p, a in enumerate(out))
    assert abs(zoom.composite_sum(H, out)) <= 1e-14 * scale
    # covered cells hold the mean of their children
    c = H.covered(1)
    kids = out[1].reshape(6, 2, 6, 2, 6, 2).mean(axis=(1, 3, 5))
    assert np.allclose(out[0][c], kids, rtol=0, atol=1e-15)


def test_hierarchy_without_patches_is_the_periodic_function():
    rng = np.random.default_rng(3)
    N, h = 8, 0.7
    L = 0.03 * rng.standard_normal((3, N, N, N))
    H = zoom.Hierarchy(N, h)
    assert np.array_equal(zoom.lla_hierarchy(H, [L])[0], lpt.lla_density(L, h))
