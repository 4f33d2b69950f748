"""Adaptive-multigrid oracle (Section 3.3) pinned to exactness, conservation,
brute-force composite solves and the paper's convergence statements."""

import numpy as np
import pytest

from oracle import zoom, dense, periodic
from oracle.stencil import restrict_mean8


def _centres(n, off_fine, h):
    """Cell-centre coordinates of an n-array whose first cell starts at off_fine cells."""
    idx = np.indices(n).astype(float)
    return [(idx[a] + off_fine[a] + 0.5) * h for a in range(3)]


def _poly(c, coef):
    x, y, z = c
    a = coef
    return (a[0] + a[1] * x + a[2] * y + a[3] * z + a[4] * x * x + a[5] * y * y + a[6] * z * z
            + a[7] * x * y + a[8] * y * z + a[9] * x * z)


def _two_level(N0=16, n=8, off=4):
    return zoom.Hierarchy(N0, 1.0 / N0, [((n, n, n), (off, off, off))])


def test_ghost_interpolation_exact_for_quadratics():
    """Steps 1-2 (parallel, then normal quadratic) reproduce any quadratic at the ghost centres."""
    H = _two_level(16, 8, 4)
    coef = [0.3, 1.0, -2.0, 0.5, 3.0, -1.5, 2.0, 0.7, -0.4, 1.1]
    u = [_poly(_centres(H.n[0], (0, 0, 0), H.h[0]), coef),
         _poly(_centres(H.n[1], (8, 8, 8), H.h[1]), coef)]
    up = zoom.ghosted(H, u, 1, flux_match=False)
    pp = _poly(_centres(tuple(s + 2 for s in H.n[1]), (7, 7, 7), H.h[1]), coef)
    n = H.n[1][0]
    for a in range(3):
        for side in (0, n + 1):
            sl = [slice(1, n + 1)] * 3
            sl[a] = side
            assert np.allclose(up[tuple(sl)], pp[tuple(sl)], atol=1e-13)


def test_flux_matched_ghosts_exact_for_linears():
    """With flux matching the ghost of a linear function is still exact (zero shift)."""
    H = _two_level(16, 8, 4)
    coef = [0.3, 1.0, -2.0, 0.5] + [0.0] * 6
    u = [_poly(_centres(H.n[0], (0, 0, 0), H.h[0]), coef),
         _poly(_centres(H.n[1], (8, 8, 8), H.h[1]), coef)]
    up = zoom.ghosted(H, u, 1, flux_match=True)
    pp = _poly(_centres(tuple(s + 2 for s in H.n[1]), (7, 7, 7), H.h[1]), coef)
    n = H.n[1][0]
    for a in range(3):
        for side in (0, n + 1):
            sl = [slice(1, n + 1)] * 3
            sl[a] = side
            assert np.allclose(up[tuple(sl)], pp[tuple(sl)], atol=1e-13)


@pytest.mark.parametrize("patches", [
    [((8, 8, 8), (4, 4, 4))],
    [((8, 12, 6), (3, 5, 2))],
    [((16, 16, 16), (2, 3, 4)), ((8, 8, 8), (4, 5, 4))],
])
def test_composite_operator_is_conservative(patches):
    """Flux matching makes sum(L u * vol) vanish for ANY u; without it, it does not."""
    H = zoom.Hierarchy(12, 1.0 / 12, patches)
    rng = np.random.default_rng(2)
    u = [rng.standard_normal(n) for n in H.n]
    r = zoom.composite_residual(H, u, H.zeros(), flux_match=True)
    scale = zoom.composite_sum(H, [np.abs(a) for a in r])
    assert abs(zoom.composite_sum(H, r)) < 1e-14 * scale
    r0 = zoom.composite_residual(H, u, H.zeros(), flux_match=False)
    assert abs(zoom.composite_sum(H, r0)) > 1e-8 * scale


def test_fas_matches_dense_composite_one_patch():
    H = zoom.Hierarchy(8, 1 / 8, [((8, 8, 8), (2, 2, 2))])
    rng = np.random.default_rng(1)
    f = [rng.standard_normal(n) for n in H.n]
    ud = dense.composite_solve(H, f)
    u, info = zoom.solve_hierarchy(H, f, tol=1e-14, max_cycles=40)
    scale = max(np.max(np.abs(a)) for a in ud)
    assert max(np.max(np.abs(a - b)) for a, b in zip(u, ud)) < 1e-11 * scale


@pytest.mark.slow
def test_fas_matches_dense_composite_two_patches():
    H = zoom.Hierarchy(8, 1 / 8, [((12, 12, 12), (1, 1, 1)), ((8, 8, 8), (4, 4, 4))])
    rng = np.random.default_rng(1)
    f = [rng.standard_normal(n) for n in H.n]
    ud = dense.composite_solve(H, f)
    u, info = zoom.solve_hierarchy(H, f, tol=1e-14, max_cycles=40)
    scale = max(np.max(np.abs(a)) for a in ud)
    assert max(np.max(np.abs(a - b)) for a, b in zip(u, ud)) < 1e-11 * scale


def test_tenfold_per_cycle_at_depth(golden):
    """Section 3.3: >= 10x residual reduction per cycle with any depth of sub-grids."""
    H = zoom.Hierarchy(16, 1 / 16, [((16, 16, 16), (4, 4, 4)), ((16, 16, 16), (4, 4, 4)),
                                    ((16, 16, 16), (4, 4, 4))])
    rng = np.random.default_rng(9)
    f = [rng.standard_normal(n) for n in H.n]
    _, info = zoom.solve_hierarchy(H, f, tol=1e-12, max_cycles=20)
    hist = [1.0] + info["history"]
    rates = [b / a for a, b in zip(hist[:-1], hist[1:])]
    assert max(rates) < golden["vcycle_reduction_per_cycle"]["max_ratio"]
    assert info["rel_res"] <= 1e-12


def test_no_flux_matching_stalls():
    """Section 3.3: without flux correction the residual does not vanish on all levels."""
    H = _two_level(16, 16, 4)
    rng = np.random.default_rng(3)
    f = [rng.standard_normal(n) for n in H.n]
    _, info = zoom.solve_hierarchy(H, f, tol=1e-12, max_cycles=14, flux_match=False)
    assert info["rel_res"] > 1e-6
    h = info["history"]
    assert h[-1] / h[-4] > 0.5          # stalled, not converging


def test_single_level_hierarchy_is_periodic_solve():
    rng = np.random.default_rng(5)
    f = rng.standard_normal((16, 16, 16))
    H = zoom.Hierarchy(16, 1 / 16, [])
    u, _ = zoom.solve_hierarchy(H, [f], tol=1e-13)
    assert np.max(np.abs(u[0] - periodic.fft_solve(f, 1 / 16))) < 1e-11 * np.max(np.abs(u[0]))


def test_wide_ghosts_exact_for_quadratics():
    """Post-solve tri-quadratic ghosts (faces, edges, corners) are exact for quadratics."""
    H = zoom.Hierarchy(16, 1 / 16, [((16, 16, 16), (4, 4, 4)), ((8, 8, 8), (4, 4, 4))])
    coef = [0.3, 1.0, -2.0, 0.5, 3.0, -1.5, 2.0, 0.7, -0.4, 1.1]
    offs = [(0, 0, 0), (8, 8, 8), (24, 24, 24)]
    v = [_poly(_centres(H.n[p], offs[p], H.h[p]), coef) for p in range(3)]
    for p, R in ((1, 2), (2, 4)):
        vp = zoom.wide_ghosted(H, v, p, R)
        exp = _poly(_centres(vp.shape, tuple(o - R for o in offs[p]), H.h[p]), coef)
        assert np.allclose(vp, exp, atol=1e-12)


def test_hierarchy_plane_wave_displacement_and_tau():
    """Plane wave on all levels: psi matches the G4 symbol away from patch faces, tau ~ 0."""
    N0 = 16
    H = zoom.Hierarchy(N0, 1.0, [((16, 16, 16), (4, 4, 4))])
    m = (1, 1, 0)
    def field(p, off):
        c = _centres(H.n[p], off, H.h[p])
        return 0.2 * np.cos(2 * np.pi * (m[0] * c[0] + m[1] * c[1]) / N0)
    phi = [field(0, (0, 0, 0)), field(1, (8, 8, 8))]
    psi = zoom.displacement_hierarchy(H, phi, scale=1.0)
    # interior of the patch (>= 2 cells from every face) uses no ghosts
    c = _centres(H.n[1], (8, 8, 8), H.h[1])
    ph = 2 * np.pi * (m[0] * c[0] + m[1] * c[1]) / N0
    kx = 2 * np.pi * m[0] * H.h[1] / N0
    g = -0.2 * (8 * np.sin(kx) - np.sin(2 * kx)) / 6 / H.h[1]
    assert np.allclose(psi[1][0][2:-2, 2:-2, 2:-2], (g * np.sin(ph))[2:-2, 2:-2, 2:-2], atol=1e-14)
    t = zoom.tau_hierarchy(H, phi)
    assert abs(zoom.composite_sum(H, t)) < 1e-14
    # away from the faces tau is exactly zero before the composite mean is removed,
    # so it is one constant there
    assert np.ptp(t[1][4:-4, 4:-4, 4:-4]) < 1e-14


def test_zoom_error_is_localised_at_the_coarse_fine_boundary():
    """Section 4.2: zoom vs a degraded unigrid - the error peaks at the patch faces."""
    from paper_1103_6031_amd import inputs
    N0, n, off = 32, 32, 8
    Nf = 2 * N0
    ff = inputs.gaussian_field(Nf, 77, box=100.0)
    fc = restrict_mean8(ff)
    sl = tuple(slice(2 * off, 2 * off + n) for _ in range(3))
    H = zoom.Hierarchy(N0, 100.0 / N0, [((n, n, n), (off, off, off))])
    u, _ = zoom.solve_hierarchy(H, [fc, ff[sl]], tol=1e-11)
    degraded = np.repeat(np.repeat(np.repeat(fc, 2, 0), 2, 1), 2, 2)
    degraded[sl] = ff[sl]
    ug = periodic.fft_solve(degraded, H.h[1])
    ug = ug - ug[sl].mean() + u[1].mean()
    err = np.abs(u[1] - ug[sl])
    face = max(err[0].max(), err[-1].max(), err[:, 0].max(), err[:, -1].max(), err[:, :, 0].max(),
               err[:, :, -1].max())
    centre = err[12:20, 12:20, 12:20].max()
    assert face > 3 * centre


def test_hierarchy_sixth_order_plane_wave_displacement_and_tau():
    """Sixth-order gradient on a hierarchy: the patch interior (>= 3 cells from every face) equals
    the printed symbol; tau is one constant away from the faces (>= 6 cells)."""
    N0 = 16
    H = zoom.Hierarchy(N0, 1.0, [((16, 16, 16), (4, 4, 4))])
    m = (1, 1, 0)

    def field(p, off):
        c = _centres(H.n[p], off, H.h[p])
        return 0.2 * np.cos(2 * np.pi * (m[0] * c[0] + m[1] * c[1]) / N0)
    phi = [field(0, (0, 0, 0)), field(1, (8, 8, 8))]
    psi = zoom.displacement_hierarchy(H, phi, scale=1.0, order=6)
    c = _centres(H.n[1], (8, 8, 8), H.h[1])
    ph = 2 * np.pi * (m[0] * c[0] + m[1] * c[1]) / N0
    kx = 2 * np.pi * m[0] * H.h[1] / N0
    g = -0.2 * (np.sin(3 * kx) - 9 * np.sin(2 * kx) + 45 * np.sin(kx)) / 30 / H.h[1]
    assert np.allclose(psi[1][0][3:-3, 3:-3, 3:-3], (g * np.sin(ph))[3:-3, 3:-3, 3:-3], atol=1e-14)
    t = zoom.tau_hierarchy(H, phi, order=6)
    assert abs(zoom.composite_sum(H, t)) < 1e-14
    assert np.ptp(t[1][6:-6, 6:-6, 6:-6]) < 1e-14


def test_wide_ghosts_width_six_exact_for_quadratics():
    H = zoom.Hierarchy(16, 1 / 16, [((16, 16, 16), (4, 4, 4)), ((8, 8, 8), (4, 4, 4))])
    coef = [0.3, 1.0, -2.0, 0.5, 3.0, -1.5, 2.0, 0.7, -0.4, 1.1]
    offs = [(0, 0, 0), (8, 8, 8), (24, 24, 24)]
    v = [_poly(_centres(H.n[p], offs[p], H.h[p]), coef) for p in range(3)]
    for p, R in ((1, 3), (2, 6)):
        vp = zoom.wide_ghosted(H, v, p, R)
        exp = _poly(_centres(vp.shape, tuple(o - R for o in offs[p]), H.h[p]), coef)
        assert np.allclose(vp, exp, atol=1e-12)
