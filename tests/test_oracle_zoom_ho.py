"""Higher-order adaptive multigrid oracle (Section 3.3 with Tables 1 and 2) pinned to the printed
tables, polynomial exactness, conservation, a brute-force composite solve and the paper's
convergence statements."""

import numpy as np
import pytest

from oracle import zoom, zoom_ho, dense, highorder


def _centres(n, off_fine, h):
    idx = np.indices(n).astype(float)
    return [(idx[a] + off_fine[a] + 0.5) * h for a in range(3)]


def _poly(c, coef, deg):
    """sum of coef[k] * monomials of total degree <= deg, with a fixed monomial order."""
    x, y, z = c
    out = np.zeros_like(x)
    k = 0
    for i in range(deg + 1):
        for j in range(deg + 1 - i):
            for m in range(deg + 1 - i - j):
                out = out + coef[k % len(coef)] * (x ** i) * (y ** j) * (z ** m) / (1.0 + k)
                k += 1
    return out


@pytest.mark.parametrize("order", [2, 4, 6])
def test_flux_operators_difference_to_the_laplacians(golden, order):
    """Table 2: F convolved with [-1 1] gives the Laplacian of Table 1 of the next order (row 1
    with its sign, rows 3 and 5 with the opposite one).  Both tables are the printed values."""
    fl = golden["table2_flux"][str(order - 1)]
    lp = golden["table1_laplacian"][str(order)]
    F = np.array(fl["weights"], dtype=float) * fl["scale"]
    assert np.allclose(F, zoom_ho.flux_weights(order), rtol=0, atol=1e-15)
    # net flux of cell i: F at face i+1/2 (cells i-R+1 .. i+R) minus F at face i-1/2
    R = order // 2
    net = np.zeros(2 * R + 1)
    net[1:] += F
    net[:-1] -= F
    L = np.array(lp["weights"], dtype=float) * lp["scale"]
    sign = 1.0 if order == 2 else -1.0
    assert np.allclose(net, sign * L, atol=1e-14)


def test_lagrange_weights_reproduce_the_quadratic_ghost_formula():
    """n = 2: the normal weights are the (8/15, 2/3, -1/5) of the order-2 ghost, the parallel
    ones (-3/32, 15/16, 5/32) at +1/4."""
    assert np.allclose(zoom_ho.lagrange([-1, 0.5, 1.5], -0.5), [8 / 15, 2 / 3, -0.2], atol=1e-15)
    assert np.allclose(zoom_ho.lagrange([-1, 0, 1], 0.25), [-3 / 32, 15 / 16, 5 / 32], atol=1e-15)


@pytest.mark.parametrize("patches", [[((8, 8, 8), (4, 4, 4))],
                                     [((16, 12, 16), (3, 4, 3)), ((8, 8, 8), (4, 4, 4))]])
def test_order_two_equals_the_quadratic_ghosts(patches):
    H = zoom.Hierarchy(16, 1.0 / 16, patches)
    rng = np.random.default_rng(4)
    u = [rng.standard_normal(n) for n in H.n]
    for p in range(1, H.P + 1):
        for fm in (False, True):
            a = zoom_ho.ghosted(H, u, p, 2, fm)
            b = zoom.ghosted(H, u, p, fm)
            m = ~np.isnan(b)
            assert np.array_equal(np.isnan(a), np.isnan(b))
            assert np.allclose(a[m], b[m], rtol=0, atol=1e-13)


@pytest.mark.parametrize("order", [4, 6])
def test_ghosts_exact_for_polynomials_of_the_order(order):
    """Steps 1-2 (parallel, then normal, degree n) reproduce any polynomial of total degree n at
    the ghost centres of every layer and face, when coarse and fine cells hold point values."""
    R = order // 2
    H = zoom.Hierarchy(16, 1.0 / 16, [((8, 8, 8), (4, 4, 4))])
    coef = [0.3, -1.1, 0.7, 2.0, -0.4]
    u = [_poly(_centres(H.n[0], (0, 0, 0), H.h[0]), coef, order),
         _poly(_centres(H.n[1], (8, 8, 8), H.h[1]), coef, order)]
    up = zoom_ho.ghosted(H, u, 1, order, flux_match=False)
    pp = _poly(_centres(tuple(s + 2 * R for s in H.n[1]), (8 - R,) * 3, H.h[1]), coef, order)
    m = ~np.isnan(up)
    assert m.sum() == 8 ** 3 + 6 * R * 8 * 8
    assert np.allclose(up[m], pp[m], rtol=0, atol=1e-11 * np.max(np.abs(pp)))
    # one degree more is not reproduced: the degree is the order, not higher
    u = [_poly(_centres(H.n[0], (0, 0, 0), H.h[0]), coef, order + 1),
         _poly(_centres(H.n[1], (8, 8, 8), H.h[1]), coef, order + 1)]
    up = zoom_ho.ghosted(H, u, 1, order, flux_match=False)
    pp = _poly(_centres(tuple(s + 2 * R for s in H.n[1]), (8 - R,) * 3, H.h[1]), coef, order + 1)
    assert np.max(np.abs(up[m] - pp[m])) > 1e-9 * np.max(np.abs(pp))


@pytest.mark.parametrize("order", [4, 6])
def test_flux_matched_ghosts_exact_for_linears(order):
    """A linear function has coarse means equal to centre values and exact fluxes: no shift."""
    R = order // 2
    H = zoom.Hierarchy(16, 1.0 / 16, [((8, 8, 8), (4, 4, 4))])
    coef = [0.3, -1.1, 0.7, 2.0]
    u = [_poly(_centres(H.n[0], (0, 0, 0), H.h[0]), coef, 1),
         _poly(_centres(H.n[1], (8, 8, 8), H.h[1]), coef, 1)]
    up = zoom_ho.ghosted(H, u, 1, order, flux_match=True)
    pp = _poly(_centres(tuple(s + 2 * R for s in H.n[1]), (8 - R,) * 3, H.h[1]), coef, 1)
    m = ~np.isnan(up)
    assert np.allclose(up[m], pp[m], rtol=0, atol=1e-12)


@pytest.mark.parametrize("order", [4, 6])
@pytest.mark.parametrize("patches", [[((8, 8, 8), (4, 4, 4))],
                                     [((8, 12, 10), (3, 3, 4))],
                                     [((16, 16, 16), (5, 4, 6)), ((8, 8, 8), (4, 4, 5))]])
def test_composite_operator_is_conservative(order, patches):
    """Flux matching makes sum(L u * vol) over the composite cells vanish for ANY u."""
    H = zoom.Hierarchy(16, 1.0 / 16, patches)
    rng = np.random.default_rng(8)
    u = [rng.standard_normal(n) for n in H.n]
    r = zoom_ho.composite_residual(H, u, H.zeros(), order, flux_match=True)
    scale = zoom.composite_sum(H, [np.abs(a) for a in r])
    assert abs(zoom.composite_sum(H, r)) < 1e-13 * scale
    r0 = zoom_ho.composite_residual(H, u, H.zeros(), order, flux_match=False)
    assert abs(zoom.composite_sum(H, r0)) > 1e-8 * scale


@pytest.mark.parametrize("order", [4, 6])
def test_single_level_is_the_periodic_higher_order_solve(order):
    rng = np.random.default_rng(5)
    f = rng.standard_normal((16, 16, 16))
    H = zoom.Hierarchy(16, 1 / 16, [])
    u, _ = zoom_ho.solve_hierarchy(H, [f], order, tol=1e-13)
    exact = highorder.fft_solve(f - f.mean(), 1 / 16, order)
    assert np.max(np.abs(u[0] - exact)) < 1e-11 * np.max(np.abs(exact))


@pytest.mark.parametrize("order", [4, 6])
def test_fas_matches_dense_composite_solve(order):
    H = zoom.Hierarchy(8, 1 / 8, [((8, 8, 8), (2, 2, 2))])
    rng = np.random.default_rng(1 + order)
    f = [rng.standard_normal(n) for n in H.n]
    ud = dense.composite_solve(H, f, order=order)
    u, info = zoom_ho.solve_hierarchy(H, f, order, tol=1e-14, max_cycles=60)
    scale = max(np.max(np.abs(a)) for a in ud)
    assert max(np.max(np.abs(a - b)) for a, b in zip(u, ud)) < 1e-10 * scale


@pytest.mark.parametrize("order", [4, 6])
def test_tenfold_per_cycle_at_depth_three(golden, order):
    """Section 3.3: >= 10x residual reduction per cycle with any depth of sub-grids."""
    H = zoom.Hierarchy(16, 1 / 16, [((16, 16, 16), (4, 4, 4)), ((16, 16, 16), (4, 4, 4)),
                                    ((16, 16, 16), (4, 4, 4))])
    rng = np.random.default_rng(9)
    f = [rng.standard_normal(n) for n in H.n]
    _, info = zoom_ho.solve_hierarchy(H, f, order, tol=1e-12, max_cycles=20)
    hist = [1.0] + info["history"]
    rates = [b / a for a, b in zip(hist[:-1], hist[1:])]
    assert max(rates) < golden["vcycle_reduction_per_cycle"]["max_ratio"], rates
    assert info["rel_res"] <= 1e-12


@pytest.mark.parametrize("order", [4, 6])
def test_no_flux_matching_stalls(order):
    H = zoom.Hierarchy(16, 1 / 16, [((16, 16, 16), (4, 4, 4))])
    rng = np.random.default_rng(3)
    f = [rng.standard_normal(n) for n in H.n]
    _, info = zoom_ho.solve_hierarchy(H, f, order, tol=1e-12, max_cycles=14, flux_match=False)
    assert info["rel_res"] > 1e-6
    h = info["history"]
    assert h[-1] / h[-4] > 0.5
