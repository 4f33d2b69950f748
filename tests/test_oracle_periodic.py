"""Periodic FAS oracle pinned to exact discrete solves and the paper's convergence claim."""

import numpy as np
import pytest

from oracle import periodic, dense, stencil


def _rand(N, seed):
    return np.random.default_rng(seed).standard_normal((N, N, N))


def test_dense_kronecker_matches_fft_solve():
    """Brute force on 8^3: Kronecker-sum matrix pseudo-inverse == eigenvalue division."""
    f = _rand(8, 1)
    h = 0.3
    ud = dense.periodic_solve(f, h)
    uf = periodic.fft_solve(f, h)
    assert np.max(np.abs(ud - uf)) <= 1e-13 * np.max(np.abs(uf))
    assert abs(ud.mean()) < 1e-14


@pytest.mark.parametrize("N", [8, 16, 32, 12, 24])
def test_fas_converges_to_exact_discrete_solution(N):
    """Section 3.2's V-cycle reaches exactly the discrete periodic solution (even and 3^3-coarsest grids)."""
    f = _rand(N, N)
    h = 1.0 / N
    u, info = periodic.solve_level(f, h, tol=1e-13, max_cycles=40)
    ue = periodic.fft_solve(f, h)
    assert info["rel_res"] <= 1e-13
    assert np.max(np.abs(u - ue)) <= 1e-11 * np.max(np.abs(ue))
    assert abs(np.mean(u)) < 1e-15


def test_fas_matches_dense_8cubed():
    f = _rand(8, 7) + 3.0   # non-zero mean is removed and reported
    h = 0.125
    u, info = periodic.solve_level(f, h, tol=1e-14, max_cycles=40)
    assert abs(info["f_mean"] - f.mean()) < 1e-15
    ud = dense.periodic_solve(f, h)
    assert np.max(np.abs(u - ud)) <= 1e-12 * np.max(np.abs(ud))


def test_single_fourier_mode_closed_form():
    """f = cos(2 pi m.x/N) => phi = f / lambda(m) (Table 1 order-2 symbol)."""
    N, h = 16, 0.25
    x = np.indices((N, N, N))
    m = (1, 2, 3)
    f = np.cos(2 * np.pi * sum(m[a] * x[a] for a in range(3)) / N)
    lam = -(2 / h ** 2) * sum(1 - np.cos(2 * np.pi * mi / N) for mi in m)
    u, _ = periodic.solve_level(f, h, tol=1e-13)
    assert np.max(np.abs(u - f / lam)) <= 1e-12 / abs(lam)


def test_convergence_rate_at_least_tenfold(golden):
    """Sections 3.2: >= one order of magnitude residual reduction per V(2,2) cycle."""
    f = _rand(32, 5)
    _, info = periodic.solve_level(f, 1 / 32, tol=1e-12, max_cycles=30)
    hist = [1.0] + info["history"]
    rates = [b / a for a, b in zip(hist[:-1], hist[1:])]
    assert max(rates) < golden["vcycle_reduction_per_cycle"]["max_ratio"]
    assert info["cycles"] <= 12


def test_half_sweep_solves_its_own_colour():
    """After a red half-sweep every red cell satisfies its own equation exactly."""
    N, h = 8, 0.5
    u = _rand(N, 11)
    f = _rand(N, 12)
    red = stencil.red_mask(u.shape)
    u1 = periodic.rbgs_half(u, f, h, 0)
    assert np.array_equal(u1[~red], u[~red])
    r = f - stencil.lap7(u1, h)
    assert np.max(np.abs(r[red])) < 1e-12 * np.max(np.abs(f))
    u2 = periodic.rbgs_half(u1, f, h, 1)
    r = f - stencil.lap7(u2, h)
    assert np.array_equal(u2[red], u1[red])
    assert np.max(np.abs(r[~red])) < 1e-12 * np.max(np.abs(f))


def test_cell_update_count():
    assert periodic.cell_updates(64, 1) == 4 * sum((64 >> k) ** 3 for k in range(6))
    assert periodic.cell_updates(48, 2) == 2 * 4 * (48 ** 3 + 24 ** 3 + 12 ** 3 + 6 ** 3)
