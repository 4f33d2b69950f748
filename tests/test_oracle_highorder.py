"""Pins of the oracle's higher-order periodic Laplacians and their FAS solve (Table 1, Section 3.2).

Each pin rests on something other than the oracle's own arithmetic:
* the stencils (Table 1, top rows) applied to Fourier modes must give the symbols that Table 1
  prints separately (bottom rows, typed below from the table);
* the truncation error must fall as h^order, which a wrong weight or a dropped term breaks;
* order 2 must equal the already pinned 7-point oracle;
* the half-sweep must solve each cell's own equation with its neighbours frozen, found here by
  evaluating the operator twice per cell (it is affine in the centre value);
* the FAS solve must reach the exact discrete solution and contract by at least a factor of ten
  per cycle, as Section 3.2 reports for every order up to six.
"""

import numpy as np
import pytest

from oracle import highorder as ho
from oracle import periodic, stencil

pytestmark = pytest.mark.filterwarnings("error")

# Table 1, bottom rows (Fourier symbols of the 1-D Laplacian stencils, k in grid units)
PRINTED = {
    2: lambda k: -2.0 * (-np.cos(k) + 1.0),
    4: lambda k: -(1.0 / 6.0) * (np.cos(2 * k) - 16.0 * np.cos(k) + 15.0),
    6: lambda k: -(1.0 / 90.0) * (-2.0 * np.cos(3 * k) + 27.0 * np.cos(2 * k) - 270.0 * np.cos(k) + 245.0),
}


@pytest.mark.parametrize("order", [2, 4, 6])
def test_stencil_reproduces_the_printed_symbol(order):
    N, h = 16, 0.75
    i = np.arange(N)
    for m in (1, 3, 5, 8):
        k = 2 * np.pi * m / N
        for axis in range(3):
            shape = [1, 1, 1]
            shape[axis] = N
            u = np.broadcast_to(np.cos(k * i + 0.4).reshape(shape), (N, N, N)).copy()
            got = ho.lap(u, h, order)
            assert np.max(np.abs(got - PRINTED[order](k) / h ** 2 * u)) <= 1e-12 / h ** 2
        # a 3-D mode: the symbols of the three axes add
        mx, my, mz = m, (m + 2) % N, (3 * m) % N
        X, Y, Z = np.meshgrid(i, i, i, indexing="ij")
        ks = [2 * np.pi * v / N for v in (mx, my, mz)]
        u = np.cos(ks[0] * X + ks[1] * Y + ks[2] * Z)
        lam = sum(PRINTED[order](kk) for kk in ks) / h ** 2
        assert np.max(np.abs(ho.lap(u, h, order) - lam * u)) <= 1e-11 / h ** 2
        assert np.allclose(ho.symbol_1d(k, order), PRINTED[order](k), rtol=0, atol=1e-14)


@pytest.mark.parametrize("order", [2, 4, 6])
def test_truncation_error_falls_as_h_to_the_order(order):
    errs = []
    for N in (16, 32):
        h = 1.0 / N
        x = (np.arange(N) + 0.5) * h
        X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
        k = 2 * np.pi
        u = np.sin(k * X) * np.cos(2 * k * Y) * np.sin(k * Z + 0.3)
        exact = -(k * k + 4 * k * k + k * k) * u
        errs.append(np.max(np.abs(ho.lap(u, h, order) - exact)) / np.max(np.abs(exact)))
    ratio = errs[0] / errs[1]
    assert 0.85 * 2 ** order <= ratio <= 1.15 * 2 ** order


def test_order_two_is_the_seven_point_oracle():
    rng = np.random.default_rng(11)
    u = rng.standard_normal((8, 8, 8))
    f = rng.standard_normal((8, 8, 8))
    assert np.allclose(ho.lap(u, 0.5, 2), stencil.lap7(u, 0.5), rtol=0, atol=1e-12)
    a, ia = ho.solve_level(f, 0.5, 2, tol=1e-12)
    b, ib = periodic.solve_level(f, 0.5, tol=1e-12)
    assert ia["cycles"] == ib["cycles"]
    assert np.max(np.abs(a - b)) <= 1e-12 * np.max(np.abs(b))


@pytest.mark.parametrize("order", [4, 6])
@pytest.mark.parametrize("colour", [0, 1])
def test_half_sweep_solves_each_cells_equation_with_frozen_neighbours(order, colour):
    # N = 8 >= 2R + 1, so no offset wraps onto the cell itself
    rng = np.random.default_rng(3 + order + colour)
    N, h = 8, 0.3
    u = rng.standard_normal((N, N, N))
    f = rng.standard_normal((N, N, N))
    got = ho.rbgs_half(u, f, h, order, colour)
    i, j, k = np.indices(u.shape)
    mine = ((i + j + k) % 2) == colour
    assert np.array_equal(got[~mine], u[~mine])
    for c in zip(*np.nonzero(mine)):
        v0 = u.copy()
        v1 = u.copy()
        v1[c] += 1.0
        L0, L1 = ho.lap(v0, h, order)[c], ho.lap(v1, h, order)[c]
        want = u[c] + (f[c] - L0) / (L1 - L0)
        assert abs(got[c] - want) <= 1e-12 * max(1.0, abs(want))


@pytest.mark.parametrize("order", [4, 6])
def test_exact_solution_is_a_fixed_point_of_the_smoother(order):
    rng = np.random.default_rng(order)
    N, h = 16, 1.0 / 16
    f = rng.standard_normal((N, N, N))
    f -= f.mean()
    u = ho.fft_solve(f, h, order)
    assert np.max(np.abs(ho.lap(u, h, order) - f)) <= 1e-11 * np.max(np.abs(f))
    v = ho.rbgs_sweep(u, f, h, order)
    assert np.max(np.abs(v - u)) <= 1e-13 * np.max(np.abs(u))


@pytest.mark.parametrize("order", [4, 6])
@pytest.mark.parametrize("N", [16, 32])
def test_fas_solve_reaches_the_exact_solution_a_decade_per_cycle(order, N):
    rng = np.random.default_rng(100 * order + N)
    h = 1.0 / N
    f = rng.standard_normal((N, N, N)) + 0.7
    u, info = ho.solve_level(f, h, order, tol=1e-12)
    assert info["rel_res"] <= 1e-12
    assert abs(info["f_mean"] - float(np.mean(f))) <= 1e-15
    exact = ho.fft_solve(f - np.mean(f), h, order)
    assert np.max(np.abs(u - exact)) <= 1e-10 * np.max(np.abs(exact))
    assert abs(float(np.mean(u))) <= 1e-15 * np.max(np.abs(u))
    hist = info["history"]
    assert all(hist[c + 1] <= 0.1 * hist[c] for c in range(len(hist) - 1) if hist[c] > 1e-14)


def test_odd_coarsest_grid_and_fixed_cycles():
    # 24 = 8 * 3 coarsens to a 3^3 grid, which is solved exactly; fixed cycles ignore the tolerance
    rng = np.random.default_rng(9)
    N, h = 24, 1.0 / 24
    f = rng.standard_normal((N, N, N))
    u, info = ho.solve_level(f, h, 4, tol=1e-10)
    exact = ho.fft_solve(f - f.mean(), h, 4)
    assert np.max(np.abs(u - exact)) <= 1e-8 * np.max(np.abs(exact))
    _, fx = ho.solve_level(f, h, 4, tol=1.0, max_cycles=3, fixed_cycles=True)
    assert fx["cycles"] == 3 and len(fx["history"]) == 3
