"""LPT oracle (Section 3.1) pinned to closed forms for plane waves."""

import numpy as np
import pytest

from oracle import lpt, periodic


def _g4sym(k):
    return (8 * np.sin(k) - np.sin(2 * k)) / 6.0


@pytest.mark.parametrize("m", [(1, 0, 0), (1, 2, 0), (1, 1, 1), (2, 3, 1), (0, 5, 7)])
def test_plane_wave_has_zero_tau(m):
    """A single plane wave has a rank-one deformation tensor, so tau = 0 exactly."""
    N, h = 16, 0.7
    x = np.indices((N, N, N))
    phi = 0.3 * np.cos(2 * np.pi * sum(m[a] * x[a] for a in range(3)) / N + 0.4)
    t = lpt.tau(phi, h)
    assert np.max(np.abs(t)) < 1e-13


def test_two_wave_closed_form_and_second_solve():
    """phi = A cos(a.x) + B cos(b.x) => tau = A B cos(a.x) cos(b.x) |alpha x beta|^2."""
    N, h = 16, 0.5
    x = np.indices((N, N, N))
    ma, mb = np.array([1, 2, 0]), np.array([0, 1, 3])
    A, B = 0.7, -1.3
    pa = 2 * np.pi * sum(ma[i] * x[i] for i in range(3)) / N
    pb = 2 * np.pi * sum(mb[i] * x[i] for i in range(3)) / N
    phi = A * np.cos(pa) + B * np.cos(pb)
    alpha = _g4sym(2 * np.pi * ma / N) / h
    beta = _g4sym(2 * np.pi * mb / N) / h
    cross2 = float(np.sum(np.cross(alpha, beta) ** 2))
    t_exact = A * B * np.cos(pa) * np.cos(pb) * cross2
    t = lpt.tau(phi, h)
    assert np.max(np.abs(t - t_exact)) < 1e-12 * np.max(np.abs(t_exact))
    # second solve: tau = AB|axb|^2/2 [cos((a+b).x) + cos((a-b).x)]
    lam = lambda m: -(2 / h ** 2) * np.sum(1 - np.cos(2 * np.pi * m / N))
    phi2_exact = 0.5 * A * B * cross2 * (np.cos(pa + pb) / lam(ma + mb) + np.cos(pa - pb) / lam(ma - mb))
    phi2, _ = periodic.solve_level(t, h, tol=1e-13)
    assert np.max(np.abs(phi2 - phi2_exact)) < 1e-11 * np.max(np.abs(phi2_exact))


def test_paper_double_sum_equals_i_gt_j_form():
    """The paper's -1/2 sum_ij [D_ij^2 - D_ii D_jj] equals sum_{i>j} (D_ii D_jj - D_ij^2)."""
    rng = np.random.default_rng(4)
    phi = rng.standard_normal((12, 12, 12))
    a = lpt.tau(phi, 0.9)
    b = lpt.tau_paper_form(phi, 0.9)
    assert np.max(np.abs(a - b)) < 1e-12 * np.max(np.abs(a))


def test_displacement_of_single_mode():
    N, h = 16, 2.0
    x = np.indices((N, N, N))
    m = (2, 0, 1)
    ph = 2 * np.pi * sum(m[a] * x[a] for a in range(3)) / N
    phi = np.sin(ph)
    psi = lpt.displacement(phi, h, scale=-1.0)
    for a in range(3):
        g = _g4sym(2 * np.pi * m[a] / N) / h
        assert np.allclose(psi[a], -g * np.cos(ph), atol=1e-13)


def _g6sym(k):
    """Table 1, order 6: the printed symbol -(i/30)(sin 3k - 9 sin 2k + 45 sin k), without -i."""
    return (np.sin(3 * k) - 9 * np.sin(2 * k) + 45 * np.sin(k)) / 30.0


def test_sixth_order_gradient_is_the_printed_stencil(golden):
    g = golden["table1_gradient"]["6"]
    N, h = 16, 0.5
    e = np.zeros((N, N, N))
    e[8, 3, 5] = 1.0
    from oracle.stencil import grad6
    for axis in range(3):
        d = grad6(e, h, axis)
        # the gradient at cell i reads u[i + k] with weight w[k]: the impulse at i0 shows w[k] at i0 - k
        line = []
        for k in range(-3, 4):
            idx = [8, 3, 5]
            idx[axis] = (idx[axis] - k) % N
            line.append(d[tuple(idx)])
        assert np.allclose(np.array(line) * h, np.array(g["weights"], dtype=float) * g["scale"], atol=1e-15)


@pytest.mark.parametrize("m", [(1, 0, 0), (2, 3, 1), (0, 5, 7)])
def test_sixth_order_displacement_of_single_mode(m):
    N, h = 16, 2.0
    x = np.indices((N, N, N))
    ph = 2 * np.pi * sum(m[a] * x[a] for a in range(3)) / N
    psi = lpt.displacement(np.sin(ph), h, scale=-1.0, order=6)
    for a in range(3):
        assert np.allclose(psi[a], -_g6sym(2 * np.pi * m[a] / N) / h * np.cos(ph), atol=1e-13)


def test_sixth_order_gradient_converges_at_sixth_order():
    errs = []
    for N in (16, 32):
        h = 1.0 / N
        x = (np.arange(N) + 0.5) * h
        u = np.broadcast_to(np.sin(2 * np.pi * x)[:, None, None], (N, N, N)).copy()
        from oracle.stencil import grad6
        d = grad6(u, h, 0)
        errs.append(np.max(np.abs(d[:, 0, 0] - 2 * np.pi * np.cos(2 * np.pi * x))))
    assert 2 ** 6 * 0.85 < errs[0] / errs[1] < 2 ** 6 * 1.15


@pytest.mark.parametrize("m", [(1, 0, 0), (1, 1, 1), (2, 3, 1)])
def test_sixth_order_plane_wave_has_zero_tau(m):
    N, h = 16, 0.7
    x = np.indices((N, N, N))
    phi = 0.3 * np.cos(2 * np.pi * sum(m[a] * x[a] for a in range(3)) / N + 0.4)
    assert np.max(np.abs(lpt.tau(phi, h, order=6))) < 1e-13


def test_sixth_order_two_wave_closed_form():
    N, h = 16, 0.5
    x = np.indices((N, N, N))
    ma, mb = np.array([1, 2, 0]), np.array([0, 1, 3])
    A, B = 0.7, -1.3
    pa = 2 * np.pi * sum(ma[i] * x[i] for i in range(3)) / N
    pb = 2 * np.pi * sum(mb[i] * x[i] for i in range(3)) / N
    phi = A * np.cos(pa) + B * np.cos(pb)
    alpha = _g6sym(2 * np.pi * ma / N) / h
    beta = _g6sym(2 * np.pi * mb / N) / h
    t_exact = A * B * np.cos(pa) * np.cos(pb) * float(np.sum(np.cross(alpha, beta) ** 2))
    t = lpt.tau(phi, h, order=6)
    assert np.max(np.abs(t - t_exact)) < 1e-12 * np.max(np.abs(t_exact))
