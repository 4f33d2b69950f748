"""Oracle operators pinned to Table 1 / Table 2 of the paper and to closed forms."""

import numpy as np
import pytest

from oracle import stencil, periodic


def _delta_response(op, N=16, axis=0):
    u = np.zeros((N, N, N))
    c = N // 2
    u[c, c, c] = 1.0
    out = op(u)
    line = [out[tuple(c + d if a == axis else c for a in range(3))] for d in range(-3, 4)]
    return np.array(line)


def test_laplacian_stencil_matches_table1(golden):
    """A unit impulse reproduces Table 1's order-2 stencil along each axis (h = 1)."""
    w = golden["table1_laplacian"]["2"]
    expect1d = np.array([0, 0] + w["weights"] + [0, 0], dtype=float) * w["scale"]
    for axis in range(3):
        line = _delta_response(lambda u: stencil.lap7(u, 1.0), axis=axis)
        off_centre = line.copy()
        off_centre[3] = 0
        exp = expect1d.copy()
        exp[3] = 0
        assert np.array_equal(off_centre, exp)
    # the 3-D centre weight is the sum of the three 1-D centre weights
    line = _delta_response(lambda u: stencil.lap7(u, 1.0))
    assert line[3] == 3 * w["weights"][1] * w["scale"]


def test_gradient_stencil_matches_table1(golden):
    """Impulse response of grad4 is Table 1's order-4 gradient, mirrored (correlation)."""
    w = golden["table1_gradient"]["4"]
    for axis in range(3):
        line = _delta_response(lambda u: stencil.grad4(u, 1.0, axis), axis=axis)
        # out[i] = sum_d w_d u[i+d]  =>  response at offset -d is w_d
        exp = np.array([0] + list(reversed(w["weights"])) + [0], dtype=float) * w["scale"]
        assert np.allclose(line, exp, rtol=0, atol=1e-15)


@pytest.mark.parametrize("N", [8, 12, 16])
def test_laplacian_single_modes_match_symbol(N):
    """Table 1 order-2 symbol -2(1 - cos k) per axis is the eigenvalue on every Fourier mode."""
    h = 0.37
    x = np.indices((N, N, N))
    rng = np.random.default_rng(N)
    for _ in range(6):
        m = rng.integers(-N // 2, N // 2 + 1, size=3)
        phase = 2 * np.pi * sum(m[a] * x[a] for a in range(3)) / N
        for f in (np.cos(phase), np.sin(phase)):
            k = 2 * np.pi * m / N
            lam = -(2.0 / h ** 2) * np.sum(1 - np.cos(k))
            assert np.allclose(stencil.lap7(f, h), lam * f, rtol=0, atol=1e-11 * max(1, abs(lam)))


@pytest.mark.parametrize("N", [8, 16])
def test_gradient_single_modes_match_symbol(N):
    """Table 1 order-4 gradient symbol (i/6)(8 sin k - sin 2k) on sine/cosine modes."""
    h = 0.5
    x = np.indices((N, N, N))
    for m in [(1, 0, 0), (0, 3, 0), (2, 1, 5), (N // 2, 0, 1)]:
        phase = 2 * np.pi * sum(m[a] * x[a] for a in range(3)) / N
        f = np.sin(phase)
        for axis in range(3):
            k = 2 * np.pi * m[axis] / N
            g = (8 * np.sin(k) - np.sin(2 * k)) / 6.0 / h
            assert np.allclose(stencil.grad4(f, h, axis), g * np.cos(phase), atol=1e-12)


def test_flux_operator_order1_gives_laplacian_order2(golden):
    """Table 2: order-1 flux [-1 1] convolved with [-1 1] is Table 1's order-2 Laplacian."""
    F = np.array(golden["table2_flux"]["1"]["weights"], dtype=float)
    conv = np.convolve(F, [-1.0, 1.0])
    L2 = np.array(golden["table1_laplacian"]["2"]["weights"], dtype=float)
    assert np.array_equal(conv, L2)


def test_attenuation_order2_at_half_nyquist(golden):
    """Section 3.4.1: order-2 L and G attenuate by ~78% at k_Ny/2 (exactly pi/4)."""
    N, h = 8, 1.0
    m = 2                              # k h = pi/2 = k_Ny / 2
    x = np.indices((N, N, N))[0]
    f = np.cos(2 * np.pi * m * x / N)
    phi = periodic.fft_solve(f, h)
    wg = golden["table1_gradient"]["2"]
    g2 = wg["scale"] * sum(wd * np.roll(phi, -d, 0) for d, wd in zip((-1, 0, 1), wg["weights"]))
    k = 2 * np.pi * m / (N * h)
    exact = -np.sin(2 * np.pi * m * x / N) * (-1.0 / k)   # d/dx of (-f/k^2)
    ratio = g2[1, 0, 0] / exact[1, 0, 0]
    ref = golden["attenuation_kny_half_order2"]
    assert abs(ratio - ref["value"]) < ref["tolerance"]
    assert abs(ratio - np.pi / 4) < 1e-12
    # the build's 4th-order gradient over the 2nd-order Laplacian: 1.0472 (>1, overshoot)
    g4 = stencil.grad4(phi, h, 0)
    assert abs(g4[1, 0, 0] / exact[1, 0, 0] - np.pi / 3) < 1e-12


def test_restriction_and_injection_geometry():
    """Cell-centred children sit at -+1/4 H from the parent centre (Fig. grid_structure)."""
    N = 8
    h = 1.0 / N
    xc = (np.indices((N, N, N)) + 0.5) * h
    lin = 3.0 * xc[0] - 2.0 * xc[1] + 0.5 * xc[2] + 1.0
    H = 2 * h
    Xc = (np.indices((N // 2,) * 3) + 0.5) * H
    lin_c = 3.0 * Xc[0] - 2.0 * Xc[1] + 0.5 * Xc[2] + 1.0
    assert np.allclose(stencil.restrict_mean8(lin), lin_c, atol=1e-14)
    rng = np.random.default_rng(3)
    c = rng.standard_normal((4, 4, 4))
    assert np.array_equal(stencil.restrict_mean8(stencil.inject(c)), c)
