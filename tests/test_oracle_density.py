"""Pins for the multi-scale density field of Sections 2.1-2.3 (oracle/density.py).

Independent routes: closed-form Gaussian transforms, brute-force convolution sums and child-pair
means by explicit loops, band-limited trigonometric fields, polynomial exactness, and a comparison
of the nested field with the full-resolution periodic field built from the same noise.
"""

import numpy as np
import pytest

from oracle import density
from oracle.zoom import Hierarchy
from paper_1103_6031_amd import inputs


def _gauss_table(sigma, r_max=40.0, count=1 << 16):
    dr = r_max / count
    r = np.arange(count) * dr
    return (2 * np.pi * sigma ** 2) ** -1.5 * np.exp(-r * r / (2 * sigma ** 2)), dr


def test_radial_table_of_a_gaussian_spectrum():
    """inputs.radial_transfer_table: T~ = exp(-k^2 s^2 / 2) (with the k_c cut folded in) has the
    closed-form transform (2 pi sig^2)^(-3/2) exp(-r^2 / (2 sig^2)), sig^2 = s^2 + 1 / k_c^2."""
    s, h = 0.7, 0.1
    kc = 2 * np.pi / h
    table, dr = inputs.radial_transfer_table(1.0, h, spectrum=lambda k: np.exp(-(k * s) ** 2), r_max=40.0,
                                             count=1 << 16)
    sig2 = s * s + 1.0 / kc ** 2
    r = np.arange(len(table)) * dr
    want = (2 * np.pi * sig2) ** -1.5 * np.exp(-r * r / (2 * sig2))
    np.testing.assert_allclose(table[:20000], want[:20000], atol=1e-9 * want[0])


def test_unigrid_convolution_is_the_direct_sum():
    """Section 2.2 on a periodic 4^3 grid: delta(a) = sum_b h^3 T(|a - b| wrapped) mu(b)."""
    rng = np.random.default_rng(1)
    N, h = 4, 0.5
    table = rng.standard_normal(64)
    dr = 0.1
    H = Hierarchy(N, h)
    xi = [rng.standard_normal((N,) * 3)]
    delta, mu, T = density.multiscale_density(H, table, dr, xi, subgrid=False)
    want = np.zeros((N,) * 3)
    for a in np.ndindex(N, N, N):
        for b in np.ndindex(N, N, N):
            d = [(a[i] - b[i]) % N for i in range(3)]
            d = [v if v < N // 2 else v - N for v in d]
            r = h * np.sqrt(sum(v * v for v in d))
            t = r / dr
            i = int(np.floor(t))
            w = t - i
            want[a] += h ** 3 * ((1 - w) * table[i] + w * table[i + 1]) * mu[0][b]
    np.testing.assert_allclose(delta[0], want, atol=1e-12)
    np.testing.assert_allclose(mu[0], xi[0] / h ** 1.5, atol=0)


def test_kernel_restriction_is_the_mean_over_child_pairs():
    """eq. transfer_average as read: coarse T(J) = mean over the 8 children a of the target and
    the 8 children b of the source (coarse cell 0) of the fine kernel at a - b."""
    rng = np.random.default_rng(2)
    Pf = (8, 16, 8)
    fine = rng.standard_normal(Pf)
    table = np.linspace(1.0, 0.0, 4096)
    coarse = density.kernel_restrict(fine, (8, 8, 8), 1.0, table, 0.01)
    for J in [(0, 0, 0), (1, -2, 1), (-1, 3, 0), (1, 1, -1)]:
        acc = 0.0
        for a in np.ndindex(2, 2, 2):
            for b in np.ndindex(2, 2, 2):
                idx = tuple((2 * J[i] + a[i] - b[i]) % Pf[i] for i in range(3))
                acc += fine[idx]
        got = coarse[tuple(J[i] % 8 for i in range(3))]
        assert abs(got - acc / 64.0) < 1e-14
    # outside the finer kernel's reach (|J_x| = 2 > 8/4 - 1): T sampled directly at |D|
    r = np.sqrt(4.0 + 0.0 + 0.0)
    assert abs(coarse[2, 0, 0] - density.radial(table, 0.01, r)) < 1e-15


def test_subgrid_kernel_transform_carries_the_cos_window():
    """Section 3.5.3: the 8-sub-cell mean multiplies the kernel's transform by prod cos(k h / 4)."""
    sigma, h, N = 2.0, 1.0, 32
    table, dr = _gauss_table(sigma)
    plain = density.kernel_direct((N,) * 3, h, table, dr, subgrid=False)
    sub = density.kernel_direct((N,) * 3, h, table, dr, subgrid=True)
    k = 2 * np.pi * np.fft.fftfreq(N, d=h)
    kx, ky, kz = np.meshgrid(k, k, k, indexing="ij")
    cont = np.exp(-0.5 * sigma ** 2 * (kx ** 2 + ky ** 2 + kz ** 2))
    win = np.cos(kx * h / 4) * np.cos(ky * h / 4) * np.cos(kz * h / 4)
    Fp = np.real(np.fft.fftn(plain)) * h ** 3
    Fs = np.real(np.fft.fftn(sub)) * h ** 3
    low = (np.abs(kx) < 1.0) & (np.abs(ky) < 1.0) & (np.abs(kz) < 1.0)
    np.testing.assert_allclose(Fp[low], cont[low], atol=2e-4)
    # the ratio tests the window itself (the sampled Gaussian's own aliasing cancels in it)
    np.testing.assert_allclose(Fs[low] / Fp[low], win[low], atol=2e-4)


def test_mode_replacement_reproduces_band_limited_parent():
    """Section 2.3.1: with zero fine noise, the refined noise on the padded domain is the parent's
    band-limited trigonometric field evaluated at the fine cell centres."""
    N0, n, off = 16, 8, 4
    H = Hierarchy(N0, 1.0, [((n,) * 3, (off,) * 3)])
    lo = off - n // 4
    m = np.array([1, -2, 3])
    I = np.arange(N0) - lo + 0.5
    X = np.meshgrid(I, I, I, indexing="ij")
    phase = 0.4
    parent = np.cos(2 * np.pi * sum(mi * xi for mi, xi in zip(m, X)) / n + phase)
    xi = [parent * H.h[0] ** 1.5, np.zeros((2 * n,) * 3)]
    mu = density.refine_noise(H, xi)
    i = (np.arange(2 * n) + 0.5) / 2.0
    x = np.meshgrid(i, i, i, indexing="ij")
    want = np.cos(2 * np.pi * sum(mi * xi_ for mi, xi_ in zip(m, x)) / n + phase)
    np.testing.assert_allclose(mu[1], want, atol=1e-12)
    # reverse Hoffman-Ribak: covered parent cells hold the mean of their children
    c = mu[1][n // 2:3 * n // 2, n // 2:3 * n // 2, n // 2:3 * n // 2]
    m8 = c.reshape(n // 2, 2, n // 2, 2, n // 2, 2).mean(axis=(1, 3, 5))
    np.testing.assert_allclose(mu[0][H.covered(1)], m8, atol=1e-14)


def test_refined_noise_keeps_eight_times_the_parent_variance():
    rng = np.random.default_rng(4)
    N0, n = 32, 16
    H = Hierarchy(N0, 2.0, [((n,) * 3, (8,) * 3)])
    xi = [rng.standard_normal((N0,) * 3), rng.standard_normal((2 * n,) * 3)]
    mu = density.refine_noise(H, xi)
    v0 = np.var(xi[0] / H.h[0] ** 1.5)
    v1 = np.var(mu[1])
    assert abs(v1 / (8 * v0) - 1.0) < 0.05


def test_conservative_tricubic_exactness_and_conservation():
    N0, n, off = 16, 16, 4
    H = Hierarchy(N0, 1.0, [((n,) * 3, (off,) * 3), ((8,) * 3, (4,) * 3)])
    X = np.meshgrid(*[np.arange(N0) + 0.5] * 3, indexing="ij")
    # linear field away from the wrap: exact at the fine centres
    U = 0.3 * X[0] - 0.2 * X[1] + 0.7 * X[2]
    fine = density.interpolate_conservative(H, 1, U)
    x = np.meshgrid(*[off + (np.arange(n) + 0.5) / 2 for _ in range(3)], indexing="ij")
    np.testing.assert_allclose(fine, 0.3 * x[0] - 0.2 * x[1] + 0.7 * x[2], atol=1e-12)
    # a cubic along x: tri-cubic exact at the fine centres, then shifted by the parent value minus
    # the children's mean
    U3 = X[0] ** 3
    fine3 = density.interpolate_conservative(H, 1, U3)
    xf = x[0]
    Xc = np.floor(xf) + 0.5
    shift = Xc ** 3 - 0.5 * ((Xc - 0.25) ** 3 + (Xc + 0.25) ** 3)
    np.testing.assert_allclose(fine3, xf ** 3 + shift, atol=1e-10)
    # conservation on a patch inside a patch, random data
    V = np.random.default_rng(5).standard_normal((n,) * 3)
    f2 = density.interpolate_conservative(H, 2, V)
    m8 = f2.reshape(4, 2, 4, 2, 4, 2).mean(axis=(1, 3, 5))
    np.testing.assert_allclose(m8, V[H.covered(2)], atol=1e-14)


def test_nested_field_matches_full_resolution_field():
    """One refinement level whose padded domain is the whole box: the nested density on the patch
    is close to the full-resolution periodic convolution of the same refined noise (the coarse
    contributions approximate the noise outside the patch at coarse resolution).  A missing or
    sign-flipped contribution (delta_bnd, delta_coarse) gives errors of order one."""
    sigma = 3.0
    table, dr = _gauss_table(sigma, r_max=80.0, count=1 << 17)
    N0, n, off = 16, 16, 4
    H = Hierarchy(N0, 2.0, [((n,) * 3, (off,) * 3)])
    rng = np.random.default_rng(6)
    xi = [rng.standard_normal((N0,) * 3), rng.standard_normal((2 * n,) * 3)]
    delta, mu, T = density.multiscale_density(H, table, dr, xi, subgrid=False)
    # full resolution: the refined noise lives on the whole (periodic) fine grid here
    ref = np.real(np.fft.ifftn(np.fft.fftn(mu[1]) * np.fft.fftn(T[1]))) * H.h[1] ** 3
    ps = tuple(slice(n // 2, 3 * n // 2) for _ in range(3))
    err = delta[1] - ref[ps]
    rel = np.sqrt(np.mean(err ** 2)) / np.sqrt(np.mean(ref[ps] ** 2))
    assert rel < 0.05, rel
    # without the boundary term the error is large
    H1 = H
    inside = np.zeros(mu[1].shape, dtype=bool)
    inside[ps] = True
    nu_self = np.where(inside, mu[1], 0.0)
    d_self = np.real(np.fft.ifftn(np.fft.fftn(nu_self) * np.fft.fftn(T[1]))) * H1.h[1] ** 3
    rel_self = np.sqrt(np.mean((d_self[ps] - ref[ps]) ** 2)) / np.sqrt(np.mean(ref[ps] ** 2))
    assert rel_self > 4 * rel
    # composite: covered base cells are the means of their children
    m8 = delta[1].reshape(8, 2, 8, 2, 8, 2).mean(axis=(1, 3, 5))
    np.testing.assert_allclose(delta[0][H.covered(1)], m8, atol=1e-15)


def test_geometry_checks():
    with pytest.raises(ValueError):
        density.check_geometry(Hierarchy(12, 1.0))
    with pytest.raises(ValueError):
        density.check_geometry(Hierarchy(32, 1.0, [((12, 12, 12), (8, 8, 8))]))
    # the padded domain of the second patch leaves the first
    with pytest.raises(ValueError):
        density.check_geometry(Hierarchy(64, 1.0, [((32,) * 3, (16,) * 3), ((32,) * 3, (4,) * 3)]))
    density.check_geometry(Hierarchy(32, 1.0, [((16,) * 3, (8,) * 3), ((8,) * 3, (4,) * 3)]))


def _m8(v):
    a, b, c = v.shape
    return v.reshape(a // 2, 2, b // 2, 2, c // 2, 2).mean(axis=(1, 3, 5))


def _inj(c):
    return np.repeat(np.repeat(np.repeat(c, 2, 0), 2, 1), 2, 2)


def test_two_levels_match_full_resolution_field():
    """Two refinement levels (Section 2.3.4), noise built consistent by construction: the first
    patch's padding carries no sub-coarse fluctuation (the one thing the paper's sum of coarse
    contributions does not pass down), every 8-child group averages to its parent.  Then patch 2's
    density is close to the full-resolution field of the same noise; dropping the parent's own
    coarse term (delta_coarse of the parent patch) makes the error about 0.5."""
    sigma = 3.0
    table, dr = _gauss_table(sigma, r_max=80.0, count=1 << 17)
    H = Hierarchy(16, 2.0, [((16,) * 3, (4,) * 3), ((16,) * 3, (4,) * 3)])
    rng = np.random.default_rng(7)

    def fluct(shape, s):
        e = rng.standard_normal(shape) * s
        return e - _inj(_m8(e))

    mu0 = rng.standard_normal((16,) * 3) / H.h[0] ** 1.5
    mu1 = _inj(mu0)                                    # D'_1 is the whole box
    p1 = tuple(slice(8, 24) for _ in range(3))         # patch 1 inside D'_1
    mu1[p1] += fluct((16,) * 3, 1 / H.h[1] ** 1.5)
    mu2 = _inj(mu1[p1]) + fluct((32,) * 3, 1 / H.h[2] ** 1.5)   # D'_2 is patch 1
    mu1[12:20, 12:20, 12:20] = _m8(mu2[8:24, 8:24, 8:24])
    mu0[4:12, 4:12, 4:12] = _m8(mu1[8:24, 8:24, 8:24])
    T = density.kernels(H, table, dr, subgrid=False)
    delta = density.convolve_levels(H, T, [mu0, mu1, mu2])
    nu = _inj(mu1)
    nu[16:48, 16:48, 16:48] = mu2
    K = density.kernel_direct((64,) * 3, H.h[2], table, dr, subgrid=False)
    ref = np.real(np.fft.ifftn(np.fft.fftn(nu) * np.fft.fftn(K))) * H.h[2] ** 3
    r = ref[24:40, 24:40, 24:40]
    rel = np.sqrt(np.mean((delta[2] - r) ** 2)) / np.sqrt(np.mean(r ** 2))
    assert rel < 0.06, rel
