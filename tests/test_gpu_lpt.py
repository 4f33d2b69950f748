"""LPT (displacements and the second-order source) on the GPU against the oracle."""

import numpy as np
import pytest

from gpu_util import needs_gpu, note, to_dev, to_host, rel_rms, rel_max
from oracle import lpt, zoom, periodic
from paper_1103_6031_amd import inputs

pytestmark = [pytest.mark.gpu, needs_gpu]


@pytest.fixture(scope="module")
def mg():
    from paper_1103_6031_amd import mgic
    return mgic


# 2: the smallest base (stencil offsets wrap once); 20: a partial group of rows in the row-group
# kernels; 64: 8 groups per plane; 128: the x-marched tiles
@pytest.mark.parametrize("N", [2, 4, 8, 16, 20, 48, 64, 128])
def test_periodic_grad_and_tau_bit_exact(mg, N):
    rng = np.random.default_rng(N)
    phi = rng.standard_normal((N, N, N))
    h = 100.0 / N
    note("periodic grad/tau N=%d" % N)
    Hg = mg.Hier(N, h)
    psi = mg.lpt_displacements(Hg, [to_dev(phi)], scale=-0.7)[0]
    pe = lpt.displacement(phi, h, scale=-0.7)
    for c in range(3):
        assert np.array_equal(to_host(psi[c]), pe[c])
    t = mg.lpt2_source(Hg, [to_dev(phi)])[0]
    te = lpt.tau(phi, h)
    te = te - te.mean()
    assert rel_max(to_host(t), te) < 1e-14


@pytest.mark.parametrize("layout", [
    (16, [((16, 16, 16), (4, 4, 4))]),
    (32, [((32, 32, 32), (8, 8, 8)), ((24, 16, 32), (4, 8, 8))]),
])
def test_hierarchy_grad_and_tau_match_oracle(mg, layout):
    N0, patches = layout
    H = zoom.Hierarchy(N0, 100.0 / N0, patches)
    Hg = mg.Hier(N0, 100.0 / N0, patches)
    rng = np.random.default_rng(4)
    phi = [rng.standard_normal(n) for n in H.n]
    note("hierarchy grad/tau N0=%d P=%d" % (N0, H.P))
    psi = mg.lpt_displacements(Hg, [to_dev(a) for a in phi], scale=1.5)
    pe = zoom.displacement_hierarchy(H, phi, scale=1.5)
    for p in range(H.P + 1):
        for c in range(3):
            assert rel_max(to_host(psi[p][c]), pe[p][c]) < 1e-13
    t = mg.lpt2_source(Hg, [to_dev(a) for a in phi])
    te = zoom.tau_hierarchy(H, phi)
    for p in range(H.P + 1):
        assert rel_max(to_host(t[p]), te[p]) < 1e-12
    assert abs(zoom.composite_sum(H, [to_host(x) for x in t])) < 1e-12 * zoom.composite_sum(
        H, [np.abs(x) for x in te])


def test_2lpt_chain_on_gpu_matches_oracle(mg):
    """phi1 = solve(delta), psi1 = -G phi1, tau, phi2 = solve(tau), psi2 = D2 G phi2 (D2 = -3/7)."""
    N = 32
    h = 100.0 / N
    f = inputs.gaussian_field(N, 31)
    note("2LPT chain N=%d" % N)
    Hg = mg.Hier(N, h)
    o = mg.make_opts(tol=1e-10)
    phi1, _ = mg.mg_solve_level(to_dev(f), h, opts=o)
    psi1 = mg.lpt_displacements(Hg, [phi1], scale=-1.0)[0]
    tau = mg.lpt2_source(Hg, [phi1])[0]
    phi2, _ = mg.mg_solve_level(tau, h, opts=o)
    psi2 = mg.lpt_displacements(Hg, [phi2], scale=-3.0 / 7.0)[0]
    e1, _ = periodic.solve_level(f, h, tol=1e-10)
    te = lpt.tau(e1, h)
    e2, _ = periodic.solve_level(te, h, tol=1e-10)
    assert rel_rms(to_host(phi1), e1) < 1e-10
    assert rel_rms(to_host(tau), te - te.mean()) < 1e-9
    assert rel_rms(to_host(phi2), e2) < 1e-9
    p1 = lpt.displacement(e1, h, -1.0)
    p2 = lpt.displacement(e2, h, -3.0 / 7.0)
    for c in range(3):
        assert rel_rms(to_host(psi1[c]), p1[c]) < 1e-10
        assert rel_rms(to_host(psi2[c]), p2[c]) < 1e-9


def test_plane_wave_tau_vanishes_on_gpu(mg):
    N = 32
    x = np.indices((N, N, N))
    phi = 0.3 * np.cos(2 * np.pi * (x[0] + 2 * x[1] + 3 * x[2]) / N)
    note("plane wave tau")
    t = mg.lpt2_source(mg.Hier(N, 1.0), [to_dev(phi)])[0]
    assert np.max(np.abs(to_host(t))) < 1e-13


@pytest.mark.parametrize("layout", ["periodic", "periodic128", "deep"])
def test_displacements_and_source_in_one_call(mg, layout):
    """psi and tau from the combined entry point equal the separate calls: bit for bit with
    scale -1, within rounding with another scale (128^3: the x-marched tile kernels)."""
    if layout.startswith("periodic"):
        N = 128 if layout == "periodic128" else 32
        Hg = mg.Hier(N, 100.0 / N)
        phi = [to_dev(inputs.gaussian_field(N, 41))]
    else:
        patches = [((16, 16, 16), (4, 4, 4)), ((12, 12, 16), (4, 4, 4))]
        Hg = mg.Hier(16, 100.0 / 16, patches)
        f = inputs.nested_fields(16, patches, 43)
        phi, _ = mg.mg_solve_hierarchy(Hg, [to_dev(a) for a in f], opts=mg.make_opts(tol=1e-12, max_cycles=60))
    note("combined displacements and tau, %s" % layout)
    for scale, exact in ((-1.0, True), (-3.0 / 7.0, False)):
        psi, tau = mg.lpt_displacements_and_source(Hg, phi, scale=scale)
        psi_s = mg.lpt_displacements(Hg, phi, scale=scale)
        tau_s = mg.lpt2_source(Hg, phi)
        for p in range(Hg.nlev):
            for c in range(3):
                assert np.array_equal(to_host(psi[p][c]), to_host(psi_s[p][c]))
            if exact:
                assert np.array_equal(to_host(tau[p]), to_host(tau_s[p]))
            else:
                assert rel_max(to_host(tau[p]), to_host(tau_s[p])) <= 1e-13


# the sixth-order gradient of Table 1 (grad_order = 6)
@pytest.mark.parametrize("N", [4, 8, 20, 64, 128])
def test_periodic_sixth_order_grad_and_tau(mg, N):
    rng = np.random.default_rng(600 + N)
    phi = rng.standard_normal((N, N, N))
    h = 100.0 / N
    note("periodic sixth-order grad/tau N=%d" % N)
    Hg = mg.Hier(N, h)
    psi = mg.lpt_displacements(Hg, [to_dev(phi)], scale=-0.7, grad_order=6)[0]
    pe = lpt.displacement(phi, h, scale=-0.7, order=6)
    for c in range(3):
        assert rel_max(to_host(psi[c]), pe[c]) < 1e-14
    t = mg.lpt2_source(Hg, [to_dev(phi)], grad_order=6)[0]
    te = lpt.tau(phi, h, order=6)
    te = te - te.mean()
    assert rel_max(to_host(t), te) < 1e-13
    # the combined call, its tau from the displacements themselves
    psi2, t2 = mg.lpt_displacements_and_source(Hg, [to_dev(phi)], scale=-1.0, grad_order=6)
    assert rel_max(to_host(t2[0]), te) < 1e-13
    for c in range(3):
        assert rel_max(to_host(psi2[0][c]), lpt.displacement(phi, h, -1.0, order=6)[c]) < 1e-14


@pytest.mark.parametrize("layout", [
    (16, [((16, 16, 16), (4, 4, 4))]),
    (32, [((32, 32, 32), (8, 8, 8)), ((24, 16, 32), (4, 8, 8))]),
])
def test_hierarchy_sixth_order_grad_and_tau_match_oracle(mg, layout):
    N0, patches = layout
    H = zoom.Hierarchy(N0, 100.0 / N0, patches)
    Hg = mg.Hier(N0, 100.0 / N0, patches)
    rng = np.random.default_rng(14)
    phi = [rng.standard_normal(n) for n in H.n]
    note("hierarchy sixth-order grad/tau N0=%d P=%d" % (N0, H.P))
    psi = mg.lpt_displacements(Hg, [to_dev(a) for a in phi], scale=1.5, grad_order=6)
    pe = zoom.displacement_hierarchy(H, phi, scale=1.5, order=6)
    for p in range(H.P + 1):
        for c in range(3):
            assert rel_max(to_host(psi[p][c]), pe[p][c]) < 1e-13
    t = mg.lpt2_source(Hg, [to_dev(a) for a in phi], grad_order=6)
    te = zoom.tau_hierarchy(H, phi, order=6)
    for p in range(H.P + 1):
        assert rel_max(to_host(t[p]), te[p]) < 1e-12
    psi2, t2 = mg.lpt_displacements_and_source(Hg, [to_dev(a) for a in phi], scale=1.5, grad_order=6)
    for p in range(H.P + 1):
        assert rel_max(to_host(t2[p]), te[p]) < 1e-12
        for c in range(3):
            assert np.array_equal(to_host(psi2[p][c]), to_host(psi[p][c]))
