"""Periodic path on the GPU (through the C ABI) against the oracle.

Bar: single kernels bit-exact where the arithmetic order is fixed (smoother), solves within
1e-10 relative RMS (FP64) and 1e-8 (mixed precision) of the oracle.
"""

import numpy as np
import pytest

from gpu_util import needs_gpu, note, to_dev, to_host, rel_rms, rel_max
from oracle import periodic, stencil
from paper_1103_6031_amd import inputs

pytestmark = [pytest.mark.gpu, needs_gpu]


@pytest.fixture(scope="module")
def mg():
    from paper_1103_6031_amd import mgic
    return mgic


# power-of-two sizes take the 16-byte-access half-sweep (4: one run is the whole half-row, its
# z-edge wraps onto itself), 48 and 160 the scalar one in flat block order, 96 the scalar one in
# plane-chunk order (8 blocks per x plane)
@pytest.mark.parametrize("N,half", [(4, 2), (8, 1), (16, 2), (32, 3), (48, 4), (96, 2), (128, 4), (160, 3)])
def test_smoother_bit_exact_fp64(mg, N, half):
    rng = np.random.default_rng(N + half)
    u0 = rng.standard_normal((N, N, N))
    f = rng.standard_normal((N, N, N))
    h = 100.0 / N
    note("smoother fp64 N=%d half=%d" % (N, half))
    ut = to_dev(u0)
    mg.mg_smooth_level(to_dev(f), ut, h, half)
    ue = u0.copy()
    for k in range(half):
        ue = periodic.rbgs_half(ue, f, h, k % 2)
    assert np.array_equal(to_host(ut), ue)


@pytest.mark.parametrize("N,half", [(4, 2), (8, 2), (16, 2), (64, 4), (96, 3), (256, 2)])
def test_smoother_fp32_bit_exact_against_float32_oracle(mg, N, half):
    rng = np.random.default_rng(7 * N)
    u0 = rng.standard_normal((N, N, N)).astype(np.float32)
    f = rng.standard_normal((N, N, N)).astype(np.float32)
    h = 100.0 / N
    note("smoother fp32 N=%d" % N)
    ut = to_dev(u0.astype(np.float64))
    mg.mg_smooth_level(to_dev(f.astype(np.float64)), ut, h, half, prec="mixed")
    ue = u0.copy()
    for k in range(half):
        ue = periodic.rbgs_half(ue, f, h, k % 2)
    assert ue.dtype == np.float32
    assert np.array_equal(to_host(ut).astype(np.float32), ue)


@pytest.mark.parametrize("N", [8, 16, 48, 64, 128])   # 64 and 128 take the fused 64^3 / 32^3 levels
def test_one_vcycle_matches_oracle(mg, N):
    f = inputs.gaussian_field(N, 11 + N)
    h = 100.0 / N
    note("one V-cycle N=%d" % N)
    u, st = mg.mg_solve_level(to_dev(f), h, opts=mg.make_opts(max_cycles=1, fixed_cycles=True))
    fz = f - f.mean()
    ue = periodic.vcycle(np.zeros_like(f), fz, h)
    ue -= ue.mean()
    assert st["cycles"] == 1
    assert rel_max(to_host(u), ue) < 1e-13


@pytest.mark.parametrize("N", [16, 24, 48, 64, 96])
def test_fp64_solve_matches_oracle(mg, N):
    f = inputs.gaussian_field(N, 100 + N) + 0.25     # non-zero mean is removed and reported
    h = 100.0 / N
    note("fp64 solve N=%d" % N)
    u, st = mg.mg_solve_level(to_dev(f), h, opts=mg.make_opts(tol=1e-10))
    ue, info = periodic.solve_level(f, h, tol=1e-10)
    ug = to_host(u)
    assert st["cycles"] == info["cycles"]
    assert abs(st["f_mean"] - info["f_mean"]) < 1e-14
    assert st["rel_res"] <= 1e-10
    assert rel_rms(ug, ue) <= 1e-10
    assert rel_rms(ug, periodic.fft_solve(f, h)) <= 1e-9
    hist = np.array(st["history"])
    ref = np.array(info["history"])
    assert np.allclose(hist[:4], ref[:4], rtol=1e-6)      # rounding-limited later on
    assert np.allclose(hist, ref, rtol=0.05)
    assert st["cell_updates"] == periodic.cell_updates(N, st["cycles"])


# the outer step takes pairs of cells (every valid base above 16^3 has even half-rows); 20, 40,
# 48 and 96 are not powers of two, so the z-edge of a pair wraps by comparison
@pytest.mark.parametrize("N", [20, 32, 40, 48, 64, 96])
def test_mixed_solve_matches_fp64_oracle(mg, N):
    f = inputs.gaussian_field(N, 200 + N)
    h = 100.0 / N
    note("mixed solve N=%d" % N)
    u, st = mg.mg_solve_level(to_dev(f), h, opts=mg.make_opts(tol=1e-10, prec="mixed", max_cycles=40))
    ue, _ = periodic.solve_level(f, h, tol=1e-12)
    assert st["rel_res"] <= 1e-10
    assert rel_rms(to_host(u), ue) <= 1e-8
    assert st["cycles"] <= 16


def test_c1_64cubed_workload(mg):
    """64^3 BBKS field, V(2,2) to 1e-10 relative residual."""
    f = inputs.c1_input()
    h = inputs.BOX / 64
    note("C1 64^3")
    u, st = mg.mg_solve_level(to_dev(f), h, opts=mg.make_opts(tol=1e-10))
    ue, info = periodic.solve_level(f, h, tol=1e-10)
    assert st["cycles"] == info["cycles"] <= 12
    assert rel_rms(to_host(u), ue) <= 1e-10


def test_errors_are_reported(mg):
    N = 16
    h = 1.0
    f = inputs.gaussian_field(N, 5)
    note("error paths")
    with pytest.raises(mg.MGError) as e:
        mg.mg_solve_level(to_dev(f), h, opts=mg.make_opts(tol=1e-14, max_cycles=1))
    assert e.value.code == mg.MG_ENOCONV and e.value.stats["cycles"] == 1
    bad = f.copy()
    bad[3, 4, 5] = np.nan
    with pytest.raises(mg.MGError) as e:
        mg.mg_solve_level(to_dev(bad), h, opts=mg.make_opts(max_cycles=5))
    assert e.value.code == mg.MG_EDIVERGED
    # the library still works after a failed call
    u, st = mg.mg_solve_level(to_dev(f), h)
    assert st["rel_res"] <= 1e-10


def test_nan_initial_guess_is_reported(mg):
    # a NaN in the initial guess ends the solve before any cycle runs on it, in both precisions,
    # on a single level (16^3: generic path, 32^3: fused mixed path), on a hierarchy and in a batch
    for prec in ("fp64", "mixed"):
        o = mg.make_opts(prec=prec, initial_guess=True, max_cycles=40)
        for N in (16, 32):
            h = 100.0 / N
            f = inputs.gaussian_field(N, 6)
            g = np.zeros_like(f)
            g[1, 2, 3] = np.nan
            note("NaN initial guess, level %d^3, %s" % (N, prec))
            with pytest.raises(mg.MGError) as e:
                mg.mg_solve_level(to_dev(f), h, u=to_dev(g), opts=o)
            assert e.value.code == mg.MG_EDIVERGED and e.value.stats["cycles"] == 0
        Hg = mg.Hier(N, h, [((8, 8, 8), (4, 4, 4))])
        fl = [to_dev(f), to_dev(np.ones((8, 8, 8)))]
        ul = [to_dev(g), to_dev(np.zeros((8, 8, 8)))]
        note("NaN initial guess, hierarchy, %s" % prec)
        with pytest.raises(mg.MGError) as e:
            mg.mg_solve_hierarchy(Hg, fl, u=ul, opts=o)
        assert e.value.code == mg.MG_EDIVERGED and e.value.stats["cycles"] == 0
        fb = inputs.gaussian_field(32, 7)

        def guesses():
            ub = [to_dev(np.zeros_like(fb)), to_dev(np.zeros_like(fb))]
            ub[1][0, 0, 1] = float("nan")
            return ub

        note("NaN initial guess, batch, %s" % prec)
        with pytest.raises(mg.MGError) as e:
            mg.mg_solve_batch([to_dev(fb), to_dev(fb)], [100.0 / 32] * 2, u=guesses(), opts=o)
        assert e.value.code == mg.MG_EDIVERGED
        _, sts = mg.mg_solve_batch([to_dev(fb), to_dev(fb)], [100.0 / 32] * 2, u=guesses(), opts=o, check=False)
        assert sts[1]["cycles"] == 0 and sts[0]["rel_res"] <= 1e-10


def test_warm_start_resumes(mg):
    N = 32
    h = 100.0 / N
    f = inputs.gaussian_field(N, 9)
    note("warm start")
    u, st1 = mg.mg_solve_level(to_dev(f), h, opts=mg.make_opts(tol=1e-4))
    u, st2 = mg.mg_solve_level(to_dev(f), h, u=u, opts=mg.make_opts(tol=1e-10, initial_guess=True))
    ue, info = periodic.solve_level(f, h, tol=1e-10)
    assert st1["cycles"] + st2["cycles"] <= info["cycles"] + 1
    assert rel_rms(to_host(u), ue) < 1e-9


def test_batch_equals_solo(mg):
    inst = inputs.c4_instances(count=6)
    fs = [inputs.c4_field(N, s, seed) for N, s, seed in inst]
    hs = [inputs.BOX / N for N, _, _ in inst]
    note("batch of %d" % len(inst))
    for prec in ("fp64", "mixed"):
        o = mg.make_opts(tol=1e-10, prec=prec, max_cycles=40)
        ub, sts = mg.mg_solve_batch([to_dev(f) for f in fs], hs, opts=o)
        for f, h, u, s in zip(fs, hs, ub, sts):
            us, _ = mg.mg_solve_level(to_dev(f), h, opts=o)
            assert np.array_equal(to_host(u), to_host(us))
            ue, _ = periodic.solve_level(f, h, tol=1e-12)
            assert rel_rms(to_host(u), ue) <= (1e-10 if prec == "fp64" else 1e-8)


@pytest.mark.parametrize("N", [32, 64])
def test_mixed_zero_start_stopping_at_once_returns_zero(mg, N):
    # the first outer step of a zero start leaves u = 0 implicit: a solve that stops right there
    # (a constant f is zero once its mean is removed; or no cycle allowed) must still return 0
    h = 100.0 / N
    note("mixed zero start, immediate stop, N=%d" % N)
    f = np.full((N, N, N), 2.5)
    u, st = mg.mg_solve_level(to_dev(f), h, opts=mg.make_opts(tol=1e-10, prec="mixed", max_cycles=40))
    assert st["cycles"] == 0 and st["f_mean"] == 2.5
    assert np.array_equal(to_host(u), np.zeros_like(f))
    g = inputs.gaussian_field(N, 4242)
    u0 = to_dev(np.full((N, N, N), 7.0))   # the output array starts non-zero
    u, st = mg.mg_solve_level(to_dev(g), h, u=u0, opts=mg.make_opts(prec="mixed", max_cycles=0, fixed_cycles=True))
    assert st["cycles"] == 0
    assert np.array_equal(to_host(u), np.zeros_like(g))
