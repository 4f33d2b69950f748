"""Batched periodic solves (mg_solve_batch) on the GPU.

Every instance of a batch must come out bit-identical to its own mg_solve_level solve (same
cycles, same residual history, same u), whatever else is in the batch, whether the launches are
replayed from graphs or issued directly, and on repeated calls that replay cached graphs.  The
full 64-instance workload is checked against the oracle's exact periodic solve.
"""

import math

import numpy as np
import pytest

from gpu_util import needs_gpu, note, to_dev, to_host, rel_rms
from oracle import periodic
from paper_1103_6031_amd import inputs

pytestmark = [pytest.mark.gpu, needs_gpu]


@pytest.fixture(scope="module")
def mg():
    from paper_1103_6031_amd import mgic
    return mgic


def _fields(sizes, seed0=500):
    fs = [inputs.gaussian_field(N, seed0 + i, spectrum=inputs.spectrum_power_law(-2.0)) for i, N in enumerate(sizes)]
    hs = [inputs.BOX / N for N in sizes]
    return fs, hs


def _same_stats(a, b):
    assert a["cycles"] == b["cycles"]
    assert a["cell_updates"] == b["cell_updates"]
    assert a["f_mean"] == b["f_mean"]
    ha, hb = np.array(a["history"]), np.array(b["history"])
    assert np.array_equal(np.isnan(ha), np.isnan(hb))
    assert np.array_equal(ha[~np.isnan(ha)], hb[~np.isnan(hb)])
    if math.isnan(b["rel_res"]):
        assert math.isnan(a["rel_res"])
    else:
        assert a["rel_res"] == b["rel_res"]


# 16^3 and 6^3 (odd coarsening 6 -> 3) are too small for the batched schedule and are solved on
# their own inside the call; the rest share the batched launches
SIZES = [32, 48, 16, 64, 20, 96, 24, 6, 40, 128]


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
@pytest.mark.parametrize("graph", [True, False])
def test_batch_bit_identical_to_solo(mg, prec, graph):
    fs, hs = _fields(SIZES)
    o = mg.make_opts(tol=1e-10, prec=prec, max_cycles=40, graph=graph)
    note("batch %s graph=%s sizes=%s" % (prec, graph, SIZES))
    ws = mg.Workspace(mg.mg_batch_workspace_bytes(SIZES, o))
    for rep in range(2):          # the second call replays the cached graphs
        ub, sts = mg.mg_solve_batch([to_dev(f) for f in fs], hs, opts=o, workspace=ws)
        for N, f, h, u, s in zip(SIZES, fs, hs, ub, sts):
            us, ss = mg.mg_solve_level(to_dev(f), h, opts=o)
            assert np.array_equal(to_host(u), to_host(us)), (N, rep)
            _same_stats(s, ss)


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
@pytest.mark.parametrize("nu", [(1, 1), (1, 2), (2, 1), (2, 2), (3, 1)])
def test_fused_levels_match_one_step_kernels(mg, prec, nu):
    """Solo solves run the 64^3, 32^3 and 16^3 coarsenings as fused tile launches (and the LDS
    tail from 8^3), batched instances run the one-step kernels and a tail from 16^3: the bits must
    agree for every sweep count the fused kernels take, and for one they do not take (both sides
    then run the one-step kernels)."""
    sizes = [32, 64, 128]
    fs, hs = _fields(sizes, seed0=950)
    o = mg.make_opts(prec=prec, max_cycles=4, fixed_cycles=True, nu1=nu[0], nu2=nu[1])
    note("fused levels %s nu=%s" % (prec, nu))
    ub, sts = mg.mg_solve_batch([to_dev(f) for f in fs], hs, opts=o)
    for N, f, h, u, s in zip(sizes, fs, hs, ub, sts):
        us, ss = mg.mg_solve_level(to_dev(f), h, opts=o)
        assert np.array_equal(to_host(u), to_host(us)), N
        _same_stats(s, ss)


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_full_size_instance_bit_identical(mg, prec):
    """A 256^3 instance: the solo solve takes the power-of-two kernels at 256^3 and 128^3 (16-byte
    half-sweeps, the correction folded into the first red half-sweep, the FAS right-hand side by
    runs, the residual-restriction by 4x4x4 neighbourhoods), the batched one the generic kernels."""
    sizes = [256, 32]
    fs, hs = _fields(sizes, seed0=990)
    o = mg.make_opts(prec=prec, max_cycles=3, fixed_cycles=True)
    note("256^3 instance, batch vs solo, %s" % prec)
    ub, sts = mg.mg_solve_batch([to_dev(f) for f in fs], hs, opts=o)
    for N, f, h, u, s in zip(sizes, fs, hs, ub, sts):
        us, ss = mg.mg_solve_level(to_dev(f), h, opts=o)
        assert np.array_equal(to_host(u), to_host(us)), N
        _same_stats(s, ss)


def test_batch_graph_equals_direct_repeated(mg):
    sizes = [64, 32, 96, 48]
    fs, hs = _fields(sizes, seed0=700)
    res = []
    for graph in (True, False, True):
        o = mg.make_opts(tol=1e-10, prec="mixed", max_cycles=40, graph=graph)
        note("batch graph=%s" % graph)
        ub, _ = mg.mg_solve_batch([to_dev(f) for f in fs], hs, opts=o)
        res.append([to_host(u) for u in ub])
    for a, b in zip(res[0], res[1]):
        assert np.array_equal(a, b)
    for a, b in zip(res[0], res[2]):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_batch_fixed_cycles_and_warm_start(mg, prec):
    sizes = [32, 64, 48]
    fs, hs = _fields(sizes, seed0=800)
    o = mg.make_opts(prec=prec, max_cycles=3, fixed_cycles=True)
    note("batch fixed cycles %s" % prec)
    ub, sts = mg.mg_solve_batch([to_dev(f) for f in fs], hs, opts=o)
    for f, h, u, s in zip(fs, hs, ub, sts):
        us, ss = mg.mg_solve_level(to_dev(f), h, opts=o)
        assert np.array_equal(to_host(u), to_host(us))
        assert s["cycles"] == ss["cycles"] == 3
    og = mg.make_opts(tol=1e-10, prec=prec, max_cycles=40, initial_guess=True)
    note("batch warm start %s" % prec)
    uw, stw = mg.mg_solve_batch([to_dev(f) for f in fs], hs, u=[x.clone() for x in ub], opts=og)
    for f, h, u0, u, s in zip(fs, hs, ub, uw, stw):
        us, ss = mg.mg_solve_level(to_dev(f), h, u=u0.clone(), opts=og)
        assert np.array_equal(to_host(u), to_host(us))
        _same_stats(s, ss)


def test_batch_with_a_bad_instance(mg):
    sizes = [32, 64, 48]
    fs, hs = _fields(sizes, seed0=900)
    fs[1] = fs[1].copy()
    fs[1][3, 4, 5] = np.nan
    o = mg.make_opts(tol=1e-10, prec="mixed", max_cycles=40)
    note("batch with a NaN instance")
    with pytest.raises(mg.MGError) as e:
        mg.mg_solve_batch([to_dev(f) for f in fs], hs, opts=o)
    assert e.value.code == mg.MG_EDIVERGED
    ub, sts = mg.mg_solve_batch([to_dev(f) for f in fs], hs, opts=o, check=False)
    for i in (0, 2):
        us, ss = mg.mg_solve_level(to_dev(fs[i]), hs[i], opts=o)
        assert np.array_equal(to_host(ub[i]), to_host(us))
        _same_stats(sts[i], ss)
    assert math.isnan(sts[1]["rel_res"])


def test_c4_batch_matches_oracle(mg):
    inst = inputs.c4_instances()
    sizes = [N for N, _, _ in inst]
    hs = [inputs.BOX / N for N in sizes]
    fs = [inputs.c4_field(N, s, seed) for N, s, seed in inst]
    o = mg.make_opts(tol=1e-10, prec="mixed", max_cycles=40)
    note("C4 batch: %d instances, %d cells" % (len(sizes), sum(N ** 3 for N in sizes)))
    ub, sts = mg.mg_solve_batch([to_dev(f) for f in fs], hs, opts=o)
    worst = 0.0
    for f, h, u, s in zip(fs, hs, ub, sts):
        assert s["rel_res"] <= 1e-10
        ue = periodic.fft_solve(f - f.mean(), h)
        worst = max(worst, rel_rms(to_host(u), ue))
    note("C4 worst rel RMS vs exact solve: %.3e" % worst)
    assert worst <= 1e-8


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_every_tuning_candidate_gives_the_same_bits(mg, prec, tmp_path):
    """The autotuner only picks a launch shape: each of its candidates (block size, cells per
    thread), forced at every depth, gives every instance the bits of its solo solve; the tuned
    shapes then persist in the JSON cache."""
    import json
    sizes = [32, 48, 64, 96, 128]
    fs, hs = _fields(sizes, seed0=700)
    o = mg.make_opts(tol=1e-10, prec=prec, max_cycles=40)
    solo = [mg.mg_solve_level(to_dev(f), h, opts=o) for f, h in zip(fs, hs)]
    ws = mg.Workspace(mg.mg_batch_workspace_bytes(sizes, o))
    try:
        for k in range(mg.mg_batch_tune_candidates()):
            note("batch %s forced candidate %d" % (prec, k))
            mg.mg_batch_force_shape(k)
            ub, sts = mg.mg_solve_batch([to_dev(f) for f in fs], hs, opts=o, workspace=ws)
            for (us, ss), u, s in zip(solo, ub, sts):
                _same_stats(s, ss)
                assert np.array_equal(to_host(u), to_host(us)), k
    finally:
        mg.mg_batch_force_shape(-1)
    cache = tmp_path / "tune.json"
    assert mg.mg_tune_cache(str(cache)) == 0
    try:
        note("batch %s tuned, with the cache file" % prec)
        ub, sts = mg.mg_solve_batch([to_dev(f) for f in fs], hs, opts=o, workspace=ws)
        for (us, ss), u in zip(solo, ub):
            assert np.array_equal(to_host(u), to_host(us))
        doc = json.loads(cache.read_text())
        assert doc["format"] == "mgic-tuning-2" and len(doc["entries"]) >= 1
        assert mg.mg_tune_cache(str(cache)) == len(doc["entries"])   # loads back
    finally:
        mg.mg_tune_cache(None)
