"""Batched hierarchy solves: every instance bit-identical to its own mg_solve_hierarchy, and the
small instances against the oracle's adaptive FAS solve (Sections 3.2-3.3)."""

import math

import numpy as np
import pytest

from gpu_util import needs_gpu, note, to_dev, to_host
from oracle import zoom
from paper_1103_6031_amd import inputs

pytestmark = [pytest.mark.gpu, needs_gpu]

BOX = 100.0
# periodic-only instances (batched launches) mixed with hierarchies of one to three patches,
# cubic and not, some larger than others
MIX = [
    (32, [((16, 16, 16), (8, 8, 8))]),
    (16, []),
    (64, [((32, 32, 32), (16, 16, 16)), ((32, 32, 32), (8, 8, 8))]),
    (48, [((24, 16, 32), (10, 14, 6))]),
    (64, []),
    (24, [((12, 16, 20), (5, 3, 2))]),
    (32, [((32, 32, 32), (8, 8, 8)), ((24, 16, 32), (4, 8, 8)), ((12, 12, 12), (5, 6, 8))]),
    (8, []),
]


@pytest.fixture(scope="module")
def mg():
    from paper_1103_6031_amd import mgic
    return mgic


def _instances(seed=5, mix=MIX):
    from paper_1103_6031_amd import mgic
    hs, fs = [], []
    for k, (N0, patches) in enumerate(mix):
        H = zoom.Hierarchy(N0, BOX / N0, patches)
        fs.append([np.random.default_rng(seed + 10 * k + p).standard_normal(n) for p, n in enumerate(H.n)])
        hs.append(mgic.Hier(N0, BOX / N0, patches))
    return hs, fs


def _same(a, b):
    assert a["cycles"] == b["cycles"]
    assert (math.isnan(a["rel_res"]) and math.isnan(b["rel_res"])) or a["rel_res"] == b["rel_res"]
    assert np.array_equal(np.array(a["history"]), np.array(b["history"]), equal_nan=True)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("fixed", [False, True])
def test_batch_equals_solo_solves(mg, prec, fixed):
    hs, fs = _instances()
    o = mg.make_opts(tol=1e-10, max_cycles=3 if fixed else 40, prec=prec, fixed_cycles=fixed)
    fd = [[to_dev(a) for a in fi] for fi in fs]
    solo = []
    for i, (H, fi) in enumerate(zip(hs, fd)):
        note("solo solve %d (%s, fixed %s)" % (i, prec, fixed))
        solo.append(mg.mg_solve_hierarchy(H, fi, opts=o))
    ws = mg.Workspace(mg.mg_batch_hier_workspace_bytes(hs, o))
    for rep in range(2):   # the second call replays the captured graphs
        note("hierarchy batch %s fixed %s call %d" % (prec, fixed, rep))
        u, st = mg.mg_solve_batch_hier(hs, fd, opts=o, workspace=ws)
        for i in range(len(hs)):
            for p in range(hs[i].nlev):
                assert np.array_equal(to_host(u[i][p]), to_host(solo[i][0][p])), (rep, i, p)
            _same(st[i], solo[i][1])


def test_batch_matches_the_oracle(mg):
    """The first instances, solved in the batch, against the oracle's solve (FP64 to 1e-10)."""
    hs, fs = _instances(seed=9, mix=MIX[:4])
    note("hierarchy batch vs oracle")
    u, st = mg.mg_solve_batch_hier(hs, [[to_dev(a) for a in fi] for fi in fs], opts=mg.make_opts(tol=1e-10))
    for i, (N0, patches) in enumerate(MIX[:4]):
        H = zoom.Hierarchy(N0, BOX / N0, patches)
        ue, info = zoom.solve_hierarchy(H, fs[i], tol=1e-10)
        assert st[i]["rel_res"] <= 1e-10
        assert abs(st[i]["cycles"] - info["cycles"]) <= 1
        ug = [to_host(x) for x in u[i]]
        num = sum(np.sum((a - b) ** 2) * H.h[p] ** 3 for p, (a, b) in enumerate(zip(ug, ue)))
        den = sum(np.sum(b ** 2) * H.h[p] ** 3 for p, b in enumerate(ue))
        assert np.sqrt(num / den) <= 1e-10, i


def test_failed_instance_leaves_the_others_intact(mg):
    hs, fs = _instances(seed=13, mix=MIX[:4])
    fs[2][1][3, 4, 5] = np.nan          # a patch of the third instance
    o = mg.make_opts(tol=1e-10)
    fd = [[to_dev(a) for a in fi] for fi in fs]
    note("hierarchy batch with a NaN instance")
    u, st = mg.mg_solve_batch_hier(hs, fd, opts=o, check=False)
    with pytest.raises(mg.MGError, match="instance 2"):
        mg.mg_solve_batch_hier(hs, fd, opts=o)
    for i in (0, 1, 3):
        ref, rst = mg.mg_solve_hierarchy(hs[i], fd[i], opts=o)
        for p in range(hs[i].nlev):
            assert np.array_equal(to_host(u[i][p]), to_host(ref[p]))
        _same(st[i], rst)
    assert math.isnan(st[2]["rel_res"])


def test_zoom_sized_batch(mg):
    """Four hierarchies of the zoom workload's shape (128^3 base, three nested 128^3 patches),
    mixed precision, each equal to its own solve."""
    patches = inputs.c3_layout(128, 128, 3)
    hs = [mg.Hier(128, BOX / 128, patches) for _ in range(4)]
    o = mg.make_opts(tol=1e-10, prec="mixed", max_cycles=60)
    fd = []
    for k in range(4):
        H = zoom.Hierarchy(128, BOX / 128, patches)
        fd.append([to_dev(np.random.default_rng(100 + 4 * k + p).standard_normal(n)) for p, n in enumerate(H.n)])
    note("zoom-sized hierarchy batch")
    u, st = mg.mg_solve_batch_hier(hs, fd, opts=o)
    for i in range(4):
        ref, rst = mg.mg_solve_hierarchy(hs[i], fd[i], opts=o)
        for p in range(4):
            assert np.array_equal(to_host(u[i][p]), to_host(ref[p])), (i, p)
        _same(st[i], rst)
        assert st[i]["rel_res"] <= 1e-10
