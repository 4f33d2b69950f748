"""Higher-order Laplacians on nested patches (Section 3.3 with Tables 1 and 2) on the GPU against
the oracle (``oracle.zoom_ho``).

Bars: the ghost layers equal the oracle's to 1e-13 of their largest value (both are FP64 sums in
different orders); after a fixed number of FP64 V-cycles every level of the GPU iterate equals
the oracle's to 1e-12 of its largest value; converged solves are within 1e-10 composite relative
RMS of the oracle's solve, whose composite residual of the GPU solution also meets the tolerance.
"""

import numpy as np
import pytest

from gpu_util import needs_gpu, note, to_dev, to_host, rel_max
from oracle import zoom, zoom_ho
from paper_1103_6031_amd import inputs

pytestmark = [pytest.mark.gpu, needs_gpu]

LAYOUTS = {
    "one": (16, [((16, 16, 16), (4, 4, 4))]),
    "rect": (16, [((12, 16, 20), (5, 3, 2))]),
    "deep": (32, [((32, 32, 32), (8, 8, 8)), ((24, 16, 32), (4, 8, 8)), ((12, 12, 12), (5, 6, 8))]),
    # long thin patches: at order 6 the rows of the 584-long finest patch exceed the 64 KB of LDS a
    # block may stage, so its half-sweep and residual norm read every neighbour from memory, while
    # the 484-long patch above it stages its rows
    "long": (128, [((16, 16, 250), (56, 56, 3)), ((16, 16, 484), (4, 4, 4)), ((8, 8, 584), (4, 4, 4))]),
}


@pytest.fixture(scope="module")
def mg():
    from paper_1103_6031_amd import mgic
    return mgic


def _case(mg, name, seed=5):
    N0, patches = LAYOUTS[name]
    H = zoom.Hierarchy(N0, 100.0 / N0, patches)
    f = [np.random.default_rng(seed + p).standard_normal(n) for p, n in enumerate(H.n)]
    return H, mg.Hier(N0, 100.0 / N0, patches), f


def _crms(H, a, b):
    num = den = 0.0
    for p in range(H.P + 1):
        m = zoom.uncovered_mask(H, p)
        num += float(np.sum((a[p] - b[p])[m] ** 2)) * H.h[p] ** 3
        den += float(np.sum(b[p][m] ** 2)) * H.h[p] ** 3
    return np.sqrt(num / den)


@pytest.mark.parametrize("order", [2, 4, 6])
@pytest.mark.parametrize("name", ["one", "rect", "deep", "long"])
def test_ghost_layers_match_oracle(mg, name, order):
    H, Hg, _ = _case(mg, name)
    R = order // 2
    rng = np.random.default_rng(11)
    u = [rng.standard_normal(n) for n in H.n]
    for p in range(1, H.P + 1):
        for fm in (True, False):
            note("ho ghost fill %s order %d p=%d flux=%s" % (name, order, p, fm))
            g = mg.mg_ghost_fill_ho(Hg, order, p, [to_dev(a) for a in u], flux_match=fm)
            faces = [to_host(x) for x in mg.split_ghosts_ho(Hg, order, p, g)]
            up = zoom_ho.ghosted(H, u, p, order, flux_match=fm)
            n = H.n[p]
            for a in range(3):
                upa = np.moveaxis(up, a, 0)
                inner = upa[:, R:-R, R:-R]
                for side in (0, 1):
                    exp = np.stack([inner[R - 1 - gl] if side == 0 else inner[R + n[a] + gl] for gl in range(R)])
                    got = faces[2 * a + side]
                    assert np.max(np.abs(got - exp)) <= 1e-13 * max(1.0, np.max(np.abs(exp))), (a, side)


@pytest.mark.parametrize("order", [4, 6])
@pytest.mark.parametrize("name", ["one", "rect", "deep", "long"])
@pytest.mark.parametrize("cycles", [1, 2])
def test_fixed_cycle_iterates_match_oracle(mg, name, order, cycles):
    H, Hg, f = _case(mg, name)
    note("ho hierarchy %s order %d, %d fixed cycles" % (name, order, cycles))
    u, st = mg.mg_solve_hierarchy_ho(Hg, order, [to_dev(a) for a in f],
                                     opts=mg.make_opts(max_cycles=cycles, fixed_cycles=True))
    ue, info = zoom_ho.solve_hierarchy(H, f, order, tol=0.0, max_cycles=cycles)
    assert st["cycles"] == cycles == info["cycles"]
    for p in range(H.P + 1):
        assert rel_max(to_host(u[p]), ue[p]) <= 1e-12, p


@pytest.mark.parametrize("order", [4, 6])
@pytest.mark.parametrize("name", ["one", "deep"])
def test_converged_solve_matches_oracle(mg, name, order):
    # white noise puts most of its power at the grid scale, where the solution error of a stopped
    # solve is several times its relative residual; these cases therefore stop at 1e-11 to be held
    # to the 1e-10 bar (the BBKS-shaped case below stops at 1e-10)
    H, Hg, f = _case(mg, name)
    note("ho hierarchy solve %s order %d" % (name, order))
    u, st = mg.mg_solve_hierarchy_ho(Hg, order, [to_dev(a) for a in f], opts=mg.make_opts(tol=1e-11))
    ue, info = zoom_ho.solve_hierarchy(H, f, order, tol=1e-13)
    ug = [to_host(x) for x in u]
    assert st["rel_res"] <= 1e-11 and abs(st["cycles"] - info["cycles"]) <= 2
    assert _crms(H, ug, ue) <= 1e-10
    fz, _ = zoom.composite_zero_mean(H, f)
    r = zoom_ho.composite_residual(H, ug, fz, order)
    rel = zoom.composite_norm(H, r) / zoom.composite_norm(H, fz)
    assert rel <= 1.05e-11 and abs(rel - st["rel_res"]) <= 0.05 * rel + 1e-13
    hist = st["history"]   # the paper's tenfold reduction per cycle, past the first cycle
    assert max(b / a for a, b in zip(hist[:-1], hist[1:])) < 0.1


def test_c3_shaped_order6_hierarchy_matches_oracle(mg):
    """A C3-shaped hierarchy at half the size: 64^3 base with three centred 64^3 patches (512^3
    effective), nested BBKS density, sixth-order operators (the order of the paper's own nested
    results)."""
    patches = inputs.c3_layout(64, 64, 3)
    f = inputs.nested_fields(64, patches, inputs.SEED_C3)
    H = zoom.Hierarchy(64, inputs.BOX / 64, patches)
    Hg = mg.Hier(64, inputs.BOX / 64, patches)
    note("ho C3-shaped 64^3 + 3 x 64^3 order 6")
    u, st = mg.mg_solve_hierarchy_ho(Hg, 6, [to_dev(a) for a in f], opts=mg.make_opts(tol=1e-10, max_cycles=40))
    ue, info = zoom_ho.solve_hierarchy(H, f, 6, tol=1e-12)
    err = _crms(H, [to_host(x) for x in u], ue)
    note("ho C3-shaped order 6: %d cycles (oracle %d), composite rel. RMS vs oracle %.2e" %
         (st["cycles"], info["cycles"], err))
    assert st["rel_res"] <= 1e-10 and err <= 1e-10


def test_argument_errors(mg):
    Hg = mg.Hier(16, 1.0, [((16, 16, 16), (4, 4, 4))])
    f = [to_dev(np.ones((16, 16, 16))), to_dev(np.ones((16, 16, 16)))]
    for kw, order in ((dict(), 5), (dict(prec="mixed"), 4)):
        with pytest.raises(mg.MGError) as e:
            mg.mg_solve_hierarchy_ho(Hg, order, f, opts=mg.make_opts(**kw))
        assert e.value.code == mg.MG_EINVAL
    with pytest.raises(mg.MGError):   # a base of 24 is not a power of two
        mg.mg_ho_hierarchy_workspace_bytes(mg.Hier(24, 1.0, [((16, 16, 16), (4, 4, 4))]), 4)
    with pytest.raises(mg.MGError):   # a patch narrower than the order
        mg.mg_ho_hierarchy_workspace_bytes(mg.Hier(16, 1.0, [((4, 8, 8), (4, 4, 4))]), 6)
