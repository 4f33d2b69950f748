"""Solo solves replayed as HIP graphs against the same solves launched directly (MG_NO_GRAPH).

A solve's repeating launch sequences (cycles, outer steps, the source preparation and the final
gauge) are captured the second time they are met for a workspace and plan, then replayed.  Each
case here solves several times in a row with graphs - with eager torch work and synchronisations
between the calls, and with a second right-hand side on the same workspace - and every result,
residual history and cycle count must equal the direct launches' bit for bit.
"""

import numpy as np
import pytest

from gpu_util import needs_gpu, note, to_dev, to_host
from paper_1103_6031_amd import inputs

pytestmark = [pytest.mark.gpu, needs_gpu]


@pytest.fixture(scope="module")
def mg():
    from paper_1103_6031_amd import mgic
    return mgic


def _same(a, sa, b, sb):
    assert sa["cycles"] == sb["cycles"]
    assert np.array_equal(np.array(sa["history"]), np.array(sb["history"]), equal_nan=True)
    assert (np.isnan(sa["rel_res"]) and np.isnan(sb["rel_res"])) or sa["rel_res"] == sb["rel_res"]
    for x, y in zip(a, b):
        assert np.array_equal(to_host(x), to_host(y))


CASES = [
    # name, base, patches, precision, options
    ("64^3 fp64", 64, [], "fp64", {}),
    ("64^3 mixed (fused outer step)", 64, [], "mixed", {}),
    ("48^3 fp64 (odd coarsest)", 48, [], "fp64", {}),
    ("32^3 + 2 patches fp64", 32, inputs.c3_layout(32, 32, 2), "fp64", {}),
    ("32^3 + 2 patches mixed", 32, inputs.c3_layout(32, 32, 2), "mixed", {}),
    ("64^3 mixed fixed cycles", 64, [], "mixed", dict(fixed_cycles=True, max_cycles=7)),
    ("32^3 + 1 patch fp64 fixed cycles", 32, inputs.c3_layout(32, 32, 1), "fp64", dict(fixed_cycles=True,
                                                                                        max_cycles=5)),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_graph_replay_equals_direct_launches(mg, case):
    import torch
    name, N0, patches, prec, extra = case
    H = mg.Hier(N0, inputs.BOX / N0, patches)
    fields = [inputs.nested_fields(N0, patches, 1103200 + k) if patches else [inputs.gaussian_field(N0, 1103200 + k)]
              for k in range(2)]
    kw = dict(tol=1e-10, prec=prec, max_cycles=60)
    kw.update(extra)
    og, od = mg.make_opts(**kw), mg.make_opts(graph=False, **kw)
    ws = mg.Workspace(mg.mg_workspace_bytes(H, og))
    for k, fl in enumerate(fields):
        f = [to_dev(a) for a in fl]
        note("graphs %s rhs %d: direct" % (name, k))
        ref, sref = mg.mg_solve_hierarchy(H, f, opts=od, workspace=ws)
        u = [torch.empty_like(x) for x in f]
        for rep in range(4):
            note("graphs %s rhs %d: replay %d" % (name, k, rep))
            got, sg = mg.mg_solve_hierarchy(H, f, u=u, opts=og, workspace=ws)
            torch.cuda.synchronize()
            _same(got, sg, ref, sref)
            junk = torch.randn(1 << 20, device="cuda", dtype=torch.float64)   # eager work between replays
            float(junk.sum())
        if not extra.get("fixed_cycles"):
            assert sg["rel_res"] <= 1e-10


def test_graph_replay_with_initial_guess(mg):
    import torch
    N = 64
    h = inputs.BOX / N
    f = to_dev(inputs.gaussian_field(N, 1103210))
    for prec in ("fp64", "mixed"):
        o1 = mg.make_opts(tol=1e-4, prec=prec)
        ws = mg.Workspace(mg.mg_workspace_bytes(mg.Hier(N, h), o1))
        u0, _ = mg.mg_solve_level(f, h, opts=o1, workspace=ws)
        og = mg.make_opts(tol=1e-10, prec=prec, initial_guess=True)
        od = mg.make_opts(tol=1e-10, prec=prec, initial_guess=True, graph=False)
        note("graphs warm start %s: direct" % prec)
        ref, sref = mg.mg_solve_level(f, h, u=u0.clone(), opts=od, workspace=ws)
        u = torch.empty_like(u0)
        for rep in range(3):
            note("graphs warm start %s: replay %d" % (prec, rep))
            u.copy_(u0)
            got, sg = mg.mg_solve_level(f, h, u=u, opts=og, workspace=ws)
            _same([got], sg, [ref], sref)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_fixed_cycle_graphs_are_not_replayed_by_a_converging_solve(mg, prec):
    """Regression: a fixed-cycle solve captures its steps without the residual readback; a later
    solve with a stopping test on the same workspace must not replay those (it would read a
    stale host value - here the NaN a failed solve left behind)."""
    N = 32
    h = inputs.BOX / N
    f = to_dev(inputs.gaussian_field(N, 1103220))
    ws = mg.Workspace(mg.mg_workspace_bytes(mg.Hier(N, h), mg.make_opts(prec=prec)))
    fixed = mg.make_opts(prec=prec, fixed_cycles=True, max_cycles=4)
    for _ in range(3):
        mg.mg_solve_level(f, h, opts=fixed, workspace=ws)
    bad = f.clone()
    bad[1, 2, 3] = float("nan")
    with pytest.raises(mg.MGError):
        mg.mg_solve_level(bad, h, opts=mg.make_opts(prec=prec))
    ref, sref = mg.mg_solve_level(f, h, opts=mg.make_opts(prec=prec, graph=False), workspace=ws)
    for _ in range(3):
        got, sg = mg.mg_solve_level(f, h, opts=mg.make_opts(prec=prec), workspace=ws)
        _same([got], sg, [ref], sref)
        assert sg["rel_res"] <= 1e-10
