"""Fixed-cycle solves under the caller's graph capture: the captured graph, replayed several times
with eager work and synchronisations in between, gives the eager solve's bits every time.  The
entry points that read back or wait refuse a capturing stream with MG_EINVAL."""

import numpy as np
import pytest

from gpu_util import needs_gpu, note, to_dev, to_host

pytestmark = [pytest.mark.gpu, needs_gpu]

BOX = 100.0
CASES = {
    "periodic32": (32, []),
    "zoom": (32, [((32, 32, 32), (8, 8, 8)), ((24, 16, 32), (4, 8, 8))]),
    "rect48": (48, [((24, 16, 32), (10, 14, 6))]),
}


@pytest.fixture(scope="module")
def mg():
    from paper_1103_6031_amd import mgic
    return mgic


def _case(mg, name, seed=3):
    N0, patches = CASES[name]
    H = mg.Hier(N0, BOX / N0, patches)
    f = [np.random.default_rng(seed + p).standard_normal(H.dims(p)) for p in range(H.nlev)]
    return H, [to_dev(a) for a in f]


@pytest.mark.parametrize("noalloc", [False, True])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("name", list(CASES))
def test_captured_fixed_cycle_solve_replays_the_eager_bits(mg, name, prec, noalloc):
    import torch
    H, fd = _case(mg, name)
    o = mg.make_opts(max_cycles=3, fixed_cycles=True, prec=prec)
    note("capture %s %s noalloc %s" % (name, prec, noalloc))
    u = [torch.zeros_like(x) for x in fd]
    ws = None if noalloc else mg.Workspace(mg.mg_workspace_bytes(H, o))

    def solve():
        if noalloc:
            return mg.mg_solve_hierarchy_noalloc(H, fd, u, opts=o)
        return mg.mg_solve_hierarchy(H, fd, u=u, opts=o, workspace=ws)

    solve()                                   # eager: the reference, and the first call's set-up
    torch.cuda.synchronize()
    ref = [to_host(x).copy() for x in u]
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        solve()
    for rep in range(3):
        for x in u:
            x.fill_(float("nan"))             # eager work between the replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for p in range(H.nlev):
            assert np.array_equal(to_host(u[p]), ref[p]), (rep, p)
        solve()                               # an eager solve between replays changes nothing
        torch.cuda.synchronize()


@pytest.mark.filterwarnings("ignore:The CUDA Graph is empty")   # every call in it is refused
def test_entry_points_that_wait_refuse_capture(mg):
    import torch
    H, fd = _case(mg, "zoom")
    Hp, fp = _case(mg, "periodic32")
    conv = mg.make_opts(tol=1e-10)
    fixed = mg.make_opts(max_cycles=2, fixed_cycles=True)
    ws = mg.Workspace(mg.mg_workspace_bytes(H, conv))
    u = [torch.zeros_like(x) for x in fd]
    up = [torch.zeros_like(x) for x in fp]
    wsb = mg.Workspace(mg.mg_batch_workspace_bytes([32], fixed))
    wsh = mg.Workspace(mg.mg_ho_workspace_bytes(32, 4))
    wsbh = mg.Workspace(mg.mg_batch_hier_workspace_bytes([H], fixed))
    note("entry points refusing capture")
    errors = []
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for call in (lambda: mg.mg_solve_hierarchy(H, fd, u=u, opts=conv, workspace=ws),
                     lambda: mg.mg_solve_batch(fp, [BOX / 32], u=up, opts=fixed, workspace=wsb),
                     lambda: mg.mg_solve_level_ho(fp[0], BOX / 32, 4, u=up[0], opts=fixed, workspace=wsh),
                     lambda: mg.mg_solve_batch_hier([H], [fd], u=[u], opts=fixed, workspace=wsbh)):
            try:
                call()
                errors.append(None)
            except mg.MGError as e:
                errors.append((e.code, str(e)))
    assert all(e is not None and e[0] == mg.MG_EINVAL and "capture" in e[1] for e in errors), errors
