"""Allocation-free solve (mg_solve_hierarchy_noalloc) against mg_solve_hierarchy on the GPU.

The two run the same kernels on the same inputs; the allocation-free call only takes its workspace
from the library's static device array.  Two calls in a row, the second on a smaller problem,
must each equal the workspace call bit for bit (residual history and cycle count included).
"""

import numpy as np
import pytest

from gpu_util import needs_gpu, note, to_dev, to_host
from paper_1103_6031_amd import inputs

pytestmark = [pytest.mark.gpu, needs_gpu]

CASES = [
    ("64^3 base + 48^3 patch", 64, [((48, 48, 48), (8, 8, 8))]),
    ("32^3 single level", 32, []),
]


def _fields(N0, patches, seed):
    if patches:
        return inputs.nested_fields(N0, patches, seed)
    return [inputs.gaussian_field(N0, seed, box=100.0)]


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_noalloc_matches_workspace_solve_twice(prec):
    from paper_1103_6031_amd import mgic
    import torch
    for k, (name, N0, patches) in enumerate(CASES):
        H = mgic.Hier(N0, 100.0 / N0, patches)
        assert mgic.mg_workspace_bytes(H, mgic.make_opts(prec=prec)) <= mgic.MG_SCRATCH_BYTES
        f = [to_dev(a) for a in _fields(N0, patches, 1103100 + k)]
        o = mgic.make_opts(tol=1e-10, prec=prec)
        note("noalloc %s %s: workspace solve" % (prec, name))
        ref, st_ref = mgic.mg_solve_hierarchy(H, f, opts=o)
        note("noalloc %s %s: static scratch solve" % (prec, name))
        u = [torch.full_like(x, float("nan")) for x in f]
        got, st = mgic.mg_solve_hierarchy_noalloc(H, f, u, opts=o)
        torch.cuda.synchronize()
        assert st["cycles"] == st_ref["cycles"] and st["rel_res"] == st_ref["rel_res"]
        assert np.array_equal(np.array(st["history"]), np.array(st_ref["history"]), equal_nan=True)
        assert st["rel_res"] <= 1e-10
        for a, b in zip(got, ref):
            assert np.array_equal(to_host(a), to_host(b)), "%s: allocation-free result differs" % name


def test_noalloc_rejects_problems_above_the_scratch_size():
    from paper_1103_6031_amd import mgic
    import torch
    H = mgic.Hier(256, 100.0 / 256)
    o = mgic.make_opts(prec="mixed")
    assert mgic.mg_workspace_bytes(H, o) > mgic.MG_SCRATCH_BYTES
    f = [torch.zeros((256,) * 3, dtype=torch.float64, device="cuda")]
    u = [torch.zeros_like(f[0])]
    note("noalloc: oversize rejection")
    with pytest.raises(mgic.MGError) as e:
        mgic.mg_solve_hierarchy_noalloc(H, f, u, opts=o)
    assert e.value.code == mgic.MG_EINVAL and "scratch" in str(e.value)
