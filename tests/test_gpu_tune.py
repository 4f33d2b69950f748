"""The mixed solve's inner-cycle tuner on the GPU: every candidate count solves the problem, the
recorded choice is what a default solve of that shape then runs (bit for bit), and it persists in
the tuning cache file."""

import json

import numpy as np
import pytest

from gpu_util import needs_gpu, note, to_dev, to_host

pytestmark = [pytest.mark.gpu, needs_gpu]


def test_inner_tuning_is_used_by_default_solves(tmp_path):
    from paper_1103_6031_amd import inputs, mgic
    patches = [((16, 12, 16), (6, 8, 10))]   # a shape no other test solves
    fl = inputs.nested_fields(32, patches, 77)
    H = mgic.Hier(32, inputs.BOX / 32, patches)
    f = [to_dev(a) for a in fl]
    path = tmp_path / "tune.json"
    assert mgic.mg_tune_cache(str(path)) == 0
    try:
        o = mgic.make_opts(prec="mixed", tol=1e-10, max_cycles=60)
        note("tune: inner cycles on 32^3 + 16x12x16")
        best, ms = mgic.mg_tune_inner(H, f, opts=o)
        assert 0 <= best <= 4
        assert all(m > 0 for m in ms), ms
        assert ms[best] == min(ms)
        entries = json.loads(path.read_text())["entries"]
        assert any(e.get("inner") == best and e["key"].startswith("inner:") for e in entries)
        note("tune: default solve against the explicit count")
        u_def, s_def = mgic.mg_solve_hierarchy(H, f, opts=mgic.make_opts(prec="mixed", tol=1e-10, max_cycles=60))
        u_exp, s_exp = mgic.mg_solve_hierarchy(H, f, opts=mgic.make_opts(prec="mixed", tol=1e-10, max_cycles=60,
                                                                          inner=best if best else 0))
        assert s_def["cycles"] == s_exp["cycles"]
        for a, b in zip(u_def, u_exp):
            assert np.array_equal(to_host(a), to_host(b))
    finally:
        mgic.mg_tune_cache(None)
