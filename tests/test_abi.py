"""The C-ABI library loads, exports every symbol include/mgic.h declares, and rejects bad
arguments on the host (no GPU needed: these paths return before any HIP call)."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mgic.h")
LIB = os.path.join(ROOT, "paper_1103_6031_amd", "libmgic.so")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(\w+)\s*\(", src, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "defined")))


def test_library_exports_every_declared_symbol():
    assert os.path.exists(LIB), "build the library first"
    lib = ctypes.CDLL(LIB)
    names = _declared()
    assert "mg_solve_level" in names and "lpt2_source" in names and "mg_solve_hierarchy" in names
    for n in names:
        assert hasattr(lib, n), "missing export " + n


def test_binding_names_match_header():
    from paper_1103_6031_amd import mgic
    assert sorted(mgic.EXPORTED) == _declared()


def test_workspace_query_and_validation():
    from paper_1103_6031_amd import mgic
    H = mgic.Hier(64, 100.0 / 64)
    b64 = mgic.mg_workspace_bytes(H, mgic.make_opts())
    bmx = mgic.mg_workspace_bytes(H, mgic.make_opts(prec="mixed"))
    assert b64 > 64 ** 3 * 8 and bmx > b64
    for bad in (mgic.Hier(44 * 3, 1.0), mgic.Hier(64, -1.0), mgic.Hier(11, 1.0)):
        with pytest.raises(mgic.MGError):
            mgic.mg_workspace_bytes(bad)
    # patch nesting rules
    ok = mgic.Hier(32, 1.0, [((16, 16, 16), (8, 8, 8)), ((8, 8, 8), (4, 4, 4))])
    assert mgic.mg_workspace_bytes(ok) > 0
    for patches in ([((16, 16, 16), (28, 8, 8))],                         # sticks out of the base
                    [((15, 16, 16), (8, 8, 8))],                          # odd size
                    [((16, 16, 16), (8, 8, 8)), ((8, 8, 8), (2, 4, 4))],  # nesting buffer < 4
                    [((64, 64, 64), (0, 0, 0))]):                         # covers the whole base
        with pytest.raises(mgic.MGError):
            mgic.mg_workspace_bytes(mgic.Hier(32, 1.0, patches))
    assert mgic.lpt_workspace_bytes(ok, 1) > 0 and mgic.lpt_workspace_bytes(ok, 2) > 0


def test_null_workspace_is_rejected_before_any_device_work():
    from paper_1103_6031_amd import mgic
    o = mgic.make_opts()
    st = mgic.mg_stats()
    rc = mgic._lib.mg_solve_level(16, 1.0, ctypes.c_void_p(16), ctypes.c_void_p(16), ctypes.byref(o),
                                  ctypes.byref(st), None, 0, None)
    assert rc == mgic.MG_EINVAL
    assert b"workspace" in mgic._lib.mg_last_error()
    rc = mgic._lib.mg_solve_level(16, 1.0, None, None, ctypes.byref(o), ctypes.byref(st), None, 0, None)
    assert rc == mgic.MG_EINVAL


def test_workspace_size_depends_on_shapes_and_precision_only():
    # the second arrays of the fused 64^3 / 32^3 coarsenings are reserved whatever the sweep
    # counts are, so a workspace sized once serves every nu1 / nu2
    from paper_1103_6031_amd import mgic
    H = mgic.Hier(128, 100.0 / 128)
    for prec in ("fp64", "mixed"):
        sizes = {mgic.mg_workspace_bytes(H, mgic.make_opts(prec=prec, nu1=a, nu2=b)) for a, b in ((1, 1), (2, 2), (3, 1), (0, 4))}
        assert len(sizes) == 1, (prec, sizes)


def test_kernel_timing_period_is_validated():
    from paper_1103_6031_amd import mgic
    for period in (0, 1, 9):
        assert mgic._lib.mg_kprof_enable(period) == mgic.MG_OK
    assert mgic._lib.mg_kprof_enable(-1) == mgic.MG_EINVAL
    assert b"period" in mgic._lib.mg_last_error()
    mgic._lib.mg_kprof_enable(0)
    ms, n, by = mgic.mg_kprof_read()   # nothing recorded: no device work
    assert n == 0 and ms == 0.0 and by == 0.0


def test_lpt_rejects_a_single_cell_base_before_any_device_work():
    from paper_1103_6031_amd import mgic
    H = mgic.Hier(1, 1.0).c_struct()
    ptrs = (ctypes.c_void_p * 3)(16, 16, 16)
    rc = mgic._lib.lpt_displacements(ctypes.byref(H), ptrs, ptrs, 4, -1.0, ctypes.c_void_p(256), 1 << 20, None)
    assert rc == mgic.MG_EINVAL
    assert b"2^3" in mgic._lib.mg_last_error()


def test_lpt_rejects_a_gradient_order_other_than_four_or_six_before_any_device_work():
    from paper_1103_6031_amd import mgic
    H = mgic.Hier(8, 1.0).c_struct()
    ptrs = (ctypes.c_void_p * 3)(16, 16, 16)
    for order in (2, 5, 8):
        rc = mgic._lib.lpt_displacements(ctypes.byref(H), ptrs, ptrs, order, -1.0, ctypes.c_void_p(256), 1 << 20, None)
        assert rc == mgic.MG_EINVAL and b"grad_order" in mgic._lib.mg_last_error()
        rc = mgic._lib.lpt2_source(ctypes.byref(H), ptrs, ptrs, order, ctypes.c_void_p(256), 1 << 20, None)
        assert rc == mgic.MG_EINVAL
    H2 = mgic.Hier(2, 1.0).c_struct()
    rc = mgic._lib.lpt_displacements(ctypes.byref(H2), ptrs, ptrs, 6, -1.0, ctypes.c_void_p(256), 1 << 20, None)
    assert rc == mgic.MG_EINVAL and b"3^3" in mgic._lib.mg_last_error()


def test_lla_validates_its_arguments_before_any_device_work():
    from paper_1103_6031_amd import mgic
    H = mgic.Hier(8, 1.0)
    assert mgic.lpt_workspace_bytes(H, 3) > 0
    ok = mgic.Hier(32, 1.0, [((16, 16, 16), (8, 8, 8))])
    # a hierarchy copies three components per level and pads three patches
    assert mgic.lpt_workspace_bytes(ok, 3) > 3 * (32 ** 3 + 16 ** 3) * 8
    Hc = H.c_struct()
    good = (ctypes.c_void_p * 3)(16, 16, 16)
    hole = (ctypes.c_void_p * 3)(16, 0, 16)
    one = (ctypes.c_void_p * 1)(16)
    lib = mgic._lib
    assert lib.lpt_lla_density(ctypes.byref(Hc), None, None, one, ctypes.c_void_p(256), 1 << 20, None) == mgic.MG_EINVAL
    assert lib.lpt_lla_density(ctypes.byref(Hc), hole, None, one, ctypes.c_void_p(256), 1 << 20, None) == mgic.MG_EINVAL
    assert lib.lpt_lla_density(ctypes.byref(Hc), good, hole, one, ctypes.c_void_p(256), 1 << 20, None) == mgic.MG_EINVAL
    assert lib.lpt_lla_density(ctypes.byref(Hc), good, None, None, ctypes.c_void_p(256), 1 << 20, None) == mgic.MG_EINVAL
    rc = lib.lpt_lla_density(ctypes.byref(Hc), good, None, one, None, 0, None)
    assert rc == mgic.MG_EINVAL and b"workspace" in lib.mg_last_error()
    H1 = mgic.Hier(1, 1.0).c_struct()
    assert lib.lpt_lla_density(ctypes.byref(H1), good, None, one, ctypes.c_void_p(256), 1 << 20, None) == mgic.MG_EINVAL


def test_higher_order_solve_validates_its_arguments_before_any_device_work():
    from paper_1103_6031_amd import mgic
    lib = mgic._lib
    assert lib.mg_ho_workspace_bytes(64, 6) > 2 * 64 ** 3 * 8
    assert lib.mg_ho_workspace_bytes(64, 4) == lib.mg_ho_workspace_bytes(64, 6)
    for n, order in ((24, 4), (1, 4), (2048, 4), (64, 3), (64, 8), (0, 2)):
        assert lib.mg_ho_workspace_bytes(n, order) == 0
    with pytest.raises(mgic.MGError):
        mgic.mg_ho_workspace_bytes(48, 6)
    st = mgic.mg_stats()
    ws = ctypes.c_void_p(256)
    big = lib.mg_ho_workspace_bytes(16, 4)
    p = ctypes.c_void_p(16)
    for o, n, order, h in ((mgic.make_opts(prec=7), 16, 4, 1.0),   # unknown precision
                           (mgic.make_opts(prec="mixed", inner=17), 16, 4, 1.0),
                           (mgic.make_opts(), 16, 5, 1.0),
                           (mgic.make_opts(), 12, 4, 1.0),
                           (mgic.make_opts(), 16, 4, -1.0),
                           (mgic.make_opts(nu1=-1), 16, 4, 1.0),
                           (mgic.make_opts(max_cycles=-1), 16, 4, 1.0),
                           (mgic.make_opts(mean_fix=False), 16, 4, 1.0)):   # the mean is always fixed here
        assert lib.mg_solve_level_ho(n, h, order, p, p, ctypes.byref(o), ctypes.byref(st), ws, big, None) == mgic.MG_EINVAL
    o = mgic.make_opts()
    assert lib.mg_solve_level_ho(16, 1.0, 4, None, p, ctypes.byref(o), ctypes.byref(st), ws, big, None) == mgic.MG_EINVAL
    rc = lib.mg_solve_level_ho(16, 1.0, 4, p, p, ctypes.byref(o), ctypes.byref(st), ws, big - 8, None)
    assert rc == mgic.MG_EINVAL and b"workspace" in lib.mg_last_error()
    rc = lib.mg_solve_level_ho(16, 1.0, 4, p, p, ctypes.byref(o), ctypes.byref(st), ctypes.c_void_p(257), big, None)
    assert rc == mgic.MG_EINVAL and b"aligned" in lib.mg_last_error()
    rc = lib.mg_solve_level_ho(16, 1.0, 4, p, ctypes.c_void_p(24), ctypes.byref(o), ctypes.byref(st), ws, big, None)
    assert rc == mgic.MG_EINVAL and b"16-byte" in lib.mg_last_error()


def test_allocation_free_solve_rejects_problems_above_its_scratch_before_any_device_work():
    from paper_1103_6031_amd import mgic
    lib = mgic._lib
    o = mgic.make_opts(prec="mixed")
    st = mgic.mg_stats()
    big = mgic.Hier(256, 100.0 / 256)
    assert mgic.mg_workspace_bytes(big, o) > mgic.MG_SCRATCH_BYTES
    Hc = big.c_struct()
    p = (ctypes.c_void_p * 1)(16)
    rc = lib.mg_solve_hierarchy_noalloc(ctypes.byref(Hc), p, p, ctypes.byref(o), ctypes.byref(st), None)
    assert rc == mgic.MG_EINVAL and b"scratch" in lib.mg_last_error()
    # the sizes the header names: 128^3 fits in both precisions, 160^3 in FP64 only
    for n, prec, fits in ((128, "fp64", True), (128, "mixed", True), (160, "fp64", True), (160, "mixed", False)):
        need = mgic.mg_workspace_bytes(mgic.Hier(n, 1.0), mgic.make_opts(prec=prec))
        assert (need <= mgic.MG_SCRATCH_BYTES) == fits, (n, prec, need)
    assert lib.mg_solve_hierarchy_noalloc(ctypes.byref(Hc), p, p, None, ctypes.byref(st), None) == mgic.MG_EINVAL


def test_tuning_cache_file_round_trip_and_validation(tmp_path):
    from paper_1103_6031_amd import mgic
    assert mgic.mg_batch_tune_candidates() == 7
    with pytest.raises(mgic.MGError):
        mgic.mg_batch_force_shape(7)
    mgic.mg_batch_force_shape(-1)
    good = tmp_path / "tune.json"
    good.write_text('{"format": "mgic-batch-smoother-tuning-1", "entries": [\n'
                    '  {"key": "0:2:64,64,", "shapes": [[256, 1], [128, 2]]},\n'
                    '  {"key": "1:2:32,", "shapes": [[512, 2]]}\n]}\n')
    assert mgic.mg_tune_cache(str(good)) == 2
    bad = tmp_path / "bad.json"
    bad.write_text('{"format": "mgic-batch-smoother-tuning-1", "entries": [{"key": "x", "shapes": [[100, 3]]}]}')
    with pytest.raises(mgic.MGError):
        mgic.mg_tune_cache(str(bad))
    other = tmp_path / "other.json"
    other.write_text('{"something": "else"}')
    with pytest.raises(mgic.MGError):
        mgic.mg_tune_cache(str(other))
    assert mgic.mg_tune_cache(str(tmp_path / "absent.json")) == 0   # created on the next tuning
    assert mgic.mg_tune_cache(None) == 0
    # the current format carries inner-cycle counts of solo solves beside the batch shapes, and a
    # loaded file is rewritten with every entry the process knows
    v2 = tmp_path / "tune2.json"
    v2.write_text('{"format": "mgic-tuning-2", "entries": [\n'
                  '  {"key": "0:2:64,", "shapes": [[256, 4]]},\n'
                  '  {"key": "inner:2,2:-10:64,64,64;", "inner": 3}\n]}\n')
    assert mgic.mg_tune_cache(str(v2)) == 2
    text = v2.read_text()
    assert '"mgic-tuning-2"' in text and '"inner": 3' in text and "[256, 4]" in text
    bad2 = tmp_path / "bad2.json"
    bad2.write_text('{"format": "mgic-tuning-2", "entries": [{"key": "inner:x", "inner": 99}]}')
    with pytest.raises(mgic.MGError):
        mgic.mg_tune_cache(str(bad2))
    assert mgic.mg_tune_cache(None) == 0
    # the tuner rejects an FP64 problem before any device work
    H = mgic.Hier(16, 1.0).c_struct()
    o = mgic.make_opts(prec="fp64")
    best = ctypes.c_int(-1)
    fake = ctypes.c_void_p(256)
    ptrs = (ctypes.c_void_p * 1)(256)
    pp = ctypes.cast(ptrs, mgic._PP)
    assert mgic._lib.mg_tune_inner(ctypes.byref(H), pp, pp, ctypes.byref(o), ctypes.byref(best), None, fake, 1 << 30,
                                   None) == mgic.MG_EINVAL


def test_spectral_calls_validate_before_any_device_work():
    from paper_1103_6031_amd import mgic
    n = (ctypes.c_int * 3)(16, 16, 16)
    assert mgic.spec_workspace_bytes((16, 16, 16)) > 3 * 16 ** 3 * 16
    # isolated 96^3 pads to 256 per axis; 513 cells exceed the 1024-point transforms
    assert mgic.spec_workspace_bytes((96, 96, 96), isolated=True) > 2 * 96 * 256 * 256 * 16
    for shape, iso in (((12, 16, 16), False), ((16, 16, 2048), False), ((0, 4, 4), True), ((513, 8, 8), True)):
        with pytest.raises(mgic.MGError):
            mgic.spec_workspace_bytes(shape, iso)
    fake = ctypes.c_void_p(256)
    outs = (ctypes.c_void_p * 3)(256, 256, 256)
    op = ctypes.cast(outs, mgic._PP)
    assert mgic._lib.spec_deconvolve(n, 3, 0, fake, fake, fake, 1 << 30, None) == mgic.MG_EINVAL
    assert mgic._lib.spec_deconvolve(n, 1, 0, fake, fake, None, 0, None) == mgic.MG_EINVAL
    assert b"workspace" in mgic._lib.mg_last_error()
    assert mgic._lib.spec_deconvolve(n, 1, 0, fake, fake, ctypes.c_void_p(257), 1 << 30, None) == mgic.MG_EINVAL
    assert b"aligned" in mgic._lib.mg_last_error()
    for lap, grad, h in ((3, 4, 1.0), (2, 5, 1.0), (2, 4, 0.0), (2, 4, float("nan"))):
        assert mgic._lib.lpt_hybrid_correction(n, h, 0, lap, grad, 1.0, fake, op, fake, 1 << 30,
                                               None) == mgic.MG_EINVAL
    assert mgic._lib.lpt_hybrid_correction(n, 1.0, 0, 2, 4, 1.0, None, op, fake, 1 << 30, None) == mgic.MG_EINVAL
    for order, h in ((3, 1.0), (2, 0.0), (4, float("inf"))):
        assert mgic._lib.spec_poisson(n, h, order, fake, fake, fake, 1 << 30, None) == mgic.MG_EINVAL
    assert mgic._lib.spec_poisson(n, 1.0, 2, fake, None, fake, 1 << 30, None) == mgic.MG_EINVAL
    assert mgic._lib.spec_poisson((ctypes.c_int * 3)(12, 16, 16), 1.0, 2, fake, fake, fake, 1 << 30,
                                  None) == mgic.MG_EINVAL


def test_density_validates_before_any_device_work():
    from paper_1103_6031_amd import mgic
    ok = mgic.Hier(32, 1.0, [((16, 16, 16), (8, 8, 8))])
    assert mgic.ic_density_workspace_bytes(ok) > 0
    for bad in (mgic.Hier(48, 1.0), mgic.Hier(32, 1.0, [((12, 12, 12), (8, 8, 8))]),
                mgic.Hier(64, 1.0, [((32,) * 3, (16,) * 3), ((32,) * 3, (4,) * 3)])):
        with pytest.raises(mgic.MGError):
            mgic.ic_density_workspace_bytes(bad)
    H = ok.c_struct()
    fake = ctypes.c_void_p(256)
    ptrs = (ctypes.c_void_p * 2)(256, 256)
    pp = ctypes.cast(ptrs, mgic._PP)
    assert mgic._lib.ic_multiscale_density(ctypes.byref(H), fake, 1 << 20, 0.01, 1, pp, pp, None, 0,
                                           None) == mgic.MG_EINVAL
    assert b"workspace" in mgic._lib.mg_last_error()
    # a table too short for the base's corners
    assert mgic._lib.ic_multiscale_density(ctypes.byref(H), fake, 100, 0.01, 1, pp, pp, fake, 1 << 40,
                                           None) == mgic.MG_EINVAL
    assert b"radial table" in mgic._lib.mg_last_error()


def test_hierarchy_batch_validates_before_any_device_work():
    from paper_1103_6031_amd import mgic
    o = mgic.make_opts()
    a = mgic.Hier(32, 1.0, [((16, 16, 16), (8, 8, 8))])
    b = mgic.Hier(16, 2.0)
    need = mgic.mg_batch_hier_workspace_bytes([a, b], o)
    # the two parts, each rounded up to 256 bytes
    up = lambda x: (x + 255) // 256 * 256
    assert need == up(mgic.mg_batch_workspace_bytes([16], o)) + up(mgic.mg_workspace_bytes(a, o))
    assert mgic.mg_batch_hier_workspace_bytes([a], o) == up(mgic.mg_workspace_bytes(a, o))
    with pytest.raises(mgic.MGError, match="instance 1"):
        mgic.mg_batch_hier_workspace_bytes([a, mgic.Hier(32, 1.0, [((14, 16, 16), (8, 8, 8)), ((8, 8, 8), (1, 1, 1))])], o)
    with pytest.raises(mgic.MGError):
        mgic.mg_batch_hier_workspace_bytes([mgic.Hier(32, 1.0, [((13, 16, 16), (8, 8, 8))])], o)
    fake = ctypes.c_void_p(256)
    hp, _keep = mgic._hier_array([a, b])
    fl = [mgic._ptr_array([256, 256]), mgic._ptr_array([256])]
    fa = (mgic._PP * 2)(*[p for p, _ in fl])
    fa_p = ctypes.cast(fa, ctypes.c_void_p)
    st = (mgic.mg_stats * 2)()
    call = mgic._lib.mg_solve_batch_hier
    assert call(2, hp, None, fa_p, ctypes.byref(o), st, fake, need, None) == mgic.MG_EINVAL
    assert call(0, hp, fa_p, fa_p, ctypes.byref(o), st, fake, need, None) == mgic.MG_EINVAL
    assert call(2, hp, fa_p, fa_p, ctypes.byref(o), st, fake, need - 1, None) == mgic.MG_EINVAL
    assert b"workspace too small" in mgic._lib.mg_last_error()
    assert call(2, hp, fa_p, fa_p, ctypes.byref(o), st, ctypes.c_void_p(257), need, None) == mgic.MG_EINVAL
    assert b"aligned" in mgic._lib.mg_last_error()
    bad_lvl = [mgic._ptr_array([256, 0]), mgic._ptr_array([256])]
    fb = (mgic._PP * 2)(*[p for p, _ in bad_lvl])
    assert call(2, hp, ctypes.cast(fb, ctypes.c_void_p), fa_p, ctypes.byref(o), st, fake, need,
                None) == mgic.MG_EINVAL
    assert b"instance 0" in mgic._lib.mg_last_error()
    bad = mgic.make_opts(max_cycles=-1)
    assert call(2, hp, fa_p, fa_p, ctypes.byref(bad), st, fake, need, None) == mgic.MG_EINVAL


def test_batched_solve_rejects_no_mean_fix_before_any_device_work():
    from paper_1103_6031_amd import mgic
    o = mgic.make_opts(mean_fix=False)
    assert o.flags & mgic.MG_NO_MEAN_FIX
    n = (ctypes.c_int * 2)(32, 64)
    h = (ctypes.c_double * 2)(1.0, 0.5)
    fp, _k1 = mgic._ptr_array([256, 512])
    st = (mgic.mg_stats * 2)()
    need = mgic.mg_batch_workspace_bytes([32, 64], o)
    rc = mgic._lib.mg_solve_batch(2, n, h, fp, fp, ctypes.byref(o), st, ctypes.c_void_p(256), need, None)
    assert rc == mgic.MG_EINVAL and b"MG_NO_MEAN_FIX" in mgic._lib.mg_last_error()
    # the hierarchy batch solves such instances on its lanes instead: its workspace has no batched part
    H = [mgic.Hier(32, 1.0), mgic.Hier(64, 0.5)]
    up = lambda x: (x + 255) // 256 * 256
    assert mgic.mg_batch_hier_workspace_bytes(H, o) == sum(up(mgic.mg_workspace_bytes(x, o)) for x in H)
