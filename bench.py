"""Benchmark of the adaptive-multigrid 2LPT hot path on one MI355X.

One step = the whole hot path over one synthetic input resident in HBM:
    phi1 = solve(delta)            FAS V(2,2) cycles to a 1e-10 relative residual
    psi1 = -G4 phi1                first-order displacements
    tau  = sum_{i>j} D_ii D_jj - D_ij^2 (D = G4 G4), composite mean removed
    phi2 = solve(tau)
    psi2 = -3/7 G4 phi2            second-order displacements
Default workload: periodic 256^3, BBKS spectrum (Gamma = 0.2), 100 Mpc/h box, density rms 0.1,
seed 1103002.  The headline path is mixed precision (FP32 smoother / transfers inside an FP64
defect-correction loop); the plain FP64 path is timed beside it.

Prints ONE JSON line.  `value` is cell-updates per second of the headline path (smoother
cell-updates summed over all levels and both solves, divided by the step time).  `roofline`
is the finest-level smoother kernel: algorithmic bytes (3 words per cell-update) over its
average launch duration, timed with HIP events on its own stream inside the timed region;
`traffic` is its HBM bytes per launch from the recorded rocprofv3 counter passes (null when the
kernel sources no longer match the ones the counters were taken on).
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Mcell-updates/s + HBM GB/s; mixed vs FP64 at 1e-8 rel. RMS; p50/p99 latency"
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline leg")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched 64-instance leg")
    ap.add_argument("--no-c1c3", action="store_true", help="skip the 64^3 solve and zoom-hierarchy legs")
    ap.add_argument("--serve-requests", type=int, default=600,
                    help="requests of the serving trace (Poisson, 20/s); 0 skips the serving leg")
    ap.add_argument("--prec", choices=["mixed", "fp64"], default="mixed", help="headline path")
    ap.add_argument("--inner", type=int, default=0, help="mixed: FP32 V-cycles per FP64 correction (0: library default)")
    ap.add_argument("--no-roof512", action="store_true", help="skip the 512^3 smoother leg")
    ap.add_argument("--no-graph", action="store_true", help="launch every kernel directly (no graph replay)")
    ap.add_argument("--only", default="",
                    help="comma-separated legs to run alone, without the headline step (profiling): "
                         "roof512, c1, c3, hoz, c4, bh, spectral, density, ho")
    ap.add_argument("--pmc-calib", action="store_true",
                    help="after the timed steps, run a plain 256 MiB device copy (counter calibration)")
    return ap.parse_args()


# HBM traffic of the finest-level smoother, from the rocprofv3 FETCH_SIZE / WRITE_SIZE passes
# recorded under profiles/; it stands only while the kernel sources hash to the recorded value.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_rbgs_vec_f32_256.md")
KERNEL_SOURCES = ("k_levels.hip", "mg_internal.h", "fastdiv.h", "p2_bodies.h")   # the smoother's sources


def kernel_source_hash():
    import hashlib
    hsh = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1103_6031_amd", "csrc", name), "rb") as fh:
            hsh.update(fh.read())
    return hsh.hexdigest()


def recorded_traffic():
    """HBM bytes per launch from the recorded counter passes, or None if absent or stale."""
    try:
        with open(TRAFFIC_FILE) as fh:
            kv = dict(line.split(":", 1) for line in fh if ":" in line and not line.startswith(("#", "`", " ")))
    except OSError:
        return None
    kv = {k.strip(): v.strip() for k, v in kv.items()}
    if kv.get("source_sha256") != kernel_source_hash():
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


KPROF_STEPS = 1   # timed steps whose finest smoother launches carry events
GRAPH = True      # replay repeating launch sequences as HIP graphs (--no-graph: direct launches)


def _opts(mg, **kw):
    return mg.make_opts(graph=GRAPH, **kw)


def run_step(mg, H, ft, h, opts, ws):
    phi1, s1 = mg.mg_solve_level(ft, h, opts=opts, workspace=ws["solve"])
    psi1, tau = mg.lpt_displacements_and_source(H, [phi1], scale=-1.0, workspace=ws["lpt2"])
    psi1, tau = psi1[0], tau[0]
    phi2, s2 = mg.mg_solve_level(tau, h, opts=opts, workspace=ws["solve"])
    psi2 = mg.lpt_displacements(H, [phi2], scale=-3.0 / 7.0, workspace=ws["lpt1"])[0]
    return (phi1, psi1, tau, phi2, psi2), (s1, s2)


def time_path(mg, torch, H, ft, h, prec, tol, steps, warmup, inner=0):
    opts = _opts(mg, tol=tol, prec=prec, max_cycles=60, inner=inner)
    ws = {"solve": mg.Workspace(mg.mg_workspace_bytes(H, opts)),
          "lpt1": mg.Workspace(mg.lpt_workspace_bytes(H, 1)),
          "lpt2": mg.Workspace(mg.lpt_workspace_bytes(H, 2))}
    for _ in range(warmup):
        out, st = run_step(mg, H, ft, h, opts, ws)
    torch.cuda.synchronize()
    mg.mg_kprof_read()            # drop anything recorded so far
    t0 = time.perf_counter()
    ups = 0
    cycles = []
    for i in range(steps):
        # every finest-level smoother launch of the first timed step carries dispatch-stamped
        # events (the regime in which rocprofv3 stamps every dispatch, so the two averages are
        # comparable); the events add several microseconds of dispatch work per launch, so the
        # other steps run without them
        mg.mg_kprof_enable(i < KPROF_STEPS)
        out, st = run_step(mg, H, ft, h, opts, ws)
        ups += st[0]["cell_updates"] + st[1]["cell_updates"]
        cycles.append((st[0]["cycles"], st[1]["cycles"]))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    mg.mg_kprof_enable(False)
    kms, klaunch, kbytes = mg.mg_kprof_read()
    achieved = kbytes / (kms * 1e-3) / 1e9 if kms > 0 else None
    res = dict(ms_per_step=1e3 * dt / steps, value=ups / dt / 1e6, cycles=cycles[-1],
               rel_res=(st[0]["rel_res"], st[1]["rel_res"]),
               kernel=dict(launches=klaunch, avg_us=1e3 * kms / max(klaunch, 1),
                           bytes_per_launch=kbytes / max(klaunch, 1), achieved_gbs=achieved))
    return res, out


def time_batch(mg, torch, reps):
    """64 independent periodic instances (sizes in {32,48,64,96,128}^3, power-law spectra): one
    batched mixed-precision solve against the same instances solved one after another."""
    from paper_1103_6031_amd import inputs
    inst = inputs.c4_instances()
    sizes = [N for N, _, _ in inst]
    hs = [inputs.BOX / N for N in sizes]
    fs = [torch.from_numpy(inputs.c4_field(N, s, seed)).to("cuda:0") for N, s, seed in inst]
    o = _opts(mg, tol=1e-10, prec="mixed", max_cycles=40)
    ws = mg.Workspace(mg.mg_batch_workspace_bytes(sizes, o))
    u = [torch.empty_like(f) for f in fs]
    mg.mg_solve_batch(fs, hs, u=u, opts=o, workspace=ws)     # warm-up (autotuning, graph capture)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        _, st = mg.mg_solve_batch(fs, hs, u=u, opts=o, workspace=ws)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    ups = sum(s["cell_updates"] for s in st)
    wss = mg.Workspace(max(mg.mg_workspace_bytes(mg.Hier(N, 1.0), o) for N in set(sizes)))
    us = [torch.empty_like(f) for f in fs]
    for f, h, x in zip(fs, hs, us):
        mg.mg_solve_level(f, h, u=x, opts=o, workspace=wss)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for f, h, x in zip(fs, hs, us):
        mg.mg_solve_level(f, h, u=x, opts=o, workspace=wss)
    torch.cuda.synchronize()
    dts = time.perf_counter() - t0
    same = all(bool(torch.equal(a, b)) for a, b in zip(u, us))
    cyc = [s["cycles"] for s in st]
    return dict(workload="64 periodic instances, sizes {32,48,64,96,128}^3, P=k^n, n in [-2.5,-1.5], mixed, tol 1e-10",
                cells=int(sum(N ** 3 for N in sizes)), ms_per_solve=round(dt * 1e3, 3),
                value=round(ups / dt / 1e6, 1), unit="Mcell-updates/s", cycles=[min(cyc), max(cyc)],
                sequential_ms=round(dts * 1e3, 3), speedup=round(dts / dt, 2), bit_identical_to_solo=same)


def time_batch_hier(mg, torch, reps=3, count=8):
    """Independent zoom hierarchies in one call (each a 128^3 base with three nested 128^3
    patches, its own nested BBKS density), mixed precision: the batched call against the same
    solves one after another on one stream.  Every instance's bits equal its solo solve."""
    from paper_1103_6031_amd import inputs
    patches = inputs.c3_layout(128, 128, 3)
    hs = [mg.Hier(128, inputs.BOX / 128, patches) for _ in range(count)]
    fs = [[torch.from_numpy(a).to("cuda:0") for a in inputs.nested_fields(128, patches, inputs.SEED_C3 + 17 * k)]
          for k in range(count)]
    o = _opts(mg, tol=1e-10, prec="mixed", max_cycles=60)
    ws = mg.Workspace(mg.mg_batch_hier_workspace_bytes(hs, o))
    u = [[torch.empty_like(x) for x in fi] for fi in fs]
    mg.mg_solve_batch_hier(hs, fs, u=u, opts=o, workspace=ws)     # warm-up (graph capture per lane)
    mg.mg_solve_batch_hier(hs, fs, u=u, opts=o, workspace=ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        _, st = mg.mg_solve_batch_hier(hs, fs, u=u, opts=o, workspace=ws)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    ups = sum(x["cell_updates"] for x in st)
    wss = [mg.Workspace(mg.mg_workspace_bytes(H, o)) for H in hs]
    us = [[torch.empty_like(x) for x in fi] for fi in fs]
    for _ in range(2):
        for H, fi, ui, w in zip(hs, fs, us, wss):
            mg.mg_solve_hierarchy(H, fi, u=ui, opts=o, workspace=w)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        for H, fi, ui, w in zip(hs, fs, us, wss):
            mg.mg_solve_hierarchy(H, fi, u=ui, opts=o, workspace=w)
    torch.cuda.synchronize()
    dts = (time.perf_counter() - t0) / reps
    same = all(bool(torch.equal(a, b)) for ai, bi in zip(u, us) for a, b in zip(ai, bi))
    return dict(workload="%d independent hierarchies of 128^3 + 3 nested 128^3 patches, mixed, tol 1e-10" % count,
                ms_per_batch=round(dt * 1e3, 3), value=round(ups / dt / 1e6, 1), unit="Mcell-updates/s",
                cycles=[x["cycles"] for x in st], sequential_ms=round(dts * 1e3, 3), speedup=round(dts / dt, 2),
                bit_identical_to_solo=same)


def time_c1(mg, torch, reps=10):
    """The 64^3 periodic workload: FP64 V(2,2) solve to a 1e-10 relative residual, then psi = -G4 phi;
    median of `reps` repeats after 2 warm-ups, each from a fresh zero start."""
    from paper_1103_6031_amd import inputs
    N = 64
    h = inputs.BOX / N
    H = mg.Hier(N, h)
    ft = torch.from_numpy(inputs.c1_input()).to("cuda:0")
    o = _opts(mg, tol=1e-10, prec="fp64", max_cycles=60)
    ws = mg.Workspace(mg.mg_workspace_bytes(H, o))
    wl = mg.Workspace(mg.lpt_workspace_bytes(H, 1))
    u = torch.empty_like(ft)
    ts, tl = [], []
    for i in range(reps + 2):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, st = mg.mg_solve_level(ft, h, u=u, opts=o, workspace=ws)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        mg.lpt_displacements(H, [u], scale=-1.0, workspace=wl)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        if i >= 2:
            ts.append(t1 - t0)
            tl.append(t2 - t0)
    ms = 1e3 * sorted(ts)[len(ts) // 2]
    # the same solve as one captured graph: the cycle count the converging solve needed, run as a
    # fixed-cycle solve (no per-cycle readback) and captured whole; replayed and timed the same way
    of = _opts(mg, prec="fp64", max_cycles=st["cycles"], fixed_cycles=True)
    uf = torch.empty_like(ft)
    mg.mg_solve_level(ft, h, u=uf, opts=of, workspace=ws)
    torch.cuda.synchronize()
    eager = uf.clone()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        mg.mg_solve_level(ft, h, u=uf, opts=of, workspace=ws)
    tg = []
    for i in range(reps + 2):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g.replay()
        torch.cuda.synchronize()
        if i >= 2:
            tg.append(time.perf_counter() - t0)
    _, rel_g = mg.mg_residual_hierarchy(H, [ft], [uf])
    return dict(workload="periodic 64^3 BBKS, FP64 V(2,2) to rel. residual 1e-10, then psi = -G4 phi",
                ms_per_solve=round(ms, 3), ms_with_displacements=round(1e3 * sorted(tl)[len(tl) // 2], 3),
                cycles=st["cycles"], rel_res=st["rel_res"],
                value=round(st["cell_updates"] / (ms * 1e-3) / 1e6, 1), unit="Mcell-updates/s", repeats=reps,
                captured_graph=dict(ms_per_solve=round(1e3 * sorted(tg)[len(tg) // 2], 3), cycles=st["cycles"],
                                    rel_res=rel_g, bit_identical_to_eager=bool(torch.equal(uf, eager)),
                                    note="the converging solve's cycle count as one fixed-cycle solve captured "
                                         "whole into a graph by the caller"))


def time_lla(mg, torch, H, psi1, psi2, reps=10):
    """LLA baryon overdensity (Section 5.3) of the step's first- plus second-order displacements:
    median of `reps` calls after 2 warm-ups, HIP events on the launch stream.  Model bytes per
    cell: 6 displacement reads + 1 write (56 B), then the renormalisation's sum (8 B) and
    subtraction (16 B)."""
    ws = mg.Workspace(mg.lpt_workspace_bytes(H, 3))
    delta = torch.empty_like(psi1[0])
    ts = []
    for i in range(reps + 2):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        mg.lpt_lla_density(H, [psi1], [psi2], delta=[delta], workspace=ws)
        e1.record()
        torch.cuda.synchronize()
        if i >= 2:
            ts.append(e0.elapsed_time(e1))
    ms = sorted(ts)[len(ts) // 2]
    cells = psi1[0].numel()
    return dict(workload="LLA baryon overdensity 1/det(I + dL/dq) - 1 of psi1 + psi2, %d^3, renormalised"
                % round(cells ** (1 / 3)), ms_per_call=round(ms, 3), value=round(cells / (ms * 1e-3) / 1e6, 1),
                unit="Mcells/s", model_bytes_per_cell=80, model_gbs=round(80 * cells / (ms * 1e-3) / 1e9, 1),
                delta_min=float(delta.min()), delta_max=float(delta.max()), repeats=reps)


def time_highorder(mg, torch, ft, h, tol, reps=3):
    """The solve with the 4th- and 6th-order Laplacians of Table 1 (13 and 19 points), FP64, on the
    step's density: median of `reps` solves after one warm-up, HIP events on the launch stream,
    and the finest half-sweep timed by the library's events.  That half-sweep is out of place:
    per cell it reads the iterate and f and writes every cell, 24 B (the colour-split in-place
    half-sweep of the 7-point path moves 12 B per cell, its updated half only)."""
    n = ft.shape[0]
    res = dict(workload="periodic %d^3 BBKS, V(2,2) with the order-4 / order-6 Laplacian, tol %g; FP64, and mixed "
                        "(FP32 inner cycles inside FP64 defect correction)" % (n, tol))
    fz = ft - ft.mean()
    wsp = mg.Workspace(mg.spec_workspace_bytes(ft.shape))
    for order in (4, 6):
        # the exact discrete solution of this order (eigenvalue division by the FFT), the fixed
        # point both solves converge to
        exact = mg.spec_poisson(fz, h, order, workspace=wsp)
        o = _opts(mg, tol=tol, max_cycles=40)
        ws = mg.Workspace(mg.mg_ho_workspace_bytes(n, order))
        u = torch.empty_like(ft)
        ts = []
        for i in range(reps + 1):
            if i == 1:
                mg.mg_kprof_read()
                mg.mg_kprof_enable(True)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            _, st = mg.mg_solve_level_ho(ft, h, order, u=u, opts=o, workspace=ws)
            e1.record()
            torch.cuda.synchronize()
            if i == 1:
                mg.mg_kprof_enable(False)
                kms, kn, kb = mg.mg_kprof_read()
            if i >= 1:
                ts.append(e0.elapsed_time(e1))
        ms = sorted(ts)[len(ts) // 2]
        u64 = u.clone()
        us = kms * 1e3 / max(kn, 1)
        res["order%d" % order] = dict(ms_per_solve=round(ms, 3), cycles=st["cycles"], rel_res=st["rel_res"],
                                      rel_rms_vs_exact=_rel_zero_mean(torch, u64, exact),
                                      value=round(st["cell_updates"] / (ms * 1e-3) / 1e6, 1),
                                      unit="Mcell-updates/s", half_sweep_avg_us=round(us, 2),
                                      half_sweep_launches=kn,
                                      half_sweep_gbs=round(kb / max(kn, 1) / (us * 1e-6) / 1e9, 1) if kn else None)
        om = _opts(mg, tol=tol, max_cycles=60, prec="mixed")
        tm = []
        for i in range(reps + 1):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            _, sm = mg.mg_solve_level_ho(ft, h, order, u=u, opts=om, workspace=ws)
            e1.record()
            torch.cuda.synchronize()
            if i >= 1:
                tm.append(e0.elapsed_time(e1))
        msm = sorted(tm)[len(tm) // 2]
        dev = float(torch.sqrt(torch.mean((u - u64) ** 2)) / torch.sqrt(torch.mean(u64 ** 2)))
        res["order%d" % order]["mixed"] = dict(ms_per_solve=round(msm, 3), cycles=sm["cycles"], rel_res=sm["rel_res"],
                                               value=round(sm["cell_updates"] / (msm * 1e-3) / 1e6, 1),
                                               rel_rms_vs_fp64=dev, rel_rms_vs_exact=_rel_zero_mean(torch, u, exact))
        del exact
    return res


def _rel_zero_mean(torch, x, exact):
    """Relative RMS of x (its mean removed: the periodic solution is fixed up to a constant)
    against the zero-mean exact solution."""
    d = (x - x.mean()) - exact
    return float(torch.sqrt(torch.mean(d * d)) / torch.sqrt(torch.mean(exact * exact)))


def time_highorder_zoom(mg, torch, reps=2):
    """The zoom hierarchy with the sixth-order operators throughout (the order of the paper's own
    nested results): 128^3 base with three centred 128^3 patches, FP64 solve with the order-6
    Laplacian (Table 1) and order-5 flux matching (Table 2), sixth-order displacements, tau with
    D = G6 o G6, the second solve and its displacements."""
    from paper_1103_6031_amd import inputs
    patches, fl = inputs.c3_input()
    H = mg.Hier(128, inputs.BOX / 128, patches)
    f = [torch.from_numpy(a).to("cuda:0") for a in fl]
    o = _opts(mg, tol=1e-10, max_cycles=60)
    ws = mg.Workspace(mg.mg_ho_hierarchy_workspace_bytes(H, 6))
    wl1 = mg.Workspace(mg.lpt_workspace_bytes(H, 1))
    wl2 = mg.Workspace(mg.lpt_workspace_bytes(H, 2))

    def step():
        phi, s1 = mg.mg_solve_hierarchy_ho(H, 6, f, opts=o, workspace=ws)
        mg.lpt_displacements(H, phi, scale=-1.0, workspace=wl1, grad_order=6)
        tau = mg.lpt2_source(H, phi, workspace=wl2, grad_order=6)
        phi2, s2 = mg.mg_solve_hierarchy_ho(H, 6, tau, opts=o, workspace=ws)
        mg.lpt_displacements(H, phi2, scale=-3.0 / 7.0, workspace=wl1, grad_order=6)
        return s1, s2

    step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        s1, s2 = step()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    return dict(workload="128^3 base + 3 nested 128^3 patches, order-6 Laplacian / order-5 flux matching / "
                         "sixth-order gradient, 2LPT, FP64, tol 1e-10",
                ms_per_step=round(dt * 1e3, 3), cycles=[s1["cycles"], s2["cycles"]],
                rel_res=[s1["rel_res"], s2["rel_res"]],
                value=round((s1["cell_updates"] + s2["cell_updates"]) / dt / 1e6, 1), unit="Mcell-updates/s")


def spectral_bytes(n, P, what):
    """Algorithmic HBM bytes of one call of the three-pass FFT pipeline on an n-cell field
    transformed on P points per axis (P = n periodic, the padded length isolated): every pass
    reads and writes each stored complex point once (16 B); the first pass reads the real field
    (8 B), the last writes real outputs (8 B each, read and written when added).  what: "deconv"
    (one multiplier, one output) or "hybrid" (two multiplier passes: x+iy and z, added to three
    outputs)."""
    n0, n1, n2 = n
    p0, p1, p2 = P
    w1 = n0 * n1 * p2
    w2 = n0 * p1 * p2
    cells = n0 * n1 * n2
    fwd = 8 * cells + 16 * w1 + 16 * w1 + 16 * w2          # z pass (real in), y pass
    mid = 16 * w2 + 16 * w2 + 16 * w2 + 16 * w1            # x pass fused, y inverse
    if what == "deconv":
        return fwd + mid + 16 * w1 + 8 * cells
    return fwd + 2 * mid + (16 * w1 + 32 * cells) + (16 * w1 + 16 * cells)


def time_spectral(mg, torch, ft, reps=5):
    """Section 3.5 on the GPU: the hybrid Poisson correction on the periodic 256^3 base (a pure
    FFT Poisson displacement when added to the multigrid one) and on a 128^3 patch zero-padded to
    256^3 (the finest level of the zoom hierarchy), and the cell-average deconvolution of the
    256^3 density.  Median of `reps` calls after one warm-up, HIP events on the launch stream;
    GB/s from the algorithmic bytes of spectral_bytes."""
    from paper_1103_6031_amd import inputs
    n = ft.shape[0]
    h = inputs.BOX / n
    res = {}

    def clock(fn):
        ts = []
        for i in range(reps + 1):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            if i:
                ts.append(e0.elapsed_time(e1))
        return sorted(ts)[len(ts) // 2]

    out = [torch.zeros_like(ft) for _ in range(3)]
    ws = mg.Workspace(mg.spec_workspace_bytes(ft.shape))
    ms = clock(lambda: mg.lpt_hybrid_correction(ft, h, out, workspace=ws))
    b = spectral_bytes(ft.shape, ft.shape, "hybrid")
    res["hybrid_periodic_%d" % n] = dict(ms=round(ms, 3), gbs=round(b / (ms * 1e-3) / 1e9, 1),
                                         algorithmic_bytes=b, transforms="1 forward + 2 inverse complex %d^3" % n)
    patch = ft[64:192, 64:192, 64:192].contiguous()
    outp = [torch.zeros_like(patch) for _ in range(3)]
    wsp = mg.Workspace(mg.spec_workspace_bytes(patch.shape, isolated=True))
    ms = clock(lambda: mg.lpt_hybrid_correction(patch, h / 2, outp, isolated=True, workspace=wsp))
    b = spectral_bytes(patch.shape, (256, 256, 256), "hybrid")
    res["hybrid_isolated_128_pad256"] = dict(ms=round(ms, 3), gbs=round(b / (ms * 1e-3) / 1e9, 1),
                                             algorithmic_bytes=b)
    dec = torch.empty_like(ft)
    ms = clock(lambda: mg.spec_deconvolve(ft, mg.SPEC_FV_DECONV, out=dec, workspace=ws))
    b = spectral_bytes(ft.shape, ft.shape, "deconv")
    res["fv_deconvolve_%d" % n] = dict(ms=round(ms, 3), gbs=round(b / (ms * 1e-3) / 1e9, 1), algorithmic_bytes=b)
    res["workload"] = ("Section 3.5 on the %d^3 BBKS density: hybrid correction periodic, the same on a 128^3 patch "
                       "isolated (zero-padded to 256^3), cell-average deconvolution; FP64" % n)
    return res


def time_c3(mg, torch, reps=3):
    """The zoom hierarchy: 128^3 base with three centred 128^3 patches, the 2LPT chain (solve,
    displacements, tau, solve, displacements) in both precisions."""
    from paper_1103_6031_amd import inputs
    patches, fl = inputs.c3_input()
    H = mg.Hier(128, inputs.BOX / 128, patches)
    f = [torch.from_numpy(a).to("cuda:0") for a in fl]
    wl1 = mg.Workspace(mg.lpt_workspace_bytes(H, 1))
    wl2 = mg.Workspace(mg.lpt_workspace_bytes(H, 2))
    res = dict(workload="128^3 base + 3 nested 128^3 patches (1024^3 effective), 2LPT, tol 1e-10",
               cells=int(128 ** 3 * 4))
    for prec in ("mixed", "fp64"):
        o = _opts(mg, tol=1e-10, prec=prec, max_cycles=60)
        ws = mg.Workspace(mg.mg_workspace_bytes(H, o))

        def step():
            phi, s1 = mg.mg_solve_hierarchy(H, f, opts=o, workspace=ws)
            mg.lpt_displacements(H, phi, scale=-1.0, workspace=wl1)
            tau = mg.lpt2_source(H, phi, workspace=wl2)
            phi2, s2 = mg.mg_solve_hierarchy(H, tau, opts=o, workspace=ws)
            mg.lpt_displacements(H, phi2, scale=-3.0 / 7.0, workspace=wl1)
            return s1, s2

        step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            s1, s2 = step()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        res[prec] = dict(ms_per_step=round(dt * 1e3, 3), cycles=[s1["cycles"], s2["cycles"]],
                         rel_res=[s1["rel_res"], s2["rel_res"]],
                         value=round((s1["cell_updates"] + s2["cell_updates"]) / dt / 1e6, 1),
                         unit="Mcell-updates/s")
        if prec == "mixed":
            # the inner-cycle tuner on this shape (outside the timed region), then the step again
            best, ms = mg.mg_tune_inner(H, f, opts=o, workspace=ws)
            step()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                s1, s2 = step()
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / reps
            res["mixed_tuned"] = dict(inner=best, solve_ms_per_count=[round(m, 3) for m in ms],
                                      ms_per_step=round(dt * 1e3, 3), cycles=[s1["cycles"], s2["cycles"]])
    return res


def time_density(mg, torch, reps=3):
    """Sections 2.1-2.3 on the zoom workload's geometry (128^3 base, three nested 128^3 patches,
    padded domains of 256^3): kernels per level, noise refinement and nested convolutions from the
    tabulated BBKS real-space transfer function and seeded unit normals already in HBM; median of
    `reps` calls after one warm-up.  Then the 2LPT chain (mixed precision, tol 1e-10) on that
    density, with the hybrid correction (Section 3.5.2) of the first-order displacement on the
    finest patch, zero-padded to 256^3."""
    from paper_1103_6031_amd import inputs
    patches, table, dr, xi = inputs.c3_multiscale_input()
    H = mg.Hier(128, inputs.BOX / 128, patches)
    tab = torch.from_numpy(table).to("cuda:0")
    xd = [torch.from_numpy(x).to("cuda:0") for x in xi]
    ws = mg.Workspace(mg.ic_density_workspace_bytes(H))
    delta = [torch.empty(H.dims(p), dtype=torch.float64, device="cuda:0") for p in range(H.nlev)]
    ts = []
    for i in range(reps + 1):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        mg.ic_multiscale_density(H, tab, dr, xd, delta=delta, workspace=ws)
        e1.record()
        torch.cuda.synchronize()
        if i:
            ts.append(e0.elapsed_time(e1))
    res = dict(workload="128^3 base + 3 nested 128^3 patches: multi-scale density (BBKS real-space kernel, "
                        "sub-grid kernel mean), then the mixed-precision 2LPT chain on it",
               density_ms=round(sorted(ts)[len(ts) // 2], 3),
               density_rms=[round(float(torch.sqrt(torch.mean(d * d))), 5) for d in delta])
    del ws
    o = _opts(mg, tol=1e-10, prec="mixed", max_cycles=60)
    wsm = mg.Workspace(mg.mg_workspace_bytes(H, o))
    wl1 = mg.Workspace(mg.lpt_workspace_bytes(H, 1))
    wl2 = mg.Workspace(mg.lpt_workspace_bytes(H, 2))
    top = H.nlev - 1
    wsh = mg.Workspace(mg.spec_workspace_bytes(H.dims(top), isolated=True))

    def step():
        phi, s1 = mg.mg_solve_hierarchy(H, delta, opts=o, workspace=wsm)
        psi = mg.lpt_displacements(H, phi, scale=-1.0, workspace=wl1)
        mg.lpt_hybrid_correction(delta[top], H.h(top), psi[top], isolated=True, scale=-1.0, workspace=wsh)
        tau = mg.lpt2_source(H, phi, workspace=wl2)
        phi2, s2 = mg.mg_solve_hierarchy(H, tau, opts=o, workspace=wsm)
        mg.lpt_displacements(H, phi2, scale=-3.0 / 7.0, workspace=wl1)
        return s1, s2

    step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        s1, s2 = step()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    res["two_lpt_mixed"] = dict(ms_per_step=round(dt * 1e3, 3), cycles=[s1["cycles"], s2["cycles"]],
                                rel_res=[s1["rel_res"], s2["rel_res"]],
                                note="includes the hybrid correction of psi_1 on the finest patch")
    return res


def time_smoother_512(mg, torch, ft, h, tol):
    """The finest-level smoother on a working set four times the 256 MB Infinity Cache: the step's
    256^3 density tiled 2 x 2 x 2 (a periodic 512^3 field with the same spectrum on its even modes),
    one 1LPT solve per precision after a warm-up solve, every finest-level smoother launch of it
    timed by the library's dispatch-stamped events.  A plain 1 GiB device copy is timed beside it
    (HIP events) as the achievable read + write bandwidth."""
    n = 2 * ft.shape[0]
    f5 = ft.repeat(2, 2, 2).contiguous()
    h5 = h / 2.0
    H5 = mg.Hier(n, h5)
    res = dict(workload="periodic %d^3 (the %d^3 density tiled 2x2x2), 1LPT solve, tol %g" % (n, n // 2, tol),
               n=n, u_plus_f_fp32_mb=round(2 * 4 * n ** 3 / 1e6, 1))
    u = torch.empty_like(f5)
    for prec, w in (("mixed", 4), ("fp64", 8)):
        o = _opts(mg, tol=tol, prec=prec, max_cycles=60)
        ws = mg.Workspace(mg.mg_workspace_bytes(H5, o))
        mg.mg_solve_level(f5, h5, u=u, opts=o, workspace=ws)
        torch.cuda.synchronize()
        mg.mg_kprof_read()
        mg.mg_kprof_enable(True)
        _, st = mg.mg_solve_level(f5, h5, u=u, opts=o, workspace=ws)
        torch.cuda.synchronize()
        mg.mg_kprof_enable(False)
        kms, kn, kb = mg.mg_kprof_read()
        us = 1e3 * kms / max(kn, 1)
        gbs = kb / (kms * 1e-3) / 1e9 if kms > 0 else 0.0
        res["fp32" if prec == "mixed" else "fp64"] = dict(
            avg_launch_us=round(us, 2), launches=kn, algorithmic_bytes_per_launch=int(kb / max(kn, 1)),
            achieved=round(gbs, 1), frac=round(gbs / HBM_PEAK_GBS, 4), cycles=st["cycles"], rel_res=st["rel_res"])
        del ws
    del u, f5
    src = torch.ones(256 * 1024 * 1024, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    ts = []
    for i in range(6):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        if i >= 1:
            ts.append(e0.elapsed_time(e1))
    ms = sorted(ts)[len(ts) // 2]
    res["copy_1gib_gbs"] = round(2 * src.numel() * 4 / (ms * 1e-3) / 1e9, 1)
    del src, dst
    torch.cuda.empty_cache()
    return res


def cpu_baseline(f, h):
    """The oracle's FAS V-cycle on the same input: a bounded sample of two cycles."""
    import numpy as np
    from oracle import periodic
    fz = f - f.mean()
    u = np.zeros_like(fz)
    t0 = time.perf_counter()
    ncyc = 2
    for _ in range(ncyc):
        u = periodic.vcycle(u, fz, h)
    dt = time.perf_counter() - t0
    ups = periodic.cell_updates(f.shape[0], ncyc)
    try:
        affinity = len(os.sched_getaffinity(0))
    except Exception:
        affinity = os.cpu_count()
    return dict(value=ups / dt / 1e6, unit="Mcell-updates/s", cores=1, kind="oracle",
                sample="%d FAS V(2,2) cycles of the numpy oracle on the same %d^3 input (%.1f s); "
                       "single-threaded numpy, 1 core used of %d" % (ncyc, f.shape[0], dt, affinity))


def calib_copies(torch):
    """Three plain 256 MiB device-to-device copies: the counter calibration of the traffic profiles."""
    src = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst


def main():
    a = parse()
    global GRAPH
    GRAPH = not a.no_graph
    if a.gpus != 1:
        print("bench.py measures one GPU only: the multigrid hot path here runs on a single device "
              "(sharding across GPUs is not built); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    serve_host = None
    if a.serve_requests > 0:
        # the serving trace's densities are made by worker processes before this process
        # touches the GPU
        from paper_1103_6031_amd import serve
        reqs = serve.trace(a.serve_requests, 20.0)
        serve_host = serve.host_fields(reqs, workers=8)
    import numpy as np
    import torch
    from paper_1103_6031_amd import inputs, mgic as mg

    N = a.n
    h = inputs.BOX / N
    f = inputs.gaussian_field(N, inputs.SEED_C2)
    ft = torch.from_numpy(f).to("cuda:0")
    H = mg.Hier(N, h)
    torch.cuda.synchronize()

    if a.only:
        line = {}
        for leg in a.only.split(","):
            if leg == "roof512":
                line["roofline_512"] = time_smoother_512(mg, torch, ft, h, a.tol)
            elif leg == "c1":
                line["solve_c1"] = time_c1(mg, torch)
            elif leg == "c3":
                line["zoom_c3"] = time_c3(mg, torch)
            elif leg == "hoz":
                line["highorder_zoom"] = time_highorder_zoom(mg, torch)
            elif leg == "c4":
                line["batch_c4"] = time_batch(mg, torch, max(2, a.steps // 2))
            elif leg == "bh":
                line["batch_hier"] = time_batch_hier(mg, torch)
            elif leg == "spectral":
                line["spectral"] = time_spectral(mg, torch, ft)
            elif leg == "density":
                line["density_c3"] = time_density(mg, torch)
            elif leg == "ho":
                line["highorder"] = time_highorder(mg, torch, ft, h, a.tol)
            else:
                raise SystemExit("unknown leg " + leg)
        if a.pmc_calib:
            calib_copies(torch)
        print(json.dumps(line), flush=True)
        return

    other = "fp64" if a.prec == "mixed" else "mixed"
    head, out_h = time_path(mg, torch, H, ft, h, a.prec, a.tol, a.steps, a.warmup, a.inner)
    side, out_s = time_path(mg, torch, H, ft, h, other, a.tol, max(1, a.steps // 2), 1)
    out_m, out_d = (out_h, out_s) if a.prec == "mixed" else (out_s, out_h)

    def rel(x, y):
        return float(torch.sqrt(torch.mean((x - y) ** 2)) / torch.sqrt(torch.mean(y ** 2)))

    acc = dict(phi1=rel(out_m[0], out_d[0]), psi1=max(rel(out_m[1][c], out_d[1][c]) for c in range(3)),
               tau=rel(out_m[2], out_d[2]), phi2=rel(out_m[3], out_d[3]),
               psi2=max(rel(out_m[4][c], out_d[4][c]) for c in range(3)))

    # each path's two solves against the exact discrete solution of the same right-hand side (the
    # 7-point symbol divided out by the FFT): phi1 from the density, phi2 from that path's tau
    wsp = mg.Workspace(mg.spec_workspace_bytes(ft.shape))
    e1 = mg.spec_poisson(ft - ft.mean(), h, 2, workspace=wsp)
    vs_exact = {}
    for name, out in (("mixed", out_m), ("fp64", out_d)):
        e2 = mg.spec_poisson(out[2] - out[2].mean(), h, 2, workspace=wsp)
        vs_exact[name] = dict(phi1=_rel_zero_mean(torch, out[0], e1), phi2=_rel_zero_mean(torch, out[3], e2))
        del e2
    del e1, wsp

    k = head["kernel"]
    roof = None
    if k["achieved_gbs"]:
        traffic = recorded_traffic() if (a.prec == "mixed" and N == 256) else None
        roof = dict(bound="hbm", achieved=round(k["achieved_gbs"], 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(k["achieved_gbs"] / HBM_PEAK_GBS, 4),
                    traffic=None if traffic is None else int(traffic),
                    kernel="finest-level red-black smoother (%s)" % ("fp32" if a.prec == "mixed" else "fp64"),
                    avg_launch_us=round(k["avg_us"], 2), launches=k["launches"], timed_steps=min(KPROF_STEPS, a.steps),
                    algorithmic_bytes_per_launch=int(k["bytes_per_launch"]))
    line = dict(metric=METRIC, value=round(head["value"], 1), unit="Mcell-updates/s", n_gpus=1, steps=a.steps,
                warmup=a.warmup, ms_per_step=round(head["ms_per_step"], 3), higher_is_better=True,
                scaling="weak", vs_baseline=None,
                dtype="f32+f64" if a.prec == "mixed" else "f64", data="synthetic",
                config=dict(workload="periodic %d^3 BBKS 2LPT (solve, grad, tau, solve, grad), tol %g" % (N, a.tol),
                            n=N, box=inputs.BOX, seed=inputs.SEED_C2, precision=a.prec, nu1=2, nu2=2),
                roofline=roof,
                cycles=dict(zip(("solve1", "solve2"), head["cycles"])),
                rel_res=head["rel_res"],
                mixed_vs_fp64_rel_rms=acc, rel_rms_vs_exact_solve=vs_exact)
    line[other + "_path"] = dict(value=round(side["value"], 1), ms_per_step=round(side["ms_per_step"], 3),
                                 cycles=side["cycles"],
                                 smoother_gbs=round(side["kernel"]["achieved_gbs"] or 0.0, 1),
                                 smoother_avg_launch_us=round(side["kernel"]["avg_us"], 2))
    if a.inner:
        line["config"]["inner"] = a.inner
    if roof is not None and not a.no_roof512 and N == 256:
        r5 = time_smoother_512(mg, torch, ft, h, a.tol)
        roof["beyond_infinity_cache"] = r5
    line["lla"] = time_lla(mg, torch, H, out_h[1], out_h[4])
    line["highorder"] = time_highorder(mg, torch, ft, h, a.tol)
    line["spectral"] = time_spectral(mg, torch, ft)
    if not a.no_c1c3:
        line["density_c3"] = time_density(mg, torch)
    if not a.no_c1c3:
        line["solve_c1"] = time_c1(mg, torch)
        line["zoom_c3"] = time_c3(mg, torch)
        line["highorder_zoom"] = time_highorder_zoom(mg, torch)
    if not a.no_batch:
        line["batch_c4"] = time_batch(mg, torch, max(2, a.steps // 2))
        line["batch_hier"] = time_batch_hier(mg, torch)
    if serve_host is not None:
        wl = ("%d requests, Poisson %g/s, base {64,128,256}^3 with 0-3 patches of {64,96,128}^3, 1LPT/2LPT 50/50, "
              "%s, tol 1e-10, %d slots, %g GB budget")
        summary, _, _ = serve.serve_trace(reqs, slots=4, budget_gb=16.0, prec="mixed", host=serve_host)
        line["serving_c5"] = dict(workload=wl % (len(reqs), 20.0, "mixed", 4, 16.0), **summary)
        # the plain FP64 path on the same trace, as the reference beside the mixed one
        summary, _, _ = serve.serve_trace(reqs, slots=4, budget_gb=16.0, prec="fp64", host=serve_host)
        line["serving_c5_fp64"] = dict(workload=wl % (len(reqs), 20.0, "fp64", 4, 16.0), **summary)
        # under load: the same requests arriving ten times faster with a 4 GB budget, so that
        # admission by footprint binds (a 256^3-base request holds about 1.5-2.5 GB)
        fast = serve.trace(a.serve_requests, 200.0)
        summary, _, _ = serve.serve_trace(fast, slots=4, budget_gb=4.0, prec="mixed", host=serve_host)
        line["serving_c5_loaded"] = dict(workload=wl % (len(fast), 200.0, "mixed", 4, 4.0), **summary)
    if a.pmc_calib:
        calib_copies(torch)
    if not a.no_cpu:
        line["cpu_baseline"] = cpu_baseline(f, h)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
