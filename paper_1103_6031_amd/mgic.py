"""Python binding of libmgic (the C ABI declared in include/mgic.h).

Argument marshalling only: every step of the computation runs in the HIP library.  PyTorch
provides device memory (inputs, outputs and workspace tensors) and the current HIP stream.
The names mirror the C entry points.  If the shared library is missing, importing this module
raises; there is no fallback.
"""

import ctypes
import math
import os
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("MGIC_LIB") or os.path.join(_HERE, "libmgic.so")   # MGIC_LIB: another build

if not os.path.exists(LIB_PATH):
    raise ImportError("libmgic.so is not built (run __graft_entry__.build() or "
                      "python paper_1103_6031_amd/build.py)")
_lib = ctypes.CDLL(LIB_PATH)

MG_MAX_LEVELS = 8
MG_OK, MG_EINVAL, MG_ENOCONV, MG_EDIVERGED, MG_EHIP = 0, -1, -2, -3, -4
MG_FP64, MG_MIXED = 0, 1
MG_USE_INITIAL_GUESS = 0x1
MG_FIXED_CYCLES = 0x2
MG_NO_GRAPH = 0x4
MG_NO_MEAN_FIX = 0x8

_ERRNAMES = {MG_EINVAL: "MG_EINVAL", MG_ENOCONV: "MG_ENOCONV", MG_EDIVERGED: "MG_EDIVERGED", MG_EHIP: "MG_EHIP"}


class mg_level(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int * 3), ("off", ctypes.c_int * 3), ("h", ctypes.c_double)]


class mg_hier(ctypes.Structure):
    _fields_ = [("nlev", ctypes.c_int), ("lev", mg_level * MG_MAX_LEVELS)]


class mg_opts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_cycles", ctypes.c_int), ("nu1", ctypes.c_int),
                ("nu2", ctypes.c_int), ("prec", ctypes.c_int), ("flags", ctypes.c_uint), ("inner", ctypes.c_int)]


class mg_stats(ctypes.Structure):
    _fields_ = [("cycles", ctypes.c_int), ("rel_res", ctypes.c_double), ("f_mean_removed", ctypes.c_double),
                ("res_hist", ctypes.c_double * 64), ("cell_updates", ctypes.c_longlong)]

    def to_dict(self):
        n = min(self.cycles, 64)
        return dict(cycles=self.cycles, rel_res=self.rel_res, f_mean=self.f_mean_removed,
                    history=list(self.res_hist[:n]), cell_updates=self.cell_updates)


_P = ctypes.c_void_p
_PP = ctypes.POINTER(ctypes.c_void_p)
_sz = ctypes.c_size_t

_sig = {
    "mg_workspace_bytes": (_sz, [ctypes.POINTER(mg_hier), ctypes.POINTER(mg_opts)]),
    "mg_solve_level": (ctypes.c_int, [ctypes.c_int, ctypes.c_double, _P, _P, ctypes.POINTER(mg_opts),
                                      ctypes.POINTER(mg_stats), _P, _sz, _P]),
    "mg_solve_hierarchy": (ctypes.c_int, [ctypes.POINTER(mg_hier), _PP, _PP, ctypes.POINTER(mg_opts),
                                          ctypes.POINTER(mg_stats), _P, _sz, _P]),
    "mg_solve_hierarchy_noalloc": (ctypes.c_int, [ctypes.POINTER(mg_hier), _PP, _PP, ctypes.POINTER(mg_opts),
                                                  ctypes.POINTER(mg_stats), _P]),
    "mg_ho_workspace_bytes": (_sz, [ctypes.c_int, ctypes.c_int]),
    "mg_solve_level_ho": (ctypes.c_int, [ctypes.c_int, ctypes.c_double, ctypes.c_int, _P, _P,
                                         ctypes.POINTER(mg_opts), ctypes.POINTER(mg_stats), _P, _sz, _P]),
    "mg_ho_hierarchy_workspace_bytes": (_sz, [ctypes.POINTER(mg_hier), ctypes.c_int]),
    "mg_solve_hierarchy_ho": (ctypes.c_int, [ctypes.POINTER(mg_hier), ctypes.c_int, _PP, _PP, ctypes.POINTER(mg_opts),
                                             ctypes.POINTER(mg_stats), _P, _sz, _P]),
    "mg_ghost_fill_ho": (ctypes.c_int, [ctypes.POINTER(mg_hier), ctypes.c_int, ctypes.c_int, _PP, _P, ctypes.c_int,
                                        _P]),
    "mg_residual_hierarchy": (ctypes.c_int, [ctypes.POINTER(mg_hier), _PP, _PP, _PP,
                                             ctypes.POINTER(ctypes.c_double), _P, _sz, _P]),
    "lpt_workspace_bytes": (_sz, [ctypes.POINTER(mg_hier), ctypes.c_int]),
    "lpt_displacements": (ctypes.c_int, [ctypes.POINTER(mg_hier), _PP, _PP, ctypes.c_int, ctypes.c_double, _P, _sz,
                                         _P]),
    "lpt2_source": (ctypes.c_int, [ctypes.POINTER(mg_hier), _PP, _PP, ctypes.c_int, _P, _sz, _P]),
    "lpt_displacements_and_source": (ctypes.c_int, [ctypes.POINTER(mg_hier), _PP, _PP, ctypes.c_int, ctypes.c_double,
                                                    _PP, _P, _sz, _P]),
    "lpt_lla_density": (ctypes.c_int, [ctypes.POINTER(mg_hier), _PP, _PP, _PP, _P, _sz, _P]),
    "spec_workspace_bytes": (_sz, [ctypes.POINTER(ctypes.c_int), ctypes.c_int]),
    "spec_deconvolve": (ctypes.c_int, [ctypes.POINTER(ctypes.c_int), ctypes.c_int, ctypes.c_int, _P, _P, _P, _sz,
                                       _P]),
    "spec_poisson": (ctypes.c_int, [ctypes.POINTER(ctypes.c_int), ctypes.c_double, ctypes.c_int, _P, _P, _P, _sz,
                                    _P]),
    "lpt_hybrid_correction": (ctypes.c_int, [ctypes.POINTER(ctypes.c_int), ctypes.c_double, ctypes.c_int,
                                             ctypes.c_int, ctypes.c_int, ctypes.c_double, _P, _PP, _P, _sz, _P]),
    "ic_density_workspace_bytes": (_sz, [ctypes.POINTER(mg_hier)]),
    "ic_multiscale_density": (ctypes.c_int, [ctypes.POINTER(mg_hier), _P, ctypes.c_int, ctypes.c_double,
                                             ctypes.c_int, _PP, _PP, _P, _sz, _P]),
    "mg_batch_workspace_bytes": (_sz, [ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(mg_opts)]),
    "mg_solve_batch": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double),
                                      _PP, _PP, ctypes.POINTER(mg_opts), ctypes.POINTER(mg_stats), _P, _sz, _P]),
    "mg_batch_hier_workspace_bytes": (_sz, [ctypes.c_int, _P, ctypes.POINTER(mg_opts)]),
    "mg_solve_batch_hier": (ctypes.c_int, [ctypes.c_int, _P, _P, _P, ctypes.POINTER(mg_opts),
                                           ctypes.POINTER(mg_stats), _P, _sz, _P]),
    "mg_smooth_level": (ctypes.c_int, [ctypes.c_int, ctypes.c_double, _P, _P, ctypes.c_int, ctypes.c_int,
                                       _P, _sz, _P]),
    "mg_ghost_fill": (ctypes.c_int, [ctypes.POINTER(mg_hier), ctypes.c_int, _PP, _P, ctypes.c_int, _P]),
    "mg_batch_tune_candidates": (ctypes.c_int, []),
    "mg_batch_force_shape": (ctypes.c_int, [ctypes.c_int]),
    "mg_tune_cache": (ctypes.c_int, [ctypes.c_char_p]),
    "mg_tune_inner": (ctypes.c_int, [ctypes.POINTER(mg_hier), _PP, _PP, ctypes.POINTER(mg_opts),
                                     ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double), _P, _sz, _P]),
    "mg_kprof_enable": (ctypes.c_int, [ctypes.c_int]),
    "mg_kprof_read": (ctypes.c_int, [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_longlong),
                                     ctypes.POINTER(ctypes.c_double)]),
    "mg_last_error": (ctypes.c_char_p, []),
}
for _name, (_res, _args) in _sig.items():
    _fn = getattr(_lib, _name)
    _fn.restype = _res
    _fn.argtypes = _args

EXPORTED = tuple(_sig)


class MGError(RuntimeError):
    def __init__(self, code, msg, stats=None):
        super().__init__("%s: %s" % (_ERRNAMES.get(code, str(code)), msg))
        self.code = code
        self.stats = stats


def _check(rc, stats=None):
    if rc != MG_OK:
        raise MGError(rc, _lib.mg_last_error().decode(), stats)


# ------------------------------------------------------------------------------------------------
# hierarchy description
# ------------------------------------------------------------------------------------------------

@dataclass
class Hier:
    """Periodic N0^3 base of spacing h0 plus nested patches [(n3, off3), ...] (outermost first)."""
    N0: int
    h0: float
    patches: List[Tuple[Tuple[int, int, int], Tuple[int, int, int]]] = field(default_factory=list)

    @property
    def nlev(self):
        return 1 + len(self.patches)

    def dims(self, p):
        return (self.N0,) * 3 if p == 0 else tuple(self.patches[p - 1][0])

    def h(self, p):
        return self.h0 / (2 ** p)

    def c_struct(self):
        H = mg_hier()
        H.nlev = self.nlev
        H.lev[0].n[:] = [self.N0] * 3
        H.lev[0].h = self.h0
        for p, (n, off) in enumerate(self.patches, start=1):
            H.lev[p].n[:] = list(n)
            H.lev[p].off[:] = list(off)
            H.lev[p].h = self.h(p)
        return H

    def cells(self):
        return sum(math.prod(self.dims(p)) for p in range(self.nlev))


def make_opts(tol=1e-10, max_cycles=50, nu1=2, nu2=2, prec="fp64", fixed_cycles=False, initial_guess=False,
              inner=0, graph=True, mean_fix=True):
    o = mg_opts()
    o.inner = inner
    o.tol = tol
    o.max_cycles = max_cycles
    o.nu1 = nu1
    o.nu2 = nu2
    o.prec = {"fp64": MG_FP64, "mixed": MG_MIXED}[prec] if isinstance(prec, str) else int(prec)
    o.flags = ((MG_FIXED_CYCLES if fixed_cycles else 0) | (MG_USE_INITIAL_GUESS if initial_guess else 0)
               | (0 if graph else MG_NO_GRAPH) | (0 if mean_fix else MG_NO_MEAN_FIX))
    return o


# ------------------------------------------------------------------------------------------------
# helpers
# ------------------------------------------------------------------------------------------------

def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dev(t, name):
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous():
        raise ValueError("%s must be a contiguous float64 CUDA tensor" % name)
    return t.data_ptr()


def _ptr_array(ptrs):
    arr = (ctypes.c_void_p * len(ptrs))(*ptrs)
    return ctypes.cast(arr, _PP), arr


class Workspace:
    """A device byte buffer aligned to 256 bytes (carved by the library)."""

    def __init__(self, nbytes, device=None):
        self.nbytes = int(nbytes)
        self.buf = torch.empty(self.nbytes + 256, dtype=torch.uint8, device=device or "cuda")
        base = self.buf.data_ptr()
        self.ptr = (base + 255) & ~255

    def fits(self, nbytes):
        return nbytes <= self.nbytes


def _ws(ws, need):
    if ws is None or not ws.fits(need):
        ws = Workspace(need)
    return ws


# ------------------------------------------------------------------------------------------------
# entry points
# ------------------------------------------------------------------------------------------------

def mg_workspace_bytes(hier: Hier, opts=None) -> int:
    H = hier.c_struct()
    o = opts or make_opts()
    n = _lib.mg_workspace_bytes(ctypes.byref(H), ctypes.byref(o))
    if n == 0:
        raise MGError(MG_EINVAL, _lib.mg_last_error().decode())
    return n


def mg_solve_level(f, h, u=None, opts=None, workspace=None, stream=None, check=True):
    """Periodic solve of L u = f - mean(f).  Returns (u, stats dict)."""
    n = f.shape[0]
    o = opts or make_opts()
    if u is None:
        u = torch.empty_like(f)
    need = mg_workspace_bytes(Hier(n, h), o)
    ws = _ws(workspace, need)
    st = mg_stats()
    rc = _lib.mg_solve_level(n, h, _dev(f, "f"), _dev(u, "u"), ctypes.byref(o), ctypes.byref(st),
                             ctypes.c_void_p(ws.ptr), ws.nbytes, _stream(stream))
    if check:
        _check(rc, st.to_dict())
    return u, st.to_dict()


def mg_ho_workspace_bytes(n: int, order: int) -> int:
    need = _lib.mg_ho_workspace_bytes(int(n), int(order))
    if need == 0:
        raise MGError(MG_EINVAL, _lib.mg_last_error().decode())
    return need


def mg_solve_level_ho(f, h, order, u=None, opts=None, workspace=None, stream=None, check=True):
    """Periodic solve of L_order u = f - mean(f) with the order-2/4/6 Laplacian.  Returns (u, stats dict)."""
    n = f.shape[0]
    if f.dim() != 3 or tuple(f.shape) != (n, n, n):
        raise ValueError("f must be an n^3 cube")
    o = opts or make_opts()
    if u is None:
        u = torch.empty_like(f)
    if tuple(u.shape) != tuple(f.shape):
        raise ValueError("u must have the shape of f")
    ws = _ws(workspace, mg_ho_workspace_bytes(n, order))
    st = mg_stats()
    rc = _lib.mg_solve_level_ho(n, h, int(order), _dev(f, "f"), _dev(u, "u"), ctypes.byref(o), ctypes.byref(st),
                                ctypes.c_void_p(ws.ptr), ws.nbytes, _stream(stream))
    if check:
        _check(rc, st.to_dict())
    return u, st.to_dict()


def mg_solve_hierarchy(hier: Hier, f: Sequence[torch.Tensor], u=None, opts=None, workspace=None, stream=None,
                       check=True):
    """Composite solve on a nested hierarchy.  Returns (u list, stats dict)."""
    o = opts or make_opts()
    if u is None:
        u = [torch.empty_like(x) for x in f]
    H = hier.c_struct()
    need = mg_workspace_bytes(hier, o)
    ws = _ws(workspace, need)
    fp, _fa = _ptr_array([_dev(x, "f") for x in f])
    up, _ua = _ptr_array([_dev(x, "u") for x in u])
    st = mg_stats()
    rc = _lib.mg_solve_hierarchy(ctypes.byref(H), fp, up, ctypes.byref(o), ctypes.byref(st),
                                 ctypes.c_void_p(ws.ptr), ws.nbytes, _stream(stream))
    if check:
        _check(rc, st.to_dict())
    return u, st.to_dict()


MG_SCRATCH_BYTES = 96 << 20   # the library's static scratch array (mgic.h)


def mg_solve_hierarchy_noalloc(hier: Hier, f: Sequence[torch.Tensor], u: Sequence[torch.Tensor], opts=None,
                               stream=None, check=True):
    """mg_solve_hierarchy without a workspace argument: the library's static device scratch array
    serves as the workspace, and the call allocates nothing.  u must be given (outputs are the
    caller's).  Returns (u list, stats dict)."""
    o = opts or make_opts()
    H = hier.c_struct()
    fp, _fa = _ptr_array([_dev(x, "f") for x in f])
    up, _ua = _ptr_array([_dev(x, "u") for x in u])
    st = mg_stats()
    rc = _lib.mg_solve_hierarchy_noalloc(ctypes.byref(H), fp, up, ctypes.byref(o), ctypes.byref(st),
                                         _stream(stream))
    if check:
        _check(rc, st.to_dict())
    return u, st.to_dict()


def mg_ho_hierarchy_workspace_bytes(hier: Hier, order: int) -> int:
    H = hier.c_struct()
    n = _lib.mg_ho_hierarchy_workspace_bytes(ctypes.byref(H), int(order))
    if n == 0:
        raise MGError(MG_EINVAL, _lib.mg_last_error().decode())
    return n


def mg_solve_hierarchy_ho(hier: Hier, order: int, f: Sequence[torch.Tensor], u=None, opts=None, workspace=None,
                          stream=None, check=True):
    """Composite solve with the order-2/4/6 Laplacian on a nested hierarchy.  Returns (u list, stats dict)."""
    o = opts or make_opts()
    if u is None:
        u = [torch.empty_like(x) for x in f]
    H = hier.c_struct()
    ws = _ws(workspace, mg_ho_hierarchy_workspace_bytes(hier, order))
    fp, _fa = _ptr_array([_dev(x, "f") for x in f])
    up, _ua = _ptr_array([_dev(x, "u") for x in u])
    st = mg_stats()
    rc = _lib.mg_solve_hierarchy_ho(ctypes.byref(H), int(order), fp, up, ctypes.byref(o), ctypes.byref(st),
                                    ctypes.c_void_p(ws.ptr), ws.nbytes, _stream(stream))
    if check:
        _check(rc, st.to_dict())
    return u, st.to_dict()


def mg_ghost_fill_ho(hier: Hier, order: int, p: int, u, flux_match=True, ghosts=None, stream=None):
    """The order/2 ghost layers of patch p (faces back to back, see split_ghosts_ho)."""
    R = order // 2
    nx, ny, nz = hier.dims(p)
    total = 2 * R * (ny * nz + nx * nz + nx * ny)
    if ghosts is None:
        ghosts = torch.empty(total, dtype=torch.float64, device=u[0].device)
    H = hier.c_struct()
    up, _ua = _ptr_array([_dev(x, "u") for x in u])
    _check(_lib.mg_ghost_fill_ho(ctypes.byref(H), int(order), int(p), up, _dev(ghosts, "ghosts"),
                                 1 if flux_match else 0, _stream(stream)))
    return ghosts


def split_ghosts_ho(hier: Hier, order: int, p: int, g):
    """View the 6 ghost faces as [(R,ny,nz), (R,ny,nz), (R,nx,nz), (R,nx,nz), (R,nx,ny), (R,nx,ny)]."""
    R = order // 2
    nx, ny, nz = hier.dims(p)
    shapes = [(R, ny, nz), (R, ny, nz), (R, nx, nz), (R, nx, nz), (R, nx, ny), (R, nx, ny)]
    out, o = [], 0
    for s in shapes:
        out.append(g[o:o + s[0] * s[1] * s[2]].view(*s))
        o += s[0] * s[1] * s[2]
    return out


def mg_residual_hierarchy(hier: Hier, f, u, r=None, workspace=None, stream=None):
    """Composite residual (covered coarse cells zero) and the relative norm."""
    if r is None:
        r = [torch.empty_like(x) for x in f]
    H = hier.c_struct()
    need = mg_workspace_bytes(hier, make_opts())
    ws = _ws(workspace, need)
    fp, _fa = _ptr_array([_dev(x, "f") for x in f])
    up, _ua = _ptr_array([_dev(x, "u") for x in u])
    rp, _ra = _ptr_array([_dev(x, "r") for x in r])
    rel = ctypes.c_double()
    _check(_lib.mg_residual_hierarchy(ctypes.byref(H), fp, up, rp, ctypes.byref(rel), ctypes.c_void_p(ws.ptr),
                                      ws.nbytes, _stream(stream)))
    return r, rel.value


def lpt_workspace_bytes(hier: Hier, what: int) -> int:
    H = hier.c_struct()
    n = _lib.lpt_workspace_bytes(ctypes.byref(H), what)
    if n == 0:
        raise MGError(MG_EINVAL, "invalid hierarchy")
    return n


def lpt_displacements(hier: Hier, phi, scale=1.0, out=None, workspace=None, stream=None, grad_order=4):
    """psi_c = scale * G_c phi per level (Table 1 gradient of order 4 or 6).  Returns a list of
    [psi_x, psi_y, psi_z] per level."""
    if out is None:
        out = [[torch.empty_like(x) for _ in range(3)] for x in phi]
    H = hier.c_struct()
    ws = _ws(workspace, lpt_workspace_bytes(hier, 1))
    pp, _pa = _ptr_array([_dev(x, "phi") for x in phi])
    op, _oa = _ptr_array([_dev(c, "out") for lvl in out for c in lvl])
    _check(_lib.lpt_displacements(ctypes.byref(H), pp, op, int(grad_order), float(scale), ctypes.c_void_p(ws.ptr),
                                  ws.nbytes, _stream(stream)))
    return out


def lpt2_source(hier: Hier, phi, tau=None, workspace=None, stream=None, grad_order=4):
    """Second-order source tau per level (composite mean removed), D = G o G of grad_order."""
    if tau is None:
        tau = [torch.empty_like(x) for x in phi]
    H = hier.c_struct()
    ws = _ws(workspace, lpt_workspace_bytes(hier, 2))
    pp, _pa = _ptr_array([_dev(x, "phi") for x in phi])
    tp, _ta = _ptr_array([_dev(x, "tau") for x in tau])
    _check(_lib.lpt2_source(ctypes.byref(H), pp, tp, int(grad_order), ctypes.c_void_p(ws.ptr), ws.nbytes,
                            _stream(stream)))
    return tau


def lpt_displacements_and_source(hier: Hier, phi, scale=1.0, out=None, tau=None, workspace=None, stream=None,
                                 grad_order=4):
    """Displacements (as lpt_displacements) and tau (as lpt2_source) in one call.
    Returns (list of [psi_x, psi_y, psi_z] per level, list of tau per level)."""
    if out is None:
        out = [[torch.empty_like(x) for _ in range(3)] for x in phi]
    if tau is None:
        tau = [torch.empty_like(x) for x in phi]
    H = hier.c_struct()
    ws = _ws(workspace, lpt_workspace_bytes(hier, 2))
    pp, _pa = _ptr_array([_dev(x, "phi") for x in phi])
    op, _oa = _ptr_array([_dev(c, "out") for lvl in out for c in lvl])
    tp, _ta = _ptr_array([_dev(x, "tau") for x in tau])
    _check(_lib.lpt_displacements_and_source(ctypes.byref(H), pp, op, int(grad_order), float(scale), tp,
                                             ctypes.c_void_p(ws.ptr), ws.nbytes, _stream(stream)))
    return out, tau


def lpt_lla_density(hier: Hier, disp, disp2=None, delta=None, workspace=None, stream=None):
    """LLA baryon overdensity 1 / det(I + G4 L) - 1 per level, L = disp (+ disp2), renormalised to
    zero composite mean.  disp / disp2: lists of [L_x, L_y, L_z] per level.  Returns delta per level."""
    if delta is None:
        delta = [torch.empty_like(lvl[0]) for lvl in disp]
    H = hier.c_struct()
    ws = _ws(workspace, lpt_workspace_bytes(hier, 3))
    ap, _aa = _ptr_array([_dev(c, "disp") for lvl in disp for c in lvl])
    bp, _ba = (None, None) if disp2 is None else _ptr_array([_dev(c, "disp2") for lvl in disp2 for c in lvl])
    dp, _da = _ptr_array([_dev(x, "delta") for x in delta])
    _check(_lib.lpt_lla_density(ctypes.byref(H), ap, bp, dp, ctypes.c_void_p(ws.ptr), ws.nbytes, _stream(stream)))
    return delta


SPEC_FV_DECONV = 1
SPEC_SG_DECONV = 2


def _shape3(shape):
    n = tuple(int(v) for v in shape)
    if len(n) != 3:
        raise ValueError("fields must be 3-D")
    return (ctypes.c_int * 3)(*n)


def spec_workspace_bytes(shape, isolated=False) -> int:
    need = _lib.spec_workspace_bytes(_shape3(shape), 1 if isolated else 0)
    if need == 0:
        raise MGError(MG_EINVAL, _lib.mg_last_error().decode())
    return need


def spec_deconvolve(f, kind, isolated=False, out=None, workspace=None, stream=None):
    """Section 3.5.1 (kind SPEC_FV_DECONV) or 3.5.3 (SPEC_SG_DECONV) deconvolution of f."""
    if out is None:
        out = torch.empty_like(f)
    ws = _ws(workspace, spec_workspace_bytes(f.shape, isolated))
    _check(_lib.spec_deconvolve(_shape3(f.shape), int(kind), 1 if isolated else 0, _dev(f, "f"), _dev(out, "out"),
                                ctypes.c_void_p(ws.ptr), ws.nbytes, _stream(stream)))
    return out


def spec_poisson(f, h, order=2, u=None, workspace=None, stream=None):
    """Exact discrete periodic solve of L u = f - mean(f) with the Table 1 Laplacian of this order."""
    if u is None:
        u = torch.empty_like(f)
    ws = _ws(workspace, spec_workspace_bytes(f.shape))
    _check(_lib.spec_poisson(_shape3(f.shape), float(h), int(order), _dev(f, "f"), _dev(u, "u"),
                             ctypes.c_void_p(ws.ptr), ws.nbytes, _stream(stream)))
    return u


def lpt_hybrid_correction(f, h, out, isolated=False, lap_order=2, grad_order=4, scale=1.0, workspace=None,
                          stream=None):
    """Section 3.5.2: adds the hybrid Poisson correction of source f to out = [psi_x, psi_y, psi_z]."""
    ws = _ws(workspace, spec_workspace_bytes(f.shape, isolated))
    op, _oa = _ptr_array([_dev(c, "out") for c in out])
    _check(_lib.lpt_hybrid_correction(_shape3(f.shape), float(h), 1 if isolated else 0, int(lap_order),
                                      int(grad_order), float(scale), _dev(f, "f"), op, ctypes.c_void_p(ws.ptr),
                                      ws.nbytes, _stream(stream)))
    return out


def ic_density_workspace_bytes(hier: Hier) -> int:
    H = hier.c_struct()
    need = _lib.ic_density_workspace_bytes(ctypes.byref(H))
    if need == 0:
        raise MGError(MG_EINVAL, _lib.mg_last_error().decode())
    return need


def ic_multiscale_density(hier: Hier, radial, dr, xi, subgrid=True, delta=None, workspace=None, stream=None):
    """Sections 2.1-2.3: the density on every level from the radial transfer function table and
    the unit normals xi (base N^3, patch p (2 n_p)^3 on its padded domain)."""
    if delta is None:
        delta = [torch.empty(hier.dims(p), dtype=torch.float64, device=xi[0].device) for p in range(hier.nlev)]
    H = hier.c_struct()
    ws = _ws(workspace, ic_density_workspace_bytes(hier))
    xp, _xa = _ptr_array([_dev(x, "xi") for x in xi])
    dp, _da = _ptr_array([_dev(d, "delta") for d in delta])
    _check(_lib.ic_multiscale_density(ctypes.byref(H), _dev(radial, "radial"), int(radial.numel()), float(dr),
                                      1 if subgrid else 0, xp, dp, ctypes.c_void_p(ws.ptr), ws.nbytes,
                                      _stream(stream)))
    return delta


def mg_batch_workspace_bytes(sizes, opts=None) -> int:
    o = opts or make_opts()
    n = (ctypes.c_int * len(sizes))(*sizes)
    b = _lib.mg_batch_workspace_bytes(len(sizes), n, ctypes.byref(o))
    if b == 0:
        raise MGError(MG_EINVAL, _lib.mg_last_error().decode())
    return b


def _hier_array(hiers):
    """Host array of pointers to mg_hier structs (the structs are kept alive with it)."""
    structs = [h.c_struct() for h in hiers]
    arr = (ctypes.POINTER(mg_hier) * len(structs))(*[ctypes.pointer(H) for H in structs])
    return ctypes.cast(arr, ctypes.c_void_p), (arr, structs)


def mg_batch_hier_workspace_bytes(hiers: Sequence[Hier], opts=None) -> int:
    o = opts or make_opts()
    hp, _keep = _hier_array(hiers)
    b = _lib.mg_batch_hier_workspace_bytes(len(hiers), hp, ctypes.byref(o))
    if b == 0:
        raise MGError(MG_EINVAL, _lib.mg_last_error().decode())
    return b


def mg_solve_batch_hier(hiers: Sequence[Hier], f: Sequence[Sequence[torch.Tensor]], u=None, opts=None,
                        workspace=None, stream=None, check=True):
    """Independent hierarchy solves in one call.  f[i][p]: level p of instance i.  Returns
    (u as a list of per-instance level lists, list of stats dicts)."""
    o = opts or make_opts()
    k = len(hiers)
    if len(f) != k:
        raise ValueError("one list of level fields per hierarchy")
    if u is None:
        u = [[torch.empty_like(x) for x in fi] for fi in f]
    need = mg_batch_hier_workspace_bytes(hiers, o)
    ws = _ws(workspace, need)
    hp, keep = _hier_array(hiers)
    fl = [_ptr_array([_dev(x, "f") for x in fi]) for fi in f]
    ul = [_ptr_array([_dev(x, "u") for x in ui]) for ui in u]
    fa = (_PP * k)(*[p for p, _ in fl])
    ua = (_PP * k)(*[p for p, _ in ul])
    st = (mg_stats * k)()
    rc = _lib.mg_solve_batch_hier(k, hp, ctypes.cast(fa, ctypes.c_void_p), ctypes.cast(ua, ctypes.c_void_p),
                                  ctypes.byref(o), st, ctypes.c_void_p(ws.ptr), ws.nbytes, _stream(stream))
    stats = [st[i].to_dict() for i in range(k)]
    if check:
        _check(rc, stats)
    return u, stats


def mg_solve_batch(f: Sequence[torch.Tensor], h: Sequence[float], u=None, opts=None, workspace=None, stream=None,
                   check=True):
    """Independent periodic solves.  Returns (u list, list of stats dicts)."""
    o = opts or make_opts()
    k = len(f)
    sizes = [x.shape[0] for x in f]
    if u is None:
        u = [torch.empty_like(x) for x in f]
    need = mg_batch_workspace_bytes(sizes, o)
    ws = _ws(workspace, need)
    n = (ctypes.c_int * k)(*sizes)
    hh = (ctypes.c_double * k)(*[float(v) for v in h])
    fp, _fa = _ptr_array([_dev(x, "f") for x in f])
    up, _ua = _ptr_array([_dev(x, "u") for x in u])
    st = (mg_stats * k)()
    rc = _lib.mg_solve_batch(k, n, hh, fp, up, ctypes.byref(o), st, ctypes.c_void_p(ws.ptr), ws.nbytes,
                             _stream(stream))
    stats = [st[i].to_dict() for i in range(k)]
    if check:
        _check(rc, stats)
    return u, stats


def mg_batch_tune_candidates() -> int:
    return _lib.mg_batch_tune_candidates()


def mg_batch_force_shape(index: int):
    """Force candidate `index` of the batched smoother at every depth (-1: back to timing)."""
    _check(_lib.mg_batch_force_shape(int(index)))


def mg_tune_cache(path) -> int:
    """Persist the batched smoother's tuned shapes in a JSON file (None: stop); returns the
    number of entries loaded from it."""
    rc = _lib.mg_tune_cache(None if path is None else os.fsencode(path))
    if rc < 0:
        _check(rc)
    return rc


def mg_tune_inner(hier: Hier, f, opts=None, u=None, workspace=None, stream=None):
    """Time the mixed solve of hier with 0..4 FP32 inner cycles per correction and record the
    fastest for this problem shape.  Returns (best, [ms per count])."""
    o = opts or make_opts(prec="mixed")
    if u is None:
        u = [torch.empty_like(x) for x in f]
    H = hier.c_struct()
    ws = _ws(workspace, mg_workspace_bytes(hier, o))
    fp, _fa = _ptr_array([_dev(x, "f") for x in f])
    up, _ua = _ptr_array([_dev(x, "u") for x in u])
    best = ctypes.c_int(-1)
    ms = (ctypes.c_double * 5)()
    _check(_lib.mg_tune_inner(ctypes.byref(H), fp, up, ctypes.byref(o), ctypes.byref(best), ms,
                              ctypes.c_void_p(ws.ptr), ws.nbytes, _stream(stream)))
    return best.value, list(ms)


def mg_smooth_level(f, u, h, half_sweeps, prec="fp64", workspace=None, stream=None):
    """In-place red/black half-sweeps (red first) on a periodic level."""
    n = f.shape[0]
    p = {"fp64": MG_FP64, "mixed": MG_MIXED}[prec]
    ws = _ws(workspace, mg_workspace_bytes(Hier(n, h), make_opts(prec=prec)))
    _check(_lib.mg_smooth_level(n, h, _dev(f, "f"), _dev(u, "u"), int(half_sweeps), p, ctypes.c_void_p(ws.ptr),
                                ws.nbytes, _stream(stream)))
    return u


def mg_ghost_fill(hier: Hier, p: int, u, flux_match=True, ghosts=None, stream=None):
    """Flux-matched ghost faces of patch p (x-lo, x-hi, y-lo, y-hi, z-lo, z-hi, back to back)."""
    nx, ny, nz = hier.dims(p)
    total = 2 * (ny * nz + nx * nz + nx * ny)
    if ghosts is None:
        ghosts = torch.empty(total, dtype=torch.float64, device=u[0].device)
    H = hier.c_struct()
    up, _ua = _ptr_array([_dev(x, "u") for x in u])
    _check(_lib.mg_ghost_fill(ctypes.byref(H), int(p), up, _dev(ghosts, "ghosts"), 1 if flux_match else 0,
                              _stream(stream)))
    return ghosts


def split_ghosts(hier: Hier, p: int, g):
    """View the 6 ghost faces as 2-D tensors: [(ny,nz), (ny,nz), (nx,nz), (nx,nz), (nx,ny), (nx,ny)]."""
    nx, ny, nz = hier.dims(p)
    shapes = [(ny, nz), (ny, nz), (nx, nz), (nx, nz), (nx, ny), (nx, ny)]
    out, o = [], 0
    for s in shapes:
        out.append(g[o:o + s[0] * s[1]].view(*s))
        o += s[0] * s[1]
    return out


def mg_kprof_enable(on=True, period=1):
    """Time every period-th finest-level smoother launch with dispatch-stamped HIP events
    (calling thread only); on=False switches timing off."""
    _check(_lib.mg_kprof_enable(int(period) if on else 0))


def mg_kprof_read():
    """(total ms, launches, algorithmic bytes) of the timed launches since the last read."""
    ms = ctypes.c_double()
    n = ctypes.c_longlong()
    by = ctypes.c_double()
    _check(_lib.mg_kprof_read(ctypes.byref(ms), ctypes.byref(n), ctypes.byref(by)))
    return ms.value, n.value, by.value
