"""Adaptive (zoom-in) multigrid on nested rectangular patches (oracle).

Test infrastructure only (see ``oracle/__init__.py``).

Follows Section 3.3 of the paper ("Adaptive multi-grid"), built on the FAS
V-cycle of Section 3.2:
* Nested rectangular sub-grids, refinement ratio 2, each inside its parent.
* Restriction and prolongation act only where a level overlaps the next finer
  one; the rest of a level is treated as if it were the finest level.
* The coarse solution is the boundary condition of the finer level through
  ghost zones: polynomial interpolation first parallel to the fine surface
  using coarse data only, then normal to it using the fine interior; the
  polynomial order equals the order of the Laplacian (2 -> quadratic).
* Flux matching (Table 2, order-1 flux operator [-1 1]/h): the ghost values
  are shifted so that the mean of the 4 fine fluxes through a coarse face
  equals the coarse flux through it.  Without it the method does not converge
  (the residual does not vanish on every level).

Data model: level 0 is the periodic base, N0^3 cells of spacing h0.  Level
p >= 1 is a patch of n = (nx, ny, nz) cells (all even) of spacing h0 / 2^p,
whose first cell is the first child of cell ``off`` of level p - 1.  Arrays
are indexed [x][y][z].

Readings (the paper is silent or ambiguous here):
* Ghost formula for the low-x face, fine cell q = (0, j, k) of a patch at
  parent offset o, parent C = o + (0, j//2, k//2), outside parent O = C - e_x:
    a_q  = sum_{dy,dz} w_dy(t_j) w_dz(t_k) U[O + (0, dy, dz)],
           w(t) = (t(t-1)/2, 1 - t^2, t(t+1)/2), t = -1/4 (even) or +1/4 (odd)
    g0_q = 8/15 a_q + 2/3 u[0,j,k] - 1/5 u[1,j,k]   (quadratic through the
           coarse centre, the first and the second fine cell, at the ghost)
    g_q  = g0_q + (mean u0 - mean g0) - 1/2 (mean8(children of C) - U[O])
  where the means run over the 2 x 2 fine cells of the face of C.  The flux
  difference is spread uniformly over the 4 ghosts.  Other faces mirror this.
* The coarse flux uses the live mean of C's current fine children, not the
  value stored on the coarse level (the stored value makes smoothing on the
  patch effectively pure-Neumann; both readings have the same fixed point).
* Ghosts are recomputed before every half-sweep and before every residual.
* Proper nesting: a patch inside a patch keeps >= 4 parent cells from its
  parent's faces; a patch inside the periodic base does not wrap, leaves at
  least 2 base cells uncovered along every axis, and reads the base with
  periodic wrap.
* The solution is the unique composite solution with zero composite mean.
  Covered coarse cells are the mean of their children; the composite mean of
  f is removed first; the residual norm is
  sqrt(sum_fine r^2 h^3 + sum_uncovered r^2 H^3) / (same for f).
* Post-solve ghosts for gradients (width 2, or 3 with the sixth-order gradient)
  and for tau (width 4, or 6), edges and corners included, are coarse-only
  tri-quadratic interpolations of the parent (whose covered cells hold the mean
  of their children).
"""

import numpy as np

from . import periodic
from .stencil import lap7, restrict_mean8, inject, red_mask, grad4


class Hierarchy:
    """Base N0^3 (periodic, spacing h0) plus patches [(n3, off3), ...], outermost first."""

    def __init__(self, N0, h0, patches=()):
        self.N0 = int(N0)
        self.n = [(self.N0,) * 3]
        self.off = [None]
        self.h = [float(h0)]
        for p, (n, off) in enumerate(patches, start=1):
            n = tuple(int(v) for v in n)
            off = tuple(int(v) for v in off)
            pn = self.n[p - 1]
            for a in range(3):
                if n[a] < 4 or n[a] % 2:
                    raise ValueError("patch sizes must be even and >= 4")
                lo, hi = off[a], off[a] + n[a] // 2
                if p == 1:
                    ok = 0 <= lo and hi <= pn[a] and n[a] // 2 <= pn[a] - 2
                else:
                    ok = lo >= 4 and hi <= pn[a] - 4
                if not ok:
                    raise ValueError("patch %d not properly nested in its parent" % p)
            self.n.append(n)
            self.off.append(off)
            self.h.append(float(h0) / 2 ** p)

    @property
    def P(self):
        return len(self.n) - 1

    def covered(self, p):
        """Slices of level p-1 covered by patch p."""
        o, n = self.off[p], self.n[p]
        return tuple(slice(o[a], o[a] + n[a] // 2) for a in range(3))

    def zeros(self):
        return [np.zeros(n) for n in self.n]


# ----------------------------------------------------------------------------- parent access

def _parent_block(H, U, p, ranges):
    """U[ranges] of the parent of patch p; ranges = 3 integer arrays (wrap on the base)."""
    idx = []
    for a, r in enumerate(ranges):
        r = np.asarray(r)
        if p == 1:
            r = np.mod(r, H.N0)
        elif r.min() < 0 or r.max() >= U.shape[a]:
            raise IndexError("parent access out of range")
        idx.append(r)
    return U[np.ix_(*idx)]


def _w2(t):
    """Quadratic Lagrange weights through nodes -1, 0, +1 evaluated at t."""
    return np.stack([0.5 * t * (t - 1.0), 1.0 - t * t, 0.5 * t * (t + 1.0)])


def _child_t(i):
    """Child offset inside its parent in parent units: -1/4 for even i, +1/4 for odd i."""
    return np.where(np.asarray(i) % 2 == 0, -0.25, 0.25)


# ----------------------------------------------------------------------------- flux-matched ghosts

def ghosted(H, u, p, flux_match=True):
    """Patch p padded by one ghost layer on its 6 faces (edges/corners are NaN)."""
    n = H.n[p]
    o = H.off[p]
    U = u[p - 1]
    v = u[p]
    up = np.full(tuple(s + 2 for s in n), np.nan)
    up[1:-1, 1:-1, 1:-1] = v
    for a in range(3):
        b, c = [x for x in range(3) if x != a]
        vf = np.moveaxis(v, a, 0)          # (n_a, n_b, n_c) view
        upf = np.moveaxis(up, a, 0)
        nb, nc = n[b], n[c]
        jb = np.arange(nb)
        kc = np.arange(nc)
        for side in (0, 1):
            if side == 0:
                L0, L1 = vf[0], vf[1]
                on = o[a] - 1                      # normal index of the outside coarse layer
            else:
                L0, L1 = vf[n[a] - 1], vf[n[a] - 2]
                on = o[a] + n[a] // 2
            # coarse layer, padded by one cell transversally
            rb = np.arange(o[b] - 1, o[b] + nb // 2 + 1)
            rc = np.arange(o[c] - 1, o[c] + nc // 2 + 1)
            ranges = [None, None, None]
            ranges[a] = np.array([on])
            ranges[b] = rb
            ranges[c] = rc
            layer = _parent_block(H, U, p, ranges)
            layer = np.moveaxis(layer, a, 0)[0]          # (nb/2+2, nc/2+2)
            # step 1: quadratic interpolation parallel to the face, coarse data only
            wb = _w2(_child_t(jb))                      # (3, nb)
            wc = _w2(_child_t(kc))                      # (3, nc)
            Jb = jb // 2 + 1
            Kc = kc // 2 + 1
            Ab = sum(wb[d][:, None] * layer[Jb + d - 1, :] for d in range(3))   # (nb, nc/2+2)
            aq = sum(wc[d][None, :] * Ab[:, Kc + d - 1] for d in range(3))      # (nb, nc)
            # step 2: quadratic normal to the face through (coarse, u0, u1)
            g0 = (8.0 / 15.0) * aq + (2.0 / 3.0) * L0 - 0.2 * L1
            g = g0
            if flux_match:
                # step 3: match the mean fine flux to the coarse flux (Table 2, order 1)
                def m4(X):
                    return X.reshape(nb // 2, 2, nc // 2, 2).mean(axis=(1, 3))
                uO = layer[1:-1, 1:-1]
                u0bar = m4(L0)
                uC = 0.5 * (m4(L0) + m4(L1))
                shift = (u0bar - m4(g0)) - 0.5 * (uC - uO)
                g = g0 + np.repeat(np.repeat(shift, 2, axis=0), 2, axis=1)
            if side == 0:
                upf[0, 1:-1, 1:-1] = g
            else:
                upf[-1, 1:-1, 1:-1] = g
    return up


def lap_padded(up, h):
    """7-point Laplacian on the interior of a ghost-padded array (faces only are read)."""
    c = up[1:-1, 1:-1, 1:-1]
    sx = up[:-2, 1:-1, 1:-1] + up[2:, 1:-1, 1:-1]
    sy = up[1:-1, :-2, 1:-1] + up[1:-1, 2:, 1:-1]
    sz = up[1:-1, 1:-1, :-2] + up[1:-1, 1:-1, 2:]
    return (((sx + sy) + sz) - 6.0 * c) / (h * h)


def level_lap(H, u, p, flux_match=True):
    """L u on the whole of level p (periodic base, or patch with fresh ghosts)."""
    if p == 0:
        return lap7(u[0], H.h[0])
    return lap_padded(ghosted(H, u, p, flux_match), H.h[p])


def patch_half_sweep(H, u, f, p, colour, flux_match=True):
    """Red or black half-sweep on patch p; ghosts refreshed from the current iterate."""
    up = ghosted(H, u, p, flux_match)
    c = up[1:-1, 1:-1, 1:-1]
    sx = up[:-2, 1:-1, 1:-1] + up[2:, 1:-1, 1:-1]
    sy = up[1:-1, :-2, 1:-1] + up[1:-1, 2:, 1:-1]
    sz = up[1:-1, 1:-1, :-2] + up[1:-1, 1:-1, 2:]
    h = H.h[p]
    new = (((sx + sy) + sz) - (h * h) * f) / 6.0
    red = red_mask(c.shape)
    mask = red if colour == 0 else ~red
    return np.where(mask, new, c)


# ----------------------------------------------------------------------------- composite helpers

def restrict_bottom_up(H, v):
    """Covered cells of every level := mean of their 8 children, finest first (in place)."""
    for p in range(H.P, 0, -1):
        v[p - 1][H.covered(p)] = restrict_mean8(v[p])
    return v


def composite_zero_mean(H, v):
    """Restrict bottom-up, then subtract the base mean (= composite volume mean) everywhere."""
    v = [np.array(a, dtype=np.float64) for a in v]
    restrict_bottom_up(H, v)
    m = float(np.mean(v[0]))
    return [a - m for a in v], m


def uncovered_mask(H, p):
    m = np.ones(H.n[p], dtype=bool)
    if p < H.P:
        m[H.covered(p + 1)] = False
    return m


def composite_residual(H, u, f, flux_match=True):
    """Per-level residual of the composite system; covered coarse cells are set to 0."""
    u = [a.copy() for a in u]
    restrict_bottom_up(H, u)
    r = []
    for p in range(H.P + 1):
        rp = f[p] - level_lap(H, u, p, flux_match)
        rp[~uncovered_mask(H, p)] = 0.0
        r.append(rp)
    return r


def composite_norm(H, v):
    """sqrt(sum over uncovered cells of v^2 * cell volume)."""
    s = 0.0
    for p in range(H.P + 1):
        s += float(np.sum(np.square(v[p][uncovered_mask(H, p)]))) * H.h[p] ** 3
    return np.sqrt(s)


def composite_sum(H, v):
    """sum over uncovered cells of v * cell volume (conservation check)."""
    return sum(float(np.sum(v[p][uncovered_mask(H, p)])) * H.h[p] ** 3 for p in range(H.P + 1))


# ----------------------------------------------------------------------------- adaptive FAS

def vcycle(H, u, fw, p, nu1=2, nu2=2, flux_match=True):
    """One adaptive FAS V-cycle entered at level p (in place on u and fw)."""
    if p == 0:
        u[0] = periodic.vcycle(u[0], fw[0], H.h[0], nu1, nu2)
        return
    h = H.h[p]
    for _ in range(nu1):
        for colour in (0, 1):
            u[p] = patch_half_sweep(H, u, fw[p], p, colour, flux_match)
    r = fw[p] - level_lap(H, u, p, flux_match)
    sl = H.covered(p)
    rc = restrict_mean8(r)
    uc = restrict_mean8(u[p])
    u[p - 1][sl] = uc
    uc_old = uc.copy()
    fw[p - 1][sl] = rc + level_lap(H, u, p - 1, flux_match)[sl]
    vcycle(H, u, fw, p - 1, nu1, nu2, flux_match)
    u[p] = u[p] + inject(u[p - 1][sl] - uc_old)
    for _ in range(nu2):
        for colour in (0, 1):
            u[p] = patch_half_sweep(H, u, fw[p], p, colour, flux_match)
    del h


def solve_hierarchy(H, f, tol=1e-10, max_cycles=40, nu1=2, nu2=2, flux_match=True, u0=None):
    """Composite solve.  Returns (u, info); u has zero composite mean."""
    f, f_mean = composite_zero_mean(H, f)
    fnorm = composite_norm(H, f)
    u = H.zeros() if u0 is None else [np.array(a, dtype=np.float64) for a in u0]
    fw = [a.copy() for a in f]
    hist = []
    cycles = 0
    rel = composite_norm(H, composite_residual(H, u, f, flux_match)) / fnorm if fnorm > 0 else 0.0
    while cycles < max_cycles and rel > tol:
        vcycle(H, u, fw, H.P, nu1, nu2, flux_match)
        cycles += 1
        rel = composite_norm(H, composite_residual(H, u, f, flux_match)) / fnorm if fnorm > 0 else 0.0
        hist.append(rel)
    u, _ = composite_zero_mean(H, u)
    return u, dict(cycles=cycles, rel_res=rel, f_mean=f_mean, history=hist)


# ----------------------------------------------------------------------------- post-solve ghosts, LPT

def wide_ghosted(H, v, p, R):
    """Patch p of v padded by R ghost layers (faces, edges, corners).

    Ghosts are coarse-only tri-quadratic interpolations of level p-1, whose
    covered cells must already hold the mean of their children.
    """
    n, o = H.n[p], H.off[p]
    U = v[p - 1]
    i_ax = [np.arange(-R, n[a] + R) for a in range(3)]
    Pc = [o[a] + np.floor_divide(i_ax[a], 2) for a in range(3)]
    lo = [int(Pc[a].min()) - 1 for a in range(3)]
    hi = [int(Pc[a].max()) + 1 for a in range(3)]
    B = _parent_block(H, U, p, [np.arange(lo[a], hi[a] + 1) for a in range(3)])
    for a in range(3):
        w = _w2(_child_t(i_ax[a]))                 # (3, m)
        base = Pc[a] - lo[a]
        Bm = np.moveaxis(B, a, 0)
        out = sum(w[d][:, None, None] * Bm[base + d - 1] for d in range(3))
        B = np.moveaxis(out, 0, a)
    vp = B
    vp[R:-R, R:-R, R:-R] = v[p]
    return vp


def _grad_padded(vp, h, axis, R, order=4):
    """Table 1 gradient (order 4 or 6) of a padded array on its interior shrunk by R."""
    weights, den = ((1.0, -8.0, 0.0, 8.0, -1.0), 12.0) if order == 4 else \
        ((-1.0, 9.0, -45.0, 0.0, 45.0, -9.0, 1.0), 60.0)
    half = len(weights) // 2
    n = [s - 2 * R for s in vp.shape]
    out = np.zeros(n)
    for off, w in zip(range(-half, half + 1), weights):
        if w == 0.0:
            continue
        sl = [slice(R, R + n[a]) for a in range(3)]
        sl[axis] = slice(R + off, R + off + n[axis])
        out = out + w * vp[tuple(sl)]
    return out / (den * h)


def displacement_hierarchy(H, phi, scale=1.0, order=4):
    """psi = scale * G phi on every level (Table 1 gradient of order 4 or 6; base periodic;
    patches via ghosts of width order / 2)."""
    from .stencil import grad
    rg = order // 2
    phi = [a.copy() for a in phi]
    restrict_bottom_up(H, phi)
    out = []
    for p in range(H.P + 1):
        if p == 0:
            out.append(np.stack([scale * grad(phi[0], H.h[0], a, order) for a in range(3)]))
        else:
            vp = wide_ghosted(H, phi, p, rg)
            out.append(np.stack([scale * _grad_padded(vp, H.h[p], a, rg, order) for a in range(3)]))
    return out


def _tau_padded(vp, h, R, order=4):
    """tau = sum_{i>j} D_ii D_jj - D_ij^2, D = G o G, on the interior (needs R = order)."""
    rg = order // 2
    g = [_grad_padded(vp, h, j, rg, order) for j in range(3)]          # valid on interior +- (R - rg)
    D = [[_grad_padded(g[j], h, i, R - rg, order) for j in range(3)] for i in range(3)]
    t = np.zeros_like(D[0][0])
    for i in range(3):
        for j in range(i):
            t = t + (D[i][i] * D[j][j] - D[i][j] * D[i][j])
    return t


def tau_hierarchy(H, phi, order=4):
    """Second-order source on every level, composite mean removed (Section 3.1); D = G o G with
    the Table 1 gradient of order 4 or 6 (patch ghosts of width = order)."""
    from .lpt import tau as tau_periodic
    phi = [a.copy() for a in phi]
    restrict_bottom_up(H, phi)
    out = []
    for p in range(H.P + 1):
        if p == 0:
            out.append(tau_periodic(phi[0], H.h[0], order))
        else:
            out.append(_tau_padded(wide_ghosted(H, phi, p, order), H.h[p], order, order))
    out, _ = composite_zero_mean(H, out)
    return out


def lla_hierarchy(H, L, renorm=True):
    """LLA baryon overdensity 1 / det(I + dL/dq) - 1 on every level (Section 5.3).

    L[p] is the displacement of level p, shape (3, *n_p).  Each component is restricted bottom-up
    (covered cells := mean of their children), the patches take width-2 ghosts of it from their
    parent (as the displacements do), and the Jacobian is the fourth-order gradient.  With renorm,
    the composite mean of the overdensity (covered cells restricted from the finer level first)
    is removed from every level.
    """
    from .lpt import lla_ratio
    comps = [[np.array(L[p][c], dtype=np.float64) for p in range(H.P + 1)] for c in range(3)]
    for c in range(3):
        restrict_bottom_up(H, comps[c])
    out = []
    for p in range(H.P + 1):
        if p == 0:
            J = [[grad4(comps[i][0], H.h[0], j) for j in range(3)] for i in range(3)]
        else:
            vp = [wide_ghosted(H, comps[i], p, 2) for i in range(3)]
            J = [[_grad_padded(vp[i], H.h[p], j, 2) for j in range(3)] for i in range(3)]
        out.append(lla_ratio(J) - 1.0)
    if renorm:
        out, _ = composite_zero_mean(H, out)
    return out
