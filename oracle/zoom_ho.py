"""Higher-order Laplacians on nested patches: the adaptive FAS of Section 3.3 with the order-4 and
order-6 operators of Table 1 and the flux operators of Table 2 (oracle).

Test infrastructure only (see ``oracle/__init__.py``).

What the paper fixes:
* Table 1: the 1-D Laplacian of order n (n = 2, 4, 6; radius R = n / 2), summed over the axes
  in 3-D as for the 7-point operator; every level uses the same order (``highorder``).
* Section 3.3: ghost zones of a patch are filled by polynomial interpolation first parallel to
  the fine surface using coarse data only, then normal to it using these intermediate values
  and fine interior values; the degree of both polynomials is the order of the Laplacian.
* Table 2: the flux operators F of order n - 1 on the cell faces, whose convolution with
  [-1 1] gives the Laplacian of order n.  The mean of the 4 fine fluxes through a coarse face,
  evaluated with F, is matched to the coarse flux through that face by adjusting the ghost
  values that enter the fine fluxes.

Readings (the paper is silent here); with n = 2 each reduces to the reading of ``zoom``:
* A star stencil of radius R reads R ghost layers on each face and nothing on edges or
  corners.
* Parallel step: along each transverse axis a polynomial of degree n through the n + 1 coarse
  cells J - R .. J + R around the parent J of the fine cell, evaluated at the child's offset
  -1/4 or +1/4 (parent units); first along the face's first transverse axis, then the second.
  It is done for each of the R coarse layers outside the face.
* Normal step: a polynomial of degree n through the R outside coarse values (at -(2k + 1) h,
  k = 0 .. R - 1, measured inwards from the face in fine units) and the first R + 1 fine cells
  (at (i + 1/2) h), evaluated at the R ghost centres -(g + 1/2) h.
* Coarse flux: F applied to the R outside coarse cells and the R covered coarse cells inside
  the face, the latter taken as the live mean of their current fine children (as ``zoom``).
* The flux difference is removed by shifting all R ghost layers of the 2 x 2 fine cells in
  front of one coarse face by the same amount; F changes by that shift times the sum of its
  ghost-side weights.
* Nesting: the outside coarse layers and the transverse stencil read R parent cells beyond the
  patch; a patch in the base reads the base with periodic wrap and needs R uncovered base
  cells along each axis, a patch in a patch keeps >= 4 >= R parent cells from the parent's
  faces (``zoom.Hierarchy``).
"""

import numpy as np

from . import highorder as ho
from .stencil import restrict_mean8, inject, red_mask
from .zoom import Hierarchy, restrict_bottom_up, composite_zero_mean, uncovered_mask, composite_norm  # noqa: F401

# Table 2: flux operator of order n - 1 for the Laplacian of order n, integer weights over the
# 2R cells around a face (outside / low side first) and their denominator
FLUX = {
    2: ((-1, 1), 1),
    4: ((-1, 15, -15, 1), 12),
    6: ((2, -25, 245, -245, 25, -2), 180),
}


def radius(order):
    return order // 2


def flux_weights(order):
    """Table 2 flux operator for the Laplacian of this order, as floats (2R weights)."""
    c, den = FLUX[order]
    return tuple(float(v) / den for v in c)


def lagrange(nodes, x):
    """Weights of the polynomial through `nodes` evaluated at x (plain Lagrange form)."""
    nodes = [float(v) for v in nodes]
    w = []
    for i, xi in enumerate(nodes):
        num, den = 1.0, 1.0
        for j, xj in enumerate(nodes):
            if j != i:
                num *= x - xj
                den *= xi - xj
        w.append(num / den)
    return w


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


def _check_nesting(H, p, R):
    if p == 1:
        for a in range(3):
            if H.N0 - H.n[1][a] // 2 < R:
                raise ValueError("base leaves fewer than R uncovered cells along axis %d" % a)


def ghosted(H, u, p, order, flux_match=True):
    """Patch p padded by R ghost layers on its 6 faces (edges and corners are NaN)."""
    R = radius(order)
    _check_nesting(H, p, R)
    n, o = H.n[p], H.off[p]
    U, v = u[p - 1], u[p]
    up = np.full(tuple(s + 2 * R for s in n), np.nan)
    up[R:-R, R:-R, R:-R] = v
    # parallel step weights: nodes -R..R (parent units), child offsets -1/4 (even), +1/4 (odd)
    wpar = {0: lagrange(range(-R, R + 1), -0.25), 1: lagrange(range(-R, R + 1), 0.25)}
    # normal step weights for ghost layer g: nodes R coarse then R + 1 fine (fine units)
    nodes = [-(2 * k + 1) for k in range(R)] + [i + 0.5 for i in range(R + 1)]
    wnor = [lagrange(nodes, -(g + 0.5)) for g in range(R)]
    F = flux_weights(order)
    S = sum(F[:R])                      # ghost-side weights of the flux operator
    h, Hc = H.h[p], H.h[p - 1]
    for a in range(3):
        b, c = [x for x in range(3) if x != a]
        nb, nc = n[b], n[c]
        jb, kc = np.arange(nb), np.arange(nc)
        for side in (0, 1):
            # fine layers counted inwards from the face: vin[i] = layer i
            vf = np.moveaxis(v, a, 0)
            vin = vf if side == 0 else vf[::-1]
            # outside coarse layers k = 0..R-1 and covered coarse layers inside k = 0..R-1,
            # with the transverse ranges padded by R parent cells
            if side == 0:
                outs = [o[a] - 1 - k for k in range(R)]
            else:
                outs = [o[a] + n[a] // 2 + k for k in range(R)]
            rb = np.arange(o[b] - R, o[b] + nb // 2 + R)
            rc = np.arange(o[c] - R, o[c] + nc // 2 + R)
            aq = []                                          # parallel step per outside layer
            for k in range(R):
                ranges = [None, None, None]
                ranges[a] = np.array([outs[k]])
                ranges[b], ranges[c] = rb, rc
                layer = np.moveaxis(_parent_block(H, U, p, ranges), a, 0)[0]   # (nb/2+2R, nc/2+2R)
                Jb, Kc = jb // 2 + R, kc // 2 + R
                Ab = np.zeros((nb, layer.shape[1]))
                for d in range(2 * R + 1):
                    wd = np.array([wpar[j % 2][d] for j in jb])
                    Ab = Ab + wd[:, None] * layer[Jb + d - R, :]
                A = np.zeros((nb, nc))
                for d in range(2 * R + 1):
                    wd = np.array([wpar[j % 2][d] for j in kc])
                    A = A + wd[None, :] * Ab[:, Kc + d - R]
                aq.append(A)
            vals = aq + [vin[i] for i in range(R + 1)]
            g0 = [sum(wnor[g][m] * vals[m] for m in range(2 * R + 1)) for g in range(R)]
            g = g0
            if flux_match:
                def m4(X):
                    return X.reshape(nb // 2, 2, nc // 2, 2).mean(axis=(1, 3))
                # fine fluxes through the face: cells g_{R-1} .. g_0 | u_0 .. u_{R-1}
                cells = [g0[R - 1 - m] for m in range(R)] + [vin[i] for i in range(R)]
                Ff = sum(F[m] * cells[m] for m in range(2 * R)) / h
                # coarse flux: O_{R-1} .. O_0 | C_0 .. C_{R-1}, C_k the live mean of its children
                sl_b = slice(o[b], o[b] + nb // 2)
                sl_c = slice(o[c], o[c] + nc // 2)
                coarse_out = []
                for k in range(R):
                    ranges = [None, None, None]
                    ranges[a] = np.array([outs[R - 1 - k]])
                    ranges[b] = np.arange(sl_b.start, sl_b.stop)
                    ranges[c] = np.arange(sl_c.start, sl_c.stop)
                    coarse_out.append(np.moveaxis(_parent_block(H, U, p, ranges), a, 0)[0])
                coarse_in = [0.5 * (m4(vin[2 * k]) + m4(vin[2 * k + 1])) for k in range(R)]
                cc = coarse_out + coarse_in
                Fc = sum(F[m] * cc[m] for m in range(2 * R)) / Hc
                delta = (Fc - m4(Ff)) * h / S
                shift = np.repeat(np.repeat(delta, 2, axis=0), 2, axis=1)
                g = [x + shift for x in g0]
            upf = np.moveaxis(up, a, 0)
            for gl in range(R):
                idx = R - 1 - gl if side == 0 else R + n[a] + gl
                upf[idx, R:R + nb, R:R + nc] = g[gl]
    return up


def off_sum_padded(up, order):
    """sum_{s=1..R} w_s sum_axes (u[i-s] + u[i+s]) on the interior of an R-padded array."""
    w = ho.weights(order)
    R = radius(order)
    n = [s - 2 * R for s in up.shape]
    acc = np.zeros(n)
    for s in range(1, R + 1):
        pair = np.zeros(n)
        for a in range(3):
            lo = [slice(R, R + n[0]), slice(R, R + n[1]), slice(R, R + n[2])]
            hi = list(lo)
            lo[a] = slice(R - s, R - s + n[a])
            hi[a] = slice(R + s, R + s + n[a])
            pair = pair + (up[tuple(lo)] + up[tuple(hi)])
        acc = acc + w[s] * pair
    return acc


def level_lap(H, u, p, order, flux_match=True):
    """L u of this order on the whole of level p (periodic base, or patch with fresh ghosts)."""
    if p == 0:
        return ho.lap(u[0], H.h[0], order)
    R = radius(order)
    up = ghosted(H, u, p, order, flux_match)
    w0 = ho.weights(order)[0]
    c = up[R:-R, R:-R, R:-R]
    return (off_sum_padded(up, order) + 3.0 * w0 * c) / (H.h[p] ** 2)


def patch_half_sweep(H, u, f, p, order, colour, flux_match=True):
    """Red or black half-sweep on patch p, Jacobi within the colour (``highorder``); ghosts
    formed from the iterate before the half-sweep."""
    R = radius(order)
    up = ghosted(H, u, p, order, flux_match)
    w0 = ho.weights(order)[0]
    c = up[R:-R, R:-R, R:-R]
    new = ((H.h[p] ** 2) * f - off_sum_padded(up, order)) / (3.0 * w0)
    red = red_mask(c.shape)
    return np.where(red if colour == 0 else ~red, new, c)


def composite_residual(H, u, f, order, flux_match=True):
    """Per-level residual of the composite system of this order; covered coarse cells set to 0."""
    u = [a.copy() for a in u]
    restrict_bottom_up(H, u)
    r = []
    for p in range(H.P + 1):
        rp = f[p] - level_lap(H, u, p, order, flux_match)
        rp[~uncovered_mask(H, p)] = 0.0
        r.append(rp)
    return r


def vcycle(H, u, fw, p, order, nu1=2, nu2=2, flux_match=True):
    """One adaptive FAS V-cycle entered at level p (in place on u and fw), Section 3.2 steps 1-9
    on every patch, the periodic V-cycle of ``highorder`` on the base and below."""
    if p == 0:
        u[0] = ho.vcycle(u[0], fw[0], H.h[0], order, nu1, nu2)
        return
    for _ in range(nu1):                                             # step 2
        for colour in (0, 1):
            u[p] = patch_half_sweep(H, u, fw[p], p, order, colour, flux_match)
    r = fw[p] - level_lap(H, u, p, order, flux_match)                 # step 3
    sl = H.covered(p)
    rc = restrict_mean8(r)                                           # step 4
    uc = restrict_mean8(u[p])                                        # step 5
    u[p - 1][sl] = uc
    uc_old = uc.copy()
    fw[p - 1][sl] = rc + level_lap(H, u, p - 1, order, flux_match)[sl]   # step 6
    vcycle(H, u, fw, p - 1, order, nu1, nu2, flux_match)             # step 7
    u[p] = u[p] + inject(u[p - 1][sl] - uc_old)                      # step 8
    for _ in range(nu2):                                             # step 9
        for colour in (0, 1):
            u[p] = patch_half_sweep(H, u, fw[p], p, order, colour, flux_match)


def solve_hierarchy(H, f, order, tol=1e-10, max_cycles=40, nu1=2, nu2=2, flux_match=True, u0=None):
    """Composite solve with the Laplacian of this order.  Returns (u, info); u has zero
    composite mean and covered coarse cells hold the mean of their children."""
    f, f_mean = composite_zero_mean(H, f)
    fnorm = composite_norm(H, f)
    u = H.zeros() if u0 is None else [np.array(a, dtype=np.float64) for a in u0]
    fw = [a.copy() for a in f]
    hist = []
    cycles = 0

    def rel_res():
        return composite_norm(H, composite_residual(H, u, f, order, flux_match)) / fnorm if fnorm > 0 else 0.0

    rel = rel_res()
    while cycles < max_cycles and rel > tol:
        vcycle(H, u, fw, H.P, order, nu1, nu2, flux_match)
        cycles += 1
        rel = rel_res()
        hist.append(rel)
    u, _ = composite_zero_mean(H, u)
    return u, dict(cycles=cycles, rel_res=rel, f_mean=f_mean, history=hist)


__all__ = ["FLUX", "radius", "flux_weights", "lagrange", "ghosted", "off_sum_padded", "level_lap",
           "patch_half_sweep", "composite_residual", "vcycle", "solve_hierarchy", "Hierarchy"]
