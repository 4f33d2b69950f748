"""Multi-scale Gaussian density field on nested grids (oracle): Sections 2.1-2.3 and 3.5.3.

Test infrastructure only (see ``oracle/__init__.py``).

Sources in the paper:
* Section 2.1 (eq. delta_amplitude_r): the density is the white noise convolved with the
  real-space counterpart T of sqrt(P(k)).  Section 2.2: T is sampled on the grid at the cell
  displacements, with the origin at a cell, and the convolution is done by FFT; on the periodic
  box the sampled kernel is used periodically.
* Section 2.3.1 (white-noise refinement): each refinement level gets unconstrained white noise
  with 8 times the parent's variance; the Fourier modes of the parent that overlap the fine grid
  are kept by replacing the fine field's modes up to the parent's Nyquist wave number with the
  parent's coefficients (then back-transforming); after doing this for every level, top down,
  every covered coarse cell's noise is replaced by the mean of its 8 children (reverse
  Hoffman-Ribak), starting at the finest level.
* Section 2.3.2 (kernels per level): the finest level samples T directly; each coarser level
  averages the finer level's kernel over children (eq. transfer_average) where the finer kernel
  exists (the refined region with its padding), and samples T directly elsewhere.
* Section 2.3.3 (first refinement level): the fine density is the sum of
    delta_coarse: the coarse noise with the refined region zeroed, convolved with the coarse
                  kernel and interpolated tri-cubically onto the fine grid;
    delta_self:   the fine noise inside the patch (zero on the padding) convolved with the fine
                  kernel on the grid padded to twice the patch size (isolated boundaries);
    delta_bnd:    on the padding only, the fine noise minus its parent's coarse value, convolved
                  with the fine kernel (periodic on the padded grid);
  and delta_bnd is also restricted to the coarse grid on the padding region.
* Section 2.3.4 (further levels): the same, with the coarse contribution of a patch level taken
  from its parent patch's own noise with isolated boundaries, and every coarser contribution
  interpolated down level by level with conservative tri-cubic interpolation (tri-cubic, then each
  group of 8 children shifted so that its mean equals the parent).
* Section 3.5.3 (averaging correction): the finest kernel value of a cell is the mean of T over
  the cell's 8 sub-cell centres (offsets +-h/4 on each axis).

Readings (where the paper is silent or ambiguous):
* Normalisation.  With unit-variance normals xi on level l, the noise is mu = xi / h_l^(3/2)
  (8 times the variance on each finer level) and delta(x_a) = sum_b h_l^3 T_l(x_a - x_b) mu(x_b),
  so that delta has power spectrum |T~|^2 independent of the spacing.
* T is the caller's radial table T(i dr) with linear interpolation in r (the paper's FFTlog
  output is a tabulated function as well).
* Kernel restriction.  Written on the fine displacement grid, the mean over the 8 children of a
  coarse target cell and the 8 children of a coarse source cell of the fine kernel weights the
  fine displacements 2J - 1, 2J, 2J + 1 (fine units, per axis) by 1/4, 1/2, 1/4; this exact mass-
  conserving form of eq. transfer_average is used wherever those fine displacements exist on the
  finer level's kernel grid (|J| <= n_fine / 2 - 1 per axis); elsewhere T(|D|) is sampled directly
  (no sub-grid average at coarse levels, as the paper states).
* Padded domain.  The padding is centred: patch p of n cells per axis has the padded domain D' of
  2n fine cells per axis starting n/2 fine cells (n/4 parent cells) before the patch.  D' must lie
  inside the parent patch (or wrap on the periodic base); patch sizes are powers of two so that
  the padded grid is an FFT grid of 2n points.  The fine noise is defined on all of D'.
* Mode replacement.  On D' (2n points per axis) with the parent cells under it (n per axis): the
  fine coefficient of mode m with |m_a| < n_a / 2 on every axis (strictly below the parent's
  Nyquist) becomes 8 C(m) prod_a exp(-i pi m_a / (2 n_a)), C the parent region's DFT - the DFT,
  at the fine cell centres, of the parent's band-limited trigonometric interpolant (the phase is
  the quarter-parent-cell offset of the fine centres).  Other modes keep the fine noise.
* Reverse Hoffman-Ribak acts on the cells covered by the patch itself (not on the padding).
* delta_coarse of patch p >= 2 is the parent level's noise on the parent patch (zero on its
  padding and on the cells covered by patch p) convolved with the parent's kernel on the parent's
  padded grid.  The coarse contribution carried to patch p is the conservative tri-cubic
  interpolation of (everything carried to the parent) + (that delta_coarse), on the parent patch.
* The restriction of delta_bnd (mean of 8 children) is ADDED to the parent's density on the
  parent cells under D' that patch p does not cover.
* Finally every covered coarse cell of the density is set to the mean of its children, finest
  level first (the composite representation the solver uses).  The paper's optional extra padding
  of a few cells, cut off at the end, is not applied.
"""

import numpy as np

from .zoom import Hierarchy

# cubic Lagrange weights through nodes -1, 0, 1, 2 evaluated at +1/4 (the odd child); the even
# child at -1/4 takes them mirrored through nodes 1, 0, -1, -2
CUBIC_PLUS = (-7.0 / 128.0, 105.0 / 128.0, 35.0 / 128.0, -5.0 / 128.0)
RESTRICT_W = (0.25, 0.5, 0.25)


def check_geometry(H):
    """Power-of-two base and patches; the padded domain of every patch inside its parent."""
    if H.N0 & (H.N0 - 1) or H.N0 < 2:
        raise ValueError("the base must be a power of two")
    for p in range(1, H.P + 1):
        n, o, pn = H.n[p], H.off[p], H.n[p - 1]
        for a in range(3):
            if n[a] & (n[a] - 1) or n[a] < 4:
                raise ValueError("patch sizes must be powers of two >= 4")
            lo, hi = o[a] - n[a] // 4, o[a] + 3 * n[a] // 4
            if p == 1:
                if n[a] > pn[a]:
                    raise ValueError("padded domain larger than the base")
            elif lo < 0 or hi > pn[a]:
                raise ValueError("padded domain of patch %d leaves its parent" % p)


def radial(table, dr, r):
    """T(r) by linear interpolation of table[i] = T(i dr)."""
    t = np.asarray(r) / dr
    i = np.floor(t).astype(np.int64)
    w = t - i
    return (1.0 - w) * table[i] + w * table[i + 1]


def fft_displacements(P):
    """Displacement (in cells) of FFT index j on an axis of P points: j below P/2, j - P above."""
    j = np.arange(P)
    return np.where(j < P // 2, j, j - P)


def _kernel_shape(H, l):
    return (H.N0,) * 3 if l == 0 else tuple(2 * v for v in H.n[l])


def kernel_direct(shape, h, table, dr, subgrid):
    """T sampled at the displacement grid (Section 2.2), or the mean over the 8 sub-cell centres
    of each displacement (Section 3.5.3)."""
    d = np.meshgrid(*[fft_displacements(P) * h for P in shape], indexing="ij")
    if not subgrid:
        return radial(table, dr, np.sqrt(d[0] ** 2 + d[1] ** 2 + d[2] ** 2))
    acc = np.zeros(shape)
    for sx in (-0.25, 0.25):
        for sy in (-0.25, 0.25):
            for sz in (-0.25, 0.25):
                x, y, z = d[0] + sx * h, d[1] + sy * h, d[2] + sz * h
                acc = acc + radial(table, dr, np.sqrt(x * x + y * y + z * z))
    return acc / 8.0


def kernel_restrict(fine, shape, h, table, dr):
    """Coarse kernel (spacing h) from the finer level's kernel grid (eq. transfer_average, read as
    the 1/4, 1/2, 1/4 child-pair mean) where it exists, T(|D|) sampled elsewhere."""
    out = kernel_direct(shape, h, table, dr, subgrid=False)
    Pf = fine.shape
    J = [fft_displacements(P) for P in shape]
    inside = [np.abs(j) <= Pf[a] // 4 - 1 for a, j in enumerate(J)]
    Jin = [j[m] for j, m in zip(J, inside)]
    avg = np.zeros(tuple(len(j) for j in Jin))
    for sx, wx in zip((-1, 0, 1), RESTRICT_W):
        for sy, wy in zip((-1, 0, 1), RESTRICT_W):
            for sz, wz in zip((-1, 0, 1), RESTRICT_W):
                ix = np.mod(2 * Jin[0] + sx, Pf[0])
                iy = np.mod(2 * Jin[1] + sy, Pf[1])
                iz = np.mod(2 * Jin[2] + sz, Pf[2])
                avg = avg + ((wx * wy) * wz) * fine[np.ix_(ix, iy, iz)]
    out[np.ix_(*[np.nonzero(m)[0] for m in inside])] = avg
    return out


def kernels(H, table, dr, subgrid=True):
    """T_l on every level's FFT grid (base: N0^3 periodic; patch p: (2 n_p)^3), finest first
    computed, returned base first."""
    check_geometry(H)
    T = [None] * (H.P + 1)
    T[H.P] = kernel_direct(_kernel_shape(H, H.P), H.h[H.P], table, dr, subgrid)
    for l in range(H.P - 1, -1, -1):
        T[l] = kernel_restrict(T[l + 1], _kernel_shape(H, l), H.h[l], table, dr)
    return T


# ----------------------------------------------------------------------------- noise

def _region(H, p):
    """Parent-cell index arrays of patch p's padded domain (wrapping on the base)."""
    idx = []
    for a in range(3):
        r = np.arange(H.off[p][a] - H.n[p][a] // 4, H.off[p][a] + 3 * H.n[p][a] // 4)
        if p == 1:
            r = np.mod(r, H.N0)
        idx.append(r)
    return idx


def _parent_view(H, p, mu_parent):
    """The parent noise array in the parent's own patch coordinates (the base, or the parent
    patch cut out of its padded domain)."""
    if p == 1:
        return mu_parent
    q = p - 1
    c = [slice(H.n[q][a] // 2, H.n[q][a] // 2 + H.n[q][a]) for a in range(3)]
    return mu_parent[tuple(c)]


def _inject(c):
    return np.repeat(np.repeat(np.repeat(c, 2, 0), 2, 1), 2, 2)


def _mean8(v):
    a, b, c = v.shape
    return v.reshape(a // 2, 2, b // 2, 2, c // 2, 2).mean(axis=(1, 3, 5))


def _patch_slices(H, p):
    """Patch p's own cells inside its padded domain D'."""
    return tuple(slice(H.n[p][a] // 2, H.n[p][a] // 2 + H.n[p][a]) for a in range(3))


def refine_noise(H, xi):
    """Section 2.3.1.  xi[0]: N0^3 unit normals; xi[p]: (2 n_p)^3 unit normals on D'.
    Returns mu: the base noise (N0^3) and every patch's noise on its padded domain."""
    check_geometry(H)
    mu = [np.asarray(xi[0], dtype=np.float64) / H.h[0] ** 1.5]
    for p in range(1, H.P + 1):
        w = np.asarray(xi[p], dtype=np.float64) / H.h[p] ** 1.5
        n = H.n[p]
        F = np.fft.fftn(w)
        par = _parent_view(H, p, mu[p - 1])
        C = np.fft.fftn(par[np.ix_(*_region(H, p))])
        m = [fft_displacements(2 * v) for v in n]
        keep = [np.abs(mi) < v // 2 for mi, v in zip(m, n)]
        sel = np.ix_(*[np.nonzero(k)[0] for k in keep])
        msel = [mi[k] for mi, k in zip(m, keep)]
        phase = [np.exp(-1j * np.pi * mi / (2.0 * v)) for mi, v in zip(msel, n)]
        csel = C[np.ix_(*[np.mod(mi, v) for mi, v in zip(msel, n)])]
        F[sel] = 8.0 * csel * phase[0][:, None, None] * phase[1][None, :, None] * phase[2][None, None, :]
        mu.append(np.real(np.fft.ifftn(F)))
    for p in range(H.P, 0, -1):
        child = mu[p][_patch_slices(H, p)]
        par = _parent_view(H, p, mu[p - 1])
        par[H.covered(p)] = _mean8(child)
    return mu


# ----------------------------------------------------------------------------- convolution

def _conv(x, T, h):
    """Circular convolution sum_b h^3 T(a - b) x(b) on T's grid."""
    return np.real(np.fft.ifftn(np.fft.fftn(x) * np.fft.fftn(T))) * h ** 3


def _cubic_axis(c, axis):
    """Tri-cubic step along one axis: coarse values padded by 2 on each side -> 2m children."""
    c = np.moveaxis(c, axis, 0)
    m = c.shape[0] - 4
    out = np.empty((2 * m,) + c.shape[1:])
    w = CUBIC_PLUS
    for I in range(m):
        j = I + 2
        out[2 * I] = w[3] * c[j - 2] + w[2] * c[j - 1] + w[1] * c[j] + w[0] * c[j + 1]
        out[2 * I + 1] = w[0] * c[j - 1] + w[1] * c[j] + w[2] * c[j + 1] + w[3] * c[j + 2]
    return np.moveaxis(out, 0, axis)


def interpolate_conservative(H, p, U):
    """Section 2.3.4: conservative tri-cubic interpolation of the level-(p-1) field U (the base, or
    the parent patch) onto patch p."""
    o, n = H.off[p], H.n[p]
    idx = [np.arange(o[a] - 2, o[a] + n[a] // 2 + 2) for a in range(3)]
    if p == 1:
        idx = [np.mod(i, H.N0) for i in idx]
    c = U[np.ix_(*idx)]
    for a in range(3):
        c = _cubic_axis(c, a)
    return c + _inject(U[H.covered(p)] - _mean8(c))


def convolve_levels(H, T, mu):
    """Sections 2.3.3-2.3.4: the density on every level (base N0^3, patches n_p^3)."""
    check_geometry(H)
    P = H.P
    delta = [None] * (P + 1)
    delta[0] = _conv(mu[0], T[0], H.h[0])
    carry = None                    # coarse contributions on the previous level
    if P >= 1:
        z = mu[0].copy()
        z[H.covered(1)] = 0.0
        carry = _conv(z, T[0], H.h[0])
    for p in range(1, P + 1):
        h = H.h[p]
        ps = _patch_slices(H, p)
        inside = np.zeros(mu[p].shape, dtype=bool)
        inside[ps] = True
        par = _parent_view(H, p, mu[p - 1])
        inj = _inject(par[np.ix_(*_region(H, p))])
        nu_self = np.where(inside, mu[p], 0.0)
        nu_bnd = np.where(inside, 0.0, mu[p] - inj)
        d_sb = _conv(nu_self + nu_bnd, T[p], h)
        d_bnd = _conv(nu_bnd, T[p], h)
        C = interpolate_conservative(H, p, carry)
        delta[p] = d_sb[ps] + C
        # delta_bnd restricted onto the parent cells of D' that the patch does not cover
        rb = _mean8(d_bnd)
        region = _region(H, p)
        cov = np.zeros(rb.shape, dtype=bool)
        q = [slice(H.n[p][a] // 4, H.n[p][a] // 4 + H.n[p][a] // 2) for a in range(3)]
        cov[tuple(q)] = True
        sel = np.ix_(*region)
        delta[p - 1][sel] = delta[p - 1][sel] + np.where(cov, 0.0, rb)
        if p < P:
            nc = nu_self.copy()
            cs = [slice(H.n[p][a] // 2 + H.off[p + 1][a], H.n[p][a] // 2 + H.off[p + 1][a] + H.n[p + 1][a] // 2)
                  for a in range(3)]
            nc[tuple(cs)] = 0.0
            carry = C + _conv(nc, T[p], h)[ps]
    for p in range(P, 0, -1):
        delta[p - 1][H.covered(p)] = _mean8(delta[p])
    return delta


def multiscale_density(H, table, dr, xi, subgrid=True):
    """The whole chain: kernels, refined noise, nested convolution.  Returns (delta, mu, T)."""
    T = kernels(H, table, dr, subgrid)
    mu = refine_noise(H, xi)
    return convolve_levels(H, T, mu), mu, T


__all__ = ["check_geometry", "radial", "fft_displacements", "kernel_direct", "kernel_restrict", "kernels",
           "refine_noise", "interpolate_conservative", "convolve_levels", "multiscale_density"]
