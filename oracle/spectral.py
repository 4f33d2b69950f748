"""Spectral corrections that recover small-scale power (oracle): Section 3.5.

Test infrastructure only (see ``oracle/__init__.py``).

Sources in the paper:
* Section 3.5.1 (finite-volume correction): the multigrid solution treats its source as cell
  averages, i.e. the continuous field convolved with the cell's box window W_s (nearest-grid-
  point assignment).  Dividing the Fourier transform of the source by the window's transform,
  prod_i (2 / k_i) sin(h k_i / 2), restores the sub-grid amplitudes.
* Section 3.5.3 (averaging correction): a source sampled as the mean over the 8 sub-cells of each
  cell (sub-cell centres at +-h/4 on every axis) is the field convolved with the sub-grid kernel,
  whose transform is prod_i cos(h k_i / 4); dividing by it restores the power.
* Section 3.5.2 (hybrid Poisson solver): on the finest grid the finite-difference gradient of
  the finite-difference potential is replaced by the k-space exact one.  The correction, added to
  the finite-difference result, has the transform [continuum gradient / continuum Laplacian
  minus G~_j / L~] times f~, where G~_j and L~ are the Fourier symbols of the finite-difference
  gradient and Laplacian (Table 1).  On a patch the source is set to zero outside the patch and
  the grid is zero-padded to twice its size (isolated boundaries); on a periodic grid no padding
  is needed and the corrected result equals a pure FFT Poisson solve.

Readings (where the paper is silent, ambiguous or its notation is garbled):
* Normalisation of W_s: the printed window is the indicator of the cell, whose transform is h^3
  times prod sinc(h k_i / 2).  The deconvolution divides by the cell AVERAGE's transform,
  prod_i sinc(h k_i / 2) (sinc(x) = sin(x) / x), so the k = 0 mode (the mean) is unchanged.
* Sign of the hybrid correction: the printed bracket pairs i k_j / k^2 with G~_j / L~ with a
  Laplacian symbol whose sign convention the text does not fix.  The reading is the one that makes
  the corrected field exact: with the library's convention (the finite-difference field is
  scale * G phi with L phi = f), the correction is
      scale * [ (i k_j) / (-k^2) - G~_j / L~ ] f~,
  so that  scale * G phi + correction = scale * grad(laplacian^-1 f)  mode by mode.  The gradient
  and Laplacian orders are separate arguments (the paper's n is the same for both; the library's
  default pairs the 7-point Laplacian with the fourth-order gradient).
* Nyquist planes: on a cell-centred grid the only real Nyquist pattern along an axis is
  (-1)^i, the samples of sin(pi x / h), whose continuum derivative vanishes at every cell centre;
  central differences give zero there too.  The correction of component j is therefore zero on
  the Nyquist plane of axis j.  k = 0 gets no correction.
* Padding: the grid is zero-padded to the smallest power of two that is at least twice the
  patch's length on each axis (twice the length exactly for power-of-two patches, the sizes the
  paper uses), with the patch at the origin corner of the padded grid; the result is cut back to
  the patch.  The same isolated treatment is offered for the two deconvolutions on patches (the
  paper describes them for periodic grids only).
* Wavenumbers: mode m of an axis of P points has k = 2 pi m / (P h), m in numpy's FFT order
  (0 .. P/2-1, -P/2 .. -1).  Every multiplier here depends on k alone, so the cell-centre offset
  of the samples does not matter (the operators are translation invariant).
"""

import numpy as np

from .highorder import symbol_1d
from .stencil import G4_WEIGHTS, G6_WEIGHTS


def pad_length(n):
    """Smallest power of two >= 2 n (the isolated-boundary FFT length for a patch of n cells)."""
    p = 1
    while p < 2 * n:
        p *= 2
    return p


def kappas(shape):
    """k h on every axis for a periodic grid of this shape: 2 pi m / P, broadcastable arrays."""
    out = []
    for a, P in enumerate(shape):
        m = np.fft.fftfreq(P) * P
        sh = [1, 1, 1]
        sh[a] = P
        out.append((2.0 * np.pi * m / P).reshape(sh))
    return out


def ngp_window(shape):
    """Transform of the cell average (Section 3.5.1, normalised): prod_i sinc(k_i h / 2)."""
    w = np.ones(shape)
    for kap in kappas(shape):
        half = kap / 2.0
        s = np.where(half == 0.0, 1.0, np.sin(half) / np.where(half == 0.0, 1.0, half))
        w = w * s
    return w


def subgrid_window(shape):
    """Transform of the 8-sub-cell average (Section 3.5.3): prod_i cos(k_i h / 4)."""
    w = np.ones(shape)
    for kap in kappas(shape):
        w = w * np.cos(kap / 4.0)
    return w


def grad_symbol(kap, order):
    """g(kh) such that Table 1's gradient of this order maps e^{ikx} to (i g / h) e^{ikx}."""
    if order == 4:
        w, den, offs = G4_WEIGHTS, 12.0, range(-2, 3)
    elif order == 6:
        w, den, offs = G6_WEIGHTS, 60.0, range(-3, 4)
    else:
        raise ValueError("gradient order must be 4 or 6")
    g = np.zeros_like(kap)
    for off, c in zip(offs, w):
        if c != 0.0:
            g = g + c * np.sin(off * kap)
    return g / den


def hybrid_multipliers(shape, lap_order=2, grad_order=4):
    """s_j(k) (j = x, y, z), real, with the correction of component j = i * scale * h * s_j * f~.

    s_j = -(kh)_j / (kh)^2 - g_j / lambda, lambda = sum_axes symbol_1d(k_a h) (Table 1 Laplacian
    symbol in grid units, negative); s_j = 0 at k = 0 and on the Nyquist plane of axis j.
    """
    kap = kappas(shape)
    k2 = sum(k * k for k in kap)
    lam = sum(symbol_1d(k, lap_order) for k in kap)
    zero = (k2 == 0.0)
    k2s = np.where(zero, 1.0, k2)
    lams = np.where(zero, 1.0, lam)
    out = []
    for a, P in enumerate(shape):
        s = -kap[a] / k2s - grad_symbol(kap[a], grad_order) / lams
        s = np.where(zero, 0.0, s)
        nyq = np.zeros(shape, dtype=bool)
        idx = [slice(None)] * 3
        idx[a] = P // 2
        nyq[tuple(idx)] = True
        out.append(np.where(nyq, 0.0, np.broadcast_to(s, shape)))
    return out


def _embed(f, periodic):
    """The grid the transform runs on: f itself (periodic) or f zero-padded at the origin corner."""
    f = np.asarray(f, dtype=np.float64)
    if periodic:
        return f
    P = tuple(pad_length(n) for n in f.shape)
    g = np.zeros(P)
    g[:f.shape[0], :f.shape[1], :f.shape[2]] = f
    return g


def _cut(g, shape):
    return g[:shape[0], :shape[1], :shape[2]]


def fv_deconvolve(f, periodic=True):
    """Section 3.5.1: f~ / prod sinc(k h / 2), back-transformed (real part)."""
    g = _embed(f, periodic)
    out = np.real(np.fft.ifftn(np.fft.fftn(g) / ngp_window(g.shape)))
    return _cut(out, np.shape(f))


def sg_deconvolve(f, periodic=True):
    """Section 3.5.3: f~ / prod cos(k h / 4), back-transformed (real part)."""
    g = _embed(f, periodic)
    out = np.real(np.fft.ifftn(np.fft.fftn(g) / subgrid_window(g.shape)))
    return _cut(out, np.shape(f))


def hybrid_correction(f, h, lap_order=2, grad_order=4, scale=1.0, periodic=True):
    """Section 3.5.2: the three components to ADD to scale * G phi (L phi = f) on the finest grid.

    Periodic: transforms on f's own grid.  Isolated (periodic=False): f is zero-padded at the
    origin corner to pad_length(n) per axis and the result is cut back to f's shape.
    Returns an array of shape (3,) + f.shape.
    """
    g = _embed(f, periodic)
    fh = np.fft.fftn(g)
    s = hybrid_multipliers(g.shape, lap_order, grad_order)
    comps = [np.real(np.fft.ifftn(1j * scale * h * sj * fh)) for sj in s]
    return np.stack([_cut(c, np.shape(f)) for c in comps])


def exact_displacement(f, h, scale=1.0):
    """scale * grad(laplacian^-1 f) by k-space division on a periodic grid (pure FFT solve)."""
    f = np.asarray(f, dtype=np.float64)
    kap = kappas(f.shape)
    k2 = sum(k * k for k in kap)
    fh = np.fft.fftn(f)
    zero = (k2 == 0.0)
    phih = np.where(zero, 0.0, -fh * (h * h) / np.where(zero, 1.0, k2))
    out = []
    for a, P in enumerate(f.shape):
        d = 1j * kap[a] / h * phih
        idx = [slice(None)] * 3
        idx[a] = P // 2
        d[tuple(idx)] = 0.0
        out.append(scale * np.real(np.fft.ifftn(d)))
    return np.stack(out)


__all__ = ["pad_length", "kappas", "ngp_window", "subgrid_window", "grad_symbol",
           "hybrid_multipliers", "fv_deconvolve", "sg_deconvolve", "hybrid_correction",
           "exact_displacement"]
