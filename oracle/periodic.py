"""Periodic FAS multigrid and the exact discrete periodic solve (oracle).

Test infrastructure only (see ``oracle/__init__.py``).

Follows Section 3.2 of the paper ("Multi-grid solution of Poisson's equation"):
the nine-step Full Approximation Scheme, red-black Gauss-Seidel smoothing with
nu1 = nu2 = 2, restriction by the mean of 8 children, prolongation by
injection, V-cycles repeated until the residual norm taken after step 9 falls
below a threshold, periodic boundary conditions throughout.

Readings (where the paper is silent, ambiguous or garbled):
* Restriction / prolongation names: the paper calls one operator "injection"
  when defining the notation but then uses it as prolongation; we use
  restriction = mean of 8 children, prolongation = injection (the operator
  choices paragraph of Section 3.2).
* Step 1 sets u = 0 on the coarsest level.  That is the exact solution only
  when the coarsest grid is one cell.  Grids are coarsened while N is even;
  if the coarsest N is odd and > 1 (48^3, 96^3 reach 3^3) it is solved exactly
  (zero-mean solution by eigenvalue division); red-black Gauss-Seidel never
  runs on an odd periodic grid, where red-black is not a 2-colouring.
* The periodic problem is singular: the mean of f is removed first (and
  reported), and the returned potential has zero mean.
* Residual norm: RMS of r over RMS of f (after mean removal), i.e. a
  relative residual.
* Colour order: red = (i+j+k) even first, then black.  Within a colour the
  update is u <- (neighbour_sum - h^2 f) / 6 with every neighbour read before
  any cell of that colour is written (Gauss-Seidel between colours).
"""

import numpy as np

from .stencil import neighbour_sum, lap7, restrict_mean8, inject, red_mask


def rbgs_half(u, f, h, colour):
    """One red (colour 0) or black (colour 1) half-sweep, returning a new array."""
    new = (neighbour_sum(u) - (h * h) * f) / 6.0
    red = red_mask(u.shape)
    mask = red if colour == 0 else ~red
    return np.where(mask, new, u)


def rbgs_sweep(u, f, h):
    """Red-black Gauss-Seidel: red half-sweep, then black."""
    u = rbgs_half(u, f, h, 0)
    return rbgs_half(u, f, h, 1)


def residual(u, f, h):
    """Step 3: r = f - L u."""
    return f - lap7(u, h)


def exact_coarse(f, h):
    """Exact zero-mean solution of L u = f - mean(f) on a small odd periodic grid."""
    return fft_solve(f, h)


def vcycle(u, f, h, nu1=2, nu2=2):
    """One FAS V-cycle on the periodic grid (Section 3.2, steps 1-9); returns new u."""
    N = u.shape[0]
    # step 1: coarsest level
    if N == 1:
        return np.zeros_like(u)
    if N % 2 == 1:
        return exact_coarse(f, h)
    # step 2: nu1 smoothing sweeps
    for _ in range(nu1):
        u = rbgs_sweep(u, f, h)
    # step 3: residual
    r = residual(u, f, h)
    # steps 4-5: restrict residual and solution
    rc = restrict_mean8(r)
    uc = restrict_mean8(u)
    uc_old = uc.copy()
    # step 6: tau-correction, coarse right-hand side
    H = 2.0 * h
    fc = rc + lap7(uc, H)
    # step 7: recurse
    uc = vcycle(uc, fc, H, nu1, nu2)
    # step 8: correct by injection of the coarse change
    u = u + inject(uc - uc_old)
    # step 9: nu2 smoothing sweeps
    for _ in range(nu2):
        u = rbgs_sweep(u, f, h)
    return u


def rms(a):
    return float(np.sqrt(np.mean(np.square(a))))


def solve_level(f, h, tol=1e-10, max_cycles=50, nu1=2, nu2=2, u0=None):
    """Periodic FAS solve of L u = f - mean(f).

    Returns (u, info) with u of zero mean and info = dict(cycles, rel_res,
    f_mean, history).  Stops when rms(r)/rms(f) <= tol after a cycle's step 9.
    """
    f = np.asarray(f, dtype=np.float64)
    f_mean = float(np.mean(f))
    fz = f - f_mean
    fnorm = rms(fz)
    u = np.zeros_like(fz) if u0 is None else np.array(u0, dtype=np.float64)
    hist = []
    cycles = 0
    rel = rms(residual(u, fz, h)) / fnorm if fnorm > 0 else 0.0
    while cycles < max_cycles and rel > tol:
        u = vcycle(u, fz, h, nu1, nu2)
        cycles += 1
        rel = rms(residual(u, fz, h)) / fnorm if fnorm > 0 else 0.0
        hist.append(rel)
    u = u - np.mean(u)
    return u, dict(cycles=cycles, rel_res=rel, f_mean=f_mean, history=hist)


def fft_solve(f, h):
    """Exact discrete solution: u_hat(m) = f_hat(m) / lambda(m), u_hat(0) = 0.

    lambda(m) is the 7-point Laplacian eigenvalue (Table 1 order-2 symbol
    summed over the axes).  The result is the zero-mean solution of
    L u = f - mean(f).
    """
    N = f.shape
    fh = np.fft.fftn(f)
    m = np.meshgrid(*[np.fft.fftfreq(n) * n for n in N], indexing="ij")
    lam = -(2.0 / (h * h)) * sum(1.0 - np.cos(2.0 * np.pi * mi / n) for mi, n in zip(m, N))
    lam[0, 0, 0] = 1.0
    uh = fh / lam
    uh[0, 0, 0] = 0.0
    return np.real(np.fft.ifftn(uh))


def cell_updates(N, cycles, nu1=2, nu2=2):
    """Smoother cell-updates of a periodic solve: sum over cycles and levels of (nu1+nu2) cells."""
    per_cycle = 0
    n = N
    while n > 1 and n % 2 == 0:
        per_cycle += (nu1 + nu2) * n ** 3
        n //= 2
    return per_cycle * cycles


__all__ = ["rbgs_half", "rbgs_sweep", "residual", "vcycle", "solve_level", "fft_solve",
           "rms", "cell_updates"]
