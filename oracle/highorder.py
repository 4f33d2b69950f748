"""Higher-order periodic Laplacians and their FAS multigrid solve (oracle).

Test infrastructure only (see ``oracle/__init__.py``).

Sources in the paper:
* Table 1 (Section 3.2): one-dimensional Laplacian stencils of order 2, 4 and 6 (top rows) and
  their Fourier symbols (bottom rows).  As for the 7-point operator (Section 3.4), the 3-D
  operator is the sum of the 1-D stencil over the three axes: 13 points at order 4, 19 at
  order 6.
* Section 3.2: the FAS V-cycle of ``periodic.py`` (red-black Gauss-Seidel with nu1 = nu2 = 2,
  mean-of-8 restriction, injection prolongation) converges by at least a factor of ten per
  cycle for every order of Table 1 up to 6; every level uses the operator of the same order.

Readings (where the paper is silent):
* Red-black with a stencil of radius R = order / 2: cells two apart along an axis have the same
  colour and now couple, so red-black is no longer a 2-colouring.  A half-sweep updates every
  cell of its colour from the values before that half-sweep (Jacobi within the colour,
  Gauss-Seidel between the colours), which makes the result independent of the update order.
  The update solves the cell's own equation for its centre value:
  u <- (h^2 f - sum_{s=1..R} w_s sum_axes (u[i-s] + u[i+s])) / (3 w_0).
* Offsets wrap modulo N, so on grids narrower than the stencil a neighbour can be the cell
  itself; it is read as a neighbour (its value before the half-sweep), and only the centre
  weight divides.
* Coarsest grid, mean removal, stopping test and the zero-mean gauge of the result are those of
  the 7-point solve (``periodic.py``).  Odd coarsest grids are solved exactly with the order's
  symbol.
"""

import numpy as np

from .stencil import restrict_mean8, inject, red_mask

# Table 1, Laplacian rows: integer weights for offsets 0, 1, ..., R and their common denominator
STENCILS = {
    2: ((-2, 1), 1),
    4: ((-30, 16, -1), 12),
    6: ((-490, 270, -27, 2), 180),
}


def weights(order):
    """w_0 .. w_R of the 1-D stencil of this order (Table 1), as floats."""
    c, den = STENCILS[order]
    return tuple(float(v) / den for v in c)


def off_sum(u, order):
    """sum_{s=1..R} w_s sum_axes (u[i-s] + u[i+s]) with periodic wrap (the off-centre part)."""
    w = weights(order)
    acc = np.zeros_like(u)
    for s in range(1, len(w)):
        pair = np.zeros_like(u)
        for a in range(3):
            pair = pair + (np.roll(u, s, a) + np.roll(u, -s, a))
        acc = acc + w[s] * pair
    return acc


def lap(u, h, order):
    """The 3-D Laplacian of this order: the 1-D stencil of Table 1 summed over the axes."""
    w0 = weights(order)[0]
    return (off_sum(u, order) + 3.0 * w0 * u) / (h * h)


def symbol_1d(k, order):
    """Fourier symbol of the 1-D stencil, as printed in Table 1's bottom rows (k in grid units)."""
    if order == 2:
        return -2.0 * (1.0 - np.cos(k))
    if order == 4:
        return -(np.cos(2 * k) - 16.0 * np.cos(k) + 15.0) / 6.0
    if order == 6:
        return -(-2.0 * np.cos(3 * k) + 27.0 * np.cos(2 * k) - 270.0 * np.cos(k) + 245.0) / 90.0
    raise ValueError("order must be 2, 4 or 6")


def fft_solve(f, h, order):
    """Exact discrete solution: u_hat = f_hat / lambda, lambda = sum_axes symbol_1d / h^2, u_hat(0) = 0."""
    N = f.shape
    m = np.meshgrid(*[np.fft.fftfreq(n) * n for n in N], indexing="ij")
    lam = sum(symbol_1d(2.0 * np.pi * mi / n, order) for mi, n in zip(m, N)) / (h * h)
    lam[0, 0, 0] = 1.0
    uh = np.fft.fftn(f) / lam
    uh[0, 0, 0] = 0.0
    return np.real(np.fft.ifftn(uh))


def rbgs_half(u, f, h, order, colour):
    """One red (colour 0) or black (colour 1) half-sweep, Jacobi within the colour; new array."""
    w0 = weights(order)[0]
    new = ((h * h) * f - off_sum(u, order)) / (3.0 * w0)
    red = red_mask(u.shape)
    return np.where(red if colour == 0 else ~red, new, u)


def rbgs_sweep(u, f, h, order):
    u = rbgs_half(u, f, h, order, 0)
    return rbgs_half(u, f, h, order, 1)


def residual(u, f, h, order):
    """Step 3: r = f - L u."""
    return f - lap(u, h, order)


def vcycle(u, f, h, order, nu1=2, nu2=2):
    """One FAS V-cycle (Section 3.2, steps 1-9) with the operator of this order on every level."""
    N = u.shape[0]
    if N == 1:                       # step 1: coarsest single cell
        return np.zeros_like(u)
    if N % 2 == 1:                   # odd coarsest grid: exact solve
        return fft_solve(f, h, order)
    for _ in range(nu1):             # step 2
        u = rbgs_sweep(u, f, h, order)
    r = residual(u, f, h, order)     # step 3
    rc = restrict_mean8(r)           # steps 4-5
    uc = restrict_mean8(u)
    uc_old = uc.copy()
    H = 2.0 * h
    fc = rc + lap(uc, H, order)      # step 6
    uc = vcycle(uc, fc, H, order, nu1, nu2)   # step 7
    u = u + inject(uc - uc_old)      # step 8
    for _ in range(nu2):             # step 9
        u = rbgs_sweep(u, f, h, order)
    return u


def _rms(a):
    return float(np.sqrt(np.mean(np.square(a))))


def solve_level(f, h, order, tol=1e-10, max_cycles=50, nu1=2, nu2=2, u0=None, fixed_cycles=False):
    """Periodic FAS solve of L_order u = f - mean(f); returns (u, info) as ``periodic.solve_level``.

    With ``fixed_cycles`` exactly max_cycles cycles run (no stopping test).
    """
    f = np.asarray(f, dtype=np.float64)
    f_mean = float(np.mean(f))
    fz = f - f_mean
    fnorm = _rms(fz)
    u = np.zeros_like(fz) if u0 is None else np.array(u0, dtype=np.float64)
    hist = []
    cycles = 0
    rel = _rms(residual(u, fz, h, order)) / fnorm if fnorm > 0 else 0.0
    while cycles < max_cycles and (fixed_cycles or rel > tol):
        u = vcycle(u, fz, h, order, nu1, nu2)
        cycles += 1
        rel = _rms(residual(u, fz, h, order)) / fnorm if fnorm > 0 else 0.0
        hist.append(rel)
    u = u - np.mean(u)
    return u, dict(cycles=cycles, rel_res=rel, f_mean=f_mean, history=hist)


__all__ = ["STENCILS", "weights", "off_sum", "lap", "symbol_1d", "fft_solve", "rbgs_half",
           "rbgs_sweep", "residual", "vcycle", "solve_level"]
