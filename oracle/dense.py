"""Brute-force dense linear systems for tiny grids (oracle pins).

Test infrastructure only (see ``oracle/__init__.py``).

* ``periodic_matrix`` assembles the 7-point periodic Laplacian of Table 1
  (order 2, summed over axes) as a Kronecker sum of 1-D circulant second
  differences - a construction independent of the stencil code in
  ``oracle.stencil`` - and ``periodic_solve`` returns the minimum-norm
  (= zero-mean) solution of L u = f - mean(f).
* ``composite_matrix`` assembles the composite operator of the adaptive
  multigrid (Section 3.3) column by column, by applying ``oracle.zoom``'s
  operator to unit vectors.  It pins the iterative adaptive FAS to the fixed
  point of that operator (the reading of the ghost formula itself is pinned
  separately by exactness and conservation tests).  With ``order`` 4 or 6 it
  assembles the operator of ``oracle.zoom_ho`` the same way.
"""

import numpy as np

from . import zoom, zoom_ho


def circulant_second_difference(N):
    T = -2.0 * np.eye(N)
    for i in range(N):
        T[i, (i - 1) % N] += 1.0
        T[i, (i + 1) % N] += 1.0
    return T


def periodic_matrix(N, h):
    T = circulant_second_difference(N)
    I = np.eye(N)
    return (np.kron(np.kron(T, I), I) + np.kron(np.kron(I, T), I) + np.kron(np.kron(I, I), T)) / (h * h)


def periodic_solve(f, h):
    """Zero-mean solution of L u = f - mean(f) by a dense least-squares solve."""
    N = f.shape[0]
    A = periodic_matrix(N, h)
    b = (f - f.mean()).ravel()
    x, *_ = np.linalg.lstsq(A, b, rcond=None)
    return x.reshape(f.shape)


def _unknown_masks(H):
    return [zoom.uncovered_mask(H, p) for p in range(H.P + 1)]


def _scatter(H, masks, x):
    u = H.zeros()
    k = 0
    for p in range(H.P + 1):
        m = masks[p]
        cnt = int(m.sum())
        u[p][m] = x[k:k + cnt]
        k += cnt
    return u


def _gather(H, masks, v):
    return np.concatenate([v[p][masks[p]] for p in range(H.P + 1)])


def _residual(H, u, f, flux_match, order):
    if order == 2:
        return zoom.composite_residual(H, u, f, flux_match)
    return zoom_ho.composite_residual(H, u, f, order, flux_match)


def composite_matrix(H, flux_match=True, order=2):
    """Dense matrix of u -> L_composite u over the composite unknowns (Laplacian of `order`)."""
    masks = _unknown_masks(H)
    nunk = sum(int(m.sum()) for m in masks)
    zero_f = H.zeros()
    A = np.zeros((nunk, nunk))
    for k in range(nunk):
        e = np.zeros(nunk)
        e[k] = 1.0
        u = _scatter(H, masks, e)
        r = _residual(H, u, zero_f, flux_match, order)            # = -L u on unknowns
        A[:, k] = -_gather(H, masks, r)
    return A, masks


def composite_solve(H, f, flux_match=True, order=2):
    """Zero-composite-mean solution of the composite system by a dense solve."""
    f, _ = zoom.composite_zero_mean(H, f)
    A, masks = composite_matrix(H, flux_match, order)
    vol = np.concatenate([np.full(int(masks[p].sum()), H.h[p] ** 3) for p in range(H.P + 1)])
    b = _gather(H, masks, f)
    Aa = np.vstack([A, vol[None, :]])
    ba = np.concatenate([b, [0.0]])
    x, *_ = np.linalg.lstsq(Aa, ba, rcond=None)
    u = _scatter(H, masks, x)
    zoom.restrict_bottom_up(H, u)
    return u
