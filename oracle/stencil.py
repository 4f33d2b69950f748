"""Finite-difference operators on cell-centred periodic grids (oracle).

Test infrastructure only (see ``oracle/__init__.py``).

Sources in the paper:
* Table 1 (Section 3.2): 1-D second-order Laplacian [1 -2 1] / h^2, the
  fourth-order gradient [1 -8 0 8 -1] / (12 h) and the sixth-order gradient
  [-1 9 -45 0 45 -9 1] / (60 h).
* Section 3.4: three-dimensional operators are built from the 1-D ones along
  the three axes.  Reading: the 3-D Laplacian is the SUM of the 1-D second
  differences over the axes (the 7-point Laplacian); the gradient component
  along axis c is the 1-D gradient along c.
* Section 3.2 (operator choices): restriction = mean of the 8 children of a
  coarse cell; prolongation = straight injection of the coarse value into its
  8 children.  The grid is the volume-subdivision, cell-centred structure of
  Fig. "grid_structure" (Section 2.3): children of coarse cell I are the fine
  cells 2I and 2I+1 along every axis.

Arrays are indexed [x][y][z].  Periodic neighbours use ``np.roll``:
``np.roll(u, +1, a)[i] == u[i-1]`` and ``np.roll(u, -1, a)[i] == u[i+1]``.
Neighbour sums are taken in the fixed order ((x- + x+) + (y- + y+)) + (z- + z+).
"""

import numpy as np


def neighbour_sum(u):
    """((x- + x+) + (y- + y+)) + (z- + z+) with periodic wrap."""
    sx = np.roll(u, 1, 0) + np.roll(u, -1, 0)
    sy = np.roll(u, 1, 1) + np.roll(u, -1, 1)
    sz = np.roll(u, 1, 2) + np.roll(u, -1, 2)
    return (sx + sy) + sz


def lap7(u, h):
    """7-point Laplacian, the sum over axes of Table 1's order-2 stencil [1 -2 1]/h^2."""
    return (neighbour_sum(u) - 6.0 * u) / (h * h)


G4_WEIGHTS = (1.0, -8.0, 0.0, 8.0, -1.0)  # Table 1, order 4, offsets -2..+2, times 1/12


def grad4(u, h, axis):
    """Fourth-order central gradient along ``axis`` (Table 1, order 4), periodic.

    (u[i-2] - 8 u[i-1] + 8 u[i+1] - u[i+2]) / (12 h)
    """
    acc = np.zeros_like(u)
    for off, w in zip(range(-2, 3), G4_WEIGHTS):
        if w != 0.0:
            acc = acc + w * np.roll(u, -off, axis)
    return acc / (12.0 * h)


G6_WEIGHTS = (-1.0, 9.0, -45.0, 0.0, 45.0, -9.0, 1.0)  # Table 1, order 6, offsets -3..+3, times 1/60


def grad6(u, h, axis):
    """Sixth-order central gradient along ``axis`` (Table 1, order 6), periodic.

    (-u[i-3] + 9 u[i-2] - 45 u[i-1] + 45 u[i+1] - 9 u[i+2] + u[i+3]) / (60 h)
    """
    acc = np.zeros_like(u)
    for off, w in zip(range(-3, 4), G6_WEIGHTS):
        if w != 0.0:
            acc = acc + w * np.roll(u, -off, axis)
    return acc / (60.0 * h)


def grad(u, h, axis, order=4):
    """Table 1 gradient of order 4 or 6 along ``axis``, periodic."""
    if order == 4:
        return grad4(u, h, axis)
    if order == 6:
        return grad6(u, h, axis)
    raise ValueError("gradient order must be 4 or 6")


def restrict_mean8(v):
    """Section 3.2 restriction: average over the 8 children of every coarse cell."""
    nx, ny, nz = v.shape
    assert nx % 2 == 0 and ny % 2 == 0 and nz % 2 == 0
    return v.reshape(nx // 2, 2, ny // 2, 2, nz // 2, 2).mean(axis=(1, 3, 5))


def inject(vc):
    """Section 3.2 prolongation: copy every coarse value into its 8 children."""
    return np.repeat(np.repeat(np.repeat(vc, 2, axis=0), 2, axis=1), 2, axis=2)


def red_mask(shape):
    """Red cells are those with (i+j+k) even (reading: red is updated first)."""
    i, j, k = np.indices(shape)
    return ((i + j + k) % 2) == 0
