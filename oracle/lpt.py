"""Lagrangian perturbation theory on periodic grids (oracle).

Test infrastructure only (see ``oracle/__init__.py``).

Section 3.1 of the paper:
* First order (eq. "zeldovich"): the displacement is a scalar times the
  gradient of the potential that solves Poisson's equation with the density as
  source.  The gradient is Table 1's fourth-order stencil.
* Second order: the second potential solves Poisson's equation with source
  tau = -1/2 sum_{i,j} [ (Phi_,ij)^2 - Phi_,ii Phi_,jj ], evaluated "using finite
  differences".

The gradient is Table 1's stencil of order 4 (the default) or 6; the same order is used for the
second derivatives of tau.

Readings:
* Stencil for the second derivatives: D_ij = G_i o G_j (the fourth-order
  gradient applied twice) for all i, j including i = j.  This makes tau the
  second invariant of the finite-difference deformation tensor; a single plane
  wave then gives tau = 0 exactly for any direction.
* The diagonal terms of the paper's double sum cancel, so
  tau = sum_{i>j} ( D_ii D_jj - D_ij^2 ).  ``tau_paper_form`` evaluates the
  paper's double sum literally; tests check the two agree.
* LLA baryon density (Section 5.3): rho / rho_bar = 1 / det(I + dL/dq) at the Lagrangian
  position, with dL_i/dq_j taken by the same fourth-order gradient (the paper does not name the
  stencil; this is the one the displacements use).  The paper's mass renormalisation
  "rho -> rho + rho~" is read as shifting every cell by the difference between rho_bar and the
  measured mean density, i.e. the returned overdensity has zero (composite) mean.
* Sign and normalisation of the displacements are garbled in the paper (the
  first-order equation carries D_+^{-1}, the second-order one D_+ and
  D_2 ~ +3/7 D_+^2).  The library therefore returns scale * G phi and the
  caller supplies the scalar; the defaults used by the tests follow the
  published convention the paper cites (Scoccimarro 1998): psi_1 = -G phi_1,
  psi_2 = D2 G phi_2 with D2 = -3/7 at D_+ = 1.
"""

import numpy as np

from .stencil import grad4, grad


def displacement(phi, h, scale=1.0, order=4):
    """psi_c = scale * G_c phi for c = x, y, z (periodic; Table 1 gradient of order 4 or 6);
    returns (3, ...) array."""
    return np.stack([scale * grad(phi, h, a, order) for a in range(3)])


def second_derivatives(phi, h, order=4):
    """D[i][j] = G_i (G_j phi) for all i, j (periodic)."""
    g = [grad(phi, h, j, order) for j in range(3)]
    return [[grad(g[j], h, i, order) for j in range(3)] for i in range(3)]


def tau(phi, h, order=4):
    """Second-order source: sum_{i>j} (D_ii D_jj - D_ij^2)."""
    D = second_derivatives(phi, h, order)
    t = np.zeros_like(phi)
    for i in range(3):
        for j in range(i):
            t = t + (D[i][i] * D[j][j] - D[i][j] * D[i][j])
    return t


def tau_paper_form(phi, h):
    """The paper's literal form -1/2 sum_{i,j} [D_ij^2 - D_ii D_jj]."""
    D = second_derivatives(phi, h)
    s = np.zeros_like(phi)
    for i in range(3):
        for j in range(3):
            s = s + (D[i][j] ** 2 - D[i][i] * D[j][j])
    return -0.5 * s


# ----------------------------------------------------------------------------- LLA baryon density

def lla_jacobian(L, h):
    """J[i][j] = dL_i/dq_j by Table 1's fourth-order gradient (periodic); L is (3, ...)."""
    return [[grad4(L[i], h, j) for j in range(3)] for i in range(3)]


def lla_ratio(J):
    """rho / rho_bar = 1 / det(delta_ij + J_ij) per cell (Section 5.3, eq. gasdens), with the
    determinant taken by numpy's LU routine on the stacked 3 x 3 matrices."""
    M = np.stack([np.stack(row, axis=-1) for row in J], axis=-2)   # (..., 3, 3), M[..., i, j] = J_ij
    M = M + np.eye(3)
    return 1.0 / np.linalg.det(M)


def lla_density(L, h, renorm=True):
    """Baryon overdensity rho/rho_bar - 1 of the local Lagrangian approximation (Section 5.3).

    L: displacement field x - q, shape (3, n, n, n), periodic.  With renorm, the measured mean
    overdensity is subtracted so that mass is conserved (the paper's a-posteriori correction,
    read as an additive shift of every cell by the deviation of the mean density from rho_bar).
    """
    d = lla_ratio(lla_jacobian(L, h)) - 1.0
    if renorm:
        d = d - float(np.mean(d))
    return d
