"""Lagrangian perturbation theory on periodic grids (oracle).

Test infrastructure only (see ``oracle/__init__.py``).

Section 3.1 of the paper:
* First order (eq. "zeldovich"): the displacement is a scalar times the
  gradient of the potential that solves Poisson's equation with the density as
  source.  The gradient is Table 1's fourth-order stencil.
* Second order: the second potential solves Poisson's equation with source
  tau = -1/2 sum_{i,j} [ (Phi_,ij)^2 - Phi_,ii Phi_,jj ], evaluated "using finite
  differences".

Readings:
* Stencil for the second derivatives: D_ij = G_i o G_j (the fourth-order
  gradient applied twice) for all i, j including i = j.  This makes tau the
  second invariant of the finite-difference deformation tensor; a single plane
  wave then gives tau = 0 exactly for any direction.
* The diagonal terms of the paper's double sum cancel, so
  tau = sum_{i>j} ( D_ii D_jj - D_ij^2 ).  ``tau_paper_form`` evaluates the
  paper's double sum literally; tests check the two agree.
* Sign and normalisation of the displacements are garbled in the paper (the
  first-order equation carries D_+^{-1}, the second-order one D_+ and
  D_2 ~ +3/7 D_+^2).  The library therefore returns scale * G phi and the
  caller supplies the scalar; the defaults used by the tests follow the
  published convention the paper cites (Scoccimarro 1998): psi_1 = -G phi_1,
  psi_2 = D2 G phi_2 with D2 = -3/7 at D_+ = 1.
"""

import numpy as np

from .stencil import grad4


def displacement(phi, h, scale=1.0):
    """psi_c = scale * G4_c phi for c = x, y, z (periodic); returns (3, ...) array."""
    return np.stack([scale * grad4(phi, h, a) for a in range(3)])


def second_derivatives(phi, h):
    """D[i][j] = G4_i (G4_j phi) for all i, j (periodic)."""
    g = [grad4(phi, h, j) for j in range(3)]
    return [[grad4(g[j], h, i) for j in range(3)] for i in range(3)]


def tau(phi, h):
    """Second-order source: sum_{i>j} (D_ii D_jj - D_ij^2)."""
    D = second_derivatives(phi, h)
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
