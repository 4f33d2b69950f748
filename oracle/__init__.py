"""Plain FP64 CPU oracle for the adaptive-multigrid / LPT hot path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  The product path
(``paper_1103_6031_amd``) never imports, calls or links anything here, and the
oracle imports nothing from the product package: the two share no code.

Everything is written from Hahn & Abel, "Multi-scale initial conditions for
cosmological simulations" (MNRAS 2011):

* ``stencil``  - Table 1 operators (7-point Laplacian, 4th-order gradient),
                 restriction / injection of Section 3.2, periodic wrap.
* ``periodic`` - the FAS V-cycle of Section 3.2 (nine steps, red-black
                 Gauss-Seidel, nu1 = nu2 = 2) and the exact discrete periodic
                 solve by eigenvalue division (Table 1 symbols).
* ``zoom``     - the adaptive multigrid of Section 3.3: nested patches, ghost
                 zones by polynomial interpolation parallel then normal to the
                 face, flux matching with the Table 2 order-1 flux operator,
                 composite residual, post-solve wide ghosts.
* ``lpt``      - Section 3.1: first-order displacements from the gradient of
                 the potential and the second-order source term tau.
* ``highorder``- the fourth- and sixth-order Laplacians of Table 1 (13- and
                 19-point) and the periodic FAS solve of Section 3.2 with them.
* ``zoom_ho``  - the adaptive multigrid with the order-4 / order-6 Laplacians:
                 ghost zones of width order / 2 by polynomials of that degree,
                 flux matching with the Table 2 operators of order 3 and 5.
* ``spectral`` - Section 3.5: finite-volume (cell-average) and sub-grid deconvolution, and the
                 hybrid Poisson correction (k-space exact displacement on the finest grid,
                 periodic or zero-padded isolated), by numpy FFTs.
* ``density``  - Sections 2.1-2.3: the multi-scale Gaussian density on nested grids (kernels
                 per level, mode-preserving white-noise refinement, nested FFT convolutions
                 with conservative tri-cubic interpolation of the coarse contributions).
* ``dense``    - brute-force dense assembly of the periodic and composite
                 linear systems for tiny grids (pins for the iterative solvers).

Precision: float64 throughout.  Speed: slow by design (numpy whole-array
operations, no blocking, no fusion).

Readings taken where the paper is silent or ambiguous are listed in each
module's header.  Parity unpinned: none of the functions here - every one is
checked in ``tests/test_oracle_*.py`` against closed forms, Table 1 symbols,
brute-force dense solves or invariants that do not reuse the oracle's own
arithmetic.
"""

from . import stencil, periodic, lpt, zoom, zoom_ho, dense, highorder, spectral, density  # noqa: F401
