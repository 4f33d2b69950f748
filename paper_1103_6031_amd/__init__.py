"""MI355X (gfx950) adaptive-multigrid Poisson solver and LPT for multi-scale initial conditions.

Hahn & Abel 2011 ("Multi-scale initial conditions for cosmological simulations"): the FAS
multigrid of Section 3.2 on a periodic base with nested 2x zoom-in patches (Section 3.3), the
first-order displacements and the second-order source of Section 3.1.  The computation is in
the HIP library libmgic.so (C ABI: include/mgic.h); ``paper_1103_6031_amd.mgic`` is its
Python binding and ``paper_1103_6031_amd.inputs`` the seeded input generator.
"""

__all__ = ["mgic", "inputs", "serve"]
