"""Oracle computations for the full-size hierarchy parity tests (test infrastructure, not
collected by pytest).

They take minutes of host time, so the tests run them in spawned worker processes - which share
nothing with the process driving the GPU - while the GPU side runs.  Each job takes a hierarchy
layout and seed, draws the same seeded density the GPU side gets, and returns the oracle's 2LPT
chain on it (Section 3.3 solve to a 1e-12 relative residual, Section 3.1 displacements and
second-order source, second solve, displacements).
"""

import time

from oracle import zoom
from paper_1103_6031_amd import inputs


def two_lpt_chain(N0, patches, seed, tol=1e-12):
    t0 = time.perf_counter()
    f = inputs.nested_fields(N0, patches, seed)
    H = zoom.Hierarchy(N0, inputs.BOX / N0, patches)
    phi1, i1 = zoom.solve_hierarchy(H, f, tol=tol, max_cycles=60)
    psi1 = zoom.displacement_hierarchy(H, phi1, -1.0)
    tau = zoom.tau_hierarchy(H, phi1)
    phi2, i2 = zoom.solve_hierarchy(H, tau, tol=tol, max_cycles=60)
    psi2 = zoom.displacement_hierarchy(H, phi2, -3.0 / 7.0)
    return dict(f=f, phi1=phi1, psi1=psi1, tau=tau, phi2=phi2, psi2=psi2,
                cycles=(i1["cycles"], i2["cycles"]), rel_res=(i1["rel_res"], i2["rel_res"]),
                seconds=time.perf_counter() - t0)
