"""The multi-scale density of Sections 2.1-2.3 on the GPU against the oracle, level by level.

Tolerance: both sides build the same kernel grids from the same radial table with the same
arithmetic order; the transforms differ (hand-written Stockham on the GPU, numpy's FFT on the host),
each backward stable with error ~ eps log2(P) of the field's norm, and the noise refinement and the
convolutions chain a handful of them.  Bound: 1e-11 of each level's largest magnitude.
"""

import numpy as np
import pytest

from gpu_util import needs_gpu, note, to_dev, to_host

pytestmark = [pytest.mark.gpu, needs_gpu]

TOL = 1e-11


def _gauss_table(sigma, r_max, count=1 << 16):
    dr = r_max / count
    r = np.arange(count) * dr
    return (2 * np.pi * sigma ** 2) ** -1.5 * np.exp(-r * r / (2 * sigma ** 2)), dr


def _run(N0, h0, patches, table, dr, seed, subgrid):
    from oracle import density
    from oracle.zoom import Hierarchy
    from paper_1103_6031_amd import inputs, mgic
    import torch
    xi = inputs.multiscale_noise(N0, patches, seed)
    H = Hierarchy(N0, h0, patches)
    want, _, _ = density.multiscale_density(H, table, dr, xi, subgrid=subgrid)
    note("density: N0 %d patches %s subgrid %s" % (N0, patches, subgrid))
    got = mgic.ic_multiscale_density(mgic.Hier(N0, h0, patches), torch.from_numpy(table).to("cuda:0"), dr,
                                     [to_dev(x) for x in xi], subgrid=subgrid)
    for lvl, (g, w) in enumerate(zip(got, want)):
        g = to_host(g)
        scale = float(np.max(np.abs(w)))
        err = float(np.max(np.abs(g - w)))
        assert err <= TOL * scale, (lvl, err, scale)


CASES = [
    (16, 1.0, [], 1.5, True),
    (32, 0.8, [((16, 16, 16), (8, 8, 8))], 1.2, False),
    (32, 0.8, [((16, 8, 16), (10, 6, 8))], 1.2, True),
    (32, 1.0, [((32, 32, 32), (8, 8, 8)), ((16, 16, 16), (8, 8, 8)), ((8, 8, 8), (4, 4, 4))], 1.0, True),
    (16, 2.0, [((16, 16, 16), (4, 4, 4)), ((16, 16, 16), (4, 4, 4))], 3.0, False),
]


@pytest.mark.parametrize("N0,h0,patches,sigma,subgrid", CASES)
def test_density_matches_oracle(N0, h0, patches, sigma, subgrid):
    table, dr = _gauss_table(sigma, r_max=4 * N0 * h0)
    _run(N0, h0, patches, table, dr, 1103 + N0 + len(patches), subgrid)


def test_density_full_size_c3():
    """The zoom workload's geometry: 128^3 base with three nested 128^3 patches (padded domains of
    256^3), the tabulated BBKS real-space transfer function, sub-grid kernel mean on the finest."""
    from paper_1103_6031_amd import inputs
    patches, table, dr, xi = inputs.c3_multiscale_input()
    _run(128, inputs.BOX / 128, patches, table, dr, inputs.SEED_C3 + 17, True)


def test_density_rejects_bad_geometry():
    from paper_1103_6031_amd import mgic
    import torch
    table = torch.zeros(1024, dtype=torch.float64, device="cuda:0")
    xi = [torch.zeros((32,) * 3, dtype=torch.float64, device="cuda:0"),
          torch.zeros((32,) * 3, dtype=torch.float64, device="cuda:0")]
    note("density: validation")
    with pytest.raises(mgic.MGError):      # 12-cell patch: not a power of two
        mgic.ic_multiscale_density(mgic.Hier(32, 1.0, [((12, 12, 12), (8, 8, 8))]), table, 1.0, xi)
    with pytest.raises(mgic.MGError):      # the table does not reach the base's corners
        mgic.ic_multiscale_density(mgic.Hier(32, 1.0, [((16, 16, 16), (8, 8, 8))]), table, 0.01, xi)
