"""The allocation-free sampling entry point (sdi_sample_points_noalloc) against
sdi_sample_points, bit for bit: two calls in a row on the same device, the
second with a smaller input (fewer points, another sector, shift and start),
with and without a Vegas grid, and an empty call."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1511_03614_amd as P  # noqa: E402
import sectorgen  # noqa: E402


def test_noalloc_matches_sample_points():
    ctx = P.sdi_ctx_create(0)
    prob = sectorgen.config2()
    try:
        for k, v in dict(lattice_log2=12, shifts=8, seed=11, warmup=2, warmup_log2=10, nbins=32, budget=0).items():
            P.sdi_set_param(ctx, k, v)
        h = P.sdi_problem_create(ctx, prob)
        try:
            for adapted in (False, True):
                if adapted:
                    P.sdi_integrate(ctx, h)              # leaves adapted Vegas grids on the problem
                for s, shift, i0, npts in ((5, 7, 0, 4096), (17, 2, 1000, 333)):
                    n = prob.sectors[s].n
                    x_ref, w_ref = P.sdi_sample_points(ctx, h, s, shift, i0, npts, n)
                    x = torch.full((npts, n), np.nan, dtype=torch.float64, device="cuda")
                    w = torch.full((npts,), np.nan, dtype=torch.float64, device="cuda")
                    P.sdi_sample_points_noalloc(ctx, h, s, shift, i0, x, w)
                    assert torch.equal(x, x_ref) and torch.equal(w, w_ref), (adapted, s, shift, npts)
                    if adapted:
                        assert not torch.all(w == 1.0)   # the grid was applied
            x0 = torch.empty((0, prob.sectors[0].n), dtype=torch.float64, device="cuda")
            P.sdi_sample_points_noalloc(ctx, h, 0, 0, 0, x0)
            with pytest.raises(P.SdiError):
                P.sdi_sample_points_noalloc(ctx, h, 0, 8, 0, torch.empty((4, prob.sectors[0].n),
                                                                         dtype=torch.float64, device="cuda"))
        finally:
            P.sdi_problem_destroy(h)
    finally:
        P.sdi_ctx_destroy(ctx)
