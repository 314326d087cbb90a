"""Parity of the integrator's inner steps on identical inputs: the Vegas grid
refit (sdi_vegas_refit, the kernel sdi_integrate's warm-up runs) against the
oracle's refit on the same histogram, and the flow training's loss weights
(sdi_flow_weights, the kernel sdi_flow_train runs) against the oracle's."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1511_03614_amd as P  # noqa: E402
from oracle import flow, points, vegas  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    c = P.sdi_ctx_create(0)
    yield c
    P.sdi_ctx_destroy(c)


@pytest.mark.parametrize("n,nb,k,alpha", [(3, 32, 3, 1.5), (1, 128, 1, 1.5), (5, 64, 5, 0.75), (2, 2, 2, 1.5)])
def test_refit_matches_oracle(ctx, n, nb, k, alpha):
    rng = np.random.default_rng(n * 100 + nb)
    h = rng.exponential(size=(n, nb, k)) * np.exp(rng.normal(size=(1, nb, 1)) * 2)
    h[:, rng.random(nb) < 0.2, :] = 0.0                       # empty bins
    if n > 1:
        h[n - 1] = 0.0                                        # a dimension with no weight keeps its grid
    g = np.stack([np.concatenate([[0.0], np.sort(rng.uniform(size=nb - 1)), [1.0]]) for _ in range(n)])
    want = vegas.refit(g, vegas.importance(h), alpha=alpha)
    grid = torch.from_numpy(g.copy()).cuda()
    P.sdi_vegas_refit(ctx, torch.from_numpy(h).cuda(), grid, alpha)
    got = grid.cpu().numpy()
    assert np.all(np.diff(got, axis=1) >= 0)
    assert np.max(np.abs(got - want)) <= 1e-12, float(np.max(np.abs(got - want)))
    if n > 1:
        assert np.array_equal(got[n - 1], g[n - 1])


def test_refit_rejects_bad_shapes(ctx):
    h = torch.zeros((2, 3, 1), dtype=torch.float64, device="cuda")
    g = torch.zeros((2, 4), dtype=torch.float64, device="cuda")
    with pytest.raises(P.SdiError):
        P.sdi_vegas_refit(ctx, h, g)                          # 3 bins: not a power of 2


@pytest.mark.parametrize("npts,K,weights", [(1000, 3, None), (4097, 5, [0.0, 1.0, 2.0, 0.5, 3.0]), (7, 1, None)])
def test_flow_weights_match_oracle(ctx, npts, K, weights):
    rng = np.random.default_rng(npts + K)
    f = rng.normal(size=(npts, K, 2)) * np.exp(rng.normal(size=(1, K, 1)) * 3)
    if K > 2:
        f[:, 1, :] = 0.0                                      # an order with zero total is skipped
    lq = rng.normal(size=npts)
    c = P.sdi_flow_weights(ctx, torch.from_numpy(f).cuda(), torch.from_numpy(lq).cuda(), weights).cpu().numpy()
    want = flow.importance_weights((f[..., 0] + 1j * f[..., 1]).T, lq, weights)
    np.testing.assert_allclose(c, want, rtol=1e-12, atol=0)


def test_argument_checks(ctx):
    """The binding refuses device arguments the library cannot size-check."""
    import sectorgen
    prob = sectorgen.config2()
    h = P.sdi_problem_create(ctx, prob)
    try:
        n = prob.sectors[0].n
        assert P.sdi_problem_nvars(h, 0) == n
        good = torch.full((8, n), 0.5, dtype=torch.float64, device="cuda")
        P.sdi_evaluate(ctx, h, 0, good)
        for bad in (good.float(), good.cpu(), torch.full((8, n + 1), 0.5, dtype=torch.float64, device="cuda"),
                    torch.full((8,), 0.5, dtype=torch.float64, device="cuda")):
            with pytest.raises(P.SdiError):
                P.sdi_evaluate(ctx, h, 0, bad)
        with pytest.raises(P.SdiError):
            P.sdi_problem_nvars(h, len(prob.sectors))
    finally:
        P.sdi_problem_destroy(h)
