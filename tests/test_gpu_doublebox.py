"""GPU parity on the Euclidean planar double box (s = -3, t = -1, massless):
282 sectors of 6 variables, up to 4 singular variables (84 sectors), orders
eps^-4..eps^0, two factors (U, F).  Its final pass runs the grouped instances
that evaluate every term once by singular support (the 4-singular-variable
family).  Every sector's per-shift means are compared with the oracle on the
same points, for each points-per-thread variant, at tile sizes that split a
shift into several tiles and leave threads without points in the last round;
the per-point values of the deepest sectors are compared through sdi_evaluate.

Bar per (sector, shift, order) mean: 1e-10 relative to max(|oracle|, mean |w F|),
or, where larger, the rounding bound 4e-15 mean(w cond) of the subtraction
sums (cond = sum of |terms|, from the oracle): near the faces the corner
differences of the four-fold subtraction cancel digits that fp64 cannot hold,
on either side (the endpoint-precision mode is the remedy).  The test reports
how many means needed the bound.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1511_03614_amd as P  # noqa: E402
from sectorgen.feynman import double_box_problem  # noqa: E402

from test_gpu_limits import oracle_shift_values_cond  # noqa: E402
from test_gpu_parity import REL_INT, log, pointwise_check, set_params  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    c = P.sdi_ctx_create(0)
    yield c
    P.sdi_ctx_destroy(c)


@pytest.fixture(scope="module")
def problem():
    return double_box_problem(-3.0, -1.0, 0.0, order_max=0)


@pytest.fixture(scope="module")
def oracle_means(problem):
    m, R, seed = 10, 4, 3
    return {s: oracle_shift_values_cond(problem, s, m, R, seed) for s in range(len(problem.sectors))}


def test_problem_shape(problem):
    ns = [int(np.sum(s.a == -1.0)) for s in problem.sectors]
    assert len(problem.sectors) == 282 and max(ns) == 4 and ns.count(4) == 84
    assert all(len(s.factors) == 2 and s.n == 6 for s in problem.sectors)


@pytest.mark.parametrize("ppt,tile_log2", [(1, 8), (2, 10), (0, 0)])
def test_all_sectors_against_oracle(ctx, problem, oracle_means, ppt, tile_log2):
    m, R, seed = 10, 4, 3
    log(f"doublebox parity ppt={ppt} tile_log2={tile_log2}")
    set_params(ctx, lattice_log2=m, shifts=R, seed=seed, ppt=ppt, tile_log2=tile_log2)
    h = P.sdi_problem_create(ctx, problem)
    try:
        res = P.sdi_integrate(ctx, h)
        assert res["n_nonfinite"] == 0
        widened, worst = 0, 0.0
        for s in range(len(problem.sectors)):
            _, _, per, nev = P.sdi_sector_results(ctx, h, s, R)
            assert nev == R << m
            oq, scale, bound = oracle_means[s]
            strict = REL_INT * np.maximum(np.abs(oq), scale[None, :])
            tol = np.maximum(strict, bound)
            d = np.abs(per - oq)
            assert (d <= tol).all(), (s, float(np.max(d / tol)))
            widened += int((bound > strict).sum())
            worst = max(worst, float(np.max(d / strict)))
        log(f"  ppt {res['ppt']} waves {res['waves_per_simd']} tile 2^{res['tile_log2']}: "
            f"{res['ms_eval_kernel']:.3f} ms; {widened} of {282 * R * 5} means need the rounding bound; "
            f"largest error {worst:.2e} of the 1e-10 bar")
    finally:
        P.sdi_problem_destroy(h)
        set_params(ctx)


def test_deepest_sectors_pointwise(ctx, problem):
    deep = [s for s, sec in enumerate(problem.sectors) if int(np.sum(sec.a == -1.0)) == 4][:6]
    rng = np.random.default_rng(11)
    for s in deep:
        x = rng.uniform(1e-3, 1.0, size=(512, 6))
        ok, strict = pointwise_check(ctx, problem, s, x)
        assert ok.all(), (s, int((~ok).sum()))
        assert strict.mean() > 0.95
