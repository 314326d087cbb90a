"""Real-mode factor exponents up to 7 (the x^4 bit of the term words): random
sectors with exponents 0..7 against the oracle on the same points - through
sdi_integrate's grouped final pass (two factors), its per-corner-list pass
(three factors), sdi_evaluate and the double-double endpoint pass - and the
limits of problem creation (8 rejected in real mode, 4 in complex mode)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1511_03614_amd as P  # noqa: E402
import sectorgen  # noqa: E402
from sectorgen import Factor, Problem, Sector, SplitMix64, _random_poly  # noqa: E402

from test_gpu_limits import oracle_shift_values_cond  # noqa: E402
from test_gpu_parity import REL_INT, log, pointwise_check, set_params  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    c = P.sdi_ctx_create(0)
    yield c
    P.sdi_ctx_destroy(c)


def high_exponent_problem(nfac: int, seed: int = 71) -> Problem:
    rng = SplitMix64(seed)
    secs = []
    for i in range(6):
        n = 3 + i % 3
        a = np.zeros(n)
        b = np.array([float(rng.randint(-2, 2)) for _ in range(n)])
        for j in range(min(i % 4, n)):
            a[j] = -1.0
            b[j] = float(rng.choice([-2, -1, 1, 2]))
        facs = []
        for m in range(nfac):
            coef, exps = _random_poly(rng, n, rng.randint(4, 10), emax=7)
            facs.append(Factor(float(rng.choice([-2, -1, 1])), float(rng.choice([-1, 1, 2])), coef, exps))
        secs.append(Sector(a=a, b=b, factors=facs))
    return Problem(sectors=secs, order_min=-2, order_max=0)


@pytest.mark.parametrize("nfac", [2, 3])
def test_integrate_high_exponents(ctx, nfac):
    prob = high_exponent_problem(nfac)
    assert max(int(f.exps.max()) for s in prob.sectors for f in s.factors) == 7
    m, R, seed = 9, 3, 6
    set_params(ctx, lattice_log2=m, shifts=R, seed=seed, tile_log2=0)
    h = P.sdi_problem_create(ctx, prob)
    try:
        res = P.sdi_integrate(ctx, h)
        log(f"factors {nfac}: grouped {res['grouped']}, ppt {res['ppt']}, waves {res['waves_per_simd']}")
        if nfac == 3:
            assert res["grouped"] == 0
        for s in range(len(prob.sectors)):
            per = P.sdi_sector_results(ctx, h, s, R)[2]
            q, scale, bound = oracle_shift_values_cond(prob, s, m, R, seed)
            tol = np.maximum(REL_INT * np.maximum(np.abs(q), scale[None, :]), bound)
            assert (np.abs(per - q) <= tol).all(), (s, float(np.max(np.abs(per - q) / tol)))
        # every point in double-double: the same means within the fp64 rounding bound
        P.sdi_set_param(ctx, "small_x", 1)
        P.sdi_integrate(ctx, h)
        for s in range(len(prob.sectors)):
            per = P.sdi_sector_results(ctx, h, s, R)[2]
            q, scale, bound = oracle_shift_values_cond(prob, s, m, R, seed)
            tol = np.maximum(REL_INT * np.maximum(np.abs(q), scale[None, :]), bound)
            assert (np.abs(per - q) <= tol).all(), ("dd", s)
    finally:
        P.sdi_set_param(ctx, "small_x", 0)
        P.sdi_problem_destroy(h)
        set_params(ctx)


def test_evaluate_high_exponents(ctx):
    prob = high_exponent_problem(2, seed=72)
    rng = np.random.default_rng(5)
    for s in range(len(prob.sectors)):
        x = rng.uniform(1e-3, 1.0, size=(256, prob.sectors[s].n))
        ok, strict = pointwise_check(ctx, prob, s, x)
        assert ok.all() and strict.mean() > 0.95, s


def test_exponent_limits(ctx):
    base = high_exponent_problem(2)
    sec = base.sectors[0]
    bad = sec.factors[0].exps.copy()
    bad[1, 0] = 8
    f8 = Factor(sec.factors[0].gamma, sec.factors[0].delta, sec.factors[0].coef, bad)
    p8 = Problem(sectors=[Sector(a=sec.a, b=sec.b, factors=[f8, sec.factors[1]])], order_min=-2, order_max=0)
    with pytest.raises(P.SdiError) as e:
        P.sdi_problem_create(ctx, p8)
    assert e.value.code == -4
    e4 = sec.factors[0].exps.copy()
    e4[1, 0] = 4
    f4 = Factor(sec.factors[0].gamma, sec.factors[0].delta, sec.factors[0].coef, e4)
    ok = Problem(sectors=[Sector(a=sec.a, b=sec.b, factors=[f4, sec.factors[1]])], order_min=-2, order_max=0)
    P.sdi_problem_destroy(P.sdi_problem_create(ctx, ok))                  # 4 is fine in real mode
    c4 = Problem(sectors=[Sector(a=sec.a, b=sec.b, factors=[f4, sec.factors[1]], deform_factor=1)], order_min=-2,
                 order_max=0, complex_mode=True, lam=0.1)
    with pytest.raises(P.SdiError) as e:
        P.sdi_problem_create(ctx, c4)
    assert e.value.code == -4
