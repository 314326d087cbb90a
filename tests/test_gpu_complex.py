"""GPU parity of the complex (contour-deformed) path against the oracle.

Bars as in test_gpu_parity.py: per point |gpu - oracle| <= 1e-12 |oracle| +
4e-15 cond; per (sector, shift) mean <= 1e-10 max(|oracle|, mean |wF|).
"""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1511_03614_amd as P  # noqa: E402
import sectorgen  # noqa: E402
from sectorgen import Factor, Sector  # noqa: E402
from sectorgen.feynman import double_box_problem, massive_bubble_problem, box_problem  # noqa: E402
from oracle import integrand, integrate, points  # noqa: E402

from test_gpu_parity import assert_close_shift, log, set_params  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    c = P.sdi_ctx_create(0)
    yield c
    P.sdi_ctx_destroy(c)


def oracle_shift_values_c(problem, s, m, R, seed):
    lead, pref = integrate.prefactor_for(problem)
    sec = problem.sectors[s]
    z = points.cbc_vector(m, sec.n)
    sh = points.shift_table(seed, s, R, sec.n, m)
    N = 1 << m
    K = problem.norders
    q = np.zeros((R, K), dtype=complex)
    scale = np.zeros(K)
    npos = 0
    for r in range(R):
        x, w, _ = points.sector_points(z, m, sh[r], 0, N, None, True)
        vals, _, pos = integrand.sector_orders(sec, x, problem.order_min, problem.order_max, lead, pref,
                                               True, problem.lam)
        npos += int(pos.sum())
        wf = vals * w[None, :]
        for k in range(K):
            q[r, k] = integrate.fsum_c(wf[k]) / N
            scale[k] = max(scale[k], float(np.mean(np.abs(wf[k]))))
    return q, scale, npos


def pointwise_c(ctx, prob, s, x_np):
    h = P.sdi_problem_create(ctx, prob)
    try:
        g, gc = P.sdi_evaluate(ctx, h, s, torch.from_numpy(x_np).cuda(), with_cond=True)
        g, gc = g.cpu().numpy(), gc.cpu().numpy()
    finally:
        P.sdi_problem_destroy(h)
    lead, pref = integrate.prefactor_for(prob)
    vals, cond, _ = integrand.sector_orders(prob.sectors[s], x_np, prob.order_min, prob.order_max, lead, pref,
                                            True, prob.lam)
    gv = g[..., 0].T + 1j * g[..., 1].T
    np.testing.assert_allclose(gc.T, cond, rtol=1e-10, atol=0)
    d = np.abs(gv - vals)
    return d <= 1e-12 * np.abs(vals) + 4e-15 * cond, d <= 1e-12 * np.abs(vals)


def test_pointwise_massive_bubble_and_2d(ctx):
    rng = np.random.default_rng(8)
    prob = massive_bubble_problem(5.0, 1.0, 0.5)
    for s in range(len(prob.sectors)):
        ok, _ = pointwise_c(ctx, prob, s, rng.uniform(1e-7, 1.0, size=(2048, prob.sectors[s].n)))
        assert ok.all(), s
    sec = Sector(a=np.array([-1.0, 0.0]), b=np.array([1.0, -1.0]), factors=[
        Factor(1.0, 1.0, np.array([1.0, 1.0, 0.5]), np.array([[0, 0], [1, 0], [0, 1]], dtype=np.uint8)),
        Factor(-2.0, -1.0, np.array([1.0, -2.0, 1.0]), np.array([[0, 0], [0, 1], [1, 1]], dtype=np.uint8))],
        deform_factor=1, deform_mono=np.array([1, 0], np.int32))
    p2 = sectorgen.Problem(sectors=[sec], order_min=-1, order_max=1, complex_mode=True, lam=0.3)
    ok, strict = pointwise_c(ctx, p2, 0, rng.uniform(1e-6, 1.0, size=(4096, 2)))
    assert ok.all() and strict.mean() > 0.95


def test_pointwise_massive_double_box_sectors(ctx):
    """Physical-region double box (s=5, t=-2, m^2=1): six-variable deformed sectors."""
    prob = double_box_problem(5.0, -2.0, 1.0, order_max=0, complex_mode=True, lam=0.5)
    rng = np.random.default_rng(9)
    fr = []
    for s in range(0, len(prob.sectors), max(1, len(prob.sectors) // 12)):
        ok, strict = pointwise_c(ctx, prob, s, rng.uniform(1e-5, 1.0, size=(512, prob.sectors[s].n)))
        assert ok.all(), s
        fr.append(strict.mean())
    assert min(fr) > 0.9


def test_integrate_massive_bubble(ctx):
    prob = massive_bubble_problem(5.0, 1.0, 0.5)
    m, R = 12, 8
    set_params(ctx, lattice_log2=m, shifts=R, seed=3)
    h = P.sdi_problem_create(ctx, prob)
    try:
        res = P.sdi_integrate(ctx, h)
        assert res["status"] == 0 and res["n_imf_positive"] == 0
        for s in range(len(prob.sectors)):
            _, _, per, _ = P.sdi_sector_results(ctx, h, s, R)
            oq, scale, npos = oracle_shift_values_c(prob, s, m, R, 3)
            assert npos == 0
            assert_close_shift(per, oq, scale, f"massive bubble sector {s}")
    finally:
        P.sdi_problem_destroy(h)
    beta = math.sqrt(1 - 4 / 5.0)
    fin = 2 - beta * math.log((1 + beta) / (1 - beta)) + 1j * math.pi * beta
    v = res["value"]
    assert abs(v[0].real - 1.0) < 6 * res["err_re"][0] + 1e-12
    assert abs(v[0].imag) < 6 * res["err_im"][0] + 1e-12
    assert abs(v[1].real - fin.real) < 6 * res["err_re"][1] + 1e-9
    assert abs(v[1].imag - fin.imag) < 6 * res["err_im"][1] + 1e-9


def test_lambda_zero_complex_equals_real(ctx):
    real = box_problem(3.0, 1.0)
    cplx = box_problem(3.0, 1.0)
    cplx.complex_mode, cplx.lam = True, 0.0
    set_params(ctx, lattice_log2=10, shifts=4, seed=6)
    out = []
    for prob in (real, cplx):
        h = P.sdi_problem_create(ctx, prob)
        try:
            out.append(P.sdi_integrate(ctx, h))
        finally:
            P.sdi_problem_destroy(h)
    assert np.allclose(out[0]["value"].real, out[1]["value"].real, rtol=1e-12, atol=1e-13)
    assert np.all(np.abs(out[1]["value"].imag) < 1e-13)


def test_integrate_massive_double_box_subset(ctx):
    prob = double_box_problem(5.0, -2.0, 1.0, order_max=0, complex_mode=True, lam=0.5)
    idx = list(range(0, len(prob.sectors), max(1, len(prob.sectors) // 6)))[:6]
    prob.sectors = [prob.sectors[i] for i in idx]
    m, R = 9, 2
    set_params(ctx, lattice_log2=m, shifts=R, seed=12)
    h = P.sdi_problem_create(ctx, prob)
    try:
        res = P.sdi_integrate(ctx, h)
        tot_pos = 0
        for s in range(len(prob.sectors)):
            _, _, per, _ = P.sdi_sector_results(ctx, h, s, R)
            oq, scale, npos = oracle_shift_values_c(prob, s, m, R, 12)
            tot_pos += npos
            assert_close_shift(per, oq, scale, f"double box sector {s}")
        assert res["n_imf_positive"] == tot_pos
    finally:
        P.sdi_problem_destroy(h)


def test_tuned_lambda_matches_oracle(ctx):
    """The GPU deformation-size search picks exactly the oracle's candidate per sector."""
    from oracle import deform
    set_params(ctx, seed=5)
    for prob in (double_box_problem(5.0, -2.0, 1.0, order_max=0, complex_mode=True, lam=0.5),
                 massive_bubble_problem(5.0, 1.0, 0.5)):
        h = P.sdi_problem_create(ctx, prob)
        try:
            for split, m, cons in ((4, 10, False), (3, 8, True)):
                lam = P.sdi_tune_deformation(ctx, h, 0.5, split, m, cons)
                olam = [deform.tune_lambda(sec, s, 0.5, split, m, 5, cons) for s, sec in enumerate(prob.sectors)]
                assert list(lam) == olam, (prob.name, split, m)
        finally:
            P.sdi_problem_destroy(h)


def test_integrate_with_tuned_lambda_matches_oracle(ctx):
    """After tuning, the deformed pass reproduces the oracle at each sector's own lambda."""
    prob = double_box_problem(5.0, -2.0, 1.0, order_max=0, complex_mode=True, lam=0.5)
    idx = [0, 5, 12, 24]
    prob.sectors = [prob.sectors[i] for i in idx]
    m, R = 9, 2
    set_params(ctx, lattice_log2=m, shifts=R, seed=12)
    h = P.sdi_problem_create(ctx, prob)
    try:
        lam = P.sdi_tune_deformation(ctx, h, 0.5, 4, 10)
        assert np.all(lam < 0.5) and np.all(lam > 0.0)
        res = P.sdi_integrate(ctx, h)
        tot_pos = 0
        for s in range(len(prob.sectors)):
            _, _, per, _ = P.sdi_sector_results(ctx, h, s, R)
            one = sectorgen.Problem(sectors=[prob.sectors[s]], order_min=prob.order_min, order_max=prob.order_max,
                                    feynman=prob.feynman, complex_mode=True, lam=float(lam[s]))
            oq, scale, npos = oracle_shift_values_c_sector(one, prob.sectors[s], s, m, R, 12)
            tot_pos += npos
            assert_close_shift(per, oq, scale, f"tuned double box sector {s}")
        assert res["n_imf_positive"] == tot_pos
    finally:
        P.sdi_problem_destroy(h)


def oracle_shift_values_c_sector(one, sec, s, m, R, seed):
    """oracle_shift_values_c for sector index s of a larger problem (its shifts are keyed by s)."""
    lead, pref = integrate.prefactor_for(one)
    z = points.cbc_vector(m, sec.n)
    sh = points.shift_table(seed, s, R, sec.n, m)
    N = 1 << m
    K = one.norders
    q = np.zeros((R, K), dtype=complex)
    scale = np.zeros(K)
    npos = 0
    for r in range(R):
        x, w, _ = points.sector_points(z, m, sh[r], 0, N, None, True)
        vals, _, pos = integrand.sector_orders(sec, x, one.order_min, one.order_max, lead, pref, True, one.lam)
        npos += int(pos.sum())
        wf = vals * w[None, :]
        for k in range(K):
            q[r, k] = integrate.fsum_c(wf[k]) / N
            scale[k] = max(scale[k], float(np.mean(np.abs(wf[k]))))
    return q, scale, npos


def test_physical_double_box_lambda_invariance(ctx):
    """Cauchy's theorem on the physical double box (s = 5, t = -2, all internal
    masses 1): the eps^0 coefficient with the tuned deformation and with the
    conservative (halved) one agree within 5 combined standard errors, real and
    imaginary parts; the conservative deformation leaves no point with
    Im F(z) > 0 in the pass."""
    from sectorgen.feynman import double_box_problem
    prob = double_box_problem(5.0, -2.0, 1.0, order_max=0, complex_mode=True, lam=0.5)
    set_params(ctx, lattice_log2=14, shifts=16, seed=5, tile_log2=0)
    h = P.sdi_problem_create(ctx, prob)
    try:
        P.sdi_tune_deformation(ctx, h, 0.5, 4, 10)
        a = P.sdi_integrate(ctx, h)
        P.sdi_tune_deformation(ctx, h, 0.5, 4, 10, conservative=True)
        b = P.sdi_integrate(ctx, h)
        log(f"physical double box eps^0: tuned {a['value'][-1]:.6f} +- {a['err_re'][-1]:.1e}/{a['err_im'][-1]:.1e} "
            f"({a['n_imf_positive']} points Im F > 0), conservative {b['value'][-1]:.6f} "
            f"+- {b['err_re'][-1]:.1e}/{b['err_im'][-1]:.1e} ({b['n_imf_positive']})")
        assert b["n_imf_positive"] == 0
        for part, ea, eb in ((np.real, a["err_re"], b["err_re"]), (np.imag, a["err_im"], b["err_im"])):
            d = abs(part(a["value"][-1]) - part(b["value"][-1]))
            assert d <= 5 * np.hypot(ea[-1], eb[-1]), (d, ea[-1], eb[-1])
    finally:
        P.sdi_problem_destroy(h)
        set_params(ctx)


# ---------------------------------------------------------------- complex term coefficients

def complex_coef_max_problem():
    """The 8-variable complex shape with complex coefficients in the positive factor
    (imaginary parts of either sign, so the factor's values leave the real axis)."""
    from shapes import max_complex_problem
    prob = max_complex_problem()
    rng = np.random.default_rng(77)
    for sec in prob.sectors:
        G = sec.factors[2]
        sec.factors[2] = Factor(G.gamma, G.delta, G.coef + 0.3j * rng.uniform(-1, 1, size=G.coef.size), G.exps)
    return prob


@pytest.mark.parametrize("lam", [0.0, 0.3])
def test_complex_mass_bubble(ctx, lam):
    """Complex mass m^2 = 1 - i/4: per point and per shift against the oracle, and
    the eps^0 coefficient against -int_0^1 ln(m^2 - s x(1-x)) dx within 5 sigma."""
    import mpmath
    from sectorgen.feynman import complex_mass_bubble_problem
    prob = complex_mass_bubble_problem(5.0, 1.0 - 0.25j, lam)
    rng = np.random.default_rng(12)
    for s in range(len(prob.sectors)):
        ok, strict = pointwise_c(ctx, prob, s, rng.uniform(1e-7, 1.0, size=(2048, 1)))
        assert ok.all() and strict.mean() > 0.99, s
    m, R = 12, 8
    set_params(ctx, lattice_log2=m, shifts=R, seed=3)
    h = P.sdi_problem_create(ctx, prob)
    try:
        res = P.sdi_integrate(ctx, h)
        assert res["status"] == 0 and res["n_imf_positive"] == 0
        for s in range(len(prob.sectors)):
            per = P.sdi_sector_results(ctx, h, s, R)[2]
            oq, scale, npos = oracle_shift_values_c(prob, s, m, R, 3)
            assert npos == 0
            assert_close_shift(per, oq, scale, f"complex-mass bubble sector {s}")
    finally:
        P.sdi_problem_destroy(h)
        set_params(ctx)
    with mpmath.workdps(30):
        ref = complex(-mpmath.quad(lambda x: mpmath.log(mpmath.mpc(1, -0.25) - 5 * x * (1 - x)), [0, 0.5, 1]))
    v = res["value"]
    assert abs(v[0].real - 1.0) < 5 * res["err_re"][0] + 1e-12 and abs(v[0].imag) < 5 * res["err_im"][0] + 1e-12
    assert abs(v[1].real - ref.real) < 5 * res["err_re"][1] + 1e-9
    assert abs(v[1].imag - ref.imag) < 5 * res["err_im"][1] + 1e-9
    log(f"complex-mass bubble, lambda {lam}: eps^0 {v[1]:.10f} vs {ref:.10f}")


def test_complex_coefficients_at_the_largest_shape(ctx):
    """8 variables, 4 singular, complex coefficients in one factor: per point and per
    (sector, shift) mean against the oracle (the widening by the rounding bound
    as in test_gpu_limits.py)."""
    from test_gpu_limits import oracle_shift_values_cond, pointwise
    from test_gpu_parity import REL_INT
    prob = complex_coef_max_problem()
    rng = np.random.default_rng(19)
    for s, sec in enumerate(prob.sectors):
        x = rng.uniform(1e-6, 1.0, size=(512, sec.n))
        ok, strict = pointwise(ctx, prob, s, x)
        assert ok.all(), f"sector {s}: {np.argwhere(~ok)[:5]}"
    m, R, seed = 10, 4, 5
    set_params(ctx, lattice_log2=m, shifts=R, seed=seed, tile_log2=0)
    h = P.sdi_problem_create(ctx, prob)
    try:
        P.sdi_integrate(ctx, h)
        for s in range(len(prob.sectors)):
            per = P.sdi_sector_results(ctx, h, s, R)[2]
            oq, scale, bound = oracle_shift_values_cond(prob, s, m, R, seed)
            tol = np.maximum(REL_INT * np.maximum(np.abs(oq), scale[None, :]), bound)
            d = np.abs(per - oq)
            assert (d <= tol).all(), f"sector {s}: max d/tol {np.max(d / tol)}"
    finally:
        P.sdi_problem_destroy(h)
        set_params(ctx)


def test_complex_coefficients_need_complex_mode(ctx):
    from sectorgen.feynman import complex_mass_bubble_problem
    prob = complex_mass_bubble_problem()
    prob.complex_mode = False
    with pytest.raises(P.SdiError) as e:
        h = P.sdi_problem_create(ctx, prob)
        P.sdi_problem_destroy(h)
    assert e.value.code == -1
