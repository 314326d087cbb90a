"""Endpoint precision (the small_x parameter): points whose smallest singular
coordinate lies below small_x are evaluated in double-double, and are checked
against the multiprecision oracle (oracle/integrand_mp.py) at the largest
accepted shapes (real: 16 variables, 4 singular, 4 factors, 8 orders;
complex: 8 deformed variables, 4 singular, 8 orders), where the fp64
subtraction cancels most digits near the faces; on lattice points and on the
explicit points of a learned sampler.

Bars: per point |gpu - exact| <= 1e-12 |exact| + 16 u foldabs + 1e-28 cond,
u = 2^-53, foldabs = sum of |c_s Pi_i f| over the fold of the per-order values
(rounded to fp64 before the fp64 fold), cond = sum of |subtraction terms|
(double-double leaves about 2^-104 of it); shift means at the 1e-10 bar with
no rounding-bound widening.  Points above the threshold give the fp64 values
bit for bit."""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1511_03614_amd as P  # noqa: E402
from oracle import integrand_mp, integrate, points  # noqa: E402

from test_gpu_limits import max_complex_problem, max_real_problem  # noqa: E402
from test_gpu_parity import REL_INT, log, set_params  # noqa: E402

U = 2.0 ** -53


@pytest.fixture(scope="module")
def ctx():
    c = P.sdi_ctx_create(0)
    yield c
    P.sdi_ctx_destroy(c)


def evaluate(ctx, h, s, x, small_x):
    P.sdi_set_param(ctx, "small_x", small_x)
    try:
        g = P.sdi_evaluate(ctx, h, s, torch.from_numpy(x).cuda()).cpu().numpy()
    finally:
        P.sdi_set_param(ctx, "small_x", 0)
    return g[..., 0].T + 1j * g[..., 1].T


def test_small_x_parameter(ctx):
    assert float(P.sdi_get_param(ctx, "small_x")) == 0.0
    P.sdi_set_param(ctx, "small_x", 1e-3)
    assert float(P.sdi_get_param(ctx, "small_x")) == 1e-3
    for bad in (-1e-3, 1.5, "nan", "x"):
        with pytest.raises(P.SdiError):
            P.sdi_set_param(ctx, "small_x", bad)
    assert float(P.sdi_get_param(ctx, "small_x")) == 1e-3
    P.sdi_set_param(ctx, "small_x", 0)


def test_pointwise_near_faces(ctx):
    prob = max_real_problem()
    lead, pref = integrate.prefactor_for(prob)
    rng = np.random.default_rng(41)
    h = P.sdi_problem_create(ctx, prob)
    try:
        for s, sec in enumerate(prob.sectors):
            x = rng.uniform(0.02, 1.0, size=(48, sec.n))
            x[:, :4] = 10.0 ** rng.uniform(-12, -2.5, size=(48, 4))
            x[:8, 1:4] = rng.uniform(0.02, 1.0, size=(8, 3))       # one singular coordinate near its face
            vals, cond, fabs_ = integrand_mp.sector_orders_mp(sec, x, prob.order_min, prob.order_max, lead, pref)
            gdd = evaluate(ctx, h, s, x, 0.01)
            g64 = evaluate(ctx, h, s, x, 0)
            tol = 1e-12 * np.abs(vals) + 16 * U * fabs_ + 1e-28 * cond
            d = np.abs(gdd - vals)
            assert (d <= tol).all(), f"sector {s}: {np.argwhere(d > tol)[:5]} max d/tol {np.max(d / tol)}"
            ok64 = (np.abs(g64 - vals) <= tol).mean()
            log(f"near faces, sector {s}: double-double max |d|/bar {np.max(d / tol):.2e}; fp64 meets the bar "
                f"at {ok64:.3f} of (point, order) pairs")
            # above the threshold the fp64 path runs unchanged
            xi = rng.uniform(0.02, 1.0, size=(64, sec.n))
            assert np.array_equal(evaluate(ctx, h, s, xi, 0.01), evaluate(ctx, h, s, xi, 0))
    finally:
        P.sdi_problem_destroy(h)


def mp_shift_means(prob, s, m, R, seed, small_x=1.0):
    """Exact shift means, mean |wF| per order, and the fp64 rounding bound
    4e-15 mean(w cond) of the points left in fp64 (smallest singular coordinate
    at or above small_x)."""
    lead, pref = integrate.prefactor_for(prob)
    sec = prob.sectors[s]
    sing = sec.a == -1.0
    z = points.cbc_vector(m, sec.n)
    sh = points.shift_table(seed, s, R, sec.n, m)
    N = 1 << m
    q = np.zeros((R, prob.norders), dtype=complex)
    scale = np.zeros(prob.norders)
    bound = np.zeros((R, prob.norders))
    for r in range(R):
        x, w, _ = points.sector_points(z, m, sh[r], 0, N, None, True)
        vals, cond, _ = integrand_mp.sector_orders_mp(sec, x, prob.order_min, prob.order_max, lead, pref,
                                                      complex_mode=prob.complex_mode, lam=prob.lam)
        # sectors without singular variables have nothing to cancel and stay in fp64
        fp64 = x[:, sing].min(axis=1) >= small_x if sing.any() else np.ones(x.shape[0], dtype=bool)
        wf = vals * w[None, :]
        for k in range(prob.norders):
            q[r, k] = integrate.fsum_c(wf[k]) / N
            scale[k] = max(scale[k], float(np.mean(np.abs(wf[k]))))
            bound[r, k] = 4e-15 * float(np.sum(cond[k] * w * fp64)) / N
    return q, scale, bound


def test_integrate_double_double_at_maximum_shapes(ctx):
    """small_x = 1: every point of every (singular) sector in double-double; the
    shift means meet the 1e-10 bar against the exact means with no widening."""
    prob = max_real_problem()
    m, R, seed = 6, 2, 5
    set_params(ctx, lattice_log2=m, shifts=R, seed=seed, tile_log2=0)
    h = P.sdi_problem_create(ctx, prob)
    try:
        P.sdi_set_param(ctx, "small_x", 1)
        res = P.sdi_integrate(ctx, h)
        assert res["ppt"] == 1 and res["waves_per_simd"] == 2 and res["n_nonfinite"] == 0
        per_dd = [P.sdi_sector_results(ctx, h, s, R)[2] for s in range(len(prob.sectors))]
        P.sdi_set_param(ctx, "small_x", 0)
        P.sdi_integrate(ctx, h)
        per_64 = [P.sdi_sector_results(ctx, h, s, R)[2] for s in range(len(prob.sectors))]
        miss64 = 0
        for s in range(len(prob.sectors)):
            q, scale, bound = mp_shift_means(prob, s, m, R, seed)
            assert not bound.any()
            tol = REL_INT * np.maximum(np.abs(q), scale[None, :])
            d = np.abs(per_dd[s] - q)
            assert (d <= tol).all(), f"sector {s}: max d/tol {np.max(d / tol)}"
            miss64 += int((np.abs(per_64[s] - q) > tol).sum())
        log(f"max shapes, shift means: double-double all within 1e-10; fp64 misses {miss64} of "
            f"{len(prob.sectors) * R * prob.norders}")
    finally:
        P.sdi_set_param(ctx, "small_x", 0)
        P.sdi_problem_destroy(h)
        set_params(ctx)


def test_threshold_mixes_paths(ctx):
    """A threshold between the faces and the interior: the final pass combines
    double-double and fp64 points and still meets the bar."""
    prob = max_real_problem()
    m, R, seed = 6, 2, 8
    set_params(ctx, lattice_log2=m, shifts=R, seed=seed, tile_log2=0)
    h = P.sdi_problem_create(ctx, prob)
    try:
        P.sdi_set_param(ctx, "small_x", 0.05)
        P.sdi_integrate(ctx, h)
        for s in range(len(prob.sectors)):
            per = P.sdi_sector_results(ctx, h, s, R)[2]
            q, scale, bound = mp_shift_means(prob, s, m, R, seed, small_x=0.05)
            d = np.abs(per - q)
            # the points above the threshold keep their fp64 rounding bound
            tol = np.maximum(REL_INT * np.maximum(np.abs(q), scale[None, :]), bound)
            assert (d <= tol).all(), f"sector {s}: max d/tol {np.max(d / tol)}"
    finally:
        P.sdi_set_param(ctx, "small_x", 0)
        P.sdi_problem_destroy(h)
        set_params(ctx)
    assert math.isfinite(float(P.sdi_get_param(ctx, "small_x")))


def test_two_singular_variables_keep_the_tuned_variants(ctx):
    """Problems whose sectors have at most two singular variables keep the tuned
    launch variants, in their double-double-capable copies: with every point in
    double-double the shift means meet the 1e-10 bar against the exact means."""
    import sectorgen
    full = sectorgen.config2()
    prob = sectorgen.Problem(sectors=full.sectors[:6], order_min=full.order_min, order_max=full.order_max,
                             pref_lead=full.pref_lead, pref=full.pref)
    m, R, seed = 6, 2, 4
    set_params(ctx, lattice_log2=m, shifts=R, seed=seed, tile_log2=0)
    h = P.sdi_problem_create(ctx, prob)
    try:
        P.sdi_set_param(ctx, "small_x", 1)
        res = P.sdi_integrate(ctx, h)
        assert 10 * res["ppt"] + res["waves_per_simd"] in (14, 23, 24, 42)
        for s in range(len(prob.sectors)):
            per = P.sdi_sector_results(ctx, h, s, R)[2]
            q, scale, bound = mp_shift_means(prob, s, m, R, seed)
            assert not bound.any() or not (prob.sectors[s].a == -1.0).any()
            tol = np.maximum(REL_INT * np.maximum(np.abs(q), scale[None, :]), bound)
            d = np.abs(per - q)
            assert (d <= tol).all(), f"sector {s}: max d/tol {np.max(d / tol)}"
    finally:
        P.sdi_set_param(ctx, "small_x", 0)
        P.sdi_problem_destroy(h)
        set_params(ctx)


@pytest.mark.parametrize("ppt", [2, 4])
def test_queue_carries_points_across_rounds(ctx, ppt):
    """With 2 or 4 points per thread and a threshold that flags a large share
    of the points, a wave queues more than 64 flagged points in one round: 64
    are evaluated in double-double and the rest carried to the next flush.  A
    point dropped or counted twice would move a shift mean by about |w F| / N;
    every shift mean must stay within the fp64 rounding bound of the oracle's,
    and the evaluation count is unchanged."""
    import sectorgen
    from test_gpu_limits import oracle_shift_values_cond
    full = sectorgen.config2()
    prob = sectorgen.Problem(sectors=full.sectors[:6], order_min=full.order_min, order_max=full.order_max,
                             pref_lead=full.pref_lead, pref=full.pref)
    m, R, seed = 10, 2, 9
    set_params(ctx, lattice_log2=m, shifts=R, seed=seed, tile_log2=10, ppt=ppt)
    h = P.sdi_problem_create(ctx, prob)
    try:
        base = P.sdi_integrate(ctx, h)
        P.sdi_set_param(ctx, "small_x", 0.3)
        res = P.sdi_integrate(ctx, h)
        assert res["ppt"] == ppt and res["n_evals"] == base["n_evals"]
        for s in range(len(prob.sectors)):
            per = P.sdi_sector_results(ctx, h, s, R)[2]
            q, scale, bound = oracle_shift_values_cond(prob, s, m, R, seed)
            tol = np.maximum(REL_INT * np.maximum(np.abs(q), scale[None, :]), bound)
            d = np.abs(per - q)
            assert (d <= tol).all(), f"sector {s}: max d/tol {np.max(d / tol)}"
    finally:
        P.sdi_set_param(ctx, "small_x", 0)
        P.sdi_problem_destroy(h)
        set_params(ctx)


# ---------------------------------------------------------------- complex mode

def test_complex_pointwise_near_faces(ctx):
    prob = max_complex_problem()
    lead, pref = integrate.prefactor_for(prob)
    rng = np.random.default_rng(43)
    h = P.sdi_problem_create(ctx, prob)
    try:
        for s, sec in enumerate(prob.sectors):
            x = rng.uniform(0.02, 1.0, size=(24, sec.n))
            x[:, :4] = 10.0 ** rng.uniform(-12, -2.5, size=(24, 4))
            x[:6, 1:4] = rng.uniform(0.02, 1.0, size=(6, 3))        # one singular coordinate near its face
            vals, cond, fabs_ = integrand_mp.sector_orders_mp(sec, x, prob.order_min, prob.order_max, lead, pref,
                                                              complex_mode=True, lam=prob.lam)
            gdd = evaluate(ctx, h, s, x, 0.01)
            g64 = evaluate(ctx, h, s, x, 0)
            tol = 1e-12 * np.abs(vals) + 16 * U * fabs_ + 1e-28 * cond
            d = np.abs(gdd - vals)
            assert (d <= tol).all(), f"sector {s}: {np.argwhere(d > tol)[:5]} max d/tol {np.max(d / tol)}"
            ok64 = (np.abs(g64 - vals) <= tol).mean()
            log(f"complex, near faces, sector {s}: double-double max |d|/bar {np.max(d / tol):.2e}; fp64 meets "
                f"the bar at {ok64:.3f} of (point, order) pairs")
            xi = rng.uniform(0.02, 1.0, size=(64, sec.n))
            assert np.array_equal(evaluate(ctx, h, s, xi, 0.01), evaluate(ctx, h, s, xi, 0))
    finally:
        P.sdi_problem_destroy(h)


def test_complex_integrate_double_double_at_maximum_shapes(ctx):
    """small_x = 1: every point in double-double, the shift means meet the 1e-10
    bar against the exact means with no widening; small_x = 0.05 mixes both
    paths (the fp64 points keep their rounding bound); the Im F > 0 count and
    the evaluation count do not change."""
    prob = max_complex_problem()
    m, R, seed = 5, 2, 5
    set_params(ctx, lattice_log2=m, shifts=R, seed=seed, tile_log2=0)
    h = P.sdi_problem_create(ctx, prob)
    try:
        base = P.sdi_integrate(ctx, h)
        per_64 = [P.sdi_sector_results(ctx, h, s, R)[2] for s in range(len(prob.sectors))]
        P.sdi_set_param(ctx, "small_x", 1)
        res = P.sdi_integrate(ctx, h)
        assert res["ppt"] == 1 and res["n_nonfinite"] == 0
        assert res["n_evals"] == base["n_evals"] and res["n_imf_positive"] == base["n_imf_positive"]
        per_dd = [P.sdi_sector_results(ctx, h, s, R)[2] for s in range(len(prob.sectors))]
        P.sdi_set_param(ctx, "small_x", 0.05)
        P.sdi_integrate(ctx, h)
        per_mix = [P.sdi_sector_results(ctx, h, s, R)[2] for s in range(len(prob.sectors))]
        miss64 = 0
        for s in range(len(prob.sectors)):
            q, scale, bound = mp_shift_means(prob, s, m, R, seed, small_x=0.05)
            strict = REL_INT * np.maximum(np.abs(q), scale[None, :])
            d = np.abs(per_dd[s] - q)
            assert (d <= strict).all(), f"sector {s}: max d/tol {np.max(d / strict)}"
            dm = np.abs(per_mix[s] - q)
            assert (dm <= np.maximum(strict, bound)).all(), f"sector {s} mixed: max d/tol {np.max(dm / strict)}"
            miss64 += int((np.abs(per_64[s] - q) > strict).sum())
        log(f"complex max shapes, shift means: double-double all within 1e-10; fp64 misses {miss64} of "
            f"{len(prob.sectors) * R * prob.norders}")
    finally:
        P.sdi_set_param(ctx, "small_x", 0)
        P.sdi_problem_destroy(h)
        set_params(ctx)


@pytest.mark.parametrize("which", ["real16", "complex8"])
def test_flow_sampled_points_in_double_double(ctx, which):
    """A pass with the learned sampler and small_x = 1: every explicit point of
    every flow-sampled sector in double-double; per (sector, shift) means equal
    the exact means at the flow's points (taken from the library's own sampler,
    whose map is checked against the flow oracle elsewhere) at the 1e-10 bar
    with no widening."""
    from test_gpu_flow import random_fp32_params
    prob = max_real_problem() if which == "real16" else max_complex_problem()
    if which == "real16":
        prob.sectors = prob.sectors[:2]
    m, R, seed = 5, 2, 7
    lead, pref = integrate.prefactor_for(prob)
    set_params(ctx, lattice_log2=m, shifts=R, seed=seed, sampler=1)
    h = P.sdi_problem_create(ctx, prob)
    try:
        P.sdi_flow_init(ctx, h, 3)
        for s, sec in enumerate(prob.sectors):
            P.sdi_flow_set_params(ctx, h, s, random_fp32_params(sec.n, 60 + s))
        P.sdi_set_param(ctx, "small_x", 1)
        res = P.sdi_integrate(ctx, h)
        assert res["status"] == 0 and res["n_nonfinite"] == 0
        worst = 0.0
        for s, sec in enumerate(prob.sectors):
            per = P.sdi_sector_results(ctx, h, s, R)[2]
            z = points.cbc_vector(m, sec.n)
            sh = points.shift_table(seed, s, R, sec.n, m)
            for r in range(R):
                u, _, _ = points.sector_points(z, m, sh[r], 0, 1 << m, None, True)
                x, lq = P.sdi_flow_sample(ctx, h, s, torch.from_numpy(u).cuda())
                x, w = x.cpu().numpy(), np.exp(-lq.cpu().numpy())
                vals, _, _ = integrand_mp.sector_orders_mp(sec, x, prob.order_min, prob.order_max, lead, pref,
                                                           complex_mode=prob.complex_mode, lam=prob.lam)
                wf = vals * w[None, :]
                for k in range(prob.norders):
                    q = integrate.fsum_c(wf[k]) / (1 << m)
                    tol = REL_INT * max(abs(q), float(np.mean(np.abs(wf[k]))))
                    assert abs(per[r, k] - q) <= tol, (s, r, k, abs(per[r, k] - q) / tol)
                    worst = max(worst, abs(per[r, k] - q) / tol)
        log(f"{which}: flow-sampled points in double-double, max |d|/bar {worst:.2e}")
    finally:
        P.sdi_set_param(ctx, "small_x", 0)
        P.sdi_problem_destroy(h)
        set_params(ctx)
