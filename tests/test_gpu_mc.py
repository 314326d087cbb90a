"""The Monte Carlo integrator (integrator 2): pseudo-random points from
Philox4x32-10 in place of the lattice, the sampling of the paper's default
final integrator (vegasCuba, section 4.4).

* The points are bit-identical to the oracle's (oracle/points.py mc_u), so
  per (sector, shift) means meet the 1e-10 bar against the oracle on the same
  points, in real and in complex mode.
* With a Vegas warm-up, the bubble's closed form within 5 standard errors.
* The error estimate (R independent samples) is calibrated: over 24 seeds
  the bubble's z-scores have mean square within [0.4, 2.5] and at least 80 %
  of them lie within 2.
* Refused with the flow sampler, text integrands and slices."""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1511_03614_amd as P  # noqa: E402
import sectorgen  # noqa: E402
from sectorgen import textgen  # noqa: E402
from sectorgen.feynman import massive_bubble_problem  # noqa: E402
from oracle import integrand, integrate, points  # noqa: E402

from test_gpu_parity import assert_close_shift, log, set_params  # noqa: E402

BUBBLE = [1.0, 2.0, 4.0 - math.pi ** 2 / 12.0]


@pytest.fixture(scope="module")
def ctx():
    c = P.sdi_ctx_create(0)
    yield c
    P.sdi_ctx_destroy(c)


def oracle_mc_shifts(prob, s, m, R, seed):
    lead, pref = integrate.prefactor_for(prob)
    sec = prob.sectors[s]
    q = np.zeros((R, prob.norders), complex)
    scale = np.zeros(prob.norders)
    args = (True, prob.lam) if prob.complex_mode else ()
    for r in range(R):
        x, w = points.mc_points(seed, s, r, 0, 1 << m, sec.n)
        vals, _, _ = integrand.sector_orders(sec, x, prob.order_min, prob.order_max, lead, pref, *args)
        wf = vals * w[None, :]
        for k in range(prob.norders):
            q[r, k] = integrate.fsum_c(wf[k]) / (1 << m)
            scale[k] = max(scale[k], float(np.mean(np.abs(wf[k]))))
    return q, scale


@pytest.mark.parametrize("which", ["synthetic", "massive bubble (complex)", "16 variables"])
def test_points_and_shift_means_match_the_oracle(ctx, which):
    m, R, seed = 9, 4, 11
    if which == "synthetic":
        full = sectorgen.config2()
        prob = sectorgen.Problem(sectors=full.sectors[:4], order_min=full.order_min, order_max=full.order_max,
                                 pref_lead=full.pref_lead, pref=full.pref)
    elif which == "16 variables":
        from shapes import max_real_problem
        big = max_real_problem()
        prob = sectorgen.Problem(sectors=big.sectors[:2], order_min=big.order_min, order_max=big.order_max,
                                 pref_lead=big.pref_lead, pref=big.pref)
        m = 6
    else:
        prob = massive_bubble_problem(5.0, 1.0, 0.5)
    set_params(ctx, lattice_log2=m, shifts=R, seed=seed, tile_log2=0)
    P.sdi_set_param(ctx, "integrator", 2)
    h = P.sdi_problem_create(ctx, prob)
    try:
        res = P.sdi_integrate(ctx, h)
        assert res["status"] == 0 and res["n_nonfinite"] == 0
        for s in range(len(prob.sectors)):
            per, nev = P.sdi_sector_results(ctx, h, s, R)[2:4]
            assert nev == R << m
            q, scale = oracle_mc_shifts(prob, s, m, R, seed)
            assert_close_shift(per, q, scale, f"{which} sector {s}")
    finally:
        P.sdi_problem_destroy(h)
        P.sdi_set_param(ctx, "integrator", 0)
        set_params(ctx)


def run_bubble(ctx, seed, m=12, R=8, warmup=0):
    prob = sectorgen.bubble_problem(order_max=1)
    set_params(ctx, lattice_log2=m, shifts=R, seed=seed, warmup=warmup)
    P.sdi_set_param(ctx, "integrator", 2)
    h = P.sdi_problem_create(ctx, prob)
    try:
        return P.sdi_integrate(ctx, h)
    finally:
        P.sdi_problem_destroy(h)
        P.sdi_set_param(ctx, "integrator", 0)
        set_params(ctx)


def test_bubble_closed_form_with_vegas_warmup(ctx):
    res = run_bubble(ctx, 5, m=14, R=16, warmup=3)
    v, e = res["value"].real, res["err_re"]
    for k in range(3):
        assert abs(v[k] - BUBBLE[k]) <= 5 * e[k] + 1e-12, (k, v[k], BUBBLE[k], e[k])
    log(f"Monte Carlo bubble with warm-up: errors {e}")


def test_error_estimate_is_calibrated(ctx):
    z = []
    for seed in range(24):
        res = run_bubble(ctx, 100 + seed, m=10, R=8)
        z.append((res["value"][1].real - BUBBLE[1]) / res["err_re"][1])
    z = np.array(z)
    log(f"Monte Carlo z-scores over 24 seeds: mean square {np.mean(z ** 2):.2f}, |z| < 2 for {np.mean(np.abs(z) < 2):.2f}")
    assert 0.4 <= np.mean(z ** 2) <= 2.5
    assert np.mean(np.abs(z) < 2) >= 0.8


def test_lattice_beats_monte_carlo_at_equal_evaluations(ctx):
    """Same points count, same shifts: the lattice's shift-to-shift error is well below Monte Carlo's."""
    mc = run_bubble(ctx, 9, m=14, R=16)
    prob = sectorgen.bubble_problem(order_max=1)
    set_params(ctx, lattice_log2=14, shifts=16, seed=9)
    h = P.sdi_problem_create(ctx, prob)
    try:
        lat = P.sdi_integrate(ctx, h)
    finally:
        P.sdi_problem_destroy(h)
        set_params(ctx)
    assert lat["n_evals"] == mc["n_evals"]
    assert lat["err_re"][1] < 0.1 * mc["err_re"][1]
    log(f"bubble eps^0 error at 2^18 evaluations: lattice {lat['err_re'][1]:.2e}, Monte Carlo {mc['err_re'][1]:.2e}")


def test_refusals(ctx):
    P.sdi_set_param(ctx, "integrator", 2)
    try:
        h = P.sdi_problem_from_text(ctx, textgen.PAPER_EXAMPLE)
        try:
            with pytest.raises(P.SdiError) as e:
                P.sdi_integrate(ctx, h)
            assert e.value.code == -4
        finally:
            P.sdi_problem_destroy(h)
        h = P.sdi_problem_create(ctx, sectorgen.bubble_problem())
        try:
            P.sdi_set_param(ctx, "slice_log2", 4)
            with pytest.raises(P.SdiError) as e:
                P.sdi_integrate(ctx, h)
            assert e.value.code == -4
        finally:
            P.sdi_set_param(ctx, "slice_log2", 0)
            P.sdi_problem_destroy(h)
        with pytest.raises(P.SdiError):
            P.sdi_set_param(ctx, "integrator", 5)
    finally:
        P.sdi_set_param(ctx, "integrator", 0)
