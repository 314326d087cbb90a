"""SeparateTerms (section 4.4): problems compiled term by term (separate_terms =
1) against oracle/separate.py on identical points.

* Synthetic sectors with 1..3 singular variables (some with every variable
  singular) and the config-2 sectors: the same terms in the same order, the
  per-(term, shift) means at the 1e-10 bar, the total equal to the sum of the
  oracle's terms; also with the endpoint precision on (double-double points),
  which must leave the boundary terms out as the fp64 path does.
* The separated total agrees with the whole sectors' total within their
  combined error estimates (two estimates of the same integral), under the
  lattice, the adaptive cubature, the subregion-adaptive Monte Carlo and the
  partition-then-lattice integrator.
* Under the Vegas warm-up every term adapts its own grids, as the oracle's
  terms do (per shift at the warm-up bar).
* The box of section 4.3 through the Feynman front end: the oracle's terms of
  the input tool's sectors per shift, and the closed form.
* Refusals: complex mode, a factor with no term on a face.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1511_03614_amd as P  # noqa: E402
import sectorgen  # noqa: E402
from sectorgen import Factor, Problem, Sector  # noqa: E402
from oracle import separate  # noqa: E402

from test_gpu_parity import assert_close_shift, log, oracle_shift_values, set_params  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    c = P.sdi_ctx_create(0)
    yield c
    P.sdi_ctx_destroy(c)


def problems():
    syn = sectorgen.synthetic_problem(11, 6, (2, 4), (2, 5), (1, 3), -3, 1)
    c2 = sectorgen.config2()
    c2 = Problem(c2.sectors[:6], c2.order_min, c2.order_max, c2.pref_lead, c2.pref, name="config2[:6]")
    return [syn, c2]


def create_separated(ctx, prob):
    P.sdi_set_param(ctx, "separate_terms", 1)
    try:
        return P.sdi_problem_create(ctx, prob)
    finally:
        P.sdi_set_param(ctx, "separate_terms", 0)


@pytest.mark.parametrize("which", [0, 1])
@pytest.mark.parametrize("small_x", [0.0, 0.05])
def test_terms_match_the_oracle(ctx, which, small_x):
    prob = problems()[which]
    parts, origin = separate.separate(prob)
    m, R, seed = 10, 4, 9
    h = create_separated(ctx, prob)
    try:
        assert P.sdi_problem_nsectors(h) == len(parts.sectors) > len(prob.sectors)
        assert [P.sdi_problem_sector_origin(h, s) for s in range(len(parts.sectors))] == origin
        assert [P.sdi_problem_nvars(h, s) for s in range(len(parts.sectors))] == [s.n for s in parts.sectors]
        set_params(ctx, lattice_log2=m, shifts=R, seed=seed)
        P.sdi_set_param(ctx, "small_x", small_x)
        res = P.sdi_integrate(ctx, h)
        tot = 0
        for s in range(len(parts.sectors)):
            q, scale = oracle_shift_values(parts, s, m, R, seed)
            assert_close_shift(P.sdi_sector_results(ctx, h, s, R)[2], q, scale, f"term {s} of sector {origin[s]}")
            tot = tot + q.mean(axis=0)
        assert np.allclose(res["value"], tot, rtol=1e-10, atol=1e-10 * float(np.max(np.abs(tot))))
        log(f"{prob.name or 'synthetic'} small_x={small_x}: {len(prob.sectors)} sectors -> "
            f"{len(parts.sectors)} terms at the bar")
    finally:
        P.sdi_set_param(ctx, "small_x", 0.0)
        P.sdi_problem_destroy(h)
        set_params(ctx)


ADAPTIVE = {1: dict(cub_maxeval=1 << 22, cub_epsrel="1e-7"),
            3: dict(cub_maxeval=1 << 20, cub_epsrel="1e-7", suave_nnew=1024),
            4: dict(cub_maxeval=1 << 18, cub_epsrel="1e-7", suave_nnew=256)}


@pytest.mark.parametrize("integrator", [0, 1, 3, 4])
def test_separated_total_agrees_with_whole(ctx, integrator):
    prob = problems()[0]
    out = []
    for sep in (0, 1):
        h = create_separated(ctx, prob) if sep else P.sdi_problem_create(ctx, prob)
        try:
            if integrator == 4:
                set_params(ctx, lattice_log2=8, shifts=8, seed=3)
            else:
                set_params(ctx, lattice_log2=14, shifts=16, seed=3)
            P.sdi_set_param(ctx, "integrator", integrator)
            for k, v in ADAPTIVE.get(integrator, {}).items():
                P.sdi_set_param(ctx, k, v)
            out.append(P.sdi_integrate(ctx, h))
        finally:
            for k, v in dict(integrator=0, cub_maxeval=1 << 24, cub_epsrel="1e-6", suave_nnew=1024).items():
                P.sdi_set_param(ctx, k, v)
            P.sdi_problem_destroy(h)
            set_params(ctx)
    a, b = out
    d = np.abs(np.asarray(a["value"]) - np.asarray(b["value"]))
    e = np.hypot(np.hypot(a["err_re"], a["err_im"]), np.hypot(b["err_re"], b["err_im"]))
    scale = np.max(np.abs(np.asarray(a["value"])))
    assert np.all(d <= 5.0 * e + 1e-12 * scale), (d, e)
    log(f"integrator {integrator}: separated vs whole |diff| {d}, combined errors {e}")


def test_refusals(ctx):
    syn = problems()[0]
    cplx = Problem(syn.sectors[:2], syn.order_min, syn.order_max, syn.pref_lead, syn.pref, complex_mode=True, lam=0.0)
    P.sdi_set_param(ctx, "separate_terms", 1)
    try:
        with pytest.raises(P.SdiError) as e:
            P.sdi_problem_create(ctx, cplx)
        assert e.value.code == -4
        f = Factor(1.0, 0.0, np.array([1.0]), np.array([[1, 0]], dtype=np.uint8))
        bad = Problem([Sector(np.array([-1.0, -1.0]), np.array([1.0, 1.0]), [f])], -2, 0)
        with pytest.raises(P.SdiError) as e:
            P.sdi_problem_create(ctx, bad)
        assert e.value.code == -4
    finally:
        P.sdi_set_param(ctx, "separate_terms", 0)
    with pytest.raises(P.SdiError):
        P.sdi_set_param(ctx, "separate_terms", 2)


def test_box_through_the_front_end(ctx):
    """The one-loop box of section 4.3 built by sdi_problem_from_feynman with
    separate_terms = 1: the oracle's terms of the input tool's sectors, the
    same per-(term, shift) means, and the closed form."""
    import math
    from sectorgen import feynman
    U, F = feynman.box_uf(3.0, 1.0)
    P.sdi_set_param(ctx, "separate_terms", 1)
    try:
        h = P.sdi_problem_from_feynman(ctx, U, F, 1, (1, 1, 1, 1), 0)
    finally:
        P.sdi_set_param(ctx, "separate_terms", 0)
    parts, origin = separate.separate(feynman.box_problem(3.0, 1.0))
    try:
        assert P.sdi_problem_nsectors(h) == len(parts.sectors)
        assert [P.sdi_problem_sector_origin(h, s) for s in range(len(parts.sectors))] == origin
        m, R, seed = 12, 8, 3
        set_params(ctx, lattice_log2=m, shifts=R, seed=seed)
        res = P.sdi_integrate(ctx, h)
        K = len(res["value"])
        off = res["order_min"] - parts.order_min
        for s in range(len(parts.sectors)):
            q, scale = oracle_shift_values(parts, s, m, R, seed)
            assert_close_shift(P.sdi_sector_results(ctx, h, s, R)[2], q[:, off:off + K], scale[off:off + K],
                               f"box term {s}")
        exact = [4 / 3, -2 * math.log(3) / 3, -4 * math.pi ** 2 / 9]
        assert np.all(np.abs(res["value"].real - exact) <= 5 * res["err_re"] + 1e-9), (res["value"], res["err_re"])
        log(f"box through the front end: {len(parts.sectors)} terms, values {res['value'].real}")
    finally:
        P.sdi_problem_destroy(h)
        set_params(ctx)


def test_terms_with_vegas_warmup(ctx):
    """Separated terms under the Vegas warm-up: every term adapts its own grids
    from all its eps rows (the eps shift included), as the oracle's terms do."""
    from oracle import integrate
    prob = problems()[0]
    parts, _ = separate.separate(prob)
    m, R, mw, nb, W = 10, 4, 10, 32, 2
    h = create_separated(ctx, prob)
    try:
        set_params(ctx, lattice_log2=m, shifts=R, seed=4, warmup=W, warmup_log2=mw, nbins=nb)
        P.sdi_integrate(ctx, h)
        lead, pref = integrate.prefactor_for(parts)
        for s in range(len(parts.sectors)):
            est = integrate.integrate_sector(parts, s, m, R, 4, lead, pref, True, nb, W, mw)
            per = P.sdi_sector_results(ctx, h, s, R)[2]
            # grids refit from histograms summed in different orders: 1e-9 of the absolute scale
            oq, scale = oracle_shift_values(parts, s, m, R, 4, grid=est.grid)
            tol = 1e-9 * np.maximum(np.abs(oq), scale[None, :])
            assert np.all(np.abs(per - oq) <= tol), s
    finally:
        P.sdi_problem_destroy(h)
        set_params(ctx)
