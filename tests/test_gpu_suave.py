"""Subregion-adaptive Monte Carlo (integrator 3, the role of suaveCuba among
the CurrentIntegrator options of section 4.4) against the oracle's run of the
same algorithm (oracle/suave.py): the points are bit-identical (Philox), so
the runs take the same regions, axes, rounds and evaluations, and per-region
values and standard errors agree to rounding; the bubble's closed form within
the error estimate, which is calibrated over seeds; complex mode; argument
checks."""
import dataclasses
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1511_03614_amd as P  # noqa: E402
import sectorgen  # noqa: E402
from sectorgen import feynman, textgen  # noqa: E402
from oracle import suave  # noqa: E402

from test_gpu_parity import log, set_params  # noqa: E402

BUBBLE = np.array([1.0, 2.0, 4 - math.pi ** 2 / 12, 8 - math.pi ** 2 / 6 - 7 * 1.2020569031595942 / 3])


@pytest.fixture(scope="module")
def ctx():
    c = P.sdi_ctx_create(0)
    yield c
    P.sdi_ctx_destroy(c)


def params(ctx, **kw):
    base = dict(integrator=3, suave_nnew=256, cub_maxeval=1 << 24, cub_epsrel=1e-12, cub_epsabs=0.0,
                cub_split_frac=0.25, cub_batch_min=16)
    base.update(kw)
    for k, v in base.items():
        P.sdi_set_param(ctx, k, v)


def reset(ctx):
    set_params(ctx)
    params(ctx, integrator=0, suave_nnew=1024, cub_maxeval=1 << 24, cub_epsrel=1e-6, cub_batch_min=1024)


def run_both(ctx, problem, what, seed=3, **kw):
    prm = dict(suave_nnew=256, cub_maxeval=20000, cub_epsrel=1e-12, cub_epsabs=0.0, cub_split_frac=0.25,
               cub_batch_min=16)
    prm.update(kw)
    h = P.sdi_problem_create(ctx, problem)
    try:
        set_params(ctx, seed=seed)
        params(ctx, **prm)
        res = P.sdi_integrate(ctx, h)
        regs = P.sdi_cubature_regions(ctx, h)
    finally:
        P.sdi_problem_destroy(h)
        reset(ctx)
    orc = suave.suave(problem, prm["cub_maxeval"], prm["suave_nnew"], prm["cub_epsrel"], prm["cub_epsabs"], seed,
                      prm["cub_split_frac"], prm["cub_batch_min"])
    alive = [r for r in orc.regions if r.alive]
    assert res["n_evals"] == orc.evals, what
    assert res["cub_rounds"] == orc.rounds, what
    assert bool(res["cub_converged"]) == orc.converged, what
    assert len(regs["sector"]) == len(alive) == res["cub_regions"], what

    def key(s, lev, idx):
        return (int(s), tuple(int(v) for v in lev), tuple(int(v) for v in idx))
    gk = {key(regs["sector"][i], regs["level"][i, :problem.sectors[regs["sector"][i]].n],
              regs["index"][i, :problem.sectors[regs["sector"][i]].n]): i for i in range(len(alive))}
    N = prm["suave_nnew"]
    worst = 0.0
    for r in alive:
        k = key(r.sector, r.level, r.index)
        assert k in gk, (what, k)
        i = gk[k]
        assert regs["axis"][i] == r.axis, (what, k)
        # the samples' magnitude: |mean| + sqrt(N) standard error, per order
        sc = np.abs(r.value) + math.sqrt(N) * (r.err_re + r.err_im)
        d = np.abs(regs["value"][i] - r.value)
        assert np.all(d <= 1e-10 * sc + 1e-300), (what, i, regs["value"][i], r.value)
        worst = max(worst, float(np.max(d / np.maximum(sc, 1e-300))))
        for got, want in ((regs["err_re"][i], r.err_re), (regs["err_im"][i], r.err_im)):
            assert np.allclose(got, want, rtol=1e-8, atol=1e-12 * float(np.max(sc))), (what, i, got, want)
    scale = np.abs(orc.value) + math.sqrt(N) * (orc.err_re + orc.err_im)
    assert np.all(np.abs(res["value"] - orc.value) <= 1e-10 * scale), what
    assert np.allclose(res["err_re"], orc.err_re, rtol=1e-8, atol=1e-300), what
    log(f"{what}: {len(alive)} regions, {orc.rounds} rounds, {orc.evals} evals, worst relative {worst:.2e}")
    return res, orc


def test_bubble_against_oracle_and_closed_form(ctx):
    prob = sectorgen.config1()
    res, _ = run_both(ctx, prob, "bubble", suave_nnew=256, cub_maxeval=40000, cub_batch_min=4)
    z = (res["value"].real - BUBBLE) / res["err_re"]
    assert np.all(np.abs(z) < 5), z
    res, _ = run_both(ctx, prob, "bubble converged", suave_nnew=512, cub_maxeval=1 << 20, cub_epsrel=1e-3,
                      cub_batch_min=4)
    assert res["cub_converged"] == 1 and res["n_evals"] < 1 << 20


def test_synthetic_sectors_against_oracle(ctx):
    prob = sectorgen.config2()
    run_both(ctx, dataclasses.replace(prob, sectors=prob.sectors[:6]), "synthetic64[:6]", suave_nnew=128,
             cub_maxeval=30000, cub_batch_min=8)


def test_complex_mode_against_oracle(ctx):
    prob = feynman.double_box_problem(5.0, -2.0, 1.0, order_max=0, complex_mode=True, lam=0.5)
    run_both(ctx, dataclasses.replace(prob, sectors=prob.sectors[:2]), "physical double box[:2]", suave_nnew=128,
             cub_maxeval=2 * 128 * 7, cub_batch_min=2)


def test_error_estimate_is_calibrated(ctx):
    prob = sectorgen.config1()
    z = []
    h = P.sdi_problem_create(ctx, prob)
    try:
        for seed in range(16):
            set_params(ctx, seed=200 + seed)
            params(ctx, suave_nnew=256, cub_maxeval=1 << 14, cub_batch_min=4)
            res = P.sdi_integrate(ctx, h)
            z.append((res["value"][1].real - BUBBLE[1]) / res["err_re"][1])
    finally:
        P.sdi_problem_destroy(h)
        reset(ctx)
    z = np.array(z)
    log(f"subregion-adaptive Monte Carlo z-scores over 16 seeds: mean square {np.mean(z ** 2):.2f}")
    assert 0.3 <= np.mean(z ** 2) <= 3.0 and np.mean(np.abs(z) < 2) >= 0.75


def test_argument_checks(ctx):
    for bad in (8, 1 << 21):
        with pytest.raises(P.SdiError):
            P.sdi_set_param(ctx, "suave_nnew", bad)
    P.sdi_set_param(ctx, "integrator", 3)
    try:
        h = P.sdi_problem_from_text(ctx, textgen.PAPER_EXAMPLE)
        try:
            with pytest.raises(P.SdiError) as e:
                P.sdi_integrate(ctx, h)
            assert e.value.code == -4
        finally:
            P.sdi_problem_destroy(h)
        h = P.sdi_problem_create(ctx, sectorgen.config1())
        try:
            P.sdi_set_param(ctx, "suave_nnew", 1 << 20)
            P.sdi_set_param(ctx, "cub_maxeval", 1000)
            with pytest.raises(P.SdiError) as e:
                P.sdi_integrate(ctx, h)
            assert e.value.code == -1
        finally:
            P.sdi_problem_destroy(h)
    finally:
        reset(ctx)


def test_largest_variable_classes(ctx):
    """The 10- and 16-variable instances (a few rounds), against the oracle."""
    from shapes import max_real_problem
    rng = np.random.default_rng(10)
    n = 10
    exps = np.zeros((12, n), dtype=np.uint8)
    for t in range(1, 12):
        exps[t, rng.choice(n, 3, replace=False)] = rng.integers(1, 4, 3)
    sec10 = sectorgen.Sector(a=np.r_[-1.0, -1.0, np.zeros(n - 2)], b=np.r_[1.0, -2.0, np.zeros(n - 2)],
                             factors=[sectorgen.Factor(-1.5, 1.0, rng.uniform(0.2, 1.0, 12), exps)])
    p10 = sectorgen.Problem(sectors=[sec10, sec10], order_min=-2, order_max=0)
    run_both(ctx, p10, "10 variables", suave_nnew=64, cub_maxeval=64 * 14, cub_batch_min=2)
    big = max_real_problem()
    p16 = dataclasses.replace(big, sectors=big.sectors[:2])
    run_both(ctx, p16, "16 variables", suave_nnew=64, cub_maxeval=64 * 10, cub_batch_min=2)
