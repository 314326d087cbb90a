"""The adaptive deterministic cubature (integrator 1, the cuhreCuba option of
section 4.4) against the oracle's run of the same algorithm.

Checks: identical region sets (sector, halvings and index per variable), split
axes, rounds and evaluation counts; per-region values and errors at the 1e-10
bar relative to the region's conditioning (sum of |w F| vol over its nodes);
totals; the bubble's closed form within the error estimate and convergence;
complex mode (the physical double box); the 10- and 16-variable instances;
consistency of a long run (tiling, sums, sampled regions); argument checks."""
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
from sectorgen import feynman  # noqa: E402
from oracle import cubature, integrate  # noqa: E402

from test_gpu_parity import log, set_params  # noqa: E402
from test_gpu_limits import max_real_problem  # noqa: E402

BAR = 1e-10


@pytest.fixture(scope="module")
def ctx():
    c = P.sdi_ctx_create(0)
    yield c
    P.sdi_ctx_destroy(c)


def cub_params(ctx, **kw):
    base = dict(integrator=1, cub_maxeval=1 << 24, cub_epsrel=1e-6, cub_epsabs=0.0, cub_split_frac=0.25,
                cub_batch_min=1024)
    base.update(kw)
    for k, v in base.items():
        P.sdi_set_param(ctx, k, v)


def reset(ctx):
    set_params(ctx)
    cub_params(ctx, integrator=0)


def region_scale(problem, reg, lead, pref):
    """Sum over the region's nodes of |w7| |F_k| vol per order (the rounding scale)."""
    sec = problem.sectors[reg.sector]
    xi, cls = cubature.nodes(sec.n)
    centre, half = cubature.box(reg)
    x = centre[None, :] + xi * half[None, :]
    vals, _, _ = integrate.sector_values(problem, reg.sector, x, lead, pref)
    w7, _ = cubature.weights(sec.n)
    a7 = np.abs(np.array([w7[c] for c in cls]))
    vol = float(np.prod(2.0 * half))
    return vol * (np.abs(vals) * a7[None, :]).sum(axis=1)


def run_both(ctx, problem, what, **kw):
    """GPU run and oracle run with the same settings; compares everything."""
    prm = dict(cub_maxeval=20000, cub_epsrel=1e-9, cub_epsabs=0.0, cub_split_frac=0.25, cub_batch_min=16)
    prm.update(kw)
    h = P.sdi_problem_create(ctx, problem)
    try:
        set_params(ctx)
        cub_params(ctx, **prm)
        res = P.sdi_integrate(ctx, h)
        regs = P.sdi_cubature_regions(ctx, h)
        per = [P.sdi_sector_results(ctx, h, s, 2) for s in range(len(problem.sectors))]
    finally:
        P.sdi_problem_destroy(h)
        reset(ctx)
    orc = cubature.cubature(problem, prm["cub_maxeval"], prm["cub_epsrel"], prm["cub_epsabs"],
                            prm["cub_split_frac"], prm["cub_batch_min"])
    alive = [r for r in orc.regions if r.alive]
    assert res["n_evals"] == orc.evals, what
    assert res["cub_rounds"] == orc.rounds, what
    assert bool(res["cub_converged"]) == orc.converged, what
    assert len(regs["sector"]) == len(alive) == res["cub_regions"], what
    # the same regions (in canonical order: regions of equal priority may be
    # halved in another order within a round, which only renumbers them)
    def key(s, lev, idx):
        return (int(s), tuple(int(v) for v in lev), tuple(int(v) for v in idx))
    gk = {key(regs["sector"][i], regs["level"][i, :problem.sectors[regs["sector"][i]].n],
              regs["index"][i, :problem.sectors[regs["sector"][i]].n]): i for i in range(len(alive))}
    lead, pref = integrate.prefactor_for(problem)
    worst = 0.0
    tot_scale = 0.0
    for r in alive:
        k = key(r.sector, r.level, r.index)
        assert k in gk, (what, k)
        i = gk[k]
        assert regs["axis"][i] == r.axis, (what, k)
        sc = region_scale(problem, r, lead, pref)
        tot_scale = tot_scale + sc
        for got, want in ((regs["value"][i], r.value), (regs["err_re"][i], r.err_re), (regs["err_im"][i], r.err_im)):
            d = np.abs(got - want)
            bar = BAR * np.maximum(np.abs(want), sc)
            assert np.all(d <= bar), (what, i, got, want, sc)
            worst = max(worst, float(np.max(d / np.maximum(np.maximum(np.abs(want), sc), 1e-300))))
    assert np.all(np.abs(res["value"] - orc.value) <= BAR * np.maximum(np.abs(orc.value), tot_scale)), what
    assert np.allclose(res["err_re"], orc.err_re, rtol=1e-8, atol=BAR * float(np.max(tot_scale)))
    # per-sector results add up to the totals
    assert np.allclose(sum(m[0] for m in per), res["value"], rtol=1e-13, atol=1e-300)
    log(f"{what}: {len(alive)} regions, {orc.rounds} rounds, {orc.evals} evals, worst relative {worst:.2e}")
    return res, orc


def test_bubble_against_oracle_and_closed_form(ctx):
    prob = sectorgen.config1()
    res, _ = run_both(ctx, prob, "bubble", cub_maxeval=20000, cub_epsrel=1e-12, cub_batch_min=4)
    z3 = 1.2020569031595942
    exact = np.array([1.0, 2.0, 4 - math.pi ** 2 / 12, 8 - math.pi ** 2 / 6 - 7 * z3 / 3])
    assert np.all(np.abs(res["value"] - exact) <= res["err_re"] + 1e-15)
    res, _ = run_both(ctx, prob, "bubble converged", cub_maxeval=20000, cub_epsrel=1e-6, cub_batch_min=4)
    assert res["cub_converged"] == 1 and res["n_evals"] < 20000


def test_synthetic_sectors_against_oracle(ctx):
    prob = sectorgen.config2()
    sub = dataclasses.replace(prob, sectors=prob.sectors[:12])
    run_both(ctx, sub, "synthetic64[:12]", cub_maxeval=60000, cub_batch_min=8)


def test_box_section_4_3(ctx):
    prob = feynman.box_problem(3.0, 1.0)
    res, _ = run_both(ctx, prob, "box", cub_maxeval=30000, cub_epsrel=1e-8, cub_batch_min=16)
    exact = [4 / 3, -2 * math.log(3) / 3, -4 * math.pi ** 2 / 9]
    for k, v in enumerate(exact):
        assert abs(res["value"][k] - v) <= 3 * res["err_re"][k] + 1e-12


def test_complex_mode_against_oracle(ctx):
    prob = feynman.double_box_problem(5.0, -2.0, 1.0, order_max=0, complex_mode=True, lam=0.5)
    sub = dataclasses.replace(prob, sectors=prob.sectors[:4])
    run_both(ctx, sub, "physical double box[:4]", cub_maxeval=4 * 149 * 9, cub_batch_min=4)


def test_largest_variable_classes(ctx):
    """A 10-variable and the 16-variable instances: one round of halving."""
    rng = np.random.default_rng(10)
    n = 10
    exps = np.zeros((12, n), dtype=np.uint8)
    for t in range(1, 12):
        exps[t, rng.choice(n, 3, replace=False)] = rng.integers(1, 4, 3)
    sec10 = sectorgen.Sector(a=np.r_[-1.0, -1.0, np.zeros(n - 2)], b=np.r_[1.0, -2.0, np.zeros(n - 2)],
                             factors=[sectorgen.Factor(-1.5, 1.0, rng.uniform(0.2, 1.0, 12), exps)])
    p10 = sectorgen.Problem(sectors=[sec10, sec10], order_min=-2, order_max=0)
    run_both(ctx, p10, "10 variables", cub_maxeval=2 * 1245 + 2 * 2 * 1245, cub_batch_min=2)
    big = max_real_problem()
    p16 = dataclasses.replace(big, sectors=big.sectors[:2])
    run_both(ctx, p16, "16 variables", cub_maxeval=2 * 66081 + 2 * 66081, cub_batch_min=1, cub_split_frac=0.01)


def test_long_run_consistency(ctx):
    """The 64-sector synthetic set with 2^22 evaluations: alive regions tile every cube, totals are
    their sums, sampled regions match the oracle's rule, and a run with 4x the
    evaluations has smaller errors and agrees within them."""
    prob = sectorgen.config2()
    lead, pref = integrate.prefactor_for(prob)
    h = P.sdi_problem_create(ctx, prob)
    try:
        set_params(ctx)
        cub_params(ctx, cub_maxeval=1 << 20, cub_epsrel=1e-12)
        small = P.sdi_integrate(ctx, h)
        cub_params(ctx, cub_maxeval=1 << 22, cub_epsrel=1e-12)
        res = P.sdi_integrate(ctx, h)
        regs = P.sdi_cubature_regions(ctx, h)
    finally:
        P.sdi_problem_destroy(h)
        reset(ctx)
    assert small["n_evals"] <= 1 << 20 and res["n_evals"] <= 1 << 22
    assert res["n_evals"] > (1 << 22) * 0.9
    N = len(regs["sector"])
    assert N == res["cub_regions"] and N > 10000
    for s in range(len(prob.sectors)):
        sel = regs["sector"] == s
        n = prob.sectors[s].n
        vol = np.sum(np.ldexp(1.0, -regs["level"][sel, :n].astype(int).sum(axis=1)))
        assert vol == 1.0
    assert np.allclose(regs["value"].sum(axis=0), res["value"], rtol=1e-12, atol=1e-14)
    assert np.sum(res["err_re"] + res["err_im"]) < np.sum(small["err_re"] + small["err_im"])
    assert np.all(np.abs(res["value"] - small["value"]) <= small["err_re"] + small["err_im"] + 1e-13)
    rng = np.random.default_rng(5)
    for i in rng.choice(N, 12, replace=False):
        s = int(regs["sector"][i])
        n = prob.sectors[s].n
        r = cubature.Region(s, regs["level"][i, :n].astype(np.int64), regs["index"][i, :n].astype(np.int64))
        cubature.apply_rule(prob, r, lead, pref, np.ones(prob.norders))
        sc = region_scale(prob, r, lead, pref)
        assert np.all(np.abs(regs["value"][i] - r.value) <= BAR * np.maximum(np.abs(r.value), sc)), i
        assert np.all(np.abs(regs["err_re"][i] - r.err_re) <= BAR * np.maximum(r.err_re, sc)), i
    log(f"synthetic64 at 2^22: {N} regions, {res['cub_rounds']} rounds, kernel {res['ms_eval_kernel']:.1f} ms, "
        f"total {res['ms_total']:.1f} ms")


def test_argument_checks(ctx):
    prob = sectorgen.config1()
    h = P.sdi_problem_create(ctx, prob)
    try:
        with pytest.raises(P.SdiError):
            P.sdi_cubature_regions(ctx, h)                 # no run yet
        set_params(ctx)
        for bad in (dict(budget=1 << 20), dict(warmup=2), dict(slice_log2=8)):
            set_params(ctx, **bad)
            cub_params(ctx)
            with pytest.raises(P.SdiError):
                P.sdi_integrate(ctx, h)
            set_params(ctx)
        cub_params(ctx, cub_maxeval=10)                   # below one rule per sector (2 x 7)
        with pytest.raises(P.SdiError):
            P.sdi_integrate(ctx, h)
        for key, val in (("cub_split_frac", 0), ("cub_epsrel", -1), ("cub_batch_min", 0), ("integrator", 5)):
            with pytest.raises(P.SdiError):
                P.sdi_set_param(ctx, key, val)
    finally:
        P.sdi_problem_destroy(h)
        reset(ctx)
    t = P.sdi_problem_from_text(ctx, "1; 0; x[1]+0.2; |")
    try:
        cub_params(ctx)
        with pytest.raises(P.SdiError):
            P.sdi_integrate(ctx, t)
    finally:
        P.sdi_problem_destroy(t)
        reset(ctx)
