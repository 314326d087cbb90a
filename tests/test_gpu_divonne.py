"""Partition by spreads, then lattice rules (integrator 4, the role of
divonneCuba among the CurrentIntegrator options of section 4.4) against the
oracle's run of the same algorithm (oracle/divonne.py): the partition's
Philox samples and the final rule's lattice points are bit-identical, so the
runs take the same regions, axes, refinements and evaluations, and the
per-region values agree to rounding; the bubble's closed form within the error
estimate; complex mode; the 10- and 16-variable instances; argument checks."""
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
from oracle import divonne  # noqa: E402

from test_gpu_parity import log, set_params  # noqa: E402

BUBBLE = np.array([1.0, 2.0, 4 - math.pi ** 2 / 12, 8 - math.pi ** 2 / 6 - 7 * 1.2020569031595942 / 3])


@pytest.fixture(scope="module")
def ctx():
    c = P.sdi_ctx_create(0)
    yield c
    P.sdi_ctx_destroy(c)


def reset(ctx):
    set_params(ctx)
    for k, v in dict(integrator=0, suave_nnew=1024, cub_maxeval=1 << 24, cub_epsrel=1e-6, cub_epsabs=0.0,
                     cub_split_frac=0.25, cub_batch_min=1024).items():
        P.sdi_set_param(ctx, k, v)


def run_both(ctx, problem, what, seed=3, m=8, R=8, baker=1, **kw):
    prm = dict(suave_nnew=256, cub_maxeval=20000, cub_epsrel=1e-6, cub_epsabs=0.0, cub_split_frac=0.25,
               cub_batch_min=16)
    prm.update(kw)
    h = P.sdi_problem_create(ctx, problem)
    try:
        set_params(ctx, seed=seed, lattice_log2=m, shifts=R, baker=baker)
        P.sdi_set_param(ctx, "integrator", 4)
        for k, v in prm.items():
            P.sdi_set_param(ctx, k, v)
        res = P.sdi_integrate(ctx, h)
        regs = P.sdi_cubature_regions(ctx, h)
    finally:
        P.sdi_problem_destroy(h)
        reset(ctx)
    orc = divonne.divonne(problem, prm["cub_maxeval"], prm["suave_nnew"], prm["cub_epsrel"], prm["cub_epsabs"],
                          seed, m, R, bool(baker), prm["cub_split_frac"], prm["cub_batch_min"])
    alive = [r for r in orc.regions if r.alive]
    assert res["n_evals"] == orc.evals, what
    assert res["cub_rounds"] == orc.rounds, what
    assert len(regs["sector"]) == len(alive) == res["cub_regions"], what

    def key(s, lev, idx):
        return (int(s), tuple(int(v) for v in lev), tuple(int(v) for v in idx))
    gk = {key(regs["sector"][i], regs["level"][i, :problem.sectors[regs["sector"][i]].n],
              regs["index"][i, :problem.sectors[regs["sector"][i]].n]): i for i in range(len(alive))}
    worst = 0.0
    for r in alive:
        k = key(r.sector, r.level, r.index)
        assert k in gk, (what, k)
        i = gk[k]
        assert regs["axis"][i] == r.axis, (what, k)
        # the lattice rule's magnitude: |value| + sqrt(R) standard error of the shift means, per order
        sc = np.abs(r.value) + math.sqrt(R) * (r.err_re + r.err_im)
        d = np.abs(regs["value"][i] - r.value)
        assert np.all(d <= 1e-10 * sc + 1e-300), (what, i, regs["value"][i], r.value)
        worst = max(worst, float(np.max(d / np.maximum(sc, 1e-300))))
        for got, want in ((regs["err_re"][i], r.err_re), (regs["err_im"][i], r.err_im)):
            # the shift means' deviations carry their rounding relative to the means themselves
            assert np.allclose(got, want, rtol=1e-6, atol=1e-13 * float(np.max(sc))), (what, i, got, want)
    scale = np.abs(orc.value) + math.sqrt(R) * (orc.err_re + orc.err_im)
    assert np.all(np.abs(res["value"] - orc.value) <= 1e-10 * scale), what
    assert np.allclose(res["err_re"], orc.err_re, rtol=1e-6, atol=1e-12 * float(np.max(scale))), what
    log(f"{what}: {len(alive)} regions ({orc.refined} refined), {orc.rounds} rounds, {orc.evals} evals, "
        f"worst relative {worst:.2e}")
    return res, orc


def test_bubble_against_oracle_and_closed_form(ctx):
    prob = sectorgen.config1()
    res, _ = run_both(ctx, prob, "bubble", suave_nnew=256, cub_maxeval=20000, cub_batch_min=4)
    z = (res["value"].real - BUBBLE) / res["err_re"]
    assert np.all(np.abs(z) < 5), z
    res, _ = run_both(ctx, prob, "bubble, no tent map", baker=0, m=10, R=4, cub_maxeval=6000, cub_batch_min=2)
    z = (res["value"].real - BUBBLE) / res["err_re"]
    assert np.all(np.abs(z) < 5), z


def test_synthetic_sectors_against_oracle(ctx):
    prob = sectorgen.config2()
    run_both(ctx, dataclasses.replace(prob, sectors=prob.sectors[:6]), "synthetic64[:6]", suave_nnew=128,
             cub_maxeval=30000, cub_batch_min=8, m=7, R=4)


def test_complex_mode_against_oracle(ctx):
    prob = feynman.double_box_problem(5.0, -2.0, 1.0, order_max=0, complex_mode=True, lam=0.5)
    run_both(ctx, dataclasses.replace(prob, sectors=prob.sectors[:2]), "physical double box[:2]", suave_nnew=128,
             cub_maxeval=2 * 128 * 7, cub_batch_min=2, m=6, R=4)


def test_argument_checks(ctx):
    with pytest.raises(P.SdiError) as e:   # the final rule's error needs two shifts at least
        P.sdi_set_param(ctx, "shifts", 1)
    assert e.value.code == -1
    h = P.sdi_problem_from_text(ctx, textgen.PAPER_EXAMPLE)
    try:
        P.sdi_set_param(ctx, "integrator", 4)
        with pytest.raises(P.SdiError) as e:
            P.sdi_integrate(ctx, h)
        assert e.value.code == -4
    finally:
        P.sdi_problem_destroy(h)
        reset(ctx)
    with pytest.raises(P.SdiError):
        P.sdi_set_param(ctx, "integrator", 5)


def test_largest_variable_classes(ctx):
    """The 10- and 16-variable instances of both phases (a few rounds, small
    lattices), against the oracle."""
    from shapes import max_real_problem
    rng = np.random.default_rng(10)
    n = 10
    exps = np.zeros((12, n), dtype=np.uint8)
    for t in range(1, 12):
        exps[t, rng.choice(n, 3, replace=False)] = rng.integers(1, 4, 3)
    sec10 = sectorgen.Sector(a=np.r_[-1.0, -1.0, np.zeros(n - 2)], b=np.r_[1.0, -2.0, np.zeros(n - 2)],
                             factors=[sectorgen.Factor(-1.5, 1.0, rng.uniform(0.2, 1.0, 12), exps)])
    p10 = sectorgen.Problem(sectors=[sec10, sec10], order_min=-2, order_max=0)
    run_both(ctx, p10, "10 variables", suave_nnew=64, cub_maxeval=64 * 14, cub_batch_min=2, m=5, R=4)
    big = max_real_problem()
    p16 = dataclasses.replace(big, sectors=big.sectors[:2])
    run_both(ctx, p16, "16 variables", suave_nnew=64, cub_maxeval=64 * 10, cub_batch_min=2, m=4, R=2)
