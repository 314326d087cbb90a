"""GPU parity: the HIP library against the fp64 oracle on identical points.

Bars:
* sampling points: bit-exact (integer lattice arithmetic, one rounding per op);
* per point: |gpu - oracle| <= 1e-12 |oracle| + 4e-15 * cond, cond = sum of the
  absolute values of every subtraction/series term (the oracle returns it);
* per (sector, shift) mean and per integral: <= 1e-10 relative to
  max(|oracle|, mean |w F|) - the second term covers cancellation to ~0.
"""
import math
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1511_03614_amd as P  # noqa: E402
import sectorgen  # noqa: E402
from oracle import integrand, integrate, points  # noqa: E402

REL_INT = 1e-10


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    c = P.sdi_ctx_create(0)
    log("device: " + P.sdi_device_info(c))
    yield c
    P.sdi_ctx_destroy(c)


def set_params(ctx, **kw):
    base = dict(lattice_log2=10, shifts=4, seed=1, baker=1, warmup=0, warmup_log2=10, nbins=32,
                tile_log2=14, ppt=0, graph=1, sampler=0, budget=0, slice_log2=0)
    base.update(kw)
    for k, v in base.items():
        P.sdi_set_param(ctx, k, v)
    return base


def oracle_shift_values(problem, s, m, R, seed, baker=True, grid=None):
    """Per-shift means Q[r, k] and mean |wF| scale from the oracle on the same points."""
    lead, pref = integrate.prefactor_for(problem)
    sec = problem.sectors[s]
    z = points.cbc_vector(m, sec.n)
    sh = points.shift_table(seed, s, R, sec.n, m)
    N = 1 << m
    K = problem.norders
    q = np.zeros((R, K), dtype=complex)
    scale = np.zeros(K)
    for r in range(R):
        x, w, _ = points.sector_points(z, m, sh[r], 0, N, grid, baker)
        vals, _, _ = integrand.sector_orders(sec, x, problem.order_min, problem.order_max, lead, pref)
        wf = vals * w[None, :]
        for k in range(K):
            q[r, k] = integrate.fsum_c(wf[k]) / N
            scale[k] = max(scale[k], float(np.mean(np.abs(wf[k]))))
    return q, scale


def assert_close_shift(gq, oq, scale, what):
    tol = REL_INT * np.maximum(np.abs(oq), scale[None, :])
    bad = ~(np.abs(gq - oq) <= tol)        # a NaN on either side fails
    assert not bad.any(), f"{what}: max rel {np.max(np.abs(gq - oq) / np.maximum(tol / REL_INT, 1e-300))}"


# ---------------------------------------------------------------- points

@pytest.mark.parametrize("m,baker", [(10, 1), (13, 0), (4, 1)])
def test_sample_points_bit_exact(ctx, m, baker):
    prob = sectorgen.config2()
    set_params(ctx, lattice_log2=m, shifts=3, seed=7, baker=baker)
    h = P.sdi_problem_create(ctx, prob)
    try:
        for s in (0, 5, 17, 63):
            sec = prob.sectors[s]
            N = 1 << m
            x, w = P.sdi_sample_points(ctx, h, s, 2, 0, N, sec.n)
            z = points.cbc_vector(m, sec.n)
            sh = points.shift_table(7, s, 3, sec.n, m)[2]
            ox, ow, _ = points.sector_points(z, m, sh, 0, N, None, bool(baker))
            assert np.array_equal(x.cpu().numpy(), ox), (m, s)
            assert np.all(w.cpu().numpy() == 1.0)
    finally:
        P.sdi_problem_destroy(h)


# ---------------------------------------------------------------- per point

def pointwise_check(ctx, prob, s, x_np):
    h = P.sdi_problem_create(ctx, prob)
    try:
        x = torch.from_numpy(x_np).cuda()
        g, gc = P.sdi_evaluate(ctx, h, s, x, with_cond=True)
        g, gc = g.cpu().numpy(), gc.cpu().numpy()
    finally:
        P.sdi_problem_destroy(h)
    lead, pref = integrate.prefactor_for(prob)
    vals, cond, _ = integrand.sector_orders(prob.sectors[s], x_np, prob.order_min, prob.order_max, lead, pref)
    gv = g[..., 0].T + 1j * g[..., 1].T
    # the library's own conditioning sums: sums of absolute values, so both sides agree closely
    np.testing.assert_allclose(gc.T, cond, rtol=1e-10, atol=0)
    d = np.abs(gv - vals)
    strict = d <= 1e-12 * np.abs(vals)
    ok = strict | (d <= 1e-12 * np.abs(vals) + 4e-15 * cond)
    return ok, strict


def test_evaluate_pointwise_config2(ctx):
    prob = sectorgen.config2()
    rng = np.random.default_rng(11)
    set_params(ctx)
    frac = []
    for s in range(0, 64, 3):
        n = prob.sectors[s].n
        x = rng.uniform(1e-6, 1.0, size=(2048, n))
        x[:64] = rng.uniform(1e-9, 1e-4, size=(64, n))          # near the faces
        ok, strict = pointwise_check(ctx, prob, s, x)
        assert ok.all(), f"sector {s}: {np.argwhere(~ok)[:5]}"
        frac.append(strict.mean())
    log(f"pointwise strict-clause fraction: min {min(frac):.4f}")
    assert min(frac) > 0.95


def test_evaluate_pointwise_bubble_and_box(ctx):
    from sectorgen.feynman import box_problem
    rng = np.random.default_rng(3)
    for prob in (sectorgen.config1(), box_problem(3.0, 1.0)):
        for s in range(len(prob.sectors)):
            x = rng.uniform(1e-8, 1.0, size=(1024, prob.sectors[s].n))
            ok, _ = pointwise_check(ctx, prob, s, x)
            assert ok.all(), (prob.name, s)


# ---------------------------------------------------------------- integrate

def test_integrate_bubble_parity_and_closed_form(ctx):
    prob = sectorgen.config1()
    m, R = 13, 8
    set_params(ctx, lattice_log2=m, shifts=R, seed=1)
    h = P.sdi_problem_create(ctx, prob)
    try:
        res = P.sdi_integrate(ctx, h)
        assert res["status"] == 0 and res["n_nonfinite"] == 0
        for s in range(2):
            mean, err, per, nev = P.sdi_sector_results(ctx, h, s, R)
            oq, scale = oracle_shift_values(prob, s, m, R, 1)
            assert_close_shift(per, oq, scale, f"bubble sector {s}")
            assert nev == R << m
    finally:
        P.sdi_problem_destroy(h)
    exact = [1.0, 2.0, 4 - math.pi ** 2 / 12, 8 - math.pi ** 2 / 6 - 7 * 1.2020569031595942 / 3]
    for k in range(4):
        assert abs(res["value"][k].real - exact[k]) < 5 * res["err_re"][k] + 1e-12


@pytest.mark.parametrize("ppt", [1, 2, 4])
def test_integrate_config2_parity(ctx, ppt):
    prob = sectorgen.config2()
    m, R = 10, 4
    set_params(ctx, lattice_log2=m, shifts=R, seed=3, ppt=ppt, tile_log2=8)
    h = P.sdi_problem_create(ctx, prob)
    try:
        res = P.sdi_integrate(ctx, h)
        assert res["status"] == 0
        tot = np.zeros(prob.norders, dtype=complex)
        scal = np.zeros(prob.norders)
        for s in range(64):
            _, _, per, _ = P.sdi_sector_results(ctx, h, s, R)
            oq, scale = oracle_shift_values(prob, s, m, R, 3)
            assert_close_shift(per, oq, scale, f"sector {s}")
            tot += oq.mean(axis=0)
            scal += scale
        tol = REL_INT * np.maximum(np.abs(tot), scal)
        assert np.all(np.abs(res["value"] - tot) <= tol)
    finally:
        P.sdi_problem_destroy(h)


def test_integrate_edge_sizes(ctx):
    """Tiny lattice (fewer points than one block), tiles larger than the lattice, two shifts."""
    prob = sectorgen.config2()
    prob.sectors = prob.sectors[:6]
    for m, tl in ((4, 14), (6, 6), (9, 7)):
        set_params(ctx, lattice_log2=m, shifts=2, seed=5, tile_log2=tl)
        h = P.sdi_problem_create(ctx, prob)
        try:
            P.sdi_integrate(ctx, h)
            for s in range(6):
                _, _, per, _ = P.sdi_sector_results(ctx, h, s, 2)
                oq, scale = oracle_shift_values(prob, s, m, 2, 5)
                assert_close_shift(per, oq, scale, f"m={m} sector {s}")
        finally:
            P.sdi_problem_destroy(h)


def test_integrate_deterministic_and_workspace(ctx):
    prob = sectorgen.config2()
    set_params(ctx, lattice_log2=11, shifts=4, seed=9)
    h = P.sdi_problem_create(ctx, prob)
    try:
        a = P.sdi_integrate(ctx, h)
        b = P.sdi_integrate(ctx, h)
        nb = P.sdi_workspace_bytes(ctx, h)
        # a caller workspace full of NaN bytes: nothing may be read before it is written
        ws = torch.full((nb,), 255, dtype=torch.uint8, device="cuda")
        c = P.sdi_integrate(ctx, h, ws)
        for r in (b, c):
            assert np.array_equal(a["value"], r["value"])
            assert np.array_equal(a["err_re"], r["err_re"])
        with pytest.raises(P.SdiError):
            P.sdi_integrate(ctx, h, ws[: nb // 2])
    finally:
        P.sdi_problem_destroy(h)


def test_integrate_with_vegas_warmup(ctx):
    prob = sectorgen.config2()
    prob.sectors = prob.sectors[:8]
    m, R, mw, nb, W = 10, 4, 10, 32, 3
    set_params(ctx, lattice_log2=m, shifts=R, seed=4, warmup=W, warmup_log2=mw, nbins=nb)
    h = P.sdi_problem_create(ctx, prob)
    try:
        P.sdi_integrate(ctx, h)
        lead, pref = integrate.prefactor_for(prob)
        for s in range(8):
            est = integrate.integrate_sector(prob, s, m, R, 4, lead, pref, True, nb, W, mw)
            _, _, per, _ = P.sdi_sector_results(ctx, h, s, R)
            # grids are refit from floating histograms summed in different orders, so
            # the points differ by a few ulp: compare at 1e-9 of the absolute scale
            oq, scale = oracle_shift_values(prob, s, m, R, 4, grid=est.grid)
            assert np.allclose(oq, est.q, rtol=0, atol=1e-300 + 1e-14 * scale.max())
            tol = 1e-9 * np.maximum(np.abs(oq), scale[None, :])
            assert np.all(np.abs(per - oq) <= tol), s
            x, w = P.sdi_sample_points(ctx, h, s, 1, 0, 256, prob.sectors[s].n)
            ox, ow, _ = points.sector_points(points.cbc_vector(m, prob.sectors[s].n), m,
                                             points.shift_table(4, s, R, prob.sectors[s].n, m)[1], 0, 256,
                                             est.grid, True)
            assert np.allclose(x.cpu().numpy(), ox, rtol=1e-12, atol=1e-15)
            assert np.allclose(w.cpu().numpy(), ow, rtol=1e-11)
    finally:
        P.sdi_problem_destroy(h)


def test_full_size_sampled_sectors(ctx):
    """The bench workload (64 sectors, 2^16 points x 16 shifts): sampled sectors against the oracle."""
    prob = sectorgen.config2()
    m, R = 16, 16
    set_params(ctx, lattice_log2=m, shifts=R, seed=1, tile_log2=14)
    h = P.sdi_problem_create(ctx, prob)
    try:
        res = P.sdi_integrate(ctx, h)
        assert res["status"] == 0 and res["n_evals"] == 64 * R << m
        for s in (0, 31, 63):
            _, _, per, _ = P.sdi_sector_results(ctx, h, s, R)
            oq, scale = oracle_shift_values(prob, s, m, R, 1)
            assert_close_shift(per, oq, scale, f"full-size sector {s}")
    finally:
        P.sdi_problem_destroy(h)


def test_errors_are_reported(ctx):
    with pytest.raises(P.SdiError):
        P.sdi_set_param(ctx, "lattice_log2", "99")
    with pytest.raises(P.SdiError):
        P.sdi_set_param(ctx, "no_such_key", "1")
    prob = sectorgen.config1()
    # a_j < -1 without an eps part (b_j = 0) has no analytic continuation to reduce
    bad = sectorgen.Problem(sectors=[sectorgen.Sector(a=np.array([-2.0]), b=np.array([0.0]), factors=[])],
                            order_min=0, order_max=0)
    with pytest.raises(P.SdiError) as ei:
        P.sdi_problem_create(ctx, bad)
    assert ei.value.code == -1
    set_params(ctx)
    h = P.sdi_problem_create(ctx, prob)
    try:
        with pytest.raises(P.SdiError):
            P.sdi_sector_results(ctx, h, 0, 4)
        with pytest.raises(P.SdiError):
            P.sdi_evaluate(ctx, h, 5, torch.zeros((4, 1), dtype=torch.float64, device="cuda"))
    finally:
        P.sdi_problem_destroy(h)


def test_graph_replays_match_eager(ctx):
    """The captured pass replayed several times, with eager torch work and syncs in between,
    gives exactly the eager result every time (no warm-up: fully deterministic sums)."""
    prob = sectorgen.config2()
    set_params(ctx, lattice_log2=11, shifts=4, seed=21, graph=0)
    h = P.sdi_problem_create(ctx, prob)
    try:
        eager = P.sdi_integrate(ctx, h)
        per_e = [P.sdi_sector_results(ctx, h, s, 4)[2] for s in range(0, 64, 7)]
        P.sdi_set_param(ctx, "graph", 1)
        for rep in range(4):
            junk = torch.randn(4096, device="cuda").mul_(3.0).sum().item()
            torch.cuda.synchronize()
            g = P.sdi_integrate(ctx, h)
            assert g["ms_eval_kernel"] > 0 and g["ms_total"] >= g["ms_eval_kernel"]
            assert np.array_equal(g["value"], eager["value"]), rep
            assert np.array_equal(g["err_re"], eager["err_re"]), rep
            per_g = [P.sdi_sector_results(ctx, h, s, 4)[2] for s in range(0, 64, 7)]
            for a, b in zip(per_e, per_g):
                assert np.array_equal(a, b)
            assert np.isfinite(junk)
    finally:
        P.sdi_problem_destroy(h)
        P.sdi_set_param(ctx, "graph", 1)


def test_graph_with_warmup_matches_eager(ctx):
    prob = sectorgen.config2()
    prob.sectors = prob.sectors[:16]
    set_params(ctx, lattice_log2=10, shifts=4, seed=2, warmup=3, warmup_log2=10, nbins=64, graph=0)
    h = P.sdi_problem_create(ctx, prob)
    try:
        eager = P.sdi_integrate(ctx, h)
        P.sdi_set_param(ctx, "graph", 1)
        for rep in range(3):
            torch.cuda.synchronize()
            g = P.sdi_integrate(ctx, h)
            scale = np.abs(eager["value"]) + 1e-300
            assert np.all(np.abs(g["value"] - eager["value"]) <= 1e-12 * scale), rep
    finally:
        P.sdi_problem_destroy(h)
        P.sdi_set_param(ctx, "graph", 1)
        P.sdi_set_param(ctx, "warmup", 0)


def test_budget_allocation_matches_oracle(ctx):
    """Pilot pass, variance-driven lattice sizes, final pass: sizes equal the oracle's rule
    applied to the oracle's own pilot, and the final per-shift means agree."""
    prob = sectorgen.config2()
    prob.sectors = prob.sectors[:12]
    R, pilot, lo, hi = 4, 8, 6, 12
    budget = 12 * R * (1 << 9)
    set_params(ctx, shifts=R, seed=31, budget=budget, pilot_log2=pilot, alloc_min_log2=lo, alloc_max_log2=hi)
    h = P.sdi_problem_create(ctx, prob)
    try:
        res = P.sdi_integrate(ctx, h)
        lead, pref = integrate.prefactor_for(prob)
        est = [integrate.integrate_sector(prob, s, pilot, R, 31, lead, pref) for s in range(12)]
        m_or = integrate.neyman_allocation(est, budget, R, lo, hi)
        m_gpu = []
        for s in range(12):
            _, _, per, nev = P.sdi_sector_results(ctx, h, s, R)
            m_gpu.append(int(nev // R).bit_length() - 1)
            if s % 4 == 0:
                oq, scale = oracle_shift_values(prob, s, m_or[s], R, 31)
                assert_close_shift(per, oq, scale, f"allocated sector {s}")
        assert m_gpu == m_or
        assert len(set(m_gpu)) > 1                      # the allocation is not uniform
        assert res["n_evals"] == sum(R << m for m in m_gpu) + 12 * (R << pilot)
    finally:
        P.sdi_problem_destroy(h)
        P.sdi_set_param(ctx, "budget", 0)
