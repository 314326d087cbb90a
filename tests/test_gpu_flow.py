"""GPU parity of the learned sampler (coupling flow) against the flow oracle.

Bars:
* initial parameters and one Adam step: bit-exact (the same Philox draws and
  the same fp64-then-fp32 roundings);
* sampling x(u) and log q: the network runs in bf16 with fp32 accumulation on
  the GPU and with fp64 accumulation in the oracle, so a hidden activation can
  land on the other side of a bf16 rounding boundary (relative change 2^-8 of
  that unit), while fp32 softmax against fp64 moves the bin probabilities by
  ~1e-7 relative.  Bar: |dx| <= 1e-7 and |d log q| <= 1e-6 for 99% of the
  points, |dx| <= 1e-3 for all (x is continuous in the bin probabilities);
  log q may jump where a point sits on a bin edge.  At the identity initialisation the
  map is exact: x = u, log q = 0;
* gradient: the back-propagated operands are rounded to bf16 before each
  matrix product and the sums over samples run in fp32, so each gradient
  element carries a relative error of order 2^-9 sqrt(terms) / cancellation.
  Bar per parameter tensor: ||g_gpu - g_oracle|| <= 1e-2 ||g_oracle||;
* a pass with the flow sampler: per (sector, shift) means equal the oracle's
  integrand averaged over the flow hook's own points and weights (1e-10, the
  evaluation bar), i.e. the pass uses exactly the map the hook exposes.
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
from oracle import flow, integrand, integrate, points  # noqa: E402

from test_gpu_parity import assert_close_shift, log, oracle_shift_values, set_params  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    c = P.sdi_ctx_create(0)
    yield c
    P.sdi_ctx_destroy(c)


def flatten(params):
    return np.concatenate([d[k].numpy().ravel() for d in params for k in ("W1", "b1", "W2", "b2", "W3", "b3")])


def unflatten(vec, n):
    out, off = [], 0
    for shp in flow.layer_shapes(n):
        d = {}
        for name, shape in shp:
            size = int(np.prod(shape))
            d[name] = torch.tensor(vec[off:off + size].astype(np.float64).reshape(shape))
            off += size
        out.append(d)
    assert off == vec.size
    return out


def random_fp32_params(n, seed, scale=0.6):
    P0 = flow.init_params(n, seed, 0)
    g = np.random.default_rng(seed)
    v = flatten(P0)
    v = (v + scale * g.standard_normal(v.size) / 8.0).astype(np.float32)
    return v


def problem_with_dims(dims):
    """Sectors of the given dimensions (no singular variables) from the synthetic generator."""
    secs = []
    for i, n in enumerate(dims):
        s = sectorgen.synthetic_sectors(100 + i, 1, (n, n), (4, 8), (0, 0))[0]
        secs.append(s)
    return sectorgen.Problem(sectors=secs, order_min=0, order_max=1)


def lattice_latent(n, m, seed, s=0, r=0, baker=True):
    z = points.cbc_vector(m, n)
    sh = points.shift_table(seed, s, r + 1, n, m)[r]
    x, _, _ = points.sector_points(z, m, sh, 0, 1 << m, None, baker)
    return x


def test_flow_init_matches_oracle_bit_exact(ctx):
    prob = problem_with_dims([1, 2, 3, 6])
    h = P.sdi_problem_create(ctx, prob)
    try:
        P.sdi_flow_init(ctx, h, 77)
        for s, sec in enumerate(prob.sectors):
            g = P.sdi_flow_params(ctx, h, s)
            o = flatten(flow.init_params(sec.n, 77, s)).astype(np.float32)
            assert g.size == o.size
            assert np.array_equal(g.view(np.uint32), o.view(np.uint32)), s
    finally:
        P.sdi_problem_destroy(h)


def test_identity_map_is_exact(ctx):
    prob = problem_with_dims([3])
    h = P.sdi_problem_create(ctx, prob)
    try:
        P.sdi_flow_init(ctx, h, 5)
        u = lattice_latent(3, 10, 4)
        x, lq = P.sdi_flow_sample(ctx, h, 0, torch.from_numpy(u).cuda())
        assert np.array_equal(x.cpu().numpy(), u)
        assert np.all(lq.cpu().numpy() == 0.0)
    finally:
        P.sdi_problem_destroy(h)


@pytest.mark.parametrize("n,npts", [(1, 1000), (2, 4096), (3, 777), (6, 2048), (9, 1100), (13, 512)])
def test_flow_sample_matches_oracle(ctx, n, npts):
    prob = problem_with_dims([n])
    h = P.sdi_problem_create(ctx, prob)
    try:
        P.sdi_flow_init(ctx, h, 1)
        v = random_fp32_params(n, 10 + n)
        P.sdi_flow_set_params(ctx, h, 0, v)
        assert np.array_equal(P.sdi_flow_params(ctx, h, 0), v)
        u = lattice_latent(n, 12, 3)[:npts]
        x, lq = P.sdi_flow_sample(ctx, h, 0, torch.from_numpy(u).cuda())
        x, lq = x.cpu().numpy(), lq.cpu().numpy()
        ox, olq = flow.sample(unflatten(v, n), u)
        dx = np.abs(x - ox).max(axis=1)
        dl = np.abs(lq - olq)
        log(f"n={n}: max dx {dx.max():.3e}, 99% dx {np.quantile(dx, 0.99):.3e}, "
            f"max dlq {dl.max():.3e}, 99% dlq {np.quantile(dl, 0.99):.3e}")
        assert np.all((x >= 0) & (x <= 1))
        assert np.mean(dx <= 1e-7) >= 0.99 and np.mean(dl <= 1e-6) >= 0.99
        assert dx.max() <= 1e-3
        assert not np.array_equal(x, u)     # the map is not the identity
    finally:
        P.sdi_problem_destroy(h)


@pytest.mark.parametrize("n,npts", [(1, 300), (2, 1000), (3, 2048), (5, 4096), (9, 1500)])
def test_flow_gradient_matches_oracle(ctx, n, npts):
    prob = problem_with_dims([n])
    h = P.sdi_problem_create(ctx, prob)
    try:
        P.sdi_flow_init(ctx, h, 1)
        v = random_fp32_params(n, 20 + n)
        P.sdi_flow_set_params(ctx, h, 0, v)
        rng = np.random.default_rng(n)
        x = rng.uniform(0.0, 1.0, size=(npts, n))
        c = rng.uniform(0.0, 1.0, size=npts) / npts
        g = P.sdi_flow_grad(ctx, h, 0, torch.from_numpy(x).cuda(), torch.from_numpy(c).cuda())
        _, G = flow.loss_and_grad(unflatten(v, n), x, c)
        og = flatten(G)
        off = 0
        worst = 0.0
        for l, shp in enumerate(flow.layer_shapes(n)):
            for name, shape in shp:
                size = int(np.prod(shape))
                a, b = g[off:off + size].astype(np.float64), og[off:off + size]
                off += size
                nb = np.linalg.norm(b)
                if nb == 0.0:
                    assert np.all(a == 0.0), (l, name)
                    continue
                rel = np.linalg.norm(a - b) / nb
                worst = max(worst, rel)
                assert rel <= 1e-2, (l, name, rel)
        log(f"n={n}: worst tensor relative gradient error {worst:.3e}")
    finally:
        P.sdi_problem_destroy(h)


def test_adam_step_bit_exact(ctx):
    prob = problem_with_dims([3, 2])
    h = P.sdi_problem_create(ctx, prob)
    try:
        P.sdi_flow_init(ctx, h, 1)
        states, params = [], []
        for s, sec in enumerate(prob.sectors):
            v = random_fp32_params(sec.n, 30 + s)
            P.sdi_flow_set_params(ctx, h, s, v)
            params.append(unflatten(v, sec.n))
            states.append(flow.adam_init(params[-1]))
        rng = np.random.default_rng(3)
        for step in range(3):
            for s, sec in enumerate(prob.sectors):
                gv = (rng.standard_normal(P.sdi_flow_nparams(h, s)) * 10.0 ** rng.integers(-6, 1)).astype(np.float32)
                gv[rng.random(gv.size) < 0.05] = 0.0
                P.sdi_flow_set_grad(ctx, h, s, gv)
                flow.adam_step(params[s], unflatten(gv, sec.n), states[s], lr=1e-3)
            P.sdi_flow_adam(ctx, h, 1e-3)
            for s, sec in enumerate(prob.sectors):
                g = P.sdi_flow_params(ctx, h, s)
                o = flatten(params[s]).astype(np.float32)
                assert np.array_equal(g.view(np.uint32), o.view(np.uint32)), (step, s)
        # the Adam step leaves the bf16 weight copies current: sampling after it equals
        # sampling after the copies are rebuilt from the same parameters
        for s, sec in enumerate(prob.sectors):
            u = torch.from_numpy(lattice_latent(sec.n, 10, 3)).cuda()
            x1, lq1 = P.sdi_flow_sample(ctx, h, s, u)
            P.sdi_flow_set_params(ctx, h, s, P.sdi_flow_params(ctx, h, s))
            x2, lq2 = P.sdi_flow_sample(ctx, h, s, u)
            assert torch.equal(x1, x2) and torch.equal(lq1, lq2), s
    finally:
        P.sdi_problem_destroy(h)


def peaked_sector(e0=0.003):
    """2-D sector whose integrand peaks sharply near (0.2, 0.7): 1 / (e0 + |x - p|^2)^2.

    With e0 = 0.003 the peak (width ~0.05) is narrow enough that 2^10 lattice
    points per shift resolve it poorly, the regime an adapted map is for; on
    smooth integrands the tent-transformed lattice converges faster than any
    piecewise-linear map allows."""
    # (e0 + (x-0.2)^2 + (y-0.7)^2) expanded as a polynomial, raised to the power -2
    c = np.array([e0 + 0.04 + 0.49, -0.4, 1.0, -1.4, 1.0])
    e = np.array([[0, 0], [1, 0], [2, 0], [0, 1], [0, 2]], dtype=np.uint8)
    return Sector(a=np.zeros(2), b=np.zeros(2), factors=[Factor(-2.0, 0.0, c, e)])


def test_flow_pass_uses_the_hook_map(ctx):
    """Sectors 0 and 2 sample through their flows, sector 1 (inactive) stays on the lattice."""
    prob = sectorgen.Problem(sectors=[peaked_sector(), problem_with_dims([4]).sectors[0],
                                      problem_with_dims([3]).sectors[0]], order_min=0, order_max=0)
    m, R = 10, 4
    set_params(ctx, lattice_log2=m, shifts=R, seed=7, sampler=1)
    h = P.sdi_problem_create(ctx, prob)
    try:
        P.sdi_flow_init(ctx, h, 3)
        for s in (0, 2):
            P.sdi_flow_set_params(ctx, h, s, random_fp32_params(prob.sectors[s].n, 40 + s))
        res = P.sdi_integrate(ctx, h)
        assert res["status"] == 0
        lead, pref = integrate.prefactor_for(prob)
        _, _, per, _ = P.sdi_sector_results(ctx, h, 1, R)
        oq, scale = oracle_shift_values(prob, 1, m, R, 7)
        assert_close_shift(per, oq, scale, "lattice sector in a flow pass")
        for s in (0, 2):
            sec = prob.sectors[s]
            _, _, per, _ = P.sdi_sector_results(ctx, h, s, R)
            z = points.cbc_vector(m, sec.n)
            sh = points.shift_table(7, s, R, sec.n, m)
            for r in range(R):
                u, _, _ = points.sector_points(z, m, sh[r], 0, 1 << m, None, True)
                x, lq = P.sdi_flow_sample(ctx, h, s, torch.from_numpy(u).cuda())
                x, w = x.cpu().numpy(), np.exp(-lq.cpu().numpy())
                vals, _, _ = integrand.sector_orders(sec, x, prob.order_min, prob.order_max, lead, pref)
                wf = vals * w[None, :]
                for k in range(prob.norders):
                    q = integrate.fsum_c(wf[k]) / (1 << m)
                    scale = float(np.mean(np.abs(wf[k])))
                    assert abs(per[r, k] - q) <= 1e-10 * max(abs(q), scale), (s, r, k)
    finally:
        P.sdi_problem_destroy(h)
        set_params(ctx)


def test_training_on_gpu_lowers_the_variance(ctx):
    """The trained map's shift-to-shift error on the peaked sector falls well below plain QMC's."""
    prob = sectorgen.Problem(sectors=[peaked_sector()], order_min=0, order_max=0)
    m, R = 10, 16
    h = P.sdi_problem_create(ctx, prob)
    try:
        set_params(ctx, lattice_log2=m, shifts=R, seed=11, sampler=0)
        plain = P.sdi_integrate(ctx, h)
        P.sdi_flow_init(ctx, h, 2)
        ms = P.sdi_flow_train(ctx, h, 60, 11, 5e-3)
        p1 = P.sdi_flow_params(ctx, h, 0)
        set_params(ctx, lattice_log2=m, shifts=R, seed=11, sampler=1)
        learned = P.sdi_integrate(ctx, h)
        log(f"plain {plain['value'][0].real:.8f} +- {plain['err_re'][0]:.2e}; "
            f"flow {learned['value'][0].real:.8f} +- {learned['err_re'][0]:.2e}; training {ms:.2f} ms")
        assert learned["err_re"][0] < 0.5 * plain["err_re"][0]
        diff = abs(learned["value"][0].real - plain["value"][0].real)
        assert diff < 5 * math.hypot(learned["err_re"][0], plain["err_re"][0])
        # training is deterministic
        P.sdi_flow_init(ctx, h, 2)
        P.sdi_flow_train(ctx, h, 60, 11, 5e-3)
        assert np.array_equal(P.sdi_flow_params(ctx, h, 0), p1)
    finally:
        P.sdi_problem_destroy(h)
        set_params(ctx)


def test_training_a_subset_leaves_the_rest(ctx):
    prob = sectorgen.Problem(sectors=[peaked_sector(), problem_with_dims([3]).sectors[0]], order_min=0, order_max=0)
    h = P.sdi_problem_create(ctx, prob)
    try:
        set_params(ctx, seed=11)
        P.sdi_flow_init(ctx, h, 2)
        before = [P.sdi_flow_params(ctx, h, s) for s in range(2)]
        P.sdi_flow_train(ctx, h, 5, 9, 5e-3, sectors=[0])
        assert not np.array_equal(P.sdi_flow_params(ctx, h, 0), before[0])
        assert np.array_equal(P.sdi_flow_params(ctx, h, 1), before[1])
        with pytest.raises(P.SdiError):
            P.sdi_flow_train(ctx, h, 5, 9, 5e-3, sectors=[0, 0])
        # a pass with the flow sampler: sector 1 is inactive, so it matches the plain lattice pass
        m, R = 10, 4
        set_params(ctx, lattice_log2=m, shifts=R, seed=11, sampler=1)
        P.sdi_integrate(ctx, h)
        _, _, per_flow, _ = P.sdi_sector_results(ctx, h, 1, R)
        set_params(ctx, lattice_log2=m, shifts=R, seed=11, sampler=0)
        P.sdi_integrate(ctx, h)
        _, _, per_plain, _ = P.sdi_sector_results(ctx, h, 1, R)
        assert np.allclose(per_flow, per_plain, rtol=1e-12, atol=0.0)
    finally:
        P.sdi_problem_destroy(h)
        set_params(ctx)


def test_validation_keeps_only_flows_that_help(ctx):
    """sdi_flow_validate's kept flags equal the criterion recomputed from the two passes'
    per-sector results: with S_k = max(|I_k|^2, V_k) from the lattice pass, a flow
    stays where sum_k var_flow(s,k)/S_k < sum_k var_lattice(s,k)/S_k and every
    order's two estimates agree within 5 combined standard errors.  The trained flow
    of the peaked sector stays; flows with random weights on smooth sectors go."""
    smooth = [problem_with_dims([3]).sectors[0], problem_with_dims([4]).sectors[0]]
    prob = sectorgen.Problem(sectors=[peaked_sector()] + smooth, order_min=0, order_max=0)
    m, R = 10, 16
    h = P.sdi_problem_create(ctx, prob)
    try:
        set_params(ctx, lattice_log2=m, shifts=R, seed=5)
        P.sdi_flow_init(ctx, h, 4)
        P.sdi_flow_train(ctx, h, 60, 11, 5e-3, sectors=[0])
        P.sdi_flow_set_params(ctx, h, 1, random_fp32_params(smooth[0].n, 9, scale=2.0))
        P.sdi_flow_set_params(ctx, h, 2, random_fp32_params(smooth[1].n, 10, scale=40.0))
        passes = []
        for sampler in (0, 1):
            set_params(ctx, lattice_log2=m, shifts=R, seed=5, sampler=sampler)
            P.sdi_integrate(ctx, h)
            passes.append([P.sdi_sector_results(ctx, h, s, R) for s in range(3)])
        set_params(ctx, lattice_log2=m, shifts=R, seed=5, sampler=0)
        kept, ms = P.sdi_flow_validate(ctx, h, m)
        mean = [np.array([passes[p][s][0] for s in range(3)]) for p in (0, 1)]   # [sector][order]
        var = [np.array([np.sum(passes[p][s][1] ** 2, axis=1) for s in range(3)]) for p in (0, 1)]
        S = np.maximum(np.abs(mean[0].sum(axis=0)) ** 2, var[0].sum(axis=0))
        want = []
        for s in range(3):
            better = (var[1][s] / S).sum() < (var[0][s] / S).sum()
            agree = bool(np.all(np.abs(mean[1][s] - mean[0][s]) ** 2 <= 25.0 * (var[0][s] + var[1][s])))
            log(f"sector {s}: lattice {mean[0][s]} +- {np.sqrt(var[0][s])}, flow {mean[1][s]} +- {np.sqrt(var[1][s])}")
            want.append(better and agree)
        log(f"validation: kept {list(kept)}, criterion {want}, {ms:.2f} ms")
        assert [bool(k) for k in kept] == want
        assert want == [True, False, False]
    finally:
        P.sdi_problem_destroy(h)
        set_params(ctx)


def test_validation_order_weights(ctx):
    """With order weights the kept flags follow the weighted criterion, recomputed here
    from the two passes for weights (1, 0), (0, 1) and (1, 1) on a two-order problem."""
    secs = [problem_with_dims([3]).sectors[0], problem_with_dims([4]).sectors[0]]
    prob = sectorgen.Problem(sectors=secs, order_min=0, order_max=1)
    m, R = 9, 16
    h = P.sdi_problem_create(ctx, prob)
    try:
        for weights in ([1.0, 0.0], [0.0, 1.0], [1.0, 1.0]):
            set_params(ctx, lattice_log2=m, shifts=R, seed=6)
            P.sdi_flow_init(ctx, h, 5)
            P.sdi_flow_set_params(ctx, h, 0, random_fp32_params(secs[0].n, 21, scale=0.8))
            P.sdi_flow_set_params(ctx, h, 1, random_fp32_params(secs[1].n, 22, scale=0.8))
            passes = []
            for sampler in (0, 1):
                set_params(ctx, lattice_log2=m, shifts=R, seed=6, sampler=sampler)
                P.sdi_integrate(ctx, h)
                passes.append([P.sdi_sector_results(ctx, h, s, R) for s in range(2)])
            set_params(ctx, lattice_log2=m, shifts=R, seed=6, sampler=0)
            kept, _ = P.sdi_flow_validate(ctx, h, m, order_weights=weights)
            mean = [np.array([passes[p][s][0] for s in range(2)]) for p in (0, 1)]
            var = [np.array([np.sum(passes[p][s][1] ** 2, axis=1) for s in range(2)]) for p in (0, 1)]
            S = np.maximum(np.abs(mean[0].sum(axis=0)) ** 2, var[0].sum(axis=0))
            w = np.array(weights)
            want = []
            for s in range(2):
                better = (w * var[1][s] / S).sum() < (w * var[0][s] / S).sum()
                agree = bool(np.all(np.abs(mean[1][s] - mean[0][s]) ** 2 <= 25.0 * (var[0][s] + var[1][s])))
                want.append(bool(better and agree))
            log(f"weights {weights}: kept {list(kept)}, criterion {want}")
            assert [bool(k) for k in kept] == want
        with pytest.raises(ValueError):
            P.sdi_flow_validate(ctx, h, m, order_weights=[1.0])
        with pytest.raises(P.SdiError):
            P.sdi_flow_validate(ctx, h, m, order_weights=[-1.0, 1.0])
    finally:
        P.sdi_problem_destroy(h)
        set_params(ctx)


def test_learned_double_box_agrees_with_lattice(ctx):
    """End to end on the Euclidean double box (282 sectors): flows trained for the sectors
    with the largest errors, validated, then a mixed pass.  Every order agrees with a
    large lattice pass within 5 combined standard errors, and the eps^0 error at the
    same points per shift is smaller than the lattice's."""
    from sectorgen.feynman import double_box_problem
    prob = double_box_problem(-3.0, -1.0, 0.0, order_max=0)
    h = P.sdi_problem_create(ctx, prob)
    try:
        set_params(ctx, lattice_log2=16, shifts=16, seed=1)
        ref = P.sdi_integrate(ctx, h)
        set_params(ctx, lattice_log2=11, shifts=16, seed=1)
        pilot = P.sdi_integrate(ctx, h)
        err = np.array([np.hypot(*P.sdi_sector_results(ctx, h, s, 16)[1][-1]) for s in range(len(prob.sectors))])
        sel = sorted(int(s) for s in np.argsort(-err)[:16])
        P.sdi_flow_init(ctx, h, 1)
        P.sdi_flow_train(ctx, h, 20, 11, 6e-3, sectors=sel)
        kept, _ = P.sdi_flow_validate(ctx, h, 11)
        set_params(ctx, lattice_log2=13, shifts=16, seed=1, sampler=1)
        learned = P.sdi_integrate(ctx, h)
        set_params(ctx, lattice_log2=13, shifts=16, seed=1, sampler=0)
        plain = P.sdi_integrate(ctx, h)
        e_l = np.hypot(learned["err_re"], learned["err_im"])
        e_r = np.hypot(ref["err_re"], ref["err_im"])
        log(f"kept {int(kept.sum())}/{len(sel)}; eps^0: learned {learned['value'][-1].real:.5f} +- {e_l[-1]:.2e}, "
            f"lattice 2^13 +- {np.hypot(plain['err_re'], plain['err_im'])[-1]:.2e}, "
            f"lattice 2^16 {ref['value'][-1].real:.5f} +- {e_r[-1]:.2e}")
        assert kept.sum() >= len(sel) // 2
        for k in range(prob.norders):
            d = abs(learned["value"][k] - ref["value"][k])
            assert d <= 5.0 * math.hypot(e_l[k], e_r[k]) + 1e-12, (k, d, e_l[k], e_r[k])
        assert e_l[-1] < np.hypot(plain["err_re"], plain["err_im"])[-1]
    finally:
        P.sdi_problem_destroy(h)
        set_params(ctx)


@pytest.mark.parametrize("n,npts", [(2, 1000), (5, 4096), (9, 1500)])
def test_flow_gradient_elementwise(ctx, n, npts):
    """Every gradient element against the oracle's: |gpu - oracle| <= 5e-2 |oracle|
    + 2e-2 rms(tensor).  The GPU rounds each back-propagated operand to bf16
    (relative 2^-9) and sums in fp32 while the oracle keeps fp64 between its
    own bf16 roundings (straight-through, the same as the GPU's), so an element,
    a sum over the batch of products, carries bf16 roundings of each product:
    relative to the element where the products do not cancel, and a random
    walk of roundings over the batch where they do, which the tensor's scale
    bounds (measured: up to 9e-3 rms for 4096 samples).  A wrong, missing or
    misplaced contribution is of the order of the tensor's scale."""
    prob = problem_with_dims([n])
    h = P.sdi_problem_create(ctx, prob)
    try:
        P.sdi_flow_init(ctx, h, 1)
        v = random_fp32_params(n, 40 + n)
        P.sdi_flow_set_params(ctx, h, 0, v)
        rng = np.random.default_rng(100 + n)
        x = rng.uniform(0.0, 1.0, size=(npts, n))
        c = rng.uniform(0.0, 1.0, size=npts) / npts
        g = P.sdi_flow_grad(ctx, h, 0, torch.from_numpy(x).cuda(), torch.from_numpy(c).cuda())
        _, G = flow.loss_and_grad(unflatten(v, n), x, c)
        og = flatten(G)
        off = 0
        q = []
        for l, shp in enumerate(flow.layer_shapes(n)):
            for name, shape in shp:
                size = int(np.prod(shape))
                a, b = g[off:off + size].astype(np.float64), og[off:off + size]
                off += size
                rms = float(np.sqrt(np.mean(b ** 2)))
                if rms == 0.0:
                    assert np.all(a == 0.0), (l, name)
                    continue
                d = np.abs(a - b)
                tol = 5e-2 * np.abs(b) + 2e-2 * rms
                assert np.all(d <= tol), (l, name, float(np.max(d / tol)))
                q.append(float(np.max(d / tol)))
        log(f"n={n}: largest element error {max(q):.3f} of its bound")
    finally:
        P.sdi_problem_destroy(h)
