"""Pins of the oracle's adaptive cubature (oracle/cubature.py): the rule pair's
polynomial degrees on the cube and on dyadic boxes of a sector, the split
axis on integrands that vary along one axis, the dyadic region bookkeeping,
and whole adaptive runs against closed forms (the one-loop bubble and the
paper's box example of section 4.3)."""
import itertools
import math

import numpy as np
import pytest

import sectorgen
from sectorgen import Factor, Problem, Sector
from oracle import cubature


def mono_mean(alpha):
    """Mean of x^alpha over [-1, 1]^n."""
    v = 1.0
    for a in alpha:
        v *= 0.0 if a % 2 else 1.0 / (a + 1)
    return v


def rule_mean(n, alpha, deg7=True):
    xi, cls = cubature.nodes(n)
    w7, w5 = cubature.weights(n)
    w = np.array([(w7 if deg7 else w5)[c] for c in cls])
    return float(np.sum(w * np.prod(xi ** np.array(alpha)[None, :], axis=1)))


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6])
def test_rule_degrees_all_monomials(n):
    xi, _ = cubature.nodes(n)
    assert len(xi) == cubature.npoints(n)
    worst7 = worst5 = 0.0
    deg6_miss = False
    for deg in range(8):
        for alpha in itertools.product(range(deg + 1), repeat=n):
            if sum(alpha) != deg:
                continue
            worst7 = max(worst7, abs(rule_mean(n, alpha) - mono_mean(alpha)))
            e5 = abs(rule_mean(n, alpha, False) - mono_mean(alpha))
            if deg <= 5:
                worst5 = max(worst5, e5)
            elif deg == 6 and e5 > 1e-6:
                deg6_miss = True
    assert worst7 < 1e-14 and worst5 < 1e-14
    assert deg6_miss                       # the embedded rule is of degree 5 exactly


@pytest.mark.parametrize("n", [7, 8, 9])
def test_rule_degrees_sampled_monomials(n):
    rng = np.random.default_rng(n)
    for _ in range(40):
        alpha = np.zeros(n, dtype=int)
        for _ in range(int(rng.integers(0, 8))):
            alpha[rng.integers(0, n)] += 1
        assert abs(rule_mean(n, alpha) - mono_mean(alpha)) < 1e-13
    # the corner class matters: x1^2 x2^2 x3^2 ... needs the 2^n corner points
    alpha = [2, 2, 2] + [0] * (n - 3)
    assert abs(rule_mean(n, alpha) - mono_mean(alpha)) < 1e-13


def poly_problem(coef, exps):
    """A one-factor sector whose integrand is the polynomial itself (exponent 1, no eps)."""
    n = exps.shape[1]
    sec = Sector(a=np.zeros(n), b=np.zeros(n),
                 factors=[Factor(1.0, 0.0, np.asarray(coef, float), np.asarray(exps, np.uint8))])
    return Problem(sectors=[sec], order_min=0, order_max=0, pref_lead=0, pref=np.ones(1, complex))


def box_integral(coef, exps, lo, hi):
    tot = 0.0
    for c, e in zip(coef, exps):
        t = c
        for j, a in enumerate(e):
            t *= (hi[j] ** (a + 1) - lo[j] ** (a + 1)) / (a + 1)
        tot += t
    return tot


def test_rule_on_dyadic_boxes_of_a_sector():
    rng = np.random.default_rng(3)
    n = 3
    exps = np.array([[0, 0, 0], [2, 1, 0], [0, 3, 3], [1, 1, 1], [7, 0, 0], [0, 2, 4]], dtype=np.uint8)
    coef = rng.uniform(0.2, 1.0, len(exps))
    prob = poly_problem(coef, exps)
    for level, index in (([0, 0, 0], [0, 0, 0]), ([1, 2, 0], [1, 3, 0]), ([3, 1, 2], [5, 0, 2])):
        r = cubature.Region(0, np.array(level), np.array(index))
        cubature.apply_rule(prob, r, 0, [1.0], np.ones(1))
        lo = np.array(index) * 2.0 ** -np.array(level, float)
        hi = lo + 2.0 ** -np.array(level, float)
        assert r.value[0].real == pytest.approx(box_integral(coef, exps, lo, hi), rel=1e-13)
        # degree 7 > 5: the pair disagrees, and the estimate is of the size of the degree-6/7 part
        assert r.err_re[0] > 0.0 and r.err_im[0] == 0.0
    # a degree-5 integrand: both rules exact, no error
    p5 = poly_problem([1.0, 0.5, 0.25], np.array([[0, 0, 0], [2, 3, 0], [1, 1, 1]], dtype=np.uint8))
    r = cubature.apply_rule(p5, cubature.Region(0, np.zeros(3, int), np.zeros(3, int)), 0, [1.0], np.ones(1))
    assert r.err_re[0] < 1e-15
    assert r.value[0].real == pytest.approx(1.0 + 0.5 / 12 + 0.25 / 8, rel=1e-14)


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_split_axis_follows_the_fourth_difference(axis):
    e = np.zeros((2, 3), dtype=np.uint8)
    e[1, axis] = 6                                           # 1 + x_axis^6: quartic part only along axis
    prob = poly_problem([1.0, 1.0], e)
    r = cubature.apply_rule(prob, cubature.Region(0, np.zeros(3, int), np.zeros(3, int)), 0, [1.0], np.ones(1))
    assert r.axis == axis
    # ties go to the lowest index: x1^6 + x2^6 + x3^6 is symmetric
    sym = poly_problem([1.0, 1.0, 1.0], np.array([[6, 0, 0], [0, 6, 0], [0, 0, 6]], dtype=np.uint8))
    r = cubature.apply_rule(sym, cubature.Region(0, np.zeros(3, int), np.zeros(3, int)), 0, [1.0], np.ones(1))
    assert r.axis == 0


def test_coarse_rounding():
    assert cubature.coarse(1.0) == 1.0
    assert cubature.coarse(1.0 + 2.0 ** -9) == 1.0                     # below the half step
    assert cubature.coarse(1.0 + 2.0 ** -8) == 1.0 + 2.0 ** -7          # half step rounds up
    assert cubature.coarse(1.0 + 2.0 ** -8 - 2.0 ** -40) == 1.0
    assert cubature.coarse(255.0) == 255.0 and cubature.coarse(255.5) == 256.0
    assert cubature.coarse(0.0) == 0.0 and cubature.coarse(float("nan")) == math.inf
    v = np.random.default_rng(1).uniform(0, 1, 1000)
    q = np.array([cubature.coarse(float(t)) for t in v])
    assert np.all(np.abs(q - v) <= v * 2.0 ** -8)
    assert np.all(np.diff(q[np.argsort(v)]) >= 0)           # monotone


def check_tiling(res, problem):
    """Alive regions of each sector cover its cube exactly once (dyadic volumes add to 1
    and no two overlap)."""
    from fractions import Fraction
    for s in range(len(problem.sectors)):
        regs = [r for r in res.regions if r.alive and r.sector == s]
        vol = sum(Fraction(1, 2 ** int(np.sum(r.level))) for r in regs)
        assert vol == 1
        for a, b in itertools.combinations(regs, 2):
            apart = False
            for j in range(len(a.level)):
                la, lb = int(a.level[j]), int(b.level[j])
                m = max(la, lb)
                ia = (int(a.index[j]) << (m - la), (int(a.index[j]) + 1) << (m - la))
                ib = (int(b.index[j]) << (m - lb), (int(b.index[j]) + 1) << (m - lb))
                if ia[1] <= ib[0] or ib[1] <= ia[0]:
                    apart = True
                    break
            assert apart


def test_adaptive_bubble_closed_form():
    """Bubble: 1/eps + 2 + (4 - pi^2/12) eps + (8 - pi^2/6 - 7 zeta(3)/3) eps^2.  A
    budget-limited run's error estimates bound the true errors; a run with a
    reachable tolerance converges within it."""
    prob = sectorgen.config1()
    z3 = 1.2020569031595942
    exact = np.array([1.0, 2.0, 4 - math.pi ** 2 / 12, 8 - math.pi ** 2 / 6 - 7 * z3 / 3])
    res = cubature.cubature(prob, maxeval=20000, epsrel=1e-12, epsabs=0.0, batch_min=4)
    assert not res.converged and res.evals <= 20000
    assert np.all(np.abs(res.value - exact) <= res.err_re + 1e-15)
    assert abs(res.value[3] - exact[3]) < 1e-6
    check_tiling(res, prob)
    res = cubature.cubature(prob, maxeval=20000, epsrel=1e-6, epsabs=0.0, batch_min=4)
    assert res.converged and res.evals < 20000
    assert np.all(res.err_re <= 1e-6 * np.abs(res.value))
    assert np.all(np.abs(res.value - exact) <= 1e-6 * np.abs(exact))


def test_adaptive_box_section_4_3():
    """The paper's box example (S = 3, T = 1): 4/(3 eps^2) - (2 ln 3 / 3)/eps - 4 pi^2 / 9,
    three-variable sectors with logarithmic endpoint behaviour after the subtraction."""
    from sectorgen.feynman import box_problem
    prob = box_problem(3.0, 1.0)
    res = cubature.cubature(prob, maxeval=60000, epsrel=1e-7, epsabs=0.0, batch_min=16)
    exact = [4 / 3, -2 * math.log(3) / 3, -4 * math.pi ** 2 / 9]
    for k, v in enumerate(exact):
        assert abs(res.value[k] - v) <= 3 * res.err_re[k] + 1e-12, (k, res.value[k], v, res.err_re[k])
        assert abs(res.value[k] - v) < 1e-4
    check_tiling(res, prob)
    # more evaluations, smaller error on the order that limits the run
    res2 = cubature.cubature(prob, maxeval=20000, epsrel=1e-7, epsabs=0.0, batch_min=16)
    assert res2.err_re[2] > res.err_re[2]
    assert res2.evals <= 20000 and res.evals <= 60000


def test_batches_take_the_highest_priorities():
    """With batch_min 1 and a tiny split fraction each round halves exactly one
    region: the run allowed k splits equals the run allowed k - 1 splits plus the
    halving of that run's alive region of largest weighted error (older first)."""
    from sectorgen.feynman import box_problem
    prob = box_problem(3.0, 1.0)
    per = 2 * cubature.npoints(3)
    base = len(prob.sectors) * cubature.npoints(3)
    kw = dict(epsrel=1e-14, epsabs=0.0, split_frac=1e-9, batch_min=1)
    prev = cubature.cubature(prob, maxeval=base, **kw)
    assert prev.rounds == 1
    for k in range(1, 6):
        cur = cubature.cubature(prob, maxeval=base + k * per, **kw)
        assert cur.rounds == k + 1 and cur.evals == base + k * per
        alive = [(i, r) for i, r in enumerate(prev.regions) if r.alive]
        total = sum(r.value for _, r in alive)
        omega, _ = cubature.order_weights(total, 1e-14, 0.0)
        pri = [(-cubature.priority(r, omega), i) for i, r in alive]
        want = min(pri)[1]
        assert not cur.regions[want].alive
        assert [r.alive for i, r in enumerate(cur.regions[:len(prev.regions)]) if i != want] == \
            [r.alive for i, r in enumerate(prev.regions) if i != want]
        # the two children halve the parent along its split axis
        a, b = cur.regions[-2:]
        p = prev.regions[want]
        assert a.level[p.axis] == b.level[p.axis] == p.level[p.axis] + 1
        assert (a.index[p.axis], b.index[p.axis]) == (2 * p.index[p.axis], 2 * p.index[p.axis] + 1)
        assert abs(a.value + b.value - p.value).max() <= 10 * (p.err_re + p.err_im).max() + 1e-15
        prev = cur


def test_regions_at_rounding_noise_are_not_halved():
    """A degree-5 integrand is integrated exactly by both rules: its rule
    difference is rounding noise, so no region is ever halved, even with a
    zero tolerance; a degree-7 one is halved."""
    p5 = poly_problem([1.0, 0.5, 0.25], np.array([[0, 0, 0], [2, 3, 0], [1, 1, 1]], dtype=np.uint8))
    res = cubature.cubature(p5, maxeval=10000, epsrel=0.0, epsabs=0.0, batch_min=4)
    assert res.rounds == 1 and not res.converged and len(res.regions) == 1
    r = res.regions[0]
    assert r.err_re[0] <= cubature.NOISE * r.sigma[0]
    assert cubature.priority(r, np.ones(1)) == 0.0
    p7 = poly_problem([1.0, 0.5], np.array([[0, 0, 0], [7, 0, 0]], dtype=np.uint8))
    res = cubature.cubature(p7, maxeval=10000, epsrel=0.0, epsabs=0.0, batch_min=4)
    assert res.rounds > 1 and res.regions[0].axis == 0
    # the rounding scale is the weighted absolute mass times 2^-52
    w7, w5 = cubature.weights(3)
    xi, cls = cubature.nodes(3)
    mass = sum((abs(w7[c]) + abs(w5[c])) * (1.0 + 0.5 * ((1 + x[0]) / 2) ** 7) for x, c in zip(xi, cls))
    assert res.regions[0].sigma[0] == pytest.approx(mass * 2.0 ** -52, rel=1e-12)


def test_suave_oracle_on_the_bubble_and_a_product():
    """The subregion-adaptive Monte Carlo oracle (oracle/suave.py): the bubble's
    closed form within 5 standard errors, regions that tile each cube, and on a
    separable integrand that varies along one variable only the splits follow it."""
    import math
    import sectorgen
    from oracle import suave
    exact = [1.0, 2.0, 4 - math.pi ** 2 / 12]
    r = suave.suave(sectorgen.bubble_problem(order_max=1), 60000, 256, 1e-12, 0.0, 5, 0.25, 4)
    z = (r.value.real - exact) / r.err_re
    assert np.all(np.abs(z) < 5), z
    alive = [g for g in r.regions if g.alive]
    for s in range(2):
        assert sum(math.ldexp(1.0, -int(g.level.sum())) for g in alive if g.sector == s) == 1.0
    # (1 + 9 x_1)^-2 in two variables: all fluctuation is along x_1
    sec = sectorgen.Sector(a=np.zeros(2), b=np.zeros(2), factors=[
        sectorgen.Factor(-2.0, 0.0, np.array([1.0, 9.0]), np.array([[0, 0], [1, 0]], dtype=np.uint8))])
    prob = sectorgen.Problem(sectors=[sec], order_min=0, order_max=0)
    r = suave.suave(prob, 256 * 15, 256, 1e-12, 0.0, 1, 1.0, 1)
    assert all(g.level[1] == 0 for g in r.regions)
    assert abs(r.value[0].real - 0.1) < 5 * r.err_re[0]


def test_divonne_oracle_pins():
    """The partition-then-lattice oracle (oracle/divonne.py): a linear
    integrand on any dyadic box is integrated exactly by the tent-transformed
    shifted lattice (the tent map of a shifted equispaced grid has mean 1/2), so
    every region's value is exact and its error 0; the bubble's closed form
    within 5 standard errors with regions that tile each cube; on an integrand
    that varies along x_1 only, the partition never cuts x_2."""
    import math
    import sectorgen
    from oracle import divonne, integrate, suave
    # 1 + 3 x_1 + 2 x_2 on [1/4, 1/2] x [1/2, 1]: vol (1 + 3 * 3/8 + 2 * 3/4) = 1/8 * 3.625
    sec = sectorgen.Sector(a=np.zeros(2), b=np.zeros(2), factors=[
        sectorgen.Factor(1.0, 0.0, np.array([1.0, 3.0, 2.0]), np.array([[0, 0], [1, 0], [0, 1]], dtype=np.uint8))])
    prob = sectorgen.Problem(sectors=[sec], order_min=0, order_max=0)
    lead, pref = integrate.prefactor_for(prob)
    reg = suave.MCRegion(0, np.array([2, 1]), np.array([1, 1]), 0)
    v, er, ei, nf = divonne.lattice_rule(prob, reg, 7, 6, 4, 3, True, lead, pref)
    assert abs(v[0].real - 0.125 * 3.625) < 1e-14 and er[0] < 1e-15 and nf == 0
    exact = [1.0, 2.0, 4 - math.pi ** 2 / 12]
    r = divonne.divonne(sectorgen.bubble_problem(order_max=1), 30000, 256, 1e-6, 0.0, 5, 8, 8)
    z = (r.value.real - exact) / r.err_re
    assert np.all(np.abs(z) < 5), z
    alive = [g for g in r.regions if g.alive]
    for s in range(2):
        assert sum(math.ldexp(1.0, -int(g.level.sum())) for g in alive if g.sector == s) == 1.0
    # (1 + 9 x_1)^-2 in two variables
    sec = sectorgen.Sector(a=np.zeros(2), b=np.zeros(2), factors=[
        sectorgen.Factor(-2.0, 0.0, np.array([1.0, 9.0]), np.array([[0, 0], [1, 0]], dtype=np.uint8))])
    prob = sectorgen.Problem(sectors=[sec], order_min=0, order_max=0)
    r = divonne.divonne(prob, 256 * 15, 256, 1e-12, 0.0, 1, 8, 4, split_frac=1.0, batch_min=1)
    assert r.rounds > 1 and all(g.level[1] == 0 for g in r.regions)
    assert abs(r.value[0].real - 0.1) < 5 * r.err_re[0] + 1e-12
