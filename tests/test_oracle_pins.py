"""Pins of the fp64 oracle against what the paper and the mathematics fix.

None of these re-types the oracle's own formulas: each compares the oracle with
an independent route - a hypergeometric closed form, a Gamma-function closed
form, the paper's printed worked example, a direct integral at finite eps,
Cauchy's theorem (lambda invariance) or exact integer facts of the lattice.
"""
import math

import mpmath as mp
import numpy as np
import pytest

import sectorgen
from sectorgen import Factor, Sector
from oracle import integrand, integrate, points, prefactor, vegas

EULER = float(mp.euler)


# ------------------------------------------------------------------ helpers

def gl_nodes(nodes: int, power: int):
    """Gauss-Legendre on [0,1] after x = t^power (smooths log endpoint singularities)."""
    t, w = np.polynomial.legendre.leggauss(nodes)
    t = 0.5 * (t + 1.0)
    w = 0.5 * w
    return t ** power, w * power * t ** (power - 1)


def quad_sector_f(sec, kf_max, nodes=80, power=5, complex_mode=False, lam=0.0):
    """Integral over [0,1]^n of the oracle's f_k, tensor Gauss-Legendre."""
    x1, w1 = gl_nodes(nodes, power)
    n = sec.n
    grids = np.meshgrid(*([x1] * n), indexing="ij")
    wts = np.meshgrid(*([w1] * n), indexing="ij")
    x = np.stack([g.ravel() for g in grids], axis=1)
    w = np.prod(np.stack([g.ravel() for g in wts], axis=1), axis=1)
    f, _, _ = integrand.sector_f(sec, x, kf_max, complex_mode, lam)
    return f @ w


def taylor(fn, n, dps=40):
    with mp.workdps(dps):
        return [complex(c) for c in mp.taylor(fn, 0, n, singular=True)]


def one_var_sector(a, b, c, gam, dlt):
    return Sector(a=np.array([a]), b=np.array([b]),
                  factors=[Factor(gam, dlt, np.array([1.0, c]), np.array([[0], [1]], dtype=np.uint8))])


def hyp_series(a, b, c, gam, dlt, n):
    """Laurent coefficients of int_0^1 x^(a+b eps) (1+cx)^(gam+dlt eps) dx (leading eps^-1 if a=-1).

    int_0^1 x^(s-1) (1+cx)^(-nu) dx = 2F1(nu, s; s+1; -c)/s  with s = a+1+b eps.
    """
    def h(e):
        s = a + 1 + b * e
        v = mp.hyp2f1(-(gam + dlt * e), s, s + 1, -c) / s
        return v * e if a == -1.0 else v
    return taylor(h, n)


# ------------------------------------------------------------------ prefactor

@pytest.mark.parametrize("loops,indices,d0", [
    (1, (1, 1), 4), (1, (1, 1, 1, 1), 4), (2, (1,) * 7, 4), (1, (1,), 4), (2, (1, 1, 1, 1, 2), 4),
    (1, (2, 1), 6), (2, (1, 1, 1), 4), (3, (1, 1, 1, 1), 4),
])
def test_prefactor_vs_gamma_taylor(loops, indices, d0):
    lead, ser = prefactor.feynman_prefactor(loops, indices, d0, 6)
    A = sum(indices)

    def fn(e):
        v = mp.exp(loops * mp.euler * e) * mp.gamma(A - loops * (d0 - 2 * e) / 2)
        for a in indices:
            v /= mp.gamma(a)
        return v * e ** (-lead)
    ref = taylor(fn, 5)
    assert np.allclose(ser, np.real(ref), rtol=1e-13, atol=1e-13)


def test_prefactor_bubble_constants():
    lead, ser = prefactor.feynman_prefactor(1, (1, 1), 4, 4)
    assert lead == -1
    assert ser[0] == pytest.approx(1.0, abs=1e-15)
    assert ser[1] == pytest.approx(0.0, abs=1e-15)
    assert ser[2] == pytest.approx(math.pi ** 2 / 12, rel=1e-14)
    assert ser[3] == pytest.approx(-float(mp.zeta(3)) / 3, rel=1e-14)


# ------------------------------------------------------------------ integrand, real

@pytest.mark.parametrize("a,b,c,gam,dlt", [
    (-1.0, 1.0, 1.0, -2.0, 2.0), (-1.0, -2.0, 0.5, -1.0, -1.0), (-1.0, 0.5, 2.0, 1.0, 3.0),
    (0.0, -1.0, 1.0, -2.0, 2.0), (0.5, 1.0, 0.3, -3.0, -2.0), (2.0, -2.0, 1.5, 1.0, 1.0),
])
def test_one_variable_vs_hypergeometric(a, b, c, gam, dlt):
    sec = one_var_sector(a, b, c, gam, dlt)
    kf = 4
    got = quad_sector_f(sec, kf, nodes=120, power=6)
    ref = hyp_series(a, b, c, gam, dlt, kf + (1 if a == -1.0 else 0))
    ns = 1 if a == -1.0 else 0
    for i in range(got.shape[0]):
        assert got[i] == pytest.approx(ref[i].real, rel=1e-10, abs=1e-12), i
    assert got.shape[0] == kf + ns + 1


def test_two_singular_variables_separable():
    # (1 + 0.7 x1)^(-2+eps) (1 + 1.3 x2)^(-1-2eps) x1^(-1+eps) x2^(-1-2eps): product of 1-D series
    sec = Sector(a=np.array([-1.0, -1.0]), b=np.array([1.0, -2.0]), factors=[
        Factor(-2.0, 1.0, np.array([1.0, 0.7]), np.array([[0, 0], [1, 0]], dtype=np.uint8)),
        Factor(-1.0, -2.0, np.array([1.0, 1.3]), np.array([[0, 0], [0, 1]], dtype=np.uint8))])
    kf = 3
    got = quad_sector_f(sec, kf, nodes=90, power=6)
    s1 = hyp_series(-1.0, 1.0, 0.7, -2.0, 1.0, kf + 2)
    s2 = hyp_series(-1.0, -2.0, 1.3, -1.0, -2.0, kf + 2)
    prod = np.convolve(np.real(s1), np.real(s2))            # starts at eps^-2
    for i in range(got.shape[0]):
        assert got[i] == pytest.approx(prod[i], rel=1e-9, abs=1e-11), i


def test_mixed_singular_and_regular_variable():
    # x1^(-1-eps) x2^(0.5+eps) (1+2 x1)^(-1+eps) (1+0.5 x2)^(2-eps): product again
    sec = Sector(a=np.array([-1.0, 0.5]), b=np.array([-1.0, 1.0]), factors=[
        Factor(-1.0, 1.0, np.array([1.0, 2.0]), np.array([[0, 0], [1, 0]], dtype=np.uint8)),
        Factor(2.0, -1.0, np.array([1.0, 0.5]), np.array([[0, 0], [0, 1]], dtype=np.uint8))])
    kf = 3
    got = quad_sector_f(sec, kf, nodes=90, power=6)
    s1 = hyp_series(-1.0, -1.0, 2.0, -1.0, 1.0, kf + 1)
    s2 = hyp_series(0.5, 1.0, 0.5, 2.0, -1.0, kf + 1)
    prod = np.convolve(np.real(s1), np.real(s2))
    for i in range(got.shape[0]):
        assert got[i] == pytest.approx(prod[i], rel=1e-9, abs=1e-11), i


def test_nonseparable_against_direct_integral():
    """int x^(-1+eps) y^(-1+2eps) (1+x+2y)^(-1+eps): series vs direct integral at finite eps."""
    sec = Sector(a=np.array([-1.0, -1.0]), b=np.array([1.0, 2.0]), factors=[
        Factor(-1.0, 1.0, np.array([1.0, 1.0, 2.0]),
               np.array([[0, 0], [1, 0], [0, 1]], dtype=np.uint8))])
    kf = 7
    coeffs = quad_sector_f(sec, kf, nodes=100, power=6)        # eps^-2 .. eps^7
    assert coeffs[0] == pytest.approx(0.5, rel=1e-12)          # G(0)/(b1 b2)
    t, w = np.polynomial.legendre.leggauss(600)
    t = 0.5 * (t + 1)
    w = 0.5 * w
    for eps in (0.02, 0.03):
        # x = s^(1/eps), y = u^(1/(2 eps)) absorb the singular monomials exactly
        X = t[:, None] ** (1.0 / eps)
        Y = t[None, :] ** (1.0 / (2 * eps))
        direct = (w[:, None] * w[None, :] * (1 + X + 2 * Y) ** (-1 + eps)).sum() / (eps * 2 * eps)
        series = sum(c * eps ** (k - 2) for k, c in enumerate(coeffs))
        assert series == pytest.approx(direct, rel=5e-10)


def test_bubble_whole_chain_closed_form():
    """Both primary sectors plus the prefactor against e^(gE eps) Gamma(eps) Gamma(1-eps)^2 / Gamma(2-2eps)."""
    prob = sectorgen.config1()
    lead, pref = integrate.prefactor_for(prob)
    x, w = gl_nodes(200, 6)
    tot = 0
    for sec in prob.sectors:
        vals, _, _ = integrand.sector_orders(sec, x[:, None], prob.order_min, prob.order_max, lead, pref)
        tot = tot + vals @ w
    ref = taylor(lambda e: e * mp.exp(mp.euler * e) * mp.gamma(e) * mp.gamma(1 - e) ** 2
                 / mp.gamma(2 - 2 * e), 3)
    assert np.allclose(tot, np.real(ref), rtol=1e-11, atol=1e-12)
    # the analytic values 4 - pi^2/12 and 8 - pi^2/6 - 7 zeta(3)/3
    assert tot[2] == pytest.approx(4 - math.pi ** 2 / 12, rel=1e-11)
    assert tot[3] == pytest.approx(8 - math.pi ** 2 / 6 - 7 * float(mp.zeta(3)) / 3, rel=1e-11)


# ------------------------------------------------------------------ integrand, complex

def massive_bubble_sector(s, m2):
    """Primary sector x1 = 1 of the equal-mass bubble: U = 1+t, F = m2 (1+t)^2 - s t."""
    F = np.array([m2, 2 * m2 - s, m2])
    return Sector(a=np.array([0.0]), b=np.array([0.0]), factors=[
        Factor(-2.0, 2.0, np.array([1.0, 1.0]), np.array([[0], [1]], dtype=np.uint8)),
        Factor(0.0, -1.0, F, np.array([[0], [1], [2]], dtype=np.uint8))],
        deform_factor=1, deform_mono=np.zeros(1, np.int32))


@pytest.mark.parametrize("lam", [0.3, 0.5, 0.8])
def test_massive_bubble_above_threshold(lam):
    """s = 5, m^2 = 1: finite part 2 - ln m^2 - beta ln((1+beta)/(1-beta)) + i pi beta."""
    s, m2 = 5.0, 1.0
    sec = massive_bubble_sector(s, m2)
    lead, pref = prefactor.feynman_prefactor(1, (1, 1), 4, 3)
    x, w = gl_nodes(400, 1)
    vals, _, pos = integrand.sector_orders(sec, x[:, None], -1, 0, lead, pref, True, lam)
    tot = 2 * (vals @ w)
    beta = math.sqrt(1 - 4 * m2 / s)
    fin = 2 - math.log(m2) - beta * math.log((1 + beta) / (1 - beta)) + 1j * math.pi * beta
    assert tot[0] == pytest.approx(1.0, abs=1e-12)
    assert abs(tot[1] - fin) < 1e-10
    assert not pos.any()


def test_minus_i0_on_negative_real_axis():
    """A factor that is real and negative takes Log = ln|P| - i pi (F - i0 of eq. (1))."""
    sec = Sector(a=np.array([0.0]), b=np.array([0.0]), factors=[
        Factor(0.0, -1.0, np.array([-1.0, -1.0]), np.array([[0], [1]], dtype=np.uint8))])
    got = quad_sector_f(sec, 1, nodes=60, power=1, complex_mode=True, lam=0.0)
    # int (-(1+x) - i0)^(-eps) dx = 1 - eps int_0^1 (ln(1+x) - i pi) dx + ...
    assert got[0] == pytest.approx(1.0, abs=1e-14)
    assert abs(got[1] - (-(2 * math.log(2) - 1) + 1j * math.pi)) < 1e-13


def deformable_2d_sector():
    # Euclidean sector: F = x1 (1 + 2 x2 + x1 x2) > 0, so deformation may not change the integral
    return Sector(a=np.array([-1.0, 0.0]), b=np.array([1.0, -1.0]), factors=[
        Factor(1.0, 1.0, np.array([1.0, 1.0, 0.5]), np.array([[0, 0], [1, 0], [0, 1]], dtype=np.uint8)),
        Factor(-2.0, -1.0, np.array([1.0, 2.0, 1.0]), np.array([[0, 0], [0, 1], [1, 1]], dtype=np.uint8))],
        deform_factor=1, deform_mono=np.array([1, 0], np.int32))


def test_lambda_invariance_two_variables():
    sec = deformable_2d_sector()
    ref = quad_sector_f(sec, 2, nodes=70, power=5, complex_mode=True, lam=0.0)
    real = quad_sector_f(sec, 2, nodes=70, power=5, complex_mode=False)
    assert np.allclose(ref.real, real, rtol=1e-13, atol=1e-14)
    assert np.all(ref.imag == 0.0)
    for lam in (0.05, 0.15):
        got = quad_sector_f(sec, 2, nodes=70, power=5, complex_mode=True, lam=lam)
        assert np.allclose(got, ref, rtol=1e-9, atol=1e-11), lam


def test_deformation_jacobian_by_finite_differences():
    """det(dz/dx) from the oracle against central differences of z(x) (3 variables)."""
    sec = Sector(a=np.zeros(3), b=np.zeros(3), factors=[
        Factor(1.0, 0.0, np.array([1.0]), np.zeros((1, 3), dtype=np.uint8)),
        Factor(1.0, 0.0, np.array([0.5, -1.0, 2.0, 0.7]),
               np.array([[0, 0, 0], [1, 1, 0], [0, 1, 2], [2, 0, 1]], dtype=np.uint8))],
        deform_factor=1, deform_mono=np.array([0, 1, 0], np.int32))
    lam = 0.4
    rng = np.random.default_rng(5)
    y = rng.uniform(0.05, 0.95, size=(6, 3))
    # G0 = det * prod_m P_m(z)^gamma_m; with the first factor 1 and gamma_F = 1, det = G0 / F(z)
    g0, _, _ = integrand.regular_part(sec, y, True, lam)
    coef, exps = integrand.full_f_terms(sec)

    def zmap(v):
        grad, _ = integrand.f_derivatives(sec, v)
        return v - 1j * lam * v * (1 - v) * grad
    z = zmap(y)
    pf = integrand.poly(sec.factors[1].coef, sec.factors[1].exps, z)
    det_o = g0 / pf
    h = 1e-6
    for p in range(y.shape[0]):
        J = np.zeros((3, 3), dtype=complex)
        for k in range(3):
            e = np.zeros(3)
            e[k] = h
            J[:, k] = (zmap((y[p] + e)[None, :])[0] - zmap((y[p] - e)[None, :])[0]) / (2 * h)
        assert abs(np.linalg.det(J) - det_o[p]) < 1e-8 * max(1.0, abs(det_o[p]))
    assert coef.shape[0] == 4 and exps[1, 1] == 2


# ------------------------------------------------------------------ points

def test_philox_known_answers():
    """Random123 known-answer vectors for philox4x32_10."""
    assert points.philox4x32_10((0, 0, 0, 0), (0, 0)) == [0x6627e8d5, 0xe169c58d, 0xbc57ac4c, 0x9b00dbd8]
    assert points.philox4x32_10((0xFFFFFFFF,) * 4, (0xFFFFFFFF,) * 2) == \
        [0x408f276d, 0x41c83b0e, 0xa20bc7c6, 0x6d5451fd]
    assert points.philox4x32_10((0x243f6a88, 0x85a308d3, 0x13198a2e, 0x03707344),
                                (0xa4093822, 0x299f31d0)) == [0xd16cfe09, 0x94fdcceb, 0x5001e420, 0x24126ea1]


@pytest.mark.parametrize("m", [4, 10, 13])
def test_lattice_projections_and_shift_mean(m):
    N = 1 << m
    z = points.cbc_vector(m, 5)
    assert z[0] == 1 and all(v % 2 == 1 for v in z)
    u = points.lattice_u(z, m, np.zeros(5, dtype=np.uint64), 0, N)
    for j in range(5):
        assert np.array_equal(np.sort(u[:, j]), np.arange(N) / N)
    D = np.array([points.shift_int(7, 3, 1, j, m) for j in range(5)], dtype=np.uint64)
    us = points.lattice_u(z, m, D, 0, N)
    assert np.all(us > 0) and np.all(us < 1)
    for j in range(5):
        # mean of {k/N + delta mod 1} = (N-1)/(2N) + (D mod 2^(53-m)) / 2^53, exactly
        exact = (N - 1) / (2 * N) + (int(D[j]) % (1 << (53 - m))) / 2.0 ** 53
        assert math.fsum(us[:, j].tolist()) / N == pytest.approx(exact, rel=1e-15)


def test_tent_and_identity_vegas_map_exact():
    rng = np.random.default_rng(1)
    u = rng.integers(1, 1 << 53, size=4096).astype(np.float64) * 2.0 ** -53
    t = points.tent(u)
    assert np.all(t > 0) and np.all(t <= 1)
    back = np.where(u < 0.5, t / 2, 1 - t / 2)
    assert np.array_equal(back, u)                       # the tent map loses no bits
    x, w, _ = points.vegas_map(points.identity_grid(1, 128), t[:, None])
    assert np.array_equal(x[:, 0], t) and np.all(w == 1.0)


def test_vegas_map_weight_integrates_to_one():
    rng = np.random.default_rng(2)
    nb = 64
    edges = np.concatenate([[0.0], np.sort(rng.uniform(size=nb - 1)), [1.0]])
    grid = edges[None, :]
    u = ((np.arange(nb) + 0.5) / nb)[:, None]          # one point per bin: exact midpoint rule
    x, w, _ = points.vegas_map(grid, u)
    assert math.fsum(w.tolist()) / nb == pytest.approx(1.0, rel=1e-14)
    assert np.all(np.diff(x[:, 0]) > 0)


# ------------------------------------------------------------------ vegas refit

def test_refit_keeps_grid_for_flat_histogram():
    g = points.identity_grid(2, 32)
    new = vegas.refit(g, np.ones((2, 32)))
    assert np.allclose(new, g, rtol=0, atol=1e-15)
    keep = vegas.refit(g, np.zeros((2, 32)))
    assert np.array_equal(keep, g)


def test_refit_moves_edges_towards_importance():
    nb = 32
    g = points.identity_grid(1, nb)
    d = np.ones((1, nb))
    d[0, :4] = 50.0
    new = vegas.refit(g, d)
    assert np.all(np.diff(new[0]) > 0) and new[0, 0] == 0.0 and new[0, -1] == 1.0
    assert new[0, nb // 2] < 0.5                          # bins crowd into the heavy end
    assert (new[0, 1] - new[0, 0]) < (new[0, -1] - new[0, -2])


def test_vegas_reduces_error_on_peaked_integrand():
    """Warm-up adaptation on x^(-1/2)-like structure reduces the shift-to-shift error."""
    sec = Sector(a=np.array([-1.0]), b=np.array([1.0]),
                 factors=[Factor(-1.0, 1.0, np.array([0.01, 1.0]), np.array([[0], [1]], dtype=np.uint8))])
    prob = sectorgen.Problem(sectors=[sec], order_min=-1, order_max=1)
    lead, pref = integrate.prefactor_for(prob)
    plain = integrate.integrate_sector(prob, 0, 10, 8, 11, lead, pref)
    adapt = integrate.integrate_sector(prob, 0, 10, 8, 11, lead, pref, warmup=4, warmup_m=10, nbins=32)
    assert adapt.err_re[1] < 0.5 * plain.err_re[1]


# ------------------------------------------------------------------ integrate

def test_bubble_estimates_calibrated():
    prob = sectorgen.config1()
    exact = [1.0, 2.0, 4 - math.pi ** 2 / 12, 8 - math.pi ** 2 / 6 - 7 * float(mp.zeta(3)) / 3]
    zs = []
    for seed in range(1, 9):
        _, val, er, _ = integrate.integrate(prob, 10, 8, seed, warmup=2, warmup_m=10, nbins=32)
        for k in range(1, 4):
            zs.append((val[k].real - exact[k]) / er[k])
    zs = np.array(zs)
    assert np.all(np.abs(zs) < 5.0)
    assert np.mean(np.abs(zs) < 2.0) > 0.7


# ------------------------------------------------------------------ the paper's worked example

def test_box_worked_example_section_4_3():
    """Massless on-shell box, S = 3, T = 1 (section 4.3): the paper prints
    -4.38658 + (1.3333 +- 0.000019)/ep^2 - (0.732466 +- 0.000667)/ep +- 0.001.
    Textbook value in the same normalisation: 4/(3 ep^2) - (2 ln 3 / 3)/ep - 4 pi^2 / 9."""
    from sectorgen.feynman import box_problem
    prob = box_problem(3.0, 1.0)
    lead, pref = integrate.prefactor_for(prob)
    x1, w1 = gl_nodes(36, 5)
    g = np.meshgrid(x1, x1, x1, indexing="ij")
    gw = np.meshgrid(w1, w1, w1, indexing="ij")
    x = np.stack([v.ravel() for v in g], axis=1)
    w = np.prod(np.stack([v.ravel() for v in gw], axis=1), axis=1)
    tot = 0
    for sec in prob.sectors:
        vals, _, _ = integrand.sector_orders(sec, x, prob.order_min, prob.order_max, lead, pref)
        tot = tot + vals @ w
    printed = [(1.3333, 0.000019), (-0.732466, 0.000667), (-4.38658, 0.001)]
    for (v, e), got in zip(printed, tot):
        assert abs(got - v) < 3 * e + 5e-5
    exact = [4 / 3, -2 * math.log(3) / 3, -4 * math.pi ** 2 / 9]
    assert np.allclose(tot, exact, rtol=2e-6, atol=2e-6)


def test_neyman_allocation_properties():
    """Shares follow the errors, clamps hold, equal errors give equal sizes, and
    the budget is spent to within one doubling."""
    from oracle.integrate import SectorEstimate, neyman_allocation

    def est(e):
        return SectorEstimate(np.zeros((2, 1), complex), np.zeros(1, complex), np.array([e]), np.array([0.0]), 0, 0, None)
    R = 16
    budget = 3 * R * 1024
    m = neyman_allocation([est(1.0), est(4.0), est(0.25)], budget, R, 4, 20)
    assert m[1] > m[0] >= m[2]
    assert m[1] - m[0] == 2
    used = sum(R << v for v in m)
    assert used <= budget and all(used + (R << v) > budget for v in m)   # no doubling fits any more
    assert neyman_allocation([est(1.0)] * 4, 4 * R * 1024, R, 4, 20) == [10] * 4
    assert neyman_allocation([est(0.0)] * 3, 3 * R * 256, R, 4, 20) == [8] * 3
    assert neyman_allocation([est(1e9), est(1e-9)], (R << 12) + (R << 6), R, 6, 12) == [12, 6]
    assert neyman_allocation([est(1e9), est(1e-9)], 1 << 40, R, 6, 12) == [12, 12]   # budget left over: filled
    # a large problem: total within one smallest doubling of the budget, sizes ordered by error
    rng = np.random.default_rng(3)
    errs = np.exp(rng.normal(size=300) * 2)
    b = 1 << 26
    m = neyman_allocation([est(e) for e in errs], b, R, 8, 18)
    used = sum(R << v for v in m)
    assert b - (R << 18) < used <= b
    order = np.argsort(errs)
    assert all(m[order[i]] <= m[order[i + 2]] + 1 for i in range(len(order) - 2))
