"""Pins of the multiprecision sector integrand (oracle/integrand_mp.py), the
reference for the double-double evaluation of points near the faces x_j = 0.

* One singular variable, x^(-1 + b eps) (1 + c x)^(gamma + delta eps): the
  subtracted coefficients are f_-1 = 1/b and, for k >= 0,
  f_k = [G0 (b L + Lambda)^k - (b L)^k] / (k! x), L = ln x, G0 = (1 + c x)^gamma,
  Lambda = delta ln(1 + c x).  Written as (b L)^k expm1(gamma log1p(c x)) +
  sum_{i>=1} C(k, i) (b L)^(k-i) G0 Lambda^i with signs chosen so that no two
  terms cancel, it is exact to a few ulp in fp64 at any x: a closed form of the
  subtraction that does not cancel at the face.
* Two singular variables with one factor each: the integrand is the product of
  two such one-variable sectors, so its eps series is the Cauchy product of
  theirs (every corner W and subset T of the two-variable subtraction enters).
* Away from the faces the fp64 oracle is accurate to its rounding bound; the
  multiprecision values agree with it there, at the largest accepted shapes.
* The value does not depend on the working precision beyond 32 digits.
* The ln 2 split used by the device double-double exp is ln 2 to 106 bits.

Complex mode (contour deformation, section 4.4):

* The equal-mass bubble above threshold (p^2 = 5, m^2 = 1): the eps^-1 and
  eps^0 coefficients of its closed form, 1 and
  2 - beta ln((1 + beta)/(1 - beta)) + i pi beta with beta^2 = 1 - 4m^2/p^2,
  from the integrand integrated by tanh-sinh quadrature (whose nodes crowd
  both faces), at two deformation sizes (Cauchy's theorem).
* One singular variable with a factor that changes sign inside the cube,
  x^(-1 + b eps) (1 - s x - i0)^(gamma + delta eps), s > 1: the integral is
  2F1(-gamma - delta eps, b eps; b eps + 1; s + i0) / (b eps); its Laurent
  coefficients from the integrand by the same quadrature.
* A factor that is real and negative at the face x = 0 (arg = -pi there):
  the closed form is the phase e^(-i pi (gamma + delta eps)) times the real
  hypergeometric integral.
* Two singular variables, the deformation acting on one of them: the
  integrand is the product of a complex and a real one-variable integrand,
  so its eps series at any point is the Cauchy product of theirs (at points
  down to 1e-14 from the faces).
* Away from the faces it agrees with the fp64 oracle to its rounding bound,
  at the largest complex shape (8 variables, 4 singular); near the faces it
  does not depend on the working precision beyond 32 digits.
"""
import math
import re
from pathlib import Path

import mpmath
import numpy as np
import pytest

from oracle import integrand, integrate
from oracle import integrand_mp as M
from sectorgen import Factor, Sector, SplitMix64
from sectorgen.feynman import massive_bubble_problem

from shapes import max_complex_problem

U = 2.0 ** -53


def one_var(b, c, gamma, delta):
    return Sector(a=np.array([-1.0]), b=np.array([b]),
                  factors=[Factor(gamma, delta, np.array([1.0, c]), np.array([[0], [1]], dtype=np.uint8))])


def closed_one_var(x, k, b, c, gamma, delta):
    """f_k of one_var(...) at x without cancellation (see the module docstring)."""
    if k == -1:
        return 1.0 / b
    L = b * math.log(x)
    lp = math.log1p(c * x)
    g0 = math.exp(gamma * lp)
    lam = delta * lp
    s = L ** k * math.expm1(gamma * lp)
    for i in range(1, k + 1):
        s += math.comb(k, i) * L ** (k - i) * g0 * lam ** i
    return s / (math.factorial(k) * x)


# b > 0 and gamma, delta of opposite signs keep every term of the closed form of one sign
PARAMS = [(1.0, 2.0, 1.5, -0.7), (2.0, 0.5, 2.0, -1.0), (1.0, 1.0, 1.0, -2.0)]


@pytest.mark.parametrize("par", PARAMS)
def test_one_variable_closed_form_at_the_face(par):
    sec = one_var(*par)
    for x in (0.5, 1e-2, 1e-5, 1e-9, 1e-13, 3e-16):
        f, _ = M.sector_f_point(sec, [x], 4)
        for k in range(-1, 5):
            ref = closed_one_var(x, k, *par)
            assert abs(float(f[k + 1]) - ref) <= 1e-13 * abs(ref), (x, k, float(f[k + 1]), ref)


def test_fp64_oracle_loses_digits_at_the_face():
    """What the multiprecision reference is for: at x = 1e-13 the fp64 subtraction
    keeps only about three digits of f_0 (and this is within its rounding bound)."""
    par = PARAMS[0]
    sec = one_var(*par)
    x = np.array([[1e-13]])
    f, cond, _ = integrand.sector_f(sec, x, 2)
    ref = closed_one_var(1e-13, 0, *par)
    err = abs(f[1, 0] - ref)
    assert err > 1e-8 * abs(ref)
    assert err <= 8 * U * cond[1, 0]


def test_two_variables_cauchy_product():
    p1, p2 = (1.0, 2.0, 1.5, -0.7), (2.0, 0.5, 2.0, -1.0)
    sec = Sector(a=np.array([-1.0, -1.0]), b=np.array([p1[0], p2[0]]),
                 factors=[Factor(p1[2], p1[3], np.array([1.0, p1[1]]), np.array([[0, 0], [1, 0]], dtype=np.uint8)),
                          Factor(p2[2], p2[3], np.array([1.0, p2[1]]), np.array([[0, 0], [0, 1]], dtype=np.uint8))])
    for x1, x2 in ((0.3, 0.7), (1e-7, 0.2), (1e-11, 1e-14), (0.9, 1e-12)):
        f, _ = M.sector_f_point(sec, [x1, x2], 3)
        a = [closed_one_var(x1, k, *p1) for k in range(-1, 5)]
        b = [closed_one_var(x2, k, *p2) for k in range(-1, 5)]
        for k in range(-2, 4):
            # f_k = sum_{i + j = k} a_i b_j, i, j >= -1
            ref = sum(a[i + 1] * b[k - i + 1] for i in range(-1, k + 2))
            scale = sum(abs(a[i + 1] * b[k - i + 1]) for i in range(-1, k + 2))
            assert abs(float(f[k + 2]) - ref) <= 1e-13 * scale, (x1, x2, k)


def max_sector(kind, seed=1601):
    """A 16-variable sector with 4 singular variables and 4 factors (exponents up to 3)."""
    rng = SplitMix64(seed)
    n = 16
    a = np.zeros(n)
    b = np.array([float(rng.randint(-2, 2)) for _ in range(n)])
    a[:4] = -1.0
    b[:4] = [1.0, -2.0, 2.0, -1.0]
    if kind == "general":
        a[4:8] = [0.5, 0.25, 1.0, 2.0]
        b[4:8] = [0.5, -1.5, 1.0, 0.0]
    facs = []
    for fm in range(4):
        rows, seen = [tuple([0] * n)], {tuple([0] * n)}
        while len(rows) < 6 + 3 * fm:
            e = tuple(rng.randint(0, 3) if rng.uniform() < 0.3 else 0 for _ in range(n))
            if e not in seen:
                seen.add(e)
                rows.append(e)
        coef = np.array([1.0] + [0.1 + 0.9 * rng.uniform() for _ in rows[1:]])
        if kind == "integer":
            g, d = float(rng.choice([-3, -2, -1, 1, 2])), float(rng.choice([-2, -1, 1, 2]))
        else:
            g, d = rng.choice([-1.5, -0.5, 0.5, 1.25]), rng.choice([-1.0, -0.5, 0.75])
        facs.append(Factor(g, d, coef, np.array(rows, dtype=np.uint8)))
    return Sector(a=a, b=b, factors=facs)


@pytest.mark.parametrize("kind", ["integer", "general"])
def test_agrees_with_fp64_oracle_away_from_faces(kind):
    sec = max_sector(kind)
    rng = np.random.default_rng(3)
    x = rng.uniform(0.05, 1.0, size=(6, 16))
    f64, cond, _ = integrand.sector_f(sec, x, 3)
    for p in range(x.shape[0]):
        f, _ = M.sector_f_point(sec, x[p], 3)
        for k in range(f64.shape[0]):
            assert abs(float(f[k]) - f64[k, p]) <= 8 * U * cond[k, p] + 1e-300, (p, k)


def test_independent_of_working_precision():
    sec = max_sector("general")
    rng = np.random.default_rng(5)
    x = rng.uniform(0.0, 1.0, size=(3, 16))
    x[:, :4] = 10.0 ** rng.uniform(-12, -2, size=(3, 4))
    for p in range(3):
        d = M.point_dps(sec, x[p])
        f1, c1 = M.sector_f_point(sec, x[p], 3)
        f2, _ = M.sector_f_point(sec, x[p], 3, dps=d + 30)
        for k in range(len(f1)):
            with mpmath.workdps(d + 30):
                assert abs(f1[k] - f2[k]) <= mpmath.mpf(10) ** -34 * (abs(f2[k]) + mpmath.mpf(10) ** -300)


def test_orders_fold_matches_fp64_oracle():
    sec = max_sector("integer")
    sec.coeff = 1.0 + 0.5j
    rng = np.random.default_rng(9)
    x = rng.uniform(0.1, 1.0, size=(4, 16))
    pref = np.array([1.0, -0.25, 0.125])
    v64, c64, _ = integrand.sector_orders(sec, x, -4, 3, 0, pref)
    vmp, cmp_, fabs_ = M.sector_orders_mp(sec, x, -4, 3, 0, pref)
    assert vmp.dtype == np.complex128
    assert np.all(np.abs(vmp - v64) <= 8 * U * c64 + 4 * U * fabs_)
    np.testing.assert_allclose(cmp_, c64, rtol=1e-12)


def test_device_ln2_split():
    src = (Path(__file__).resolve().parents[1] / "paper_1511_03614_amd" / "csrc" / "eval_dd.hpp").read_text()
    hi = float.fromhex(re.search(r"LN2_HI = (0x[0-9a-fp.+-]+);", src).group(1))
    lo = float.fromhex(re.search(r"LN2_LO = (0x[0-9a-fp.+-]+);", src).group(1))
    with mpmath.workdps(60):
        ln2 = mpmath.log(2)
        assert hi == float(ln2)
        assert lo == float(ln2 - mpmath.mpf(hi))
        assert abs(mpmath.mpf(hi) + mpmath.mpf(lo) - ln2) <= mpmath.mpf(2) ** -106


# ---------------------------------------------------------------- complex mode

def quad_order(sec, k, lam, dps=30):
    """int_0^1 f_k(x) dx of a one-variable sector by tanh-sinh quadrature at dps digits."""
    ns = len(integrand.singular_set(sec))
    with mpmath.workdps(dps):
        return mpmath.quad(lambda x: M.sector_f_point(sec, [x], k, dps=dps, complex_mode=True, lam=lam)[0][k + ns],
                           [0, 1])


@pytest.mark.parametrize("lam", [0.5, 0.3])
def test_complex_massive_bubble_closed_form(lam):
    prob = massive_bubble_problem(5.0, 1.0, lam)
    lead, pref = integrate.prefactor_for(prob)
    assert lead == -1 and pref[0] == 1.0 and pref[1] == 0.0
    with mpmath.workdps(30):
        f0 = sum(quad_order(sec, 0, lam) for sec in prob.sectors)       # eps^-1 of the result
        f1 = sum(quad_order(sec, 1, lam) for sec in prob.sectors)       # eps^0
        beta = mpmath.sqrt(1 - mpmath.mpf(4) / 5)
        fin = 2 - beta * mpmath.log((1 + beta) / (1 - beta)) + 1j * mpmath.pi * beta
        assert abs(f0 - 1) < mpmath.mpf(10) ** -28
        assert abs(f1 - fin) < mpmath.mpf(10) ** -28


def hyp_complex_series(b, s, g, d, n, dps=40):
    """Laurent coefficients eps^-1 .. eps^(n-1) of int_0^1 x^(-1+b eps) (1 - s x - i0)^(g + d eps) dx."""
    with mpmath.workdps(dps):
        z = mpmath.mpf(s) + mpmath.mpc(0, mpmath.mpf(10) ** -(dps + 15))     # the -i0 side of 1 - s x
        return mpmath.taylor(lambda e: mpmath.hyp2f1(-(g + d * e), b * e, b * e + 1, z) / b, 0, n - 1)


@pytest.mark.parametrize("b,s,g,d,lam", [(1.0, 2.0, -1.0, 1.0, 0.4), (-2.0, 3.0, 1.5, -1.0, 0.2),
                                         (0.5, 1.5, -2.0, 0.5, 0.5)])
def test_complex_one_variable_through_the_cut(b, s, g, d, lam):
    sec = Sector(a=np.array([-1.0]), b=np.array([b]),
                 factors=[Factor(g, d, np.array([1.0, -s]), np.array([[0], [1]], dtype=np.uint8))],
                 deform_factor=0, deform_mono=np.zeros(1, np.int32))
    ref = hyp_complex_series(b, s, g, d, 4)
    with mpmath.workdps(30):
        for k in range(-1, 3):
            got = quad_order(sec, k, lam)
            assert abs(got - ref[k + 1]) < mpmath.mpf(10) ** -24 * max(1, abs(ref[k + 1])), k


@pytest.mark.parametrize("b,c,g,d,lam", [(1.0, 0.5, -1.5, 1.0, 0.3), (-1.0, 2.0, 0.5, -0.5, 0.2)])
def test_complex_factor_negative_at_the_face(b, c, g, d, lam):
    """x^(-1+b eps) (-(1 + c x) - i0)^(g + d eps) = e^(-i pi (g + d eps)) x^(-1+b eps) (1 + c x)^(g + d eps):
    the factor is real and negative at the corner x = 0, where its argument is -pi."""
    sec = Sector(a=np.array([-1.0]), b=np.array([b]),
                 factors=[Factor(g, d, np.array([-1.0, -c]), np.array([[0], [1]], dtype=np.uint8))],
                 deform_factor=0, deform_mono=np.zeros(1, np.int32))
    with mpmath.workdps(40):
        ref = mpmath.taylor(lambda e: mpmath.exp(-1j * mpmath.pi * (g + d * e))
                            * mpmath.hyp2f1(-(g + d * e), b * e, b * e + 1, -c) / b, 0, 3)
    with mpmath.workdps(30):
        for k in range(-1, 3):
            got = quad_order(sec, k, lam)
            assert abs(got - ref[k + 1]) < mpmath.mpf(10) ** -24 * max(1, abs(ref[k + 1])), k


def test_complex_two_variables_cauchy_product():
    b1, s1, g1, d1, lam = 1.0, 2.5, -1.0, 0.5, 0.3
    b2, c2, g2, d2 = -1.0, 0.7, 2.0, -1.0
    one_c = Sector(a=np.array([-1.0]), b=np.array([b1]),
                   factors=[Factor(g1, d1, np.array([1.0, -s1]), np.array([[0], [1]], dtype=np.uint8))],
                   deform_factor=0, deform_mono=np.zeros(1, np.int32))
    one_r = one_var(b2, c2, g2, d2)
    two = Sector(a=np.array([-1.0, -1.0]), b=np.array([b1, b2]), factors=[
        Factor(g1, d1, np.array([1.0, -s1]), np.array([[0, 0], [1, 0]], dtype=np.uint8)),
        Factor(g2, d2, np.array([1.0, c2]), np.array([[0, 0], [0, 1]], dtype=np.uint8))],
        deform_factor=0, deform_mono=np.zeros(2, np.int32))
    for x1, x2 in [(0.3, 0.6), (1e-3, 0.8), (1e-9, 1e-5), (1e-14, 0.4), (0.7, 1e-13), (1e-12, 1e-14)]:
        fa, _ = M.sector_f_point(one_c, [x1], 3, complex_mode=True, lam=lam)
        fb, _ = M.sector_f_point(one_r, [x2], 3)
        f, _ = M.sector_f_point(two, [x1, x2], 2, complex_mode=True, lam=lam)
        with mpmath.workdps(60):
            for k in range(-2, 3):
                ref = sum(fa[i + 1] * fb[k - i + 1] for i in range(-1, k + 2))
                scale = sum(abs(fa[i + 1] * fb[k - i + 1]) for i in range(-1, k + 2))
                assert abs(f[k + 2] - ref) <= mpmath.mpf(10) ** -30 * scale, (x1, x2, k)


def test_complex_agrees_with_fp64_oracle_away_from_faces():
    prob = max_complex_problem()
    rng = np.random.default_rng(3)
    for sec in prob.sectors:
        x = rng.uniform(0.05, 1.0, size=(3, sec.n))
        f64, cond, _ = integrand.sector_f(sec, x, 3, True, prob.lam)
        for p in range(x.shape[0]):
            f, _ = M.sector_f_point(sec, x[p], 3, complex_mode=True, lam=prob.lam)
            for k in range(f64.shape[0]):
                assert abs(complex(f[k]) - f64[k, p]) <= 32 * U * cond[k, p], (p, k)


def test_complex_independent_of_working_precision():
    prob = max_complex_problem()
    sec = prob.sectors[1]
    rng = np.random.default_rng(6)
    x = rng.uniform(0.0, 1.0, size=(2, sec.n))
    x[:, :4] = 10.0 ** rng.uniform(-12, -2, size=(2, 4))
    for p in range(2):
        d = M.point_dps(sec, x[p])
        f1, _ = M.sector_f_point(sec, x[p], 3, complex_mode=True, lam=prob.lam)
        f2, _ = M.sector_f_point(sec, x[p], 3, dps=d + 30, complex_mode=True, lam=prob.lam)
        for k in range(len(f1)):
            with mpmath.workdps(d + 30):
                assert abs(f1[k] - f2[k]) <= mpmath.mpf(10) ** -34 * (abs(f2[k]) + mpmath.mpf(10) ** -300)


def test_complex_orders_fold_matches_fp64_oracle():
    prob = max_complex_problem()
    sec = prob.sectors[0]
    lead, pref = integrate.prefactor_for(prob)
    x = np.random.default_rng(10).uniform(0.1, 1.0, size=(2, sec.n))
    v64, c64, _ = integrand.sector_orders(sec, x, prob.order_min, prob.order_max, lead, pref, True, prob.lam)
    vmp, cmp_, fabs_ = M.sector_orders_mp(sec, x, prob.order_min, prob.order_max, lead, pref,
                                          complex_mode=True, lam=prob.lam)
    assert vmp.dtype == np.complex128
    assert np.all(np.abs(vmp - v64) <= 32 * U * c64 + 4 * U * fabs_)
    np.testing.assert_allclose(cmp_, c64, rtol=1e-10)
