"""Pins of oracle/separate.py (SeparateTerms, section 4.4).

* A two-variable sector with both variables singular and the factor
  (1 + x1)(1 + x2): every term's integrand has a closed form at each point,
  T = {} : (b1 ln x1 + b2 ln x2)^k / k!           (the doubly subtracted part),
  T = {1}: (b2 ln x2)^(k+1) / ((k+1)! b1)          (1/(b1 eps) x2^(b2 eps)),
  T = {2}: the same with the variables exchanged,
  T = S  : 1/(b1 b2) at eps^-2 only,
  so a dropped 1/b, a missing eps shift, boundary terms kept inside a term, or
  a wrong face all fail.
* One singular variable, (1 + x)^(1 + delta eps): the subtracted term
  integrates (mpmath quadrature of the closed-form integrand per order) to
  the whole integral minus 1/(b eps).
* Random sectors (1..3 singular variables, some with every variable
  singular): the terms, at the face points of the same x, sum to the whole
  sector's integrand at x.
"""
import math

import numpy as np
import pytest

import sectorgen
from sectorgen import Factor, Problem, Sector
from oracle import integrand, separate


def two_var_sector(b1, b2):
    # (1 + x1)(1 + x2) = 1 + x1 + x2 + x1 x2
    f = Factor(1.0, 0.0, np.array([1.0, 1.0, 1.0, 1.0]), np.array([[0, 0], [1, 0], [0, 1], [1, 1]], dtype=np.uint8))
    return Sector(a=np.array([-1.0, -1.0]), b=np.array([b1, b2]), factors=[f], coeff=1.0)


def term_orders(face, x, order_min, order_max):
    vals, _, _ = integrand.sector_orders(face, x, order_min, order_max, 0, [1.0])
    return vals


def test_two_variable_terms_closed_forms():
    b1, b2 = 0.7, -1.3
    sec = two_var_sector(b1, b2)
    rng = np.random.default_rng(4)
    x = rng.uniform(0.01, 0.99, size=(50, 2))
    lo, hi = -2, 3
    K = hi - lo + 1
    L = b1 * np.log(x[:, 0]) + b2 * np.log(x[:, 1])
    expect = {0: np.zeros((K, 50)), 1: np.zeros((K, 50)), 2: np.zeros((K, 50)), 3: np.zeros((K, 50))}
    for ki, k in enumerate(range(lo, hi + 1)):
        if k >= 0:
            expect[0][ki] = L ** k / math.factorial(k)
        if k >= -1:
            expect[1][ki] = (b2 * np.log(x[:, 1])) ** (k + 1) / (math.factorial(k + 1) * b1)
            expect[2][ki] = (b1 * np.log(x[:, 0])) ** (k + 1) / (math.factorial(k + 1) * b2)
        if k == -2:
            expect[3][ki] = 1.0 / (b1 * b2)
    total = np.zeros((K, 50))
    for tmask in range(4):
        face = separate.face_sector(sec, tmask)
        assert face.n == max(1, 2 - bin(tmask).count("1")) and face.eps_shift == bin(tmask).count("1")
        got = term_orders(face, separate.face_point(sec, tmask, x), lo, hi)
        np.testing.assert_allclose(got, expect[tmask], rtol=1e-12, atol=1e-12, err_msg=f"T={tmask}")
        total += got
    whole = term_orders(sec, x, lo, hi)
    np.testing.assert_allclose(total, whole, rtol=1e-11, atol=1e-11)


def test_one_variable_subtracted_term_integral():
    mp = pytest.importorskip("mpmath")
    b, dl = 0.9, 0.6
    f = Factor(1.0, dl, np.array([1.0, 1.0]), np.array([[0], [1]], dtype=np.uint8))
    sec = Sector(a=np.array([-1.0]), b=np.array([b]), factors=[f], coeff=1.0)
    lo, hi = -1, 2
    parts = [separate.face_sector(sec, t) for t in range(2)]
    # the boundary term: 1/(b eps) exactly, at eps^-1 only
    bt = term_orders(parts[1], np.array([[0.3], [0.8]]), lo, hi)
    np.testing.assert_allclose(bt, [[1 / b] * 2, [0, 0], [0, 0], [0, 0]], atol=1e-15)
    # the subtracted term: eps^k coefficient of int x^(-1 + b eps) ((1+x)^(1 + dl eps) - 1) dx,
    # the integrand's coefficient written out: sum_{i+j=k} (b ln x)^i/i! [(1+x) (dl ln(1+x))^j/j! - [j=0]] / x
    mp.mp.dps = 30
    for ki, k in enumerate(range(lo, hi + 1)):
        if k < 0:
            continue

        def g(t, k=k):
            s = mp.mpf(0)
            for i in range(k + 1):
                j = k - i
                inner = (1 + t) * (dl * mp.log(1 + t)) ** j / mp.factorial(j) - (1 if j == 0 else 0)
                s += (b * mp.log(t)) ** i / mp.factorial(i) * inner / t
            return s

        ref = float(mp.quad(g, [0, 1]))
        # the oracle's subtracted integrand, integrated by a tanh-sinh rule in mpmath on its fp64 values
        val = float(mp.quad(lambda t: term_orders(parts[0], np.array([[float(t)]]), k, k)[0, 0], [0, 1]))
        assert abs(val - ref) <= 1e-9 * max(1.0, abs(ref)), (k, val, ref)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_terms_sum_to_the_sector(seed):
    prob = sectorgen.synthetic_problem(seed, 5, (2, 4), (2, 5), (1, 3), -3, 1)
    parts, origin = separate.separate(prob)
    assert origin == sorted(origin)
    rng = np.random.default_rng(seed)
    for s, sec in enumerate(prob.sectors):
        ns = len(integrand.singular_set(sec))
        idx = [i for i, o in enumerate(origin) if o == s]
        assert len(idx) == (1 << ns if ns else 1)
        x = rng.uniform(0.02, 0.98, size=(40, sec.n))
        whole = term_orders(sec, x, prob.order_min, prob.order_max)
        tot = np.zeros_like(whole)
        for i in idx:
            face = parts.sectors[i]
            tm = getattr(face, "tmask", 0)
            tot = tot + term_orders(face, separate.face_point(sec, tm, x), prob.order_min, prob.order_max)
        np.testing.assert_allclose(tot, whole, rtol=1e-9, atol=1e-9 * float(np.max(np.abs(whole))))


def test_refusals():
    sec = two_var_sector(1.0, 1.0)
    sec.factors = [Factor(1.0, 0.0, np.array([1.0]), np.array([[1, 0]], dtype=np.uint8))]
    with pytest.raises(ValueError):
        separate.face_sector(sec, 1)
    with pytest.raises(ValueError):
        separate.separate(Problem([two_var_sector(1.0, 1.0)], -2, 0, complex_mode=True))
