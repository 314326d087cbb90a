"""Pins of the deformation-size search oracle (oracle/deform.py)."""
import cmath

import numpy as np
import pytest

from oracle import deform
from oracle.integrand import singular_set
from sectorgen.feynman import double_box_problem, massive_bubble_problem


def scalar_imf(sector, x, lam):
    """Im F(z) > 0 at some corner, from plain complex arithmetic and numerical derivatives.

    Independent of the oracle: F is the deform factor times the factored
    monomial, evaluated term by term; dF/dy_j by central differences of that
    same scalar function (step 1e-6, enough to fix a sign that is not borderline)."""
    fac = sector.factors[sector.deform_factor]
    mono = sector.deform_mono

    def F(v):
        tot = 0j
        for c, e in zip(fac.coef, fac.exps):
            t = complex(c)
            for j in range(sector.n):
                t *= v[j] ** int(e[j] + mono[j])
            tot += t
        return tot

    S = singular_set(sector)
    for wmask in range(1 << len(S)):
        y = list(x)
        for i, j in enumerate(S):
            if wmask >> i & 1:
                y[j] = 0.0
        z = []
        for j in range(sector.n):
            h = 1e-6
            yp, ym = list(y), list(y)
            yp[j] += h
            ym[j] -= h
            g = (F(yp) - F(ym)).real / (2 * h)
            z.append(complex(y[j], -lam * y[j] * (1 - y[j]) * g))
        if F(z).imag > 0:
            return True
    return False


def test_imf_flags_match_plain_complex_arithmetic():
    prob = double_box_problem(5.0, -2.0, 1.0, order_max=0, complex_mode=True, lam=0.5)
    rng = np.random.default_rng(5)
    checked = 0
    for s in (0, 7, 19):
        sec = prob.sectors[s]
        x = rng.uniform(0.05, 0.95, size=(40, sec.n))
        for lam in (0.5, 0.2):
            flags = deform.imf_positive(sec, x, lam)
            for i in range(x.shape[0]):
                assert flags[i] == scalar_imf(sec, x[i], lam), (s, lam, i)
                checked += 1
    assert checked == 240


def test_first_order_deformation_never_fails():
    """Im F(z) = -lam sum_j y_j (1 - y_j) (dF/dy_j)^2 + O(lam^2) <= 0 for small lam."""
    prob = double_box_problem(5.0, -2.0, 1.0, order_max=0, complex_mode=True, lam=0.5)
    for s in (0, 11, 29):
        sec = prob.sectors[s]
        x = deform.test_points(sec, s, 8, 1)
        assert not deform.imf_positive(sec, x, 1e-7).any()
        assert deform.tune_lambda(sec, s, 1e-7, 4, 8, 1) == 1e-7


def test_tuned_lambda_is_largest_passing_candidate():
    prob = double_box_problem(5.0, -2.0, 1.0, order_max=0, complex_mode=True, lam=0.5)
    sec = prob.sectors[3]
    lam = deform.tune_lambda(sec, 3, 0.5, 4, 9, 2)
    x = deform.test_points(sec, 3, 9, 2)
    assert 0.0 < lam < 0.5
    assert not deform.imf_positive(sec, x, lam).any()
    grid = [0.5 * k / 4 for k in range(1, 5)]
    assert lam in grid
    for g in grid:
        if g > lam:
            assert deform.imf_positive(sec, x, g).any()
    assert deform.tune_lambda(sec, 3, 0.5, 4, 9, 2, conservative=True) == lam / 2


def test_massive_bubble_keeps_the_full_deformation():
    prob = massive_bubble_problem(5.0, 1.0, 0.5)
    assert [deform.tune_lambda(sec, s, 0.5, 4, 10, 1) for s, sec in enumerate(prob.sectors)] == [0.5, 0.5]
