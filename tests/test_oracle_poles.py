"""Pins of the oracle's reduction of a_j < -1 (oracle/poles.py): the reduced
sectors, integrated by quadrature and weighted by their coefficient series,
reproduce closed forms - hypergeometric Laurent series in one variable for
a = -2, -3 and -1.5, a separable product in two variables, and a polynomial
integrand whose continuation is elementary; the expansion's structure (which
sectors, which series) for a hand-checked case."""

import mpmath as mp
import numpy as np
import pytest

from sectorgen import Factor, Sector
from oracle import integrand, poles

from test_oracle_pins import quad_sector_f, taylor


def laurent_total(secs, series, kmin, kmax, nodes=90, power=6):
    """sum_i c_i(eps) I_i(eps) as Laurent coefficients eps^kmin .. eps^kmax."""
    out = np.zeros(kmax - kmin + 1, complex)
    for sec, c in zip(secs, series):
        ns = len(integrand.singular_set(sec))
        kf = kmax + ns
        f = quad_sector_f(sec, kf, nodes=nodes, power=power)       # eps^-ns ...
        for i, fk in enumerate(f):
            for q, cq in enumerate(c):
                k = i - ns + q
                if kmin <= k <= kmax:
                    out[k - kmin] += cq * fk
    return out


def hyp(a, b, c, gam, dlt, n, pole):
    """int_0^1 x^(a+b eps) (1+cx)^(gam+dlt eps) dx = 2F1(-gam-dlt eps, s; s+1; -c)/s, s = a+1+b eps."""
    def h(e):
        s = a + 1 + b * e
        v = mp.hyp2f1(-(gam + dlt * e), s, s + 1, -c) / s
        return v * e ** pole
    return taylor(h, n)


@pytest.mark.parametrize("a,b,c,gam,dlt,pole", [
    (-2.0, 1.0, 0.7, -2.0, 1.0, 1), (-2.0, -0.5, 1.3, 1.0, -2.0, 1), (-3.0, 2.0, 0.4, -1.0, 1.0, 1),
    (-1.5, 1.0, 0.9, -2.0, 1.0, 0), (-2.0, 1.0, 0.5, 0.5, 1.0, 1),
])
def test_one_variable_closed_forms(a, b, c, gam, dlt, pole):
    sec = Sector(a=np.array([a]), b=np.array([b]),
                 factors=[Factor(gam, dlt, np.array([1.0, c]), np.array([[0], [1]], dtype=np.uint8))])
    secs, series, origin = poles.expand([sec])
    assert origin == [0] * len(secs)
    assert all(s.a[0] >= -1.0 for s in secs)
    got = laurent_total(secs, series, -pole, 3, nodes=200, power=8)
    ref = hyp(a, b, c, gam, dlt, 3 + pole, pole)
    for k in range(len(got)):
        assert got[k] == pytest.approx(ref[k].real, rel=1e-9, abs=1e-11), (k, got[k], ref[k])


def test_two_variables_separable():
    """x^(-2+eps) y^(-1-2eps) (1+0.7x)^(-1+eps) (1+1.3y)^(-2-eps): product of one-variable series."""
    sec = Sector(a=np.array([-2.0, -1.0]), b=np.array([1.0, -2.0]), factors=[
        Factor(-1.0, 1.0, np.array([1.0, 0.7]), np.array([[0, 0], [1, 0]], dtype=np.uint8)),
        Factor(-2.0, -1.0, np.array([1.0, 1.3]), np.array([[0, 0], [0, 1]], dtype=np.uint8))])
    secs, series, _ = poles.expand([sec])
    got = laurent_total(secs, series, -2, 2, nodes=70)
    s1 = hyp(-2.0, 1.0, 0.7, -1.0, 1.0, 6, 1)             # from eps^-1
    s2 = hyp(-1.0, -2.0, 1.3, -2.0, -1.0, 6, 1)           # from eps^-1
    prod = np.convolve(np.real(s1), np.real(s2))         # from eps^-2
    for k in range(len(got)):
        assert got[k] == pytest.approx(prod[k], rel=1e-8, abs=1e-10), k


def test_structure_of_a_polynomial_case():
    """int x^(-2+b eps) (1 + c x) dx = 1/(-1+b eps) + c/(b eps): boundary sector with
    series 1/(-1+b eps) and P(1) = 1 + c; derivative sector x^(-1+b eps) c with
    series -1/(-1+b eps)."""
    b, c = 0.5, 3.0
    sec = Sector(a=np.array([-2.0]), b=np.array([b]),
                 factors=[Factor(1.0, 0.0, np.array([1.0, c]), np.array([[0], [1]], dtype=np.uint8))])
    secs, series, _ = poles.expand([sec])
    assert len(secs) == 2
    bnd, der = secs
    assert bnd.a[0] == 0.0 and bnd.b[0] == 0.0
    assert len(bnd.factors) == 1 and bnd.factors[0].coef.tolist() == [1.0 + c]
    assert der.a[0] == -1.0 and len(der.factors) == 1            # P^0 dropped, dP/dx = c appended
    assert der.factors[0].coef.tolist() == [c] and der.factors[0].gamma == 1.0
    inv = [(-1.0) * b ** q for q in range(poles.SERIES_LEN)]     # 1/(-1 + b eps) = -sum (b eps)^q
    assert np.allclose(series[0], inv)
    assert np.allclose(series[1], [-v for v in inv])
    got = laurent_total(secs, series, -1, 3)
    # 1/(-1+b e) + c/(b e) = c/b e^-1 - sum (b e)^q
    exact = [c / b] + [-(b ** q) for q in range(4)]
    assert np.allclose(got, exact, rtol=1e-12, atol=1e-12)


def test_reduction_leaves_other_sectors_alone_and_keeps_order():
    plain = Sector(a=np.array([-1.0, 0.0]), b=np.array([1.0, 0.0]),
                   factors=[Factor(-1.0, 1.0, np.array([1.0, 2.0]), np.array([[0, 0], [1, 1]], dtype=np.uint8))])
    low = Sector(a=np.array([0.0, -2.0]), b=np.array([0.0, 1.0]),
                 factors=[Factor(-2.0, 1.0, np.array([1.0, 2.0, 1.0]), np.array([[0, 0], [0, 1], [1, 1]],
                                                                             dtype=np.uint8))])
    secs, series, origin = poles.expand([plain, low, plain])
    assert origin[0] == 0 and origin[-1] == 2 and set(origin[1:-1]) == {1}
    assert secs[0] is plain and secs[-1] is plain
    assert series[0][0] == 1.0 and np.all(series[0][1:] == 0)
    # the boundary sector of `low` merged the rows (0,1)->(0,0) and (1,1)->(1,0): 1 + 2 = 3 and 1
    bnd = secs[1]
    assert bnd.factors[0].coef.tolist() == [3.0, 1.0]
    assert bnd.factors[0].exps.tolist() == [[0, 0], [1, 0]]
