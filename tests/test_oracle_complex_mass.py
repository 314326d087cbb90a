"""Pins of complex term coefficients in the sector oracle (complex masses in
complex mode; oracle/integrand.py and oracle/integrand_mp.py).

The equal-mass bubble at p^2 = s has, in the normalisation of the prefactor
(eps^-1 coefficient 1), the eps^0 coefficient -int_0^1 ln(m^2 - s x(1 - x)) dx
(for a real mass the logarithm takes the -i0 side).  With m^2 = M^2 - i M Gamma
the logarithm's argument stays below the real axis on [0, 1], so that integral
of an elementary function, by mpmath quadrature, is the reference.  The sector
integrand with complex coefficients, integrated over its primary sectors, must
reproduce it without deformation and with one (Cauchy's theorem: the
deformation follows Re F and keeps Im F below zero).  Complex coefficients are
refused in real mode."""
import mpmath
import numpy as np
import pytest

from oracle import integrand, integrate
from oracle import integrand_mp as M
from sectorgen.feynman import complex_mass_bubble_problem, massive_bubble_problem


def gl_orders(prob, kf, nodes=80):
    t, w = np.polynomial.legendre.leggauss(nodes)
    t, w = 0.5 * (t + 1.0), 0.5 * w
    tot = 0
    for sec in prob.sectors:
        f, _, _ = integrand.sector_f(sec, t[:, None], kf, True, prob.lam)
        tot = tot + f @ w
    return tot


def reference(s, m2, dps=30):
    with mpmath.workdps(dps):
        m = mpmath.mpc(m2.real, m2.imag)
        return -mpmath.quad(lambda x: mpmath.log(m - s * x * (1 - x)), [0, 0.5, 1])


@pytest.mark.parametrize("m2,lam", [(1.0 - 0.25j, 0.0), (1.0 - 0.25j, 0.3), (0.8 - 0.05j, 0.2), (2.0 - 1.0j, 0.0)])
def test_complex_mass_bubble(m2, lam):
    prob = complex_mass_bubble_problem(5.0, m2, lam)
    lead, pref = integrate.prefactor_for(prob)
    assert lead == -1 and pref[0] == 1.0 and pref[1] == 0.0
    f = gl_orders(prob, 1)
    assert abs(f[0] - 1.0) < 1e-13
    ref = complex(reference(5.0, m2))
    assert abs(f[1] - ref) < 1e-12 * abs(ref), (f[1], ref)


def test_real_mass_limit_is_the_minus_i0_side():
    """The same formula with a real mass and the -i0 prescription gives the real-mass bubble's value."""
    prob = massive_bubble_problem(5.0, 1.0, 0.5)
    f = gl_orders(prob, 1)
    with mpmath.workdps(30):
        ref = -mpmath.quad(lambda x: mpmath.log(mpmath.mpc(1 - 5 * x * (1 - x), -mpmath.mpf(10) ** -40)),
                           [0, (5 - mpmath.sqrt(5)) / 10, (5 + mpmath.sqrt(5)) / 10, 1])
    assert abs(f[1] - complex(ref)) < 1e-12


def test_multiprecision_oracle_with_complex_coefficients():
    prob = complex_mass_bubble_problem(5.0, 1.0 - 0.25j, 0.3)
    with mpmath.workdps(30):
        tot = 0
        for sec in prob.sectors:
            tot += mpmath.quad(lambda x: M.sector_f_point(sec, [x], 1, dps=30, complex_mode=True, lam=prob.lam)[0][1],
                               [0, 1])
        assert abs(tot - reference(5.0, 1.0 - 0.25j)) < mpmath.mpf(10) ** -25


def test_complex_coefficients_need_complex_mode():
    sec = complex_mass_bubble_problem().sectors[0]
    with pytest.raises(ValueError):
        integrand.sector_f(sec, np.full((2, 1), 0.5), 1, False, 0.0)
