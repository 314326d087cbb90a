"""Oracle: the eps-expanded sector integrand at single points in multiprecision.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The same formula as oracle.integrand.sector_f (pole subtraction at x_j = 0 for
j in S, eps expansion of x_j^(b_j eps) and G = G0 exp(eps Lambda); section 1
and eq. (2)), in real mode and in complex mode (the contour deformation of
section 4.4: z_j = y_j - i lam y_j (1 - y_j) dF/dy_j at each corner y of the
subtraction, G = det(dz/dy) prod_j w_j^(a_j + b_j eps) prod_m P_m(z)^(...),
principal logarithms with arg = -pi on the negative real axis), evaluated
with mpmath.  The corner terms near a face x_j -> 0 cancel by at most about
log10(1/x_j) digits per singular variable, so the working precision is 40
decimal digits plus sum_{j in S} log10(1/x_j) at each point (or a fixed
`dps`): the result keeps well over 32 correct digits, which makes it the
exact value against which a double-double evaluation is judged.  This plays
the part of the paper's MPFR evaluation below the SmallX threshold (section
4.6, mixed arithmetic; section 4.4 for complex mode).

Parity unpinned by the paper itself (it prints no near-face values); pinned in
tests/test_oracle_mp.py against the fp64 oracle where fp64 is accurate, against
closed forms of one- and two-variable sectors that stay exact at the faces,
against itself at a higher precision, and in complex mode against the closed
forms of the massive bubble and of a one-variable sector whose factor changes
sign inside the cube (hypergeometric, with the -i0 side), integrated by
tanh-sinh quadrature whose nodes crowd the faces, and against the product
structure of a two-variable sector.
"""
from __future__ import annotations

from typing import Sequence

import mpmath
import numpy as np

from .integrand import singular_set


def _poly_mp(coef, exps, y):
    """sum_t coef_t prod_j y_j^exps_tj with mpf arithmetic (coefficients are exact binary values)."""
    s = mpmath.mpf(0)
    for t in range(coef.shape[0]):
        c = complex(coef[t])
        m = mpmath.mpc(c.real, c.imag) if c.imag else mpmath.mpf(c.real)
        for j, e in enumerate(exps[t]):
            if e:
                m *= y[j] ** int(e)
        s += m
    return s


def point_dps(sector, x: Sequence[float]) -> int:
    """40 digits plus what the corner terms at x can cancel."""
    S = singular_set(sector)
    return 40 + int(np.ceil(sum(max(0.0, -np.log10(float(x[j]))) for j in S)))


def _log_mi0(p):
    """Principal logarithm; a real negative argument takes arg = -pi (the side F - i0 approaches)."""
    p = mpmath.mpc(p)
    if p.imag == 0 and p.real < 0:
        return mpmath.mpc(mpmath.log(-p.real), -mpmath.pi)
    return mpmath.log(p)


def _deform_terms(sector):
    """Coefficients (real parts: the deformation follows Re F) and exponents of x^mono * P_F."""
    fac = sector.factors[sector.deform_factor]
    mono = sector.deform_mono if sector.deform_mono is not None else np.zeros(sector.n, np.int32)
    return np.real(fac.coef), fac.exps.astype(np.int64) + np.asarray(mono, np.int64)[None, :]


def _derivative(coef, exps, j):
    """d/dy_j of sum_t coef_t y^exps_t, as (coef, exps) lists (terms without y_j dropped)."""
    c, e = [], []
    for t in range(len(coef)):
        if exps[t][j] > 0:
            c.append(float(coef[t]) * float(exps[t][j]))
            r = np.array(exps[t], dtype=np.int64)
            r[j] -= 1
            e.append(r)
    return c, e


def _corner(sector, y, complex_mode: bool, lam: float):
    """G0 and Lambda of G(y, eps) = G0 exp(eps Lambda) at the corner point y (a list of mpf)."""
    if not complex_mode:
        g0 = mpmath.mpf(1)
        lm = mpmath.mpf(0)
        for fac in sector.factors:
            p = _poly_mp(fac.coef, fac.exps, y)
            g0 *= mpmath.power(p, mpmath.mpf(float(fac.gamma)))
            if fac.delta != 0.0:           # P^gamma alone has no eps dependence (and may vanish)
                lp = mpmath.log(p) if p > 0 else mpmath.mpf("nan")
                lm += mpmath.mpf(float(fac.delta)) * lp
        return g0, lm
    n = sector.n
    lam_ = mpmath.mpf(float(lam))
    grad = [mpmath.mpf(0)] * n
    hess = [[mpmath.mpf(0)] * n for _ in range(n)]
    if sector.deform_factor >= 0:
        coef, exps = _deform_terms(sector)
        for j in range(n):
            cj, ej = _derivative(coef, exps, j)
            if not cj:
                continue
            grad[j] = _poly_mp(np.array(cj), np.array(ej), y)
            for k in range(n):
                ck, ek = _derivative(cj, ej, k)
                if ck:
                    hess[j][k] = _poly_mp(np.array(ck), np.array(ek), y)
    z = [y[j] - 1j * lam_ * y[j] * (1 - y[j]) * grad[j] for j in range(n)]
    w = [1 - 1j * lam_ * (1 - y[j]) * grad[j] for j in range(n)]
    jac = mpmath.matrix(n, n)
    for j in range(n):
        for k in range(n):
            v = -1j * lam_ * y[j] * (1 - y[j]) * hess[j][k]
            if j == k:
                v += 1 - 1j * lam_ * (1 - 2 * y[j]) * grad[j]
            jac[j, k] = v
    g0 = mpmath.mpc(mpmath.det(jac))
    lm = mpmath.mpc(0)
    for j in range(n):
        lw = _log_mi0(w[j])
        g0 *= mpmath.exp(mpmath.mpf(float(sector.a[j])) * lw)
        lm += mpmath.mpf(float(sector.b[j])) * lw
    for fac in sector.factors:
        lp = _log_mi0(_poly_mp(fac.coef, fac.exps, z))
        g0 *= mpmath.exp(mpmath.mpf(float(fac.gamma)) * lp)
        lm += mpmath.mpf(float(fac.delta)) * lp
    return g0, lm


def sector_f_point(sector, x: Sequence[float], kf_max: int, dps: int = 0, complex_mode: bool = False,
                   lam: float = 0.0):
    """f_k(x) for k = -|S| .. kf_max at one point, as mpf (mpc in complex mode)
    values, and the sums of |term| per order (cond), both lists indexed k + |S|;
    dps 0: point_dps."""
    S = singular_set(sector)
    ns = len(S)
    dps = dps or point_dps(sector, x)
    nonS = [j for j in range(sector.n) if j not in S]
    korders = kf_max + ns + 1
    with mpmath.workdps(dps):
        # fp64 points are exact binary values; mpf points (quadrature nodes) are kept as given
        xm = [v if isinstance(v, mpmath.mpf) else mpmath.mpf(float(v)) for v in x]
        lnx = [mpmath.log(v) for v in xm]
        mono = mpmath.mpf(1)
        lrest = mpmath.mpf(0)
        for j in nonS:
            mono *= mpmath.power(xm[j], mpmath.mpf(float(sector.a[j])))
            lrest += mpmath.mpf(float(sector.b[j])) * lnx[j]
        zero = mpmath.mpc(0) if complex_mode else mpmath.mpf(0)
        f = [zero] * korders
        cond = [mpmath.mpf(0)] * korders
        for wmask in range(1 << ns):
            y = list(xm)
            for i in range(ns):
                if wmask >> i & 1:
                    y[S[i]] = mpmath.mpf(0)
            g0, lm = _corner(sector, y, complex_mode, lam)
            tmask = wmask
            while True:
                sign = -1 if bin(wmask & ~tmask).count("1") % 2 else 1
                nt = bin(tmask).count("1")
                coef = mpmath.mpf(sign)
                lt = lrest
                for i in range(ns):
                    j = S[i]
                    if tmask >> i & 1:
                        coef /= mpmath.mpf(float(sector.b[j]))
                    else:
                        coef /= xm[j]
                        lt += mpmath.mpf(float(sector.b[j])) * lnx[j]
                base = coef * mono * g0
                zz = lt + lm
                for k in range(-ns, kf_max + 1):
                    q = k + nt
                    if q < 0:
                        continue
                    term = base * zz ** q / mpmath.factorial(q)
                    f[k + ns] += term
                    cond[k + ns] += abs(term)
                if tmask == 0:
                    break
                tmask = (tmask - 1) & wmask
        return f, cond


def sector_orders_mp(sector, x: np.ndarray, order_min: int, order_max: int, pref_lead: int,
                     pref: Sequence[float], dps: int = 0, complex_mode: bool = False, lam: float = 0.0):
    """F_k(x) = c_s sum_i Pi_i f_{k - lead - i}(x), k = order_min .. order_max, real
    or complex mode, at every point of x (npts, n): the multiprecision values rounded once to
    fp64 (K, npts), the term sums cond (K, npts) as in oracle.integrand, and
    foldabs (K, npts) = sum_i |c_s Pi_i f_{k-lead-i}| (what an fp64 fold of exact
    f values can lose: a few ulp of it)."""
    S = singular_set(sector)
    ns = len(S)
    kf_max = order_max - pref_lead
    K = order_max - order_min + 1
    npts = x.shape[0]
    cplx = complex_mode or any(complex(v).imag != 0.0 for v in pref) or complex(sector.coeff).imag != 0.0
    vals = np.zeros((K, npts), dtype=np.complex128 if cplx else np.float64)
    cnd = np.zeros((K, npts))
    fabs_ = np.zeros((K, npts))
    cs = complex(sector.coeff)
    for p in range(npts):
        d = dps or point_dps(sector, x[p])
        f, cond = sector_f_point(sector, x[p], max(kf_max, -ns), d, complex_mode, lam)
        with mpmath.workdps(d):
            for ki, k in enumerate(range(order_min, order_max + 1)):
                v = mpmath.mpc(0)
                for i, pv in enumerate(pref):
                    kk = k - pref_lead - i
                    if kk < -ns or kk > kf_max:
                        continue
                    t = mpmath.mpc(cs) * mpmath.mpc(complex(pv)) * f[kk + ns]
                    v += t
                    cnd[ki, p] += abs(cs) * abs(complex(pv)) * float(cond[kk + ns])
                    fabs_[ki, p] += float(abs(t))
                vals[ki, p] = complex(v) if cplx else float(v.real)
    return vals, cnd, fabs_
