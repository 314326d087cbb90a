"""Oracle: the eps-expanded sector integrand, point by point, in fp64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

A sector (eq. (2) after sector decomposition, section 1) is

    I_s = c_s int_[0,1]^n prod_j x_j^(a_j + b_j eps) G(x, eps) dx,
    G(x, eps) = prod_m P_m(x)^(gamma_m + delta_m eps),

with a_j = -1 exactly (and b_j != 0) on the singular set S and a_j > -1
elsewhere.  The paper defers pole resolution and the eps expansion to the
earlier FIESTA papers (section 1); the form used here is the standard
subtraction at x_j = 0:

    int_0^1 x^(-1 + b eps) g(x) dx = int_0^1 x^(-1 + b eps) (g(x) - g(0)) dx + g(0)/(b eps),

applied to every j in S.  Writing x^(W) for x with x_j = 0 for j in W, and
expanding x_j^(b_j eps) = exp(eps b_j ln x_j) and G = G0 exp(eps Lambda),

    f_k(x) = sum_{W subset S} sum_{T subset W} (-1)^|W\\T| prod_{j in T} 1/b_j
             prod_{j in S\\T} 1/x_j  prod_{j not in S} x_j^a_j
             G0(x^(W)) (L_T(x) + Lambda(x^(W)))^q / q!,        q = k + |T| >= 0,
    L_T = sum_{j in S\\T} b_j ln x_j + sum_{j not in S} b_j ln x_j,

is the integrand of the eps^k coefficient of I_s / c_s.

Complex mode (section 4.4, ComplexMode; the -i0 of eq. (1) and eq. (2)):
the sector variables move to z_j = x_j - i lam x_j (1 - x_j) dF/dx_j, F the
sector's deformation polynomial x^m P_F: P_F is the sector's reduced F factor
(what is left of F after the decomposition takes the monomial out; it has a
constant term and carries the F - i0 branch) and m its optional monomial
(deform_mono, zero by default, so F = P_F), so that Im F(z) <= 0 to first order.  With
z_j = x_j w_j, w_j = 1 - i lam (1 - x_j) dF/dx_j, the monomial keeps its real
form and

    G(x, eps) = det(dz/dx) prod_j w_j^(a_j + b_j eps) prod_m P_m(z)^(gamma_m + delta_m eps).

Term coefficients may be complex in complex mode (complex masses, whose
negative imaginary parts already put F below the real axis): the factors are
evaluated with them, and the deformation follows the gradient of Re F (a
reading: the paper defines the deformation for real F only).

Logarithms are principal; a factor that is real and negative takes
arg = -pi (the value approached from Im < 0, as F - i0 prescribes).  Points
with Im F(z) > 0 are counted, as the TestF check of section 4.6 does.

The result orders come from the prefactor fold
F_k(x) = c_s sum_i Pi_i f_{k - lead - i}(x) (section 4.3, SDEvaluate).
"""
from __future__ import annotations

from math import factorial
from typing import List, Sequence, Tuple

import numpy as np


def singular_set(sector) -> List[int]:
    s = [j for j in range(sector.n) if sector.a[j] == -1.0]
    for j in s:
        if sector.b[j] == 0.0:
            raise ValueError("a_j = -1 needs b_j != 0")
    for j in range(sector.n):
        if j not in s and not sector.a[j] > -1.0:
            raise ValueError("a_j must be -1 or > -1")
    return s


def poly(coef: np.ndarray, exps: np.ndarray, y: np.ndarray) -> np.ndarray:
    """sum_t coef_t prod_j y_j^exps_tj at every point of y (npts, n)."""
    out = np.zeros(y.shape[0], dtype=y.dtype)
    for t in range(coef.shape[0]):
        mono = np.full(y.shape[0], coef[t], dtype=y.dtype)
        for j in range(exps.shape[1]):
            e = int(exps[t, j])
            if e:
                mono = mono * y[:, j] ** e
        out = out + mono
    return out


def log_minus_i0(p: np.ndarray) -> np.ndarray:
    """Principal complex log; on the negative real axis the branch below the cut."""
    p = np.asarray(p, dtype=np.complex128)
    ang = np.angle(p)
    ang = np.where((p.imag == 0.0) & (p.real < 0.0), -np.pi, ang)
    return np.log(np.abs(p)) + 1j * ang


def full_f_terms(sector) -> Tuple[np.ndarray, np.ndarray]:
    """Coefficients and integer exponents of the deformation polynomial x^mono * P_F (mono = 0: P_F);
    for complex coefficients (complex masses) their real parts: the deformation follows Re F."""
    fac = sector.factors[sector.deform_factor]
    mono = sector.deform_mono if sector.deform_mono is not None else np.zeros(sector.n, np.int32)
    return np.real(fac.coef).astype(np.float64), fac.exps.astype(np.int64) + mono.astype(np.int64)[None, :]


def _poly_int(coef, exps, y):
    out = np.zeros(y.shape[0], dtype=np.float64)
    for t in range(coef.shape[0]):
        if coef[t] == 0.0:
            continue
        mono = np.full(y.shape[0], coef[t])
        for j in range(exps.shape[1]):
            e = int(exps[t, j])
            if e:
                mono = mono * y[:, j] ** e
        out = out + mono
    return out


def f_derivatives(sector, y: np.ndarray):
    """Gradient (npts, n) and Hessian (npts, n, n) of the deformation polynomial at real points y."""
    coef, exps = full_f_terms(sector)
    n = sector.n
    grad = np.zeros((y.shape[0], n))
    hess = np.zeros((y.shape[0], n, n))
    for j in range(n):
        cj = coef * exps[:, j]
        ej = exps.copy()
        ej[:, j] -= 1
        keep = cj != 0
        grad[:, j] = _poly_int(cj[keep], ej[keep], y)
        for k in range(n):
            ck = cj * ej[:, k]
            ek = ej.copy()
            ek[:, k] -= 1
            keep2 = (ck != 0)
            hess[:, j, k] = _poly_int(ck[keep2], ek[keep2], y)
    return grad, hess


def regular_part(sector, y: np.ndarray, complex_mode: bool, lam: float):
    """G0(y) and Lambda(y) of G(y, eps) = G0 exp(eps Lambda); also Im F(z) > 0 flags."""
    npts, n = y.shape
    if not complex_mode:
        if any(np.iscomplexobj(f.coef) and np.any(np.imag(f.coef) != 0) for f in sector.factors):
            raise ValueError("complex term coefficients need complex mode")
        g0 = np.ones(npts)
        lam_ = np.zeros(npts)
        for fac in sector.factors:
            p = poly(fac.coef, fac.exps, y)
            g0 = g0 * p ** fac.gamma
            if fac.delta != 0.0:            # P^gamma alone has no eps dependence (and may vanish)
                lam_ = lam_ + fac.delta * np.log(p)
        return g0, lam_, np.zeros(npts, dtype=bool)
    if sector.deform_factor >= 0:
        grad, hess = f_derivatives(sector, y)
    else:
        grad, hess = np.zeros((npts, n)), np.zeros((npts, n, n))
    z = (y - 1j * lam * y * (1.0 - y) * grad).astype(np.complex128)
    w = 1.0 - 1j * lam * (1.0 - y) * grad
    jac = np.zeros((npts, n, n), dtype=np.complex128)
    for j in range(n):
        for k in range(n):
            v = -1j * lam * y[:, j] * (1.0 - y[:, j]) * hess[:, j, k]
            if j == k:
                v = v + 1.0 - 1j * lam * (1.0 - 2.0 * y[:, j]) * grad[:, j]
            jac[:, j, k] = v
    det = np.linalg.det(jac)
    g0 = det.astype(np.complex128)
    lam_ = np.zeros(npts, dtype=np.complex128)
    for j in range(n):
        lw = log_minus_i0(w[:, j])
        g0 = g0 * np.exp(sector.a[j] * lw)
        lam_ = lam_ + sector.b[j] * lw
    for fac in sector.factors:
        lp = log_minus_i0(poly(fac.coef, fac.exps, z))
        g0 = g0 * np.exp(fac.gamma * lp)
        lam_ = lam_ + fac.delta * lp
    if sector.deform_factor < 0:
        return g0, lam_, np.zeros(npts, dtype=bool)
    coef, exps = full_f_terms(sector)
    fz = np.zeros(npts, dtype=np.complex128)
    for t in range(coef.shape[0]):
        mono = np.full(npts, coef[t], dtype=np.complex128)
        for j in range(n):
            if exps[t, j]:
                mono = mono * z[:, j] ** int(exps[t, j])
        fz = fz + mono
    return g0, lam_, fz.imag > 0.0


def sector_f(sector, x: np.ndarray, kf_max: int, complex_mode: bool = False, lam: float = 0.0):
    """f_k(x) for k = -|S| .. kf_max (rows), with the absolute term sums (cond).

    Returns (f, cond, imf_pos) with f of shape (kf_max + |S| + 1, npts).  A
    sector marked ``boundary = False`` (a separated term, oracle/separate.py)
    keeps only the subtracted integrand, the T = {} part of the sum.
    """
    boundary = getattr(sector, "boundary", True)
    S = singular_set(sector)
    ns = len(S)
    nonS = [j for j in range(sector.n) if j not in S]
    npts = x.shape[0]
    dtype = np.complex128 if complex_mode else np.float64
    korders = kf_max + ns + 1
    f = np.zeros((korders, npts), dtype=dtype)
    cond = np.zeros((korders, npts))
    lnx = np.log(x)
    mono = np.ones(npts)
    lrest = np.zeros(npts)
    for j in nonS:
        mono = mono * x[:, j] ** sector.a[j]
        lrest = lrest + sector.b[j] * lnx[:, j]
    imf_pos = np.zeros(npts, dtype=bool)
    for wmask in range(1 << ns):
        y = x.copy()
        for i in range(ns):
            if wmask >> i & 1:
                y[:, S[i]] = 0.0
        g0, lam_w, pos = regular_part(sector, y, complex_mode, lam)
        imf_pos |= pos
        tmask = wmask if boundary else 0
        while True:                                   # every T subset of W
            sign = -1.0 if bin(wmask & ~tmask).count("1") % 2 else 1.0
            nt = bin(tmask).count("1")
            coef = np.full(npts, sign)
            lt = lrest.copy()
            for i in range(ns):
                j = S[i]
                if tmask >> i & 1:
                    coef = coef / sector.b[j]
                else:
                    coef = coef / x[:, j]
                    lt = lt + sector.b[j] * lnx[:, j]
            base = coef * mono * g0
            zz = lt + lam_w
            for k in range(-ns, kf_max + 1):
                q = k + nt
                if q < 0:
                    continue
                term = base * zz ** q / factorial(q)
                f[k + ns] += term
                cond[k + ns] += np.abs(term)
            if tmask == 0:
                break
            tmask = (tmask - 1) & wmask
    return f, cond, imf_pos


def sector_orders(sector, x: np.ndarray, order_min: int, order_max: int, pref_lead: int,
                  pref: Sequence[complex], complex_mode: bool = False, lam: float = 0.0):
    """F_k(x) = c_s sum_i Pi_i f_{k - lead - i}(x) for k = order_min .. order_max.

    A sector with ``eps_shift = s`` (a separated term) stands for eps^-s times
    its own integral.  Returns (vals (K, npts), cond (K, npts), imf_pos (npts,)).
    """
    S = singular_set(sector)
    shift = getattr(sector, "eps_shift", 0)
    ns = len(S) + shift
    kf_max = order_max - pref_lead
    f, cond, pos = sector_f(sector, x, max(kf_max + shift, -len(S)), complex_mode, lam)
    K = order_max - order_min + 1
    cplx = complex_mode or any(complex(p).imag != 0.0 for p in pref) or complex(sector.coeff).imag != 0.0
    vals = np.zeros((K, x.shape[0]), dtype=np.complex128 if cplx else np.float64)
    cnd = np.zeros((K, x.shape[0]))
    cs = complex(sector.coeff) if cplx else complex(sector.coeff).real
    for ki, k in enumerate(range(order_min, order_max + 1)):
        for i, p in enumerate(pref):
            kk = k - pref_lead - i
            if kk < -ns or kk > kf_max:
                continue
            pv = complex(p) if cplx else complex(p).real
            vals[ki] += cs * pv * f[kk + ns]
            cnd[ki] += abs(cs) * abs(pv) * cond[kk + ns]
    return vals, cnd, pos
