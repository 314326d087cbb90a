"""Oracle: sectors with monomial exponents a_j < -1, reduced to a_j >= -1.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Eq. (2) leaves, after decomposition, sector integrals
int_0^1 x_j^(a_j + b_j eps) G(x) dx_j whose exponent can lie below -1 (a
propagator raised to a power, or d0 below 4).  They are defined by analytic
continuation in eps, and the subtraction of the evaluator handles a_j = -1
only.  With alpha = a_j + 1 + b_j eps, x^(a_j + b_j eps) = (1/alpha) d/dx
x^alpha, so integrating by parts

    int_0^1 x^(a+b eps) G dx = G|_(x_j=1) / alpha - (1/alpha) int_0^1 x^alpha dG/dx_j dx

(the boundary term at 0 vanishes in the continuation: it does for
Re alpha > 0 and both sides are analytic), and for G = prod_m P_m^(g_m + d_m eps)

    dG/dx_j = sum_m (g_m + d_m eps) (dP_m/dx_j) P_m^(g_m - 1 + d_m eps) prod_(m' != m) P_m'^(...).

Each step raises a_j by one; steps repeat until every a_j >= -1.  The result
is a list of sectors, each with a coefficient series in eps (products of
1/alpha and of (g_m + d_m eps)) that multiplies the problem's prefactor.
Readings (the paper says nothing about a_j < -1; its predecessors use
Taylor subtraction of higher order, which defines the same continuation):

* Order of the expansion: sectors in input order; within a sector the lowest
  variable with a_j < -1 first; the boundary sector (x_j = 1: the exponents of
  x_j set to 0, equal exponent rows merged in order of first occurrence,
  a_j = b_j = 0, so the variable stays and integrates to 1) before the
  derivative sectors, these by factor index; factors whose exponent becomes
  (0, 0) are dropped; the derivative factor dP_m/dx_j (exponent (1, 0), terms
  in P_m's order) is appended last; depth first.
* A boundary factor whose terms all cancel gives zero if its exponent is
  positive (the sector is dropped) and is an error otherwise.
* Coefficient series are truncated at SERIES_LEN terms.
"""
from __future__ import annotations

from typing import List, Tuple

import numpy as np

from sectorgen import Factor, Sector

SERIES_LEN = 12


def inv_alpha(alpha0: float, b: float) -> np.ndarray:
    """1/(alpha0 + b eps) = (1/alpha0) sum_q (-b/alpha0)^q eps^q."""
    return np.array([(1.0 / alpha0) * (-b / alpha0) ** q for q in range(SERIES_LEN)], dtype=complex)


def series_mul(s: np.ndarray, t) -> np.ndarray:
    return np.convolve(np.asarray(s, complex), np.asarray(t, complex))[:SERIES_LEN]


def at_one(f: Factor, j: int) -> Factor:
    """P with x_j = 1: x_j's exponents set to 0, equal rows merged (first occurrence order)."""
    rows, coef = [], []
    index = {}
    for c, e in zip(f.coef, f.exps):
        e2 = e.copy()
        e2[j] = 0
        key = e2.tobytes()
        if key in index:
            coef[index[key]] += c
        else:
            index[key] = len(rows)
            rows.append(e2)
            coef.append(float(c))
    keep = [i for i, c in enumerate(coef) if c != 0.0]
    n = f.exps.shape[1]
    return Factor(f.gamma, f.delta, np.array([coef[i] for i in keep]),
                  np.array([rows[i] for i in keep], dtype=np.uint8).reshape(len(keep), n))


def derivative(f: Factor, j: int):
    """dP/dx_j (terms in P's order), or None if P does not depend on x_j."""
    sel = [i for i in range(len(f.coef)) if f.exps[i, j] > 0]
    if not sel:
        return None
    exps = f.exps[sel].copy()
    coef = f.coef[sel] * exps[:, j].astype(float)
    exps[:, j] -= 1
    return Factor(1.0, 0.0, coef, exps)


def expand_sector(sec: Sector, series: np.ndarray, out: List[Tuple[Sector, np.ndarray]]):
    low = [j for j in range(sec.n) if sec.a[j] < -1.0]
    if not low:
        out.append((sec, series))
        return
    j = low[0]
    a0, b = float(sec.a[j]) + 1.0, float(sec.b[j])
    if b == 0.0:
        raise ValueError("a_j < -1 needs b_j != 0")
    inv = inv_alpha(a0, b)
    # boundary x_j = 1
    facs = [at_one(f, j) for f in sec.factors]
    if any(len(f.coef) == 0 for f in facs):
        if not all(f.gamma > 0 for f in facs if len(f.coef) == 0):
            raise ValueError("a factor vanishes at x_j = 1 with a non-positive exponent")
    else:
        a, bb = sec.a.copy(), sec.b.copy()
        a[j], bb[j] = 0.0, 0.0
        expand_sector(Sector(a=a, b=bb, factors=facs, coeff=sec.coeff), series_mul(series, inv), out)
    # derivative terms
    for m, f in enumerate(sec.factors):
        D = derivative(f, j)
        if D is None:
            continue
        facs = []
        for mm, g in enumerate(sec.factors):
            if mm != m:
                facs.append(g)
            elif not (g.gamma - 1.0 == 0.0 and g.delta == 0.0):
                facs.append(Factor(g.gamma - 1.0, g.delta, g.coef, g.exps))
        facs.append(D)
        a = sec.a.copy()
        a[j] += 1.0
        s2 = series_mul(series_mul(series, -inv), [f.gamma, f.delta])
        expand_sector(Sector(a=a, b=sec.b.copy(), factors=facs, coeff=sec.coeff), s2, out)


def expand(sectors: List[Sector]):
    """Every sector with some a_j < -1 replaced by its expansion; returns
    (sectors, coefficient series, index of the input sector) in order."""
    secs, series, origin = [], [], []
    for i, sec in enumerate(sectors):
        out: List[Tuple[Sector, np.ndarray]] = []
        one = np.zeros(SERIES_LEN, complex)
        one[0] = 1.0
        expand_sector(sec, one, out)
        for s, c in out:
            secs.append(s)
            series.append(c)
            origin.append(i)
    return secs, series, origin


def folded_prefactor(pref, series: np.ndarray) -> np.ndarray:
    """The prefactor series times a sector's coefficient series (same leading
    power; the full product, whose terms are exact as far as pref is)."""
    return np.convolve(np.asarray(pref, complex), np.asarray(series, complex))
