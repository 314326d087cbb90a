"""Feynman-integral test inputs: Symanzik polynomials and a minimal sector decomposer.

Input preparation only (the algebra that the paper performs in Mathematica
before integration, section 4.2): it builds U and F of eq. (2) from
propagator momenta, splits the simplex into primary sectors (x_k = 1) and
iterates the classic decomposition (Binoth-Heinrich) until every polynomial
has a nonzero constant term.  The output is a ``sectorgen.Problem`` whose
sectors the integrators consume.  Nothing here evaluates an integrand.

Momenta are linear combinations: q_i = sum_a alpha_ia k_a + sum_e r_ie p_e.
With sum_i x_i (-q_i^2 + m_i^2) = -k^T M k + 2 k.Q + J,
U = det M and F = Q^T adj(M) Q + U J.
"""
from __future__ import annotations

from fractions import Fraction
from itertools import combinations
from typing import Dict, List, Sequence, Tuple

import numpy as np
import sympy as sp

from . import Factor, FeynmanPrefactor, Problem, Sector

Poly = Dict[Tuple[int, ...], float]


def symanzik(alpha: Sequence[Sequence[float]], r: Sequence[Sequence[float]], gram, masses):
    """U and F as {exponent tuple: coefficient} in the Feynman parameters x_1..x_n."""
    n = len(alpha)
    nl = len(alpha[0])
    x = sp.symbols(f"x1:{n + 1}")
    gram = sp.Matrix(gram)
    M = sp.zeros(nl, nl)
    Q = [sp.zeros(gram.shape[0], 1) for _ in range(nl)]
    J = 0
    for i in range(n):
        al = [sp.nsimplify(v) for v in alpha[i]]
        ri = sp.Matrix([sp.nsimplify(v) for v in r[i]])
        for a in range(nl):
            for b in range(nl):
                M[a, b] += x[i] * al[a] * al[b]
            Q[a] += -x[i] * al[a] * ri
        J += x[i] * (-(ri.T * gram * ri)[0, 0] + sp.nsimplify(masses[i]))
    U = sp.expand(M.det())
    adj = M.adjugate()
    F = 0
    for a in range(nl):
        for b in range(nl):
            F += adj[a, b] * (Q[a].T * gram * Q[b])[0, 0]
    F = sp.expand(F + U * J)
    return _to_poly(U, x), _to_poly(F, x)


def _to_poly(expr, x) -> Poly:
    p = sp.Poly(expr, *x)
    return {tuple(int(e) for e in mon): float(c) for mon, c in zip(p.monoms(), p.coeffs()) if c != 0}


# ---------------------------------------------------------------- decomposition

def _gcd_mono(p: Poly) -> Tuple[int, ...]:
    keys = list(p.keys())
    return tuple(min(k[j] for k in keys) for j in range(len(keys[0])))


def _has_const(p: Poly, g: Tuple[int, ...]) -> bool:
    return tuple(g) in p


def _substitute(p: Poly, Z: Sequence[int], k: int) -> Poly:
    """x_i -> x_i x_k for i in Z \\ {k}: exponent e_k gains sum_{i in Z\\k} e_i."""
    out: Poly = {}
    for e, c in p.items():
        e2 = list(e)
        e2[k] = e[k] + sum(e[i] for i in Z if i != k)
        t = tuple(e2)
        out[t] = out.get(t, 0.0) + c
    return {e: c for e, c in out.items() if c != 0.0}


def _sub_vec(v: Sequence, Z: Sequence[int], k: int):
    v2 = list(v)
    v2[k] = v[k] + sum(v[i] for i in Z if i != k)
    return v2


def _vanishing_set(p: Poly, g: Tuple[int, ...]) -> List[int]:
    """Smallest set Z (first in size-then-lexicographic order) hitting every term of p / x^g."""
    n = len(g)
    terms = [tuple(e[j] - g[j] for j in range(n)) for e in p]
    for size in range(1, n + 1):
        for Z in combinations(range(n), size):
            if all(any(t[j] > 0 for j in Z) for t in terms):
                return list(Z)
    raise ValueError("polynomial is identically zero")


def decompose(polys: List[Poly], expo: List[Tuple[float, float]], mono_a: List[Fraction],
              mono_b: List[Fraction], max_depth: int = 40):
    """Iterated decomposition of prod_j x_j^(mono_a_j + mono_b_j eps) prod_m P_m^(expo_m).

    Returns a list of (polys, mono_a, mono_b) in the final variables.
    """
    out = []
    stack = [(polys, list(mono_a), list(mono_b), 0)]
    while stack:
        ps, ma, mb, depth = stack.pop()
        bad = None
        for m, p in enumerate(ps):
            g = _gcd_mono(p)
            if not _has_const(p, g):
                bad = m
                break
        if bad is None:
            out.append((ps, ma, mb))
            continue
        if depth >= max_depth:
            raise RuntimeError("sector decomposition did not terminate")
        p = ps[bad]
        Z = _vanishing_set(p, _gcd_mono(p))
        for k in Z:
            ps2 = [_substitute(q, Z, k) for q in ps]
            ma2 = _sub_vec(ma, Z, k)
            mb2 = _sub_vec(mb, Z, k)
            ma2[k] += len(Z) - 1
            stack.append((ps2, ma2, mb2, depth + 1))
    return out


def feynman_sectors(U: Poly, F: Poly, indices: Sequence[int], loops: int, d0: int = 4,
                    masses_present: bool = False, deform_full_f: bool = False) -> List[Sector]:
    """Primary sectors x_k = 1 of eq. (2), then iterated decomposition of U and F.

    In complex mode the deformation follows the gradient of the sector's
    reduced F (the factor left after the monomial is taken out, which has a
    constant term).  With ``deform_full_f`` it follows the full F = x^mono P_F
    instead: then the deformation shrinks with the monomial near the faces where
    it vanishes while P_F can still cross zero there, so Im P_F(z) only grows
    linearly away from such a face and the integrand's variance diverges.
    """
    n = len(indices)
    A = sum(indices)
    gU = Fraction(A) - Fraction((loops + 1) * d0, 2)
    dU = Fraction(loops + 1)
    gF = -(Fraction(A) - Fraction(loops * d0, 2))
    dF = Fraction(-loops)
    secs: List[Sector] = []
    for k in range(n):
        keep = [j for j in range(n) if j != k]

        def restrict(p: Poly) -> Poly:
            out: Poly = {}
            for e, c in p.items():
                t = tuple(e[j] for j in keep)
                out[t] = out.get(t, 0.0) + c
            return {e: c for e, c in out.items() if c != 0.0}
        ps = [restrict(U), restrict(F)]
        ma = [Fraction(indices[j] - 1) for j in keep]
        mb = [Fraction(0)] * (n - 1)
        for ps_f, ma_f, mb_f in decompose(ps, [(gU, dU), (gF, dF)], ma, mb):
            a = list(ma_f)
            b = list(mb_f)
            facs = []
            mono_F = None
            for m, (p, (g, d)) in enumerate(zip(ps_f, [(gU, dU), (gF, dF)])):
                gm = _gcd_mono(p)
                for j in range(n - 1):
                    a[j] += gm[j] * g
                    b[j] += gm[j] * d
                terms = sorted(p.items(), key=lambda kv: tuple(e - gg for e, gg in zip(kv[0], gm)))
                coef = np.array([c for _, c in terms])
                exps = np.array([[e[j] - gm[j] for j in range(n - 1)] for e, _ in terms], dtype=np.int64)
                if exps.max(initial=0) > 255:
                    raise ValueError("exponent exceeds uint8")
                facs.append(Factor(float(g), float(d), coef, exps.astype(np.uint8)))
                if m == 1:
                    mono_F = np.array(gm, dtype=np.int32)
            secs.append(Sector(a=np.array([float(v) for v in a]), b=np.array([float(v) for v in b]),
                               factors=facs, coeff=1.0, deform_factor=1,
                               deform_mono=mono_F if deform_full_f else np.zeros(n - 1, dtype=np.int32)))
    return secs


# ---------------------------------------------------------------- named inputs

def box_uf(S: float, T: float):
    """One-loop massless on-shell box of section 4.3: propagators k, k+p1, k+p1+p2, k+p1+p2+p4."""
    alpha = [[1], [1], [1], [1]]
    r = [[0, 0, 0], [1, 0, 0], [1, 1, 0], [1, 1, 1]]
    gram = [[0, -S / 2, (S + T) / 2], [-S / 2, 0, -T / 2], [(S + T) / 2, -T / 2, 0]]
    return symanzik(alpha, r, gram, [0, 0, 0, 0])


def box_problem(S: float = 3.0, T: float = 1.0, order_max: int = 0) -> Problem:
    U, F = box_uf(S, T)
    secs = feynman_sectors(U, F, (1, 1, 1, 1), 1)
    return Problem(sectors=secs, order_min=-2, order_max=order_max,
                   feynman=FeynmanPrefactor(1, (1, 1, 1, 1), 4), name="box")


def double_box_uf(s: float, t: float, m2: float = 0.0):
    """Planar double box: k1, k1+p1, k1+p1+p2, k2+p1+p2, k2+p1+p2+p3, k2, k1-k2; p_i^2 = 0."""
    alpha = [[1, 0], [1, 0], [1, 0], [0, 1], [0, 1], [0, 1], [1, -1]]
    r = [[0, 0, 0], [1, 0, 0], [1, 1, 0], [1, 1, 0], [1, 1, 1], [0, 0, 0], [0, 0, 0]]
    gram = [[0, s / 2, -(s + t) / 2], [s / 2, 0, t / 2], [-(s + t) / 2, t / 2, 0]]
    return symanzik(alpha, r, gram, [m2] * 7)


def double_box_problem(s: float = -3.0, t: float = -1.0, m2: float = 0.0, order_max: int = 0,
                       complex_mode: bool = False, lam: float = 0.0) -> Problem:
    U, F = double_box_uf(s, t, m2)
    secs = feynman_sectors(U, F, (1,) * 7, 2)
    return Problem(sectors=secs, order_min=-4, order_max=order_max,
                   feynman=FeynmanPrefactor(2, (1,) * 7, 4), complex_mode=complex_mode, lam=lam,
                   name="double_box")


def massive_bubble_problem(s: float = 5.0, m2: float = 1.0, lam: float = 0.5) -> Problem:
    """Equal-mass one-loop bubble at p^2 = s (complex mode with deformation)."""
    U, F = symanzik([[1], [1]], [[0], [1]], [[s]], [m2, m2])
    secs = feynman_sectors(U, F, (1, 1), 1)
    return Problem(sectors=secs, order_min=-1, order_max=1,
                   feynman=FeynmanPrefactor(1, (1, 1), 4), complex_mode=True, lam=lam,
                   name="massive_bubble")


def complex_mass_bubble_problem(s: float = 5.0, m2: complex = 1.0 - 0.25j, lam: float = 0.3) -> Problem:
    """Equal-mass one-loop bubble at p^2 = s with a complex mass m^2 = M^2 - i M Gamma:
    the two primary sectors of the real-mass bubble, F = m^2 (1 + t)^2 - s t written
    with complex coefficients (complex mode)."""
    base = massive_bubble_problem(s, 1.0, lam)
    secs = []
    for sec in base.sectors:
        F = sec.factors[sec.deform_factor]
        assert F.exps[:, 0].tolist() == [0, 1, 2] and np.allclose(F.coef, [1.0, 2.0 - s, 1.0])
        facs = list(sec.factors)
        facs[sec.deform_factor] = Factor(F.gamma, F.delta, np.array([m2, 2.0 * m2 - s, m2], dtype=complex),
                                         F.exps.copy())
        secs.append(Sector(a=sec.a.copy(), b=sec.b.copy(), factors=facs, coeff=sec.coeff,
                           deform_factor=sec.deform_factor, deform_mono=sec.deform_mono))
    return Problem(sectors=secs, order_min=base.order_min, order_max=base.order_max, feynman=base.feynman,
                   complex_mode=True, lam=lam, name="complex_mass_bubble")


def bisect_sector(sec: Sector, j: int, p: float = 0.5) -> List[Sector]:
    """Splits the integration over x_j at p (the BisectionVariables option of
    section 4.4, bisection point p): the lower part maps x_j = p y, the upper
    part x_j = 1 - (1 - p) y, so that x_j = 1 becomes the endpoint y = 0 of the
    new variable.  The Jacobians go into the coefficient; the monomial
    x_j^(a + b eps) becomes p^(a + b eps) y^(a + b eps) (a constant factor) in
    the lower part and a regular factor (1 - (1 - p) y)^(a + b eps) in the
    upper part; polynomial terms are substituted and expanded.  Returns
    [lower, upper]; their integrals add up to the sector's."""
    import math as _m
    n = sec.n
    c = 1.0 - p
    a_j, b_j = float(sec.a[j]), float(sec.b[j])
    lower_f, upper_f = [], []
    for f in sec.factors:
        lc = f.coef * np.array([p ** int(e[j]) for e in f.exps])
        lower_f.append(Factor(f.gamma, f.delta, lc, f.exps.copy()))
        terms = {}
        for coef, e in zip(f.coef, f.exps):
            for k in range(int(e[j]) + 1):
                ne = list(int(v) for v in e)
                ne[j] = k
                terms[tuple(ne)] = terms.get(tuple(ne), 0.0) + coef * _m.comb(int(e[j]), k) * (-c) ** k
        keys = sorted(terms, key=lambda t: (sum(t), t))
        keys = [t for t in keys if terms[t] != 0.0]
        zero = tuple([0] * n)
        if zero in keys:                       # the constant term first, as the generators write it
            keys.remove(zero)
            keys.insert(0, zero)
        upper_f.append(Factor(f.gamma, f.delta, np.array([terms[t] for t in keys]),
                              np.array(keys, dtype=np.uint8).reshape(len(keys), n)))
    lower_a, lower_b = sec.a.copy(), sec.b.copy()
    upper_a, upper_b = sec.a.copy(), sec.b.copy()
    upper_a[j], upper_b[j] = 0.0, 0.0
    if a_j != 0.0 or b_j != 0.0:
        lower_f.append(Factor(a_j, b_j, np.array([p]), np.zeros((1, n), dtype=np.uint8)))
        e1 = np.zeros((2, n), dtype=np.uint8)
        e1[1, j] = 1
        upper_f.append(Factor(a_j, b_j, np.array([1.0, -c]), e1))
    mono = None if sec.deform_mono is None else sec.deform_mono.copy()
    lower = Sector(a=lower_a, b=lower_b, factors=lower_f, coeff=complex(sec.coeff) * p,
                   deform_factor=sec.deform_factor, deform_mono=mono)
    upper = Sector(a=upper_a, b=upper_b, factors=upper_f, coeff=complex(sec.coeff) * c,
                   deform_factor=sec.deform_factor, deform_mono=None if mono is None else mono.copy())
    return [lower, upper]


def bisect_problem(problem: Problem, variables: Sequence[int], p: float = 0.5) -> Problem:
    """Every sector bisected at p in each variable of `variables` in turn
    (2^len(variables) parts per sector)."""
    import dataclasses
    secs = list(problem.sectors)
    for j in variables:
        secs = [part for s in secs for part in bisect_sector(s, j, p)]
    return dataclasses.replace(problem, sectors=secs)
