"""Oracle: SeparateTerms, a sector as the sum of its integrable terms.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section 4.4's SeparateTerms option hands the integrator the integrable terms
of a sector one at a time instead of the sector's whole expression.  With the
subtraction at x_j = 0 on the singular set S (oracle/integrand.py), every
subset T of S gives one term:

    I_s = sum_{T subset S} prod_{j in T} 1/(b_j eps)
          c_s int prod_{j not in T} x_j^(a_j + b_j eps) G(x^(T), eps) dx_{not T},

where x^(T) sets x_T = 0, so the integrand no longer depends on x_T, and the
remaining singular variables S \\ T are subtracted without boundary terms
(the boundary terms of S \\ T are the terms T' > T).  Each term is therefore
a sector of its own over the n - |T| variables outside T: its factors keep
the terms free of x_T (with the other exponent columns), its coefficient takes
prod_{j in T} 1/b_j, and it stands for eps^-|T| times its own integral.  A term
with no variable left (T = S = all variables) gets one constant variable
(a = b = 0) so that it is a one-dimensional integral of a constant.

The terms of a sector come in the order of T read as a bit mask over S, the
singular variables in increasing index; sectors without singular variables
stay as they are.  Real mode only: the contour deformation's factors at the
subtraction corners belong to the sector as a whole.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List

import numpy as np

from sectorgen import Factor, Problem, Sector

from .integrand import singular_set


@dataclass
class FaceSector(Sector):
    """A separated term: ``boundary = False`` keeps only the subtracted
    integrand, ``eps_shift`` the power of 1/eps the term carries."""
    boundary: bool = False
    eps_shift: int = 0
    tmask: int = 0


def face_sector(sector: Sector, tmask: int) -> FaceSector:
    """Term T = tmask (bits over the singular variables) of ``sector``."""
    S = singular_set(sector)
    T = [S[i] for i in range(len(S)) if tmask >> i & 1]
    keep = [j for j in range(sector.n) if j not in T]
    scale = 1.0
    for j in T:
        scale /= sector.b[j]
    factors = []
    for m, fac in enumerate(sector.factors):
        on_face = np.all(fac.exps[:, T] == 0, axis=1) if T else np.ones(len(fac.coef), dtype=bool)
        if not np.any(on_face):
            raise ValueError(f"factor {m} has no term on the face x_T = 0")
        ex = fac.exps[on_face][:, keep] if keep else np.zeros((int(on_face.sum()), 1), dtype=np.uint8)
        factors.append(Factor(fac.gamma, fac.delta, fac.coef[on_face], ex))
    a = sector.a[keep] if keep else np.zeros(1)
    b = sector.b[keep] if keep else np.zeros(1)
    return FaceSector(a, b, factors, complex(sector.coeff) * scale, sector.deform_factor, None,
                      boundary=False, eps_shift=len(T), tmask=tmask)


def separate(problem: Problem):
    """The problem with every sector replaced by its terms, and the input
    sector of each term."""
    if problem.complex_mode:
        raise ValueError("separated terms in real mode only")
    sectors, origin = [], []
    for s, sec in enumerate(problem.sectors):
        ns = len(singular_set(sec))
        if ns == 0:
            sectors.append(sec)
            origin.append(s)
            continue
        for tmask in range(1 << ns):
            sectors.append(face_sector(sec, tmask))
            origin.append(s)
    parts = Problem(sectors, problem.order_min, problem.order_max, problem.pref_lead, problem.pref,
                    problem.feynman, problem.complex_mode, problem.lam, problem.name + " (separated)")
    return parts, origin


def face_point(sector: Sector, tmask: int, x: np.ndarray) -> np.ndarray:
    """The term's own coordinates of points x of the whole sector cube."""
    S = singular_set(sector)
    T = [S[i] for i in range(len(S)) if tmask >> i & 1]
    keep = [j for j in range(sector.n) if j not in T]
    return x[:, keep] if keep else np.full((x.shape[0], 1), 0.5)
