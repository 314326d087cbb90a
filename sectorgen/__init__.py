"""Seeded input generators for sector integrands.

This module holds *inputs only*: the plain data layout of a sector-decomposed
integrand and seeded synthetic workloads.  It contains none of the method's
arithmetic (no polynomial evaluation, no epsilon expansion, no sampling), so
both the fp64 oracle (``oracle/``) and the HIP library binding
(``paper_1511_03614_amd``) may read what it produces.

A sector is one integral left after sector decomposition (paper, section 1 and
eq. (2)):

    I_s = c_s * int_[0,1]^n  prod_j x_j^(a_j + b_j eps)
                            * prod_m P_m(x)^(gamma_m + delta_m eps)  dx

with every P_m a polynomial with a nonzero constant term.  A problem is a list
of sectors, the requested orders eps^k, and a prefactor series Pi(eps) that
multiplies the sector sum (for Feynman integrals the Gamma-function factor of
eq. (2) with exp(l*gamma_E*eps) restored, paper section 4.3).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

__all__ = [
    "Factor", "Sector", "Problem", "FeynmanPrefactor", "SplitMix64",
    "synthetic_sectors", "synthetic_problem", "bubble_problem",
    "config1", "config2", "config4",
]

MAX_VARS = 16


@dataclass
class Factor:
    """One regular factor P_m(x)^(gamma + delta*eps) with P_m = sum_t coef_t x^exps_t."""
    gamma: float
    delta: float
    coef: np.ndarray          # (T,) float64 (complex128 for complex coefficients, complex mode only)
    exps: np.ndarray          # (T, n) uint8

    def __post_init__(self):
        c = np.asarray(self.coef)
        self.coef = np.ascontiguousarray(c, dtype=np.complex128 if np.iscomplexobj(c) else np.float64)
        self.exps = np.ascontiguousarray(self.exps, dtype=np.uint8)
        if self.exps.ndim != 2 or self.exps.shape[0] != self.coef.shape[0]:
            raise ValueError("exps must be (T, n) with T == len(coef)")


@dataclass
class Sector:
    """One sector: monomial exponents a_j + b_j eps, factors, coefficient c_s.

    ``deform_factor`` names the factor that is the sector's F polynomial (used
    by the contour deformation in complex mode).  The deformation follows the
    gradient of x^deform_mono * P_F(x); None (zeros) deforms along P_F itself,
    the polynomial with a constant term that carries the F - i0 branch.
    """
    a: np.ndarray                    # (n,) float64, -1 exactly or > -1
    b: np.ndarray                    # (n,) float64
    factors: List[Factor]
    coeff: complex = 1.0
    deform_factor: int = -1
    deform_mono: Optional[np.ndarray] = None   # (n,) int32

    def __post_init__(self):
        self.a = np.ascontiguousarray(self.a, dtype=np.float64)
        self.b = np.ascontiguousarray(self.b, dtype=np.float64)
        if self.deform_mono is not None:
            self.deform_mono = np.ascontiguousarray(self.deform_mono, dtype=np.int32)

    @property
    def n(self) -> int:
        return int(self.a.shape[0])


@dataclass
class FeynmanPrefactor:
    """Pi(eps) = exp(l*gamma_E*eps) Gamma(A - l*d/2) / prod_i Gamma(a_i), d = d0 - 2 eps.

    Eq. (2) of the paper with (i pi^(d/2))^l and exp(-l gamma_E eps) pulled out
    (section 4.3).  Each side of the parity check expands this series itself.
    """
    loops: int
    indices: Tuple[int, ...]
    d0: int = 4


@dataclass
class Problem:
    sectors: List[Sector]
    order_min: int
    order_max: int
    # Either an explicit series Pi(eps) = sum_i pref[i] eps^(pref_lead + i) ...
    pref_lead: int = 0
    pref: np.ndarray = field(default_factory=lambda: np.ones(1, dtype=np.complex128))
    # ... or a Feynman prefactor to be expanded by the consumer (takes precedence).
    feynman: Optional[FeynmanPrefactor] = None
    complex_mode: bool = False
    lam: float = 0.0
    name: str = ""

    def __post_init__(self):
        self.pref = np.ascontiguousarray(self.pref, dtype=np.complex128)

    @property
    def norders(self) -> int:
        return self.order_max - self.order_min + 1


class SplitMix64:
    """SplitMix64 (Steele, Lea and Flood, OOPSLA 2014): the published 64-bit mixer."""
    MASK = (1 << 64) - 1

    def __init__(self, seed: int):
        self.state = seed & self.MASK

    def next_u64(self) -> int:
        self.state = (self.state + 0x9E3779B97F4A7C15) & self.MASK
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & self.MASK
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & self.MASK
        return z ^ (z >> 31)

    def uniform(self) -> float:
        """Double in [0, 1) from the top 53 bits."""
        return (self.next_u64() >> 11) * (1.0 / (1 << 53))

    def randint(self, lo: int, hi: int) -> int:
        """Integer uniform on the closed range [lo, hi]."""
        return lo + self.next_u64() % (hi - lo + 1)

    def choice(self, seq: Sequence):
        return seq[self.randint(0, len(seq) - 1)]


def _random_poly(rng: SplitMix64, n: int, nextra: int, emax: int = 2) -> Tuple[np.ndarray, np.ndarray]:
    """Constant term plus ``nextra`` distinct non-constant monomials, coefficients U[0.1, 1]."""
    seen = set()
    exps = [tuple([0] * n)]
    seen.add(exps[0])
    limit = (emax + 1) ** n - 1
    nextra = min(nextra, limit)
    while len(exps) < nextra + 1:
        e = tuple(rng.randint(0, emax) for _ in range(n))
        if e in seen:
            continue
        seen.add(e)
        exps.append(e)
    coef = np.array([0.1 + 0.9 * rng.uniform() for _ in exps], dtype=np.float64)
    return coef, np.array(exps, dtype=np.uint8).reshape(len(exps), n)


def synthetic_sectors(seed: int, count: int, nvar: Tuple[int, int], terms: Tuple[int, int],
                      nsing: Tuple[int, int]) -> List[Sector]:
    """Random positive sectors with two factors ("U" and "F").

    n ~ U{nvar}; each factor is a constant term plus U{terms[0]-1 .. terms[1]-1}
    distinct monomials with exponents U{0,1,2} per variable and coefficients
    U[0.1, 1]; gamma_U in {-2,-1,1}, delta_U in {1,2,3}, gamma_F in {-3,-2,-1},
    delta_F in {-2,-1}; |S| ~ U{nsing} singular variables with a = -1 and
    b in {+-1, +-2}; the other variables have a = 0 and b in {-2..2}.
    """
    rng = SplitMix64(seed)
    out = []
    for _ in range(count):
        n = rng.randint(*nvar)
        a = np.zeros(n)
        b = np.array([float(rng.randint(-2, 2)) for _ in range(n)])
        ns = min(rng.randint(*nsing), n)
        idx = list(range(n))
        sing = []
        for _k in range(ns):
            j = idx.pop(rng.randint(0, len(idx) - 1))
            sing.append(j)
        for j in sing:
            a[j] = -1.0
            b[j] = float(rng.choice([-2, -1, 1, 2]))
        facs = []
        for (gs, ds) in (([-2, -1, 1], [1, 2, 3]), ([-3, -2, -1], [-2, -1])):
            nextra = rng.randint(terms[0] - 1, terms[1] - 1)
            coef, exps = _random_poly(rng, n, nextra)
            facs.append(Factor(float(rng.choice(gs)), float(rng.choice(ds)), coef, exps))
        out.append(Sector(a=a, b=b, factors=facs, coeff=1.0, deform_factor=1,
                          deform_mono=np.zeros(n, dtype=np.int32)))
    return out


def synthetic_problem(seed: int, count: int, nvar, terms, nsing, order_min: int, order_max: int,
                      name: str = "") -> Problem:
    return Problem(sectors=synthetic_sectors(seed, count, nvar, terms, nsing),
                   order_min=order_min, order_max=order_max, pref_lead=0,
                   pref=np.ones(1, dtype=np.complex128), name=name)


def bubble_problem(order_max: int = 2) -> Problem:
    """One-loop massless bubble, indices (1,1), p^2 = -1, d = 4 - 2 eps.

    U = x1 + x2, F = x1 x2; each of the two primary sectors (x_k = 1) leaves
    t^(-eps) (1 + t)^(-2 + 2 eps) on [0, 1].  The Feynman prefactor of eq. (2)
    is Gamma(eps) exp(gamma_E eps).
    """
    secs = []
    for _ in range(2):
        secs.append(Sector(a=np.array([0.0]), b=np.array([-1.0]),
                           factors=[Factor(-2.0, 2.0, np.array([1.0, 1.0]),
                                           np.array([[0], [1]], dtype=np.uint8))],
                           coeff=1.0))
    return Problem(sectors=secs, order_min=-1, order_max=order_max,
                   feynman=FeynmanPrefactor(loops=1, indices=(1, 1), d0=4), name="bubble")


def config1() -> Problem:
    """Tiny case: the massless bubble, orders eps^-1 .. eps^2."""
    return bubble_problem(order_max=2)


def config2() -> Problem:
    """64 synthetic sectors, 3-6 variables, 4-20 terms per factor, |S| <= 2, orders -2..0."""
    return synthetic_problem(2, 64, (3, 6), (4, 20), (0, 2), -2, 0, name="synthetic64")


def config4() -> Problem:
    """2000 synthetic sectors, 4-9 variables, 5-40 terms per factor, |S| <= 3, orders -3..0."""
    return synthetic_problem(4, 2000, (4, 9), (5, 40), (0, 3), -3, 0, name="batched2000")
