"""Oracle: globally adaptive deterministic cubature over the sector cube.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper lets the final stage use Cuba's deterministic integrator in place of
Vegas (CurrentIntegrator = cuhreCuba, section 4.4).  Cuhre is globally
adaptive subdivision driven by an embedded pair of fully symmetric cubature
rules.  This module states the algorithm that the library's cubature mode
computes, written from the published method (A. C. Genz and A. A. Malik,
J. Comput. Appl. Math. 6 (1980) 295, and the DCUHRE description of
Berntsen, Espelid and Genz, ACM TOMS 17 (1991) 437):

Rule.  On the cube [-1, 1]^n the degree-7 Genz-Malik rule uses the centre,
the 2n points +-l2 e_i, the 2n points +-l3 e_i, the 2n(n-1) points
+-l4 e_i +- l4 e_j (i < j) and the 2^n points (+-l5, ..., +-l5), with
l2^2 = 9/70, l3^2 = l4^2 = 9/10, l5^2 = 9/19; the embedded degree-5 rule uses
the first four classes.  Weights (of the mean over the cube) per class:

    degree 7: (12824 - 9120 n + 400 n^2)/19683, 980/6561, (1820 - 400 n)/19683,
              200/19683, 6859/19683 / 2^n
    degree 5: (729 - 950 n + 50 n^2)/729, 245/486, (265 - 100 n)/1458, 25/729, 0

On a box with centre c and half-widths h the node xi maps to c + xi h and the
integral is vol * sum_p w_p F(x_p) with vol = prod_j 2 h_j.

Readings where the published method leaves a choice (the same in the library):

* Vector integrand: F has K result orders, each complex.  The rule's error
  for order k is vol * |S7_k - S5_k| split into real and imaginary parts
  (the region error is the degree-7/degree-5 difference, without the null
  rules of DCUHRE); the integral of order k is the sum of vol * S7_k over the
  regions, its error the sum of the region errors (not a root-sum-square: rule
  errors are not independent random errors).
* Tolerance per order: tau_k = max(epsabs, epsrel |T_k|), T_k the current
  total; order weights omega_k = 1/tau_k (1 where tau_k = 0).
* Roundoff: the rule difference and the fourth differences are differences of
  nearly equal sums once a region is resolved, so below some size they are
  rounding noise.  Unit u = 2^-52; a region's rounding scale for order k is
  sigma_k = vol u sum_p (|w7_p| + |w5_p|) |F_k(x_p)|_1 (|z|_1 = |Re z| +
  |Im z|); order k of the region counts as converged when its error
  e_k = e_re + e_im is at most 2^20 sigma_k.
* Split axis: the fourth divided difference along each axis,
  Delta_j = (F(c + l2 h_j e_j) + F(c - l2 h_j e_j) - 2F(c))
            - (l2^2/l3^2) (F(c + l3 h_j e_j) + F(c - l3 h_j e_j) - 2F(c)),
  measured as D_j = max_k omega_k |Delta_jk|_1 with the weights of the round
  in which the region is evaluated; the region is halved along the lowest axis
  whose D_j is within 2^20 nu of the largest, nu = u max_k omega_k max_p
  |F_k(x_p)|_1 over the centre and the 4n axis nodes (differences below that
  are noise; a NaN counts as infinite).
* Region priority: max_k omega_k e_k over the orders not converged (0 if
  all are: the region is never halved), with the weights of the current
  totals.
* Batches: a round halves the B regions of highest priority (equal
  priorities: the older region first), B = max(ceil(split_frac |alive|),
  min(|alive|, batch_min)), cut to the longest prefix whose children fit in
  maxeval; it stops when every order meets its tolerance, when nothing fits,
  or when no region can be split (zero priority, or 30 halvings of its axis).
* Priorities are compared at 8 significant bits (``coarse``; equal ones: the
  older region first).  Sectors that are equal up to the order of their terms
  (the symmetries of a diagram) give regions whose errors are equal up to
  rounding noise of relative size sigma/e <= 2^-20; at 8 bits such twins
  still compare equal (unless they straddle a rounding boundary, a chance of
  about 2^-12 per pair at the noise threshold and far less above it), so
  their order does not depend on the summation order.
* Regions are dyadic: per variable a level d and an index k, the interval
  [k 2^-d, (k+1) 2^-d]; ids in creation order (sector order first, then each
  round's children, lower half before upper half, in selection order).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from itertools import product
from typing import List

import numpy as np

from . import integrate

MAX_LEVEL = 30
U = 2.0 ** -52          # unit roundoff of the rounding scales
NOISE = 2.0 ** 20       # rule differences within NOISE units of roundoff are noise


def lambdas():
    """l2, l3, l4, l5 of the Genz-Malik rule."""
    return math.sqrt(9.0 / 70.0), math.sqrt(9.0 / 10.0), math.sqrt(9.0 / 10.0), math.sqrt(9.0 / 19.0)


def weights(n: int):
    """Per-class weights (centre, l2 axis, l3 axis, l4 pairs, l5 corners) of the
    degree-7 and the embedded degree-5 rule, as means over the cube."""
    w7 = [(12824.0 - 9120.0 * n + 400.0 * n * n) / 19683.0, 980.0 / 6561.0, (1820.0 - 400.0 * n) / 19683.0,
          200.0 / 19683.0, 6859.0 / 19683.0 / 2.0 ** n]
    w5 = [(729.0 - 950.0 * n + 50.0 * n * n) / 729.0, 245.0 / 486.0, (265.0 - 100.0 * n) / 1458.0,
          25.0 / 729.0, 0.0]
    return w7, w5


def nodes(n: int):
    """Nodes on [-1, 1]^n and their classes: centre; +-l2 e_i (i ascending, + then
    -); +-l3 e_i; +-l4 e_i +-l4 e_j (pairs i < j, signs ++, +-, -+, --); the
    corners (+-l5)^n."""
    l2, l3, l4, l5 = lambdas()
    pts, cls = [np.zeros(n)], [0]
    for lam, c in ((l2, 1), (l3, 2)):
        for i in range(n):
            for sg in (1.0, -1.0):
                v = np.zeros(n)
                v[i] = sg * lam
                pts.append(v)
                cls.append(c)
    for i in range(n):
        for j in range(i + 1, n):
            for si, sj in ((1.0, 1.0), (1.0, -1.0), (-1.0, 1.0), (-1.0, -1.0)):
                v = np.zeros(n)
                v[i], v[j] = si * l4, sj * l4
                pts.append(v)
                cls.append(3)
    for sg in product((1.0, -1.0), repeat=n):
        pts.append(np.array(sg) * l5)
        cls.append(4)
    return np.array(pts), np.array(cls)


def npoints(n: int) -> int:
    return 1 + 4 * n + 2 * n * (n - 1) + (1 << n)


def coarse(v: float) -> float:
    """v >= 0 rounded to 8 significant bits (the 45 lowest of the 52 stored
    mantissa bits rounded away, half up); NaN and infinity give infinity."""
    if not math.isfinite(v) or v <= 0.0:
        return v if math.isfinite(v) else math.inf
    b = np.array([v], dtype=np.float64).view(np.uint64)[0]
    b = (int(b) + (1 << 44)) & ~((1 << 45) - 1)
    return float(np.array([b], dtype=np.uint64).view(np.float64)[0])


@dataclass
class Region:
    sector: int
    level: np.ndarray          # (n,) int
    index: np.ndarray          # (n,) int
    value: np.ndarray = None   # (K,) complex: vol * S7
    err_re: np.ndarray = None  # (K,)
    err_im: np.ndarray = None
    sigma: np.ndarray = None   # (K,) rounding scale
    axis: int = 0
    nonfinite: int = 0
    alive: bool = True


def box(region: Region):
    """Centre and half-widths of a dyadic region."""
    half = np.ldexp(0.5, -region.level.astype(np.int64))
    centre = (2.0 * region.index + 1.0) * half
    return centre, half


def apply_rule(problem, region: Region, pref_lead: int, pref, omega: np.ndarray):
    """The rule pair on one region: value, errors, split axis (the docstring's
    definitions) and the number of nodes where some order is not finite."""
    sec = problem.sectors[region.sector]
    n = sec.n
    xi, cls = nodes(n)
    centre, half = box(region)
    x = centre[None, :] + xi * half[None, :]
    vals, _, _ = integrate.sector_values(problem, region.sector, x, pref_lead, pref)   # (K, P)
    w7, w5 = weights(n)
    a7 = np.array([w7[c] for c in cls])
    a5 = np.array([w5[c] for c in cls])
    K = vals.shape[0]
    vol = float(np.prod(2.0 * half))
    s7 = np.array([integrate.fsum_c(vals[k] * a7) for k in range(K)])
    s5 = np.array([integrate.fsum_c(vals[k] * a5) for k in range(K)])
    d = s7 - s5
    region.value = vol * s7
    region.err_re = vol * np.abs(d.real)
    region.err_im = vol * np.abs(d.imag)
    region.nonfinite = int(np.sum(~np.all(np.isfinite(vals), axis=0)))
    l1 = np.abs(vals.real) + np.abs(vals.imag)                                  # (K, P)
    region.sigma = vol * U * np.array([math.fsum(l1[k] * (np.abs(a7) + np.abs(a5))) for k in range(K)])
    f0 = vals[:, 0]
    r = 1.0 / 7.0                                   # l2^2 / l3^2
    D = np.zeros(n)
    for j in range(n):
        fp2, fm2 = vals[:, 1 + 2 * j], vals[:, 2 + 2 * j]
        fp3, fm3 = vals[:, 1 + 2 * n + 2 * j], vals[:, 2 + 2 * n + 2 * j]
        delta = (fp2 + fm2 - 2.0 * f0) - r * (fp3 + fm3 - 2.0 * f0)
        d = omega * (np.abs(delta.real) + np.abs(delta.imag))
        D[j] = math.inf if np.any(np.isnan(d)) else float(np.max(d))
    nu = U * float(np.max(omega[:, None] * l1[:, :1 + 4 * n]))
    tol = NOISE * nu if math.isfinite(nu) else 0.0
    top = float(np.max(D))
    region.axis = int(np.flatnonzero(D >= top - tol)[0])
    return region


def priority(region: Region, omega: np.ndarray) -> float:
    """max_k omega_k e_k over the orders not converged (at 8 significant bits; 0: none)."""
    e = region.err_re + region.err_im
    live = ~(e <= NOISE * region.sigma)
    v = omega * e
    if np.any(np.isnan(v[live])):
        return math.inf
    return coarse(float(np.max(v[live]))) if np.any(live) else 0.0


def order_weights(total: np.ndarray, epsrel: float, epsabs: float):
    tau = np.maximum(epsabs, epsrel * np.abs(total))
    return np.where(tau > 0, 1.0 / np.where(tau > 0, tau, 1.0), 1.0), tau


@dataclass
class CubatureResult:
    value: np.ndarray
    err_re: np.ndarray
    err_im: np.ndarray
    regions: List[Region] = field(default_factory=list)
    evals: int = 0
    rounds: int = 0
    converged: bool = False


def cubature(problem, maxeval: int, epsrel: float, epsabs: float, split_frac: float = 0.25,
             batch_min: int = 1024, sectors=None) -> CubatureResult:
    """The adaptive loop of the module docstring over every sector (or the listed
    ones, which then keep their own region ids in list order)."""
    lead, pref = integrate.prefactor_for(problem)
    K = problem.order_max - problem.order_min + 1
    idx = list(range(len(problem.sectors))) if sectors is None else list(sectors)
    regs: List[Region] = []
    omega = np.ones(K)
    evals = 0
    for s in idx:
        n = problem.sectors[s].n
        regs.append(Region(s, np.zeros(n, dtype=np.int64), np.zeros(n, dtype=np.int64)))
        evals += npoints(n)
    if evals > maxeval:
        raise ValueError("maxeval below one rule per sector")
    for r in regs:
        apply_rule(problem, r, lead, pref, omega)
    rounds = 1
    while True:
        alive = [r for r in regs if r.alive]
        total = np.array([integrate.fsum_c([r.value[k] for r in alive]) for k in range(K)])
        err = np.array([math.fsum([r.err_re[k] + r.err_im[k] for r in alive]) for k in range(K)])
        omega, tau = order_weights(total, epsrel, epsabs)
        if np.all(err <= tau):
            converged = True
            break
        cand = []
        for i, r in enumerate(regs):
            if not r.alive or r.level[r.axis] >= MAX_LEVEL:
                continue
            p = priority(r, omega)
            if p > 0.0:
                cand.append((-p, i))
        cand.sort()
        B = max(math.ceil(split_frac * len(alive)), min(len(alive), batch_min))
        chosen = []
        for _, i in cand[:B]:
            cost = 2 * npoints(problem.sectors[regs[i].sector].n)
            if evals + cost > maxeval:
                break
            evals += cost
            chosen.append(i)
        if not chosen:
            converged = False
            break
        new = []
        for i in chosen:
            r = regs[i]
            r.alive = False
            for half in (0, 1):
                lev = r.level.copy()
                ind = r.index.copy()
                lev[r.axis] += 1
                ind[r.axis] = 2 * ind[r.axis] + half
                new.append(Region(r.sector, lev, ind))
        for r in new:
            apply_rule(problem, r, lead, pref, omega)
        regs.extend(new)
        rounds += 1
    alive = [r for r in regs if r.alive]
    value = np.array([integrate.fsum_c([r.value[k] for r in alive]) for k in range(K)])
    er = np.array([math.fsum([r.err_re[k] for r in alive]) for k in range(K)])
    ei = np.array([math.fsum([r.err_im[k] for r in alive]) for k in range(K)])
    return CubatureResult(value, er, ei, regs, evals, rounds, converged)
