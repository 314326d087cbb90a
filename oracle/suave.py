"""Oracle: subregion-adaptive Monte Carlo over the sector cube.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper lets the final stage use Cuba's Suave (CurrentIntegrator =
suaveCuba, section 4.4): Monte Carlo sampling in subregions that are
bisected where the samples fluctuate most.  The paper gives no more than the
name; this module states the algorithm that the library's integrator 3
computes (a reading: plain Monte Carlo per region, no per-region Vegas grid,
the parent's samples not carried into its halves):

* Regions are the dyadic boxes of the adaptive cubature (oracle/cubature.py:
  per sector, level and index per variable; the whole cube first), numbered in
  order of creation: the sectors' cubes 0 .. nsec-1, then the two halves of
  every bisected region in turn (lower half first).
* Every new region takes N = nnew points: point p, variable c from
  Philox4x32-10 with key = the seed's 32-bit halves and counter
  (p, c, region number, 0x53554156); u = (b + 1/2) 2^-52 with b the top 52
  bits of the first two words (as the Monte Carlo points of oracle/points.py),
  x_c = lo_c + u_c w_c with the box's corner lo_c and width w_c (one rounding
  each).
* The region's value for result order k is vol mean_p F_k(x_p), its errors
  vol sqrt(var_re / N) and vol sqrt(var_im / N) with the unbiased sample
  variances of the real and imaginary parts (sums of F and F^2 exact to
  rounding, var = (S2 - S1^2 / N) / (N - 1), negative values clamped to 0).
* Split axis: with g_p = sum_k omega_k (|Re F_k| + |Im F_k|) (the order
  weights of the round), the samples with u_c < 1/2 and u_c >= 1/2 give the
  two halves' spreads s = sqrt(max(0, mean(g^2) - mean(g)^2)); the region is
  halved along the variable c with the smallest s_left + s_right, compared at
  8 significant bits (equal ones: the lowest c); a half with fewer than two
  samples gives an infinite sum; if every sum is infinite, variable 0.
* Totals: the sum of the values of the regions alive; errors combine as a
  root sum of squares (independent samples).  Tolerance, order weights,
  priorities (max_k omega_k (e_re + e_im) at 8 significant bits), batches and
  the stop rule as in the cubature, a halving costing 2 N evaluations.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List

import numpy as np

from . import integrate, points
from .cubature import MAX_LEVEL, coarse, order_weights

TAG = 0x53554156


@dataclass
class MCRegion:
    sector: int
    level: np.ndarray
    index: np.ndarray
    uid: int
    value: np.ndarray = None
    err_re: np.ndarray = None
    err_im: np.ndarray = None
    axis: int = 0
    nonfinite: int = 0
    alive: bool = True


def region_u(seed: int, uid: int, n: int, N: int, tag: int = TAG) -> np.ndarray:
    key = (seed & points.M32, (seed >> 32) & points.M32)
    u = np.empty((N, n))
    p = np.arange(N, dtype=np.uint64)
    for c in range(n):
        o = points.philox4x32_10_np(p, np.full(N, c), np.full(N, uid & points.M32),
                                    np.full(N, ((uid >> 32) ^ tag) & points.M32), key)
        b = (o[0] << np.uint64(20)) | (o[1] >> np.uint64(12))
        u[:, c] = (b.astype(np.float64) + 0.5) * 2.0 ** -52
    return u


def evaluate(problem, r: MCRegion, N: int, seed: int, lead: int, pref, omega: np.ndarray):
    sec = problem.sectors[r.sector]
    n = sec.n
    width = np.ldexp(1.0, -r.level.astype(np.int64))
    lo = r.index * width
    u = region_u(seed, r.uid, n, N)
    x = lo[None, :] + u * width[None, :]
    vals, _, _ = integrate.sector_values(problem, r.sector, x, lead, pref)     # (K, N)
    vals = np.asarray(vals, dtype=complex)
    K = vals.shape[0]
    vol = float(np.prod(width))
    r.value = np.zeros(K, complex)
    r.err_re = np.zeros(K)
    r.err_im = np.zeros(K)
    for k in range(K):
        s1r, s1i = math.fsum(vals[k].real), math.fsum(vals[k].imag)
        s2r, s2i = math.fsum(vals[k].real ** 2), math.fsum(vals[k].imag ** 2)
        r.value[k] = vol * complex(s1r / N, s1i / N)
        vr = max(0.0, (s2r - s1r * s1r / N) / (N - 1))
        vi = max(0.0, (s2i - s1i * s1i / N) / (N - 1))
        r.err_re[k] = vol * math.sqrt(vr / N)
        r.err_im[k] = vol * math.sqrt(vi / N)
    r.nonfinite = int(np.sum(~np.all(np.isfinite(vals), axis=0)))
    g = np.sum(omega[:, None] * (np.abs(vals.real) + np.abs(vals.imag)), axis=0)
    best, axis = math.inf, 0
    for c in range(n):
        left = u[:, c] < 0.5
        nl, nr = int(left.sum()), int((~left).sum())
        if nl < 2 or nr < 2:
            continue
        sl = math.sqrt(max(0.0, np.mean(g[left] ** 2) - np.mean(g[left]) ** 2))
        sr = math.sqrt(max(0.0, np.mean(g[~left] ** 2) - np.mean(g[~left]) ** 2))
        phi = coarse(sl + sr)
        if phi < best:
            best, axis = phi, c
    r.axis = axis
    return r


def priority(r: MCRegion, omega: np.ndarray) -> float:
    v = omega * (r.err_re + r.err_im)
    if np.any(np.isnan(v)):
        return math.inf
    return coarse(float(np.max(v))) if np.any(v > 0) else 0.0


@dataclass
class SuaveResult:
    value: np.ndarray
    err_re: np.ndarray
    err_im: np.ndarray
    regions: List[MCRegion] = field(default_factory=list)
    evals: int = 0
    rounds: int = 0
    converged: bool = False


def suave(problem, maxeval: int, nnew: int, epsrel: float, epsabs: float, seed: int, split_frac: float = 0.25,
          batch_min: int = 1024) -> SuaveResult:
    lead, pref = integrate.prefactor_for(problem)
    K = problem.order_max - problem.order_min + 1
    regs: List[MCRegion] = []
    omega = np.ones(K)
    for s, sec in enumerate(problem.sectors):
        regs.append(MCRegion(s, np.zeros(sec.n, dtype=np.int64), np.zeros(sec.n, dtype=np.int64), s))
    evals = nnew * len(regs)
    if evals > maxeval:
        raise ValueError("maxeval below nnew points per sector")
    for r in regs:
        evaluate(problem, r, nnew, seed, lead, pref, omega)
    rounds = 1
    while True:
        alive = [r for r in regs if r.alive]
        total = np.array([integrate.fsum_c([r.value[k] for r in alive]) for k in range(K)])
        er = np.array([math.sqrt(math.fsum([r.err_re[k] ** 2 for r in alive])) for k in range(K)])
        ei = np.array([math.sqrt(math.fsum([r.err_im[k] ** 2 for r in alive])) for k in range(K)])
        omega, tau = order_weights(total, epsrel, epsabs)
        if np.all(er + ei <= tau):
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
            if evals + 2 * nnew > maxeval:
                break
            evals += 2 * nnew
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
                new.append(MCRegion(r.sector, lev, ind, len(regs) + len(new)))
        for r in new:
            evaluate(problem, r, nnew, seed, lead, pref, omega)
        regs.extend(new)
        rounds += 1
    alive = [r for r in regs if r.alive]
    value = np.array([integrate.fsum_c([r.value[k] for r in alive]) for k in range(K)])
    er = np.array([math.sqrt(math.fsum([r.err_re[k] ** 2 for r in alive])) for k in range(K)])
    ei = np.array([math.sqrt(math.fsum([r.err_im[k] ** 2 for r in alive])) for k in range(K)])
    return SuaveResult(value, er, ei, regs, evals, rounds, converged)
