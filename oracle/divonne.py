"""Oracle: a partition by spreads, then a lattice rule on every region.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper lets the final stage use Cuba's Divonne (CurrentIntegrator =
divonneCuba, section 4.4) and gives nothing beyond the name.  Divonne's idea
(Hahn, Comput. Phys. Commun. 168 (2005) 78) is stratified sampling: cut the
region into subregions of about equal spread, integrate each with a more
accurate rule, and refine where the two estimates disagree.  This module
states the version the library's integrator 4 computes (a reading):

* Partition: the region loop of oracle/suave.py (dyadic boxes numbered in
  creation order, batches, the cubature's budget), every new region sampled
  at N points from Philox4x32-10 with counter (p, c, number, (number / 2^32)
  xor 0x44495631) and valued as in suave.  With g_p = sum_k omega_k
  (|Re F_k| + |Im F_k|) (the round's order weights, 1 / tolerance), the
  region's spread is vol (max g - min g) / 2, and it would be halved along the
  variable c whose halves (u_c < 1/2, u_c >= 1/2) have the smallest larger
  range max - min of g, compared at 8 significant bits (ties: the lowest c; a
  half with fewer than two samples: infinite; all infinite: variable 0).  A
  round halves the regions of largest spread (8 significant bits; batch rule
  and budget as in the cubature) until the budget is spent or no region can
  be halved (level limit, zero spread).  Spreads are taken with the weights of
  the round a region was sampled in, so they order the halving but are no
  stopping test: the partition spends its budget.
* Final rule: the regions alive, numbered 0, 1, ... in creation order, each
  take the rank-1 lattice rule of 2^m points with the CBC vector of
  oracle/points.py and R shifts: D_{c,t} = the top 53 bits of Philox4x32-10
  with counter (c, t, number, (number / 2^32) xor 0x44495632), lowest bit set
  (so no point has u = 0); u_i = ((i z_c 2^(53-m) + D) mod 2^53) 2^-53, the
  tent map when baker, x_c = lo_c + u w_c.  Value: vol times the mean of the
  R shift means; error: vol sqrt(s^2 / R) with s^2 the unbiased variance of
  the shift means, per real and imaginary part.
* Refinement (one pass): a region whose final and partition values differ by
  more than 4 sqrt(e_final^2 + e_partition^2) in some order's real or
  imaginary part is halved along its partition axis (below the level limit);
  the halves, numbered on after the final rule's regions (lower half first,
  parents in order), take the final rule instead of it.
* Totals: sums over the regions alive; errors combine as root sums of squares.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List

import numpy as np

from . import integrate, points, suave
from .cubature import MAX_LEVEL, coarse, order_weights

PART_TAG = 0x44495631
LAT_TAG = 0x44495632
MASK53 = (1 << 53) - 1


def partition_evaluate(problem, r: suave.MCRegion, N: int, seed: int, lead: int, pref, omega: np.ndarray):
    """Value, errors, spread and axis of a new region of the partition."""
    sec = problem.sectors[r.sector]
    n = sec.n
    width = np.ldexp(1.0, -r.level.astype(np.int64))
    lo = r.index * width
    u = suave.region_u(seed, r.uid, n, N, PART_TAG)
    x = lo[None, :] + u * width[None, :]
    vals, _, _ = integrate.sector_values(problem, r.sector, x, lead, pref)
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
        r.err_re[k] = vol * math.sqrt(max(0.0, (s2r - s1r * s1r / N) / (N - 1)) / N)
        r.err_im[k] = vol * math.sqrt(max(0.0, (s2i - s1i * s1i / N) / (N - 1)) / N)
    r.nonfinite = int(np.sum(~np.all(np.isfinite(vals), axis=0)))
    g = np.zeros(N)
    for k in range(K):
        g = g + omega[k] * (np.abs(vals[k].real) + np.abs(vals[k].imag))
    r.spread = vol * (float(np.max(g)) - float(np.min(g))) * 0.5
    best, axis = math.inf, 0
    for c in range(n):
        left = u[:, c] < 0.5
        if left.sum() < 2 or (~left).sum() < 2:
            continue
        phi = coarse(max(np.max(g[left]) - np.min(g[left]), np.max(g[~left]) - np.min(g[~left])))
        if phi < best:
            best, axis = phi, c
    r.axis = axis
    return r


def lattice_rule(problem, r: suave.MCRegion, number: int, m: int, R: int, seed: int, baker: bool, lead: int, pref):
    """The final rule on region r (numbered `number`): value and errors."""
    sec = problem.sectors[r.sector]
    n = sec.n
    N = 1 << m
    width = np.ldexp(1.0, -r.level.astype(np.int64))
    lo = r.index * width
    vol = float(np.prod(width))
    z = points.cbc_vector(m, n)
    key = (seed & points.M32, (seed >> 32) & points.M32)
    i = np.arange(N, dtype=np.uint64)
    means = []
    nonfin = 0
    for t in range(R):
        u = np.empty((N, n))
        for c in range(n):
            o = points.philox4x32_10((c, t, number & points.M32, ((number >> 32) ^ LAT_TAG) & points.M32), key)
            D = (((o[0] << 21) | (o[1] >> 11)) & MASK53) | 1
            U = (i * np.uint64(int(z[c]) << (53 - m)) + np.uint64(D)) & np.uint64(MASK53)
            u[:, c] = U.astype(np.float64) * 2.0 ** -53
        if baker:
            u = points.tent(u)
        x = lo[None, :] + u * width[None, :]
        vals, _, _ = integrate.sector_values(problem, r.sector, x, lead, pref)
        vals = np.asarray(vals, dtype=complex)
        nonfin += int(np.sum(~np.all(np.isfinite(vals), axis=0)))
        means.append([complex(math.fsum(v.real) / N, math.fsum(v.imag) / N) for v in vals])
    q = np.array(means)                                  # (R, K)
    K = q.shape[1]
    value = np.zeros(K, complex)
    er = np.zeros(K)
    ei = np.zeros(K)
    for k in range(K):
        ar = math.fsum(q[:, k].real) / R
        ai = math.fsum(q[:, k].imag) / R
        vr = math.fsum((q[:, k].real - ar) ** 2) / (R - 1)
        vi = math.fsum((q[:, k].imag - ai) ** 2) / (R - 1)
        value[k] = vol * complex(ar, ai)
        er[k] = vol * math.sqrt(vr / R)
        ei[k] = vol * math.sqrt(vi / R)
    return value, er, ei, nonfin


@dataclass
class DivonneResult:
    value: np.ndarray
    err_re: np.ndarray
    err_im: np.ndarray
    regions: List[suave.MCRegion] = field(default_factory=list)
    evals: int = 0
    rounds: int = 0
    refined: int = 0


def divonne(problem, maxeval: int, nnew: int, epsrel: float, epsabs: float, seed: int, m: int, R: int,
            baker: bool = True, split_frac: float = 0.25, batch_min: int = 1024) -> DivonneResult:
    lead, pref = integrate.prefactor_for(problem)
    K = problem.order_max - problem.order_min + 1
    regs: List[suave.MCRegion] = []
    omega = np.ones(K)
    for s, sec in enumerate(problem.sectors):
        regs.append(suave.MCRegion(s, np.zeros(sec.n, dtype=np.int64), np.zeros(sec.n, dtype=np.int64), s))
    evals = nnew * len(regs)
    if evals > maxeval:
        raise ValueError("maxeval below nnew points per sector")
    for r in regs:
        partition_evaluate(problem, r, nnew, seed, lead, pref, omega)
    rounds = 1
    while True:
        alive = [r for r in regs if r.alive]
        total = np.array([integrate.fsum_c([r.value[k] for r in alive]) for k in range(K)])
        omega, _ = order_weights(total, epsrel, epsabs)
        cand = []
        for i, r in enumerate(regs):
            if not r.alive or r.level[r.axis] >= MAX_LEVEL:
                continue
            p = math.inf if math.isnan(r.spread) else coarse(r.spread)
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
                new.append(suave.MCRegion(r.sector, lev, ind, len(regs) + len(new)))
        for r in new:
            partition_evaluate(problem, r, nnew, seed, lead, pref, omega)
        regs.extend(new)
        rounds += 1
    # final rule, then one refinement
    final = [r for r in regs if r.alive]
    redo = []
    for num, r in enumerate(final):
        v, er, ei, nf = lattice_rule(problem, r, num, m, R, seed, baker, lead, pref)
        r.nonfinite += nf
        evals += R << m
        d_re, d_im = np.abs(v.real - r.value.real), np.abs(v.imag - r.value.imag)
        bad = np.any(~(d_re <= 4.0 * np.hypot(er, r.err_re))) or np.any(~(d_im <= 4.0 * np.hypot(ei, r.err_im)))
        r.value, r.err_re, r.err_im = v, er, ei
        if bad and r.level[r.axis] < MAX_LEVEL:
            redo.append(r)
    num = len(final)
    for r in redo:
        r.alive = False
        for half in (0, 1):
            lev = r.level.copy()
            ind = r.index.copy()
            lev[r.axis] += 1
            ind[r.axis] = 2 * ind[r.axis] + half
            h = suave.MCRegion(r.sector, lev, ind, len(regs))
            h.axis = r.axis
            h.value, h.err_re, h.err_im, h.nonfinite = lattice_rule(problem, h, num, m, R, seed, baker, lead, pref)
            num += 1
            evals += R << m
            regs.append(h)
    alive = [r for r in regs if r.alive]
    value = np.array([integrate.fsum_c([r.value[k] for r in alive]) for k in range(K)])
    er = np.array([math.sqrt(math.fsum([r.err_re[k] ** 2 for r in alive])) for k in range(K)])
    ei = np.array([math.sqrt(math.fsum([r.err_im[k] ** 2 for r in alive])) for k in range(K)])
    return DivonneResult(value, er, ei, regs, evals, rounds, len(redo))
