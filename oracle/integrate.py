"""Oracle: per-sector QMC estimates, shift-to-shift errors and the combination.

TEST INFRASTRUCTURE ONLY (see the package docstring).

For sector s, shift r and result order k (after the prefactor fold):

    Q_{s,r,k} = (1/N) sum_{i<N} w_i F_{s,k}(x_i)          (sum correctly rounded: math.fsum)
    Qbar_{s,k} = mean_r Q_{s,r,k}
    sigma^2_{s,k} = sum_r |Q_{s,r,k} - Qbar_{s,k}|^2 / (R (R - 1))   (real and imaginary apart)

and the problem result R_k = sum_s Qbar_{s,k} with sigma_k = sqrt(sum_s sigma^2_{s,k}):
the paper sums the integrator's error estimates "using the mean-square norm"
(section 4.3).  Optional Vegas warm-up iterations adapt each sector's grid on
their own shifts before the frozen final pass (Vegas is the paper's default
integrator, section 4.4).
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import List, Optional

import numpy as np

from . import integrand, points, prefactor, vegas


@dataclass
class SectorEstimate:
    q: np.ndarray          # (R, K) complex per-shift means
    mean: np.ndarray       # (K,) complex
    err_re: np.ndarray     # (K,)
    err_im: np.ndarray     # (K,)
    n_nonfinite: int       # points where some order is not finite
    n_imf_positive: int
    grid: Optional[np.ndarray]


def fsum_c(v: np.ndarray) -> complex:
    v = np.asarray(v)
    if np.iscomplexobj(v):
        return complex(math.fsum(v.real.tolist()), math.fsum(v.imag.tolist()))
    return complex(math.fsum(v.tolist()), 0.0)


def prefactor_for(problem):
    max_s = max(len(integrand.singular_set(s)) for s in problem.sectors)
    if problem.feynman is not None:
        lead = prefactor.feynman_prefactor(problem.feynman.loops, problem.feynman.indices,
                                           problem.feynman.d0, 1)[0]
        length = problem.order_max - lead + max_s + 1
        return prefactor.explicit_or_feynman(problem, max(length, 1))
    return problem.pref_lead, [complex(p) for p in problem.pref]


def sector_values(problem, s: int, x: np.ndarray, pref_lead: int, pref):
    sec = problem.sectors[s]
    return integrand.sector_orders(sec, x, problem.order_min, problem.order_max, pref_lead, pref,
                                   problem.complex_mode, problem.lam)


def integrate_sector(problem, s: int, m: int, nshifts: int, seed: int, pref_lead: int, pref,
                     baker: bool = True, nbins: int = 128, warmup: int = 0, warmup_m: int = 14,
                     grid: Optional[np.ndarray] = None) -> SectorEstimate:
    sec = problem.sectors[s]
    n = sec.n
    N = 1 << m
    use_grid = warmup > 0 or grid is not None
    if use_grid and grid is None:
        grid = points.identity_grid(n, nbins)
    nonfinite = 0
    imfpos = 0
    kf_max = problem.order_max - pref_lead
    for it in range(warmup):
        zw = points.cbc_vector(warmup_m, n)
        sh = points.shift_table(seed, s, nshifts + it + 1, n, warmup_m)[nshifts + it]
        x, w, b = points.sector_points(zw, warmup_m, sh, 0, 1 << warmup_m, grid, baker)
        f, _, _ = integrand.sector_f(sec, x, kf_max + getattr(sec, "eps_shift", 0), problem.complex_mode,
                                     problem.lam)
        h = vegas.histogram(b, f * w[None, :], nbins)
        grid = vegas.refit(grid, vegas.importance(h))
    z = points.cbc_vector(m, n)
    shifts = points.shift_table(seed, s, nshifts, n, m)
    K = problem.order_max - problem.order_min + 1
    q = np.zeros((nshifts, K), dtype=np.complex128)
    for r in range(nshifts):
        x, w, _ = points.sector_points(z, m, shifts[r], 0, N, grid if use_grid else None, baker)
        vals, _, pos = sector_values(problem, s, x, pref_lead, pref)
        wf = vals * w[None, :]
        nonfinite += int(np.sum(~np.all(np.isfinite(wf), axis=0)))
        imfpos += int(np.sum(pos))
        for k in range(K):
            q[r, k] = fsum_c(wf[k]) / N
    mean = np.array([fsum_c(q[:, k]) / nshifts for k in range(K)])
    if nshifts > 1:
        d = q - mean[None, :]
        err_re = np.sqrt(np.sum(d.real ** 2, axis=0) / (nshifts * (nshifts - 1)))
        err_im = np.sqrt(np.sum(d.imag ** 2, axis=0) / (nshifts * (nshifts - 1)))
    else:
        err_re = np.zeros(K)
        err_im = np.zeros(K)
    return SectorEstimate(q, mean, err_re, err_im, nonfinite, imfpos, grid)


def combine(estimates: List[SectorEstimate]):
    """R_k = sum_s Qbar_{s,k}; sigma_k = sqrt(sum_s sigma_{s,k}^2) (re and im apart)."""
    K = estimates[0].mean.shape[0]
    val = np.array([fsum_c([e.mean[k] for e in estimates]) for k in range(K)])
    er = np.sqrt(np.array([math.fsum([e.err_re[k] ** 2 for e in estimates]) for k in range(K)]))
    ei = np.sqrt(np.array([math.fsum([e.err_im[k] ** 2 for e in estimates]) for k in range(K)]))
    return val, er, ei


def integrate(problem, m: int, nshifts: int, seed: int, baker: bool = True, nbins: int = 128,
              warmup: int = 0, warmup_m: int = 14, sectors=None):
    """All (or the listed) sectors; returns (per-sector estimates, value, err_re, err_im)."""
    lead, pref = prefactor_for(problem)
    idx = range(len(problem.sectors)) if sectors is None else sectors
    est = [integrate_sector(problem, s, m, nshifts, seed, lead, pref, baker, nbins, warmup, warmup_m)
           for s in idx]
    val, er, ei = combine(est)
    return est, val, er, ei


def neyman_allocation(estimates: List[SectorEstimate], budget: int, nshifts: int, lo: int, hi: int):
    """Per-sector lattice log2 for a final-pass budget from pilot errors.

    For every order k with a nonzero total T_k = sum_s (err_re^2 + err_im^2),
    sector s gets the weight sqrt(err_re^2 + err_im^2) / sqrt(T_k); weights add
    over orders; the sector's share is n_s = budget * w_s / W (equal shares if
    every error is zero).  Lattices are powers of two: each sector starts at the
    largest m in [lo, hi] with R 2^m <= n_s (lo if none), then, while the
    budget allows, the sector furthest below its share (largest n_s / 2^m,
    ties to the lower index) among those whose doubling still fits in the
    budget and stays <= hi is doubled.  Variance-proportional (Neyman)
    allocation of sampling effort, spending the budget to within one lattice
    doubling; the paper's integrator adapts points within one integral only
    (section 4.4), so this is a reading, not the paper's rule.
    """
    import heapq
    nsec = len(estimates)
    K = estimates[0].mean.shape[0]
    w = np.zeros(nsec)
    for k in range(K):
        tot = 0.0
        for e in estimates:
            tot += e.err_re[k] ** 2 + e.err_im[k] ** 2
        if not tot > 0.0 or not math.isfinite(tot):
            continue
        rt = math.sqrt(tot)
        for s, e in enumerate(estimates):
            w[s] += math.sqrt(e.err_re[k] ** 2 + e.err_im[k] ** 2) / rt
    W = 0.0
    for v in w:
        W += float(v)
    share = [float(budget) * float(w[s]) / W if W > 0.0 else float(budget) / nsec for s in range(nsec)]
    m = []
    for s in range(nsec):
        v = lo
        while v < hi and float(nshifts) * 2.0 ** (v + 1) <= share[s]:
            v += 1
        m.append(v)
    used = sum(nshifts << v for v in m)
    heap = [(-(share[s] / 2.0 ** m[s]), s) for s in range(nsec) if m[s] < hi]
    heapq.heapify(heap)
    while heap:
        _, s = heapq.heappop(heap)
        cost = nshifts << m[s]
        if used + cost > budget:
            continue                      # never fits later: the remaining budget only shrinks
        used += cost
        m[s] += 1
        if m[s] < hi:
            heapq.heappush(heap, (-(share[s] / 2.0 ** m[s]), s))
    return m
