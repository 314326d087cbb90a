"""Oracle: Vegas histogram and grid refit (Lepage, J. Comput. Phys. 27 (1978) 192).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper's default integrator is Cuba's Vegas (section 4.4, CurrentIntegrator);
Cuba's own constants are not given there, so this is Lepage's published
refinement with these constants:

* importance of a point: rho = sum_k |w f_k|^2 / H_{j,k} over the sector's
  internal eps orders f_k (before the prefactor series multiplies them), where
  H_{j,k} is the iteration's total of |w f_k|^2 (so every order counts equally);
* per dimension j and bin b: d_b = sum of rho over the points in bin b;
* smoothing: d'_b = (d_{b-1} + d_b + d_{b+1}) / 3, two-point means at the ends;
* compression: r_b = d'_b / sum d', m_b = ((r_b - 1) / ln r_b)^alpha
  (m_b = 1 when |r_b - 1| < 1e-12, m_b = 0 when r_b = 0), alpha = 1.5;
* new edges hold equal shares sum(m)/NB, linear inside the old bins;
* a dimension whose histogram is all zero keeps its grid.
"""
from __future__ import annotations

import numpy as np

ALPHA = 1.5


def histogram(bins: np.ndarray, wf: np.ndarray, nbins: int) -> np.ndarray:
    """h[j, b, k] = sum over points with bin b in dim j of |w f_k|^2.

    bins: (npts, n) bin indices; wf: (K, npts) weighted internal orders.
    """
    npts, n = bins.shape
    a2 = np.abs(wf) ** 2
    K = a2.shape[0]
    h = np.zeros((n, nbins, K))
    for j in range(n):
        for k in range(K):
            h[j, :, k] = np.bincount(bins[:, j], weights=a2[k], minlength=nbins)
    return h


def importance(h: np.ndarray) -> np.ndarray:
    """d[j, b] = sum_k h[j, b, k] / H[j, k] over orders with H[j, k] > 0."""
    n, nb, K = h.shape
    d = np.zeros((n, nb))
    for j in range(n):
        for k in range(K):
            tot = h[j, :, k].sum()
            if tot > 0.0:
                d[j] += h[j, :, k] / tot
    return d


def refit(grid: np.ndarray, d: np.ndarray, alpha: float = ALPHA) -> np.ndarray:
    n, nb = d.shape
    new = grid.copy()
    for j in range(n):
        dj = d[j]
        if not np.any(dj > 0.0):
            continue
        sm = np.empty(nb)
        sm[0] = (dj[0] + dj[1]) / 2.0
        sm[nb - 1] = (dj[nb - 2] + dj[nb - 1]) / 2.0
        for b in range(1, nb - 1):
            sm[b] = (dj[b - 1] + dj[b] + dj[b + 1]) / 3.0
        tot = sum(sm)
        m = np.zeros(nb)
        for b in range(nb):
            r = sm[b] / tot
            if r == 0.0:
                m[b] = 0.0
            elif abs(r - 1.0) < 1e-12:
                m[b] = 1.0
            else:
                m[b] = ((r - 1.0) / np.log(r)) ** alpha
        share = sum(m) / nb
        g = grid[j]
        acc = 0.0
        b = 0
        for k in range(1, nb):
            t = k * share
            while b < nb - 1 and acc + m[b] <= t:
                acc += m[b]
                b += 1
            frac = min((t - acc) / m[b], 1.0) if m[b] > 0.0 else 1.0
            new[j, k] = g[b] + frac * (g[b + 1] - g[b])
        new[j, 0] = 0.0
        new[j, nb] = 1.0
    return new
