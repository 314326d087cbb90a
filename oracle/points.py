"""Oracle: sampling points - rank-1 lattice, random shifts, tent map, Vegas map.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper integrates with Cuba's Vegas (section 4.4, CurrentIntegrator,
default vegasCuba, maxeval 50000) and says nothing about how points are drawn
beyond that.  The point set here is a randomly shifted rank-1 lattice rule
followed by the tent ("baker's") transform and, optionally, a Vegas
piecewise-linear map; every step is integer-exact or a single correctly
rounded fp64 operation, so an independent implementation can reproduce the
points bit for bit.

* N = 2^m points per shift; generating vector z from a component-by-component
  (CBC) search on the weighted P_2 criterion (Korobov space, alpha = 2,
  product weights gamma_j = j^-2).
* Shift for (sector s, shift r, dimension j): a 53-bit integer D from
  Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) with key = seed and counter
  (j, r, s, t); t counts redraws while D is a multiple of 2^(53-m).
* Point i: U_j = (i * z_j * 2^(53-m) + D_j) mod 2^53, u_j = U_j * 2^-53, which
  lies in (0, 1) by the redraw rule.
* Tent map: u -> 2u for u < 1/2, else 2(1 - u); values in (0, 1].
* Vegas map with NB bins and edges g_0 = 0 < ... < g_NB = 1:
  b = min(floor(u NB), NB - 1), d = u NB - b, x = g_b + d (g_{b+1} - g_b),
  weight NB (g_{b+1} - g_b) per dimension.
"""
from __future__ import annotations

from functools import lru_cache
from typing import Tuple

import numpy as np

M32 = 0xFFFFFFFF
MASK53 = (1 << 53) - 1

PHILOX_M0 = 0xD2511F53
PHILOX_M1 = 0xCD9E8D57
PHILOX_W0 = 0x9E3779B9
PHILOX_W1 = 0xBB67AE85


def philox4x32_10(ctr, key):
    """Philox4x32 with 10 rounds, on Python integers (one block)."""
    c = [int(v) & M32 for v in ctr]
    k0, k1 = int(key[0]) & M32, int(key[1]) & M32
    for rnd in range(10):
        if rnd:
            k0 = (k0 + PHILOX_W0) & M32
            k1 = (k1 + PHILOX_W1) & M32
        p0 = PHILOX_M0 * c[0]
        p1 = PHILOX_M1 * c[2]
        hi0, lo0 = p0 >> 32, p0 & M32
        hi1, lo1 = p1 >> 32, p1 & M32
        c = [hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0]
    return c


def philox4x32_10_np(c0, c1, c2, c3, key):
    """philox4x32_10 on arrays of counters (the same rounds on uint64 numpy arrays
    holding 32-bit values); returns the four output words as arrays."""
    c = [np.asarray(v, dtype=np.uint64) & np.uint64(M32) for v in (c0, c1, c2, c3)]
    k0, k1 = int(key[0]) & M32, int(key[1]) & M32
    m32 = np.uint64(M32)
    for rnd in range(10):
        if rnd:
            k0 = (k0 + PHILOX_W0) & M32
            k1 = (k1 + PHILOX_W1) & M32
        p0 = np.uint64(PHILOX_M0) * c[0]
        p1 = np.uint64(PHILOX_M1) * c[2]
        hi0, lo0 = p0 >> np.uint64(32), p0 & m32
        hi1, lo1 = p1 >> np.uint64(32), p1 & m32
        c = [hi1 ^ c[1] ^ np.uint64(k0), lo1, hi0 ^ c[3] ^ np.uint64(k1), lo0]
    return c


def shift_int(seed: int, s: int, r: int, j: int, m: int) -> int:
    """53-bit shift integer D_{s,r,j} for a lattice of 2^m points."""
    key = (seed & M32, (seed >> 32) & M32)
    t = 0
    while True:
        o = philox4x32_10((j, r, s, t), key)
        d = ((o[0] << 21) | (o[1] >> 11)) & MASK53
        if d % (1 << (53 - m)) != 0:
            return d
        t += 1


def shift_table(seed: int, s: int, nshifts: int, n: int, m: int) -> np.ndarray:
    return np.array([[shift_int(seed, s, r, j, m) for j in range(n)] for r in range(nshifts)],
                    dtype=np.uint64)


# ---------------------------------------------------------------- CBC vector

CBC_CANDIDATES = 64
GOLDEN64 = 0x9E3779B97F4A7C15


def cbc_candidates(m: int):
    """Odd candidates: all odd z < 2^m when there are at most 64, else 64 hashed ones."""
    N = 1 << m
    if N // 2 <= CBC_CANDIDATES:
        return [2 * k + 1 for k in range(N // 2)]
    out = []
    for k in range(1, CBC_CANDIDATES + 1):
        h = (k * GOLDEN64) & ((1 << 64) - 1)
        out.append(2 * (h >> (64 - (m - 1))) + 1)
    return out


@lru_cache(maxsize=None)
def cbc_vector(m: int, dims: int) -> Tuple[int, ...]:
    """Component-by-component generating vector for N = 2^m points.

    Criterion for candidate z in dimension j (1-based, weight 1/j^2), given the
    running products p_k of the earlier dimensions:
        E(z) = sum_{k=0}^{N-1} p_k (1 + gamma_j * 2 pi^2 B2({k z / N})),
    B2(t) = t^2 - t + 1/6; the smallest E wins, ties (relative 1e-12) go to the
    earlier candidate.  z_1 = 1.
    """
    N = 1 << m
    k = np.arange(N, dtype=np.uint64)
    p = np.ones(N, dtype=np.float64)
    z = []
    for j in range(1, dims + 1):
        gam = 1.0 / (j * j)
        cands = [1] if j == 1 else cbc_candidates(m)
        best, best_e = None, None
        for c in cands:
            t = ((k * np.uint64(c)) & np.uint64(N - 1)).astype(np.float64) / N
            e = float(np.sum(p * (1.0 + gam * (2.0 * np.pi ** 2) * (t * t - t + 1.0 / 6.0))))
            if best is None or e < best_e * (1.0 - 1e-12):
                best, best_e = c, e
        t = ((k * np.uint64(best)) & np.uint64(N - 1)).astype(np.float64) / N
        p = p * (1.0 + gam * (2.0 * np.pi ** 2) * (t * t - t + 1.0 / 6.0))
        z.append(int(best))
    return tuple(z)


# ---------------------------------------------------------------- points

def lattice_u(z, m: int, shifts: np.ndarray, i0: int, count: int) -> np.ndarray:
    """Shifted lattice points u (count, n) for indices i0 .. i0+count-1 (exact)."""
    n = len(shifts)
    i = np.arange(i0, i0 + count, dtype=np.uint64)[:, None]
    zz = np.array([int(v) << (53 - m) for v in z[:n]], dtype=np.uint64)[None, :]
    U = (i * zz + shifts.astype(np.uint64)[None, :]) & np.uint64(MASK53)
    return U.astype(np.float64) * (2.0 ** -53)


def tent(u: np.ndarray) -> np.ndarray:
    """Baker's transform: 2u for u < 1/2, 2(1 - u) otherwise (exact in fp64)."""
    return np.where(u < 0.5, 2.0 * u, 2.0 * (1.0 - u))


def identity_grid(n: int, nbins: int) -> np.ndarray:
    return np.tile(np.arange(nbins + 1, dtype=np.float64) / nbins, (n, 1))


def vegas_map(grid: np.ndarray, u: np.ndarray):
    """x and weight for points u under per-dimension piecewise-linear grids."""
    nb = grid.shape[1] - 1
    un = u * nb
    b = np.minimum(np.floor(un), nb - 1).astype(np.int64)
    d = un - b
    x = np.empty_like(u)
    w = np.ones(u.shape[0])
    for j in range(u.shape[1]):
        lo = grid[j, b[:, j]]
        hi = grid[j, b[:, j] + 1]
        width = hi - lo
        x[:, j] = lo + d[:, j] * width
        w = w * (nb * width)
    return x, w, b


# ---------------------------------------------------------------- Monte Carlo points

MC_TAG = 0x4D433031


def mc_u(seed: int, s: int, r: int, i0: int, count: int, n: int) -> np.ndarray:
    """Pseudo-random points of the Monte Carlo integrator (the sampling of the
    paper's default vegasCuba, section 4.4): point i of shift r of sector s,
    variable c from Philox4x32-10 with key = the seed's 32-bit halves and
    counter (i, c + 16 r, s, MC_TAG); u = (b + 1/2) 2^-52 with b the top 52 bits
    of the first two output words (out0 * 2^20 + floor(out1 / 2^12)), so u lies
    strictly inside (0, 1) and is exact in fp64."""
    key = (seed & M32, (seed >> 32) & M32)
    u = np.empty((count, n))
    idx = np.arange(i0, i0 + count, dtype=np.uint64)
    for c in range(n):
        o = philox4x32_10_np(idx, np.full(count, c + 16 * r), np.full(count, s), np.full(count, MC_TAG), key)
        b = (o[0] << np.uint64(20)) | (o[1] >> np.uint64(12))
        u[:, c] = (b.astype(np.float64) + 0.5) * 2.0 ** -52
    return u


def mc_points(seed: int, s: int, r: int, i0: int, count: int, n: int, grid=None):
    """Monte Carlo points and weights of one (sector, shift): no tent map; through
    the sector's Vegas grid when there is one."""
    u = mc_u(seed, s, r, i0, count, n)
    if grid is None:
        return u, np.ones(count)
    x, w, _ = vegas_map(grid, u)
    return x, w


def sector_points(z, m: int, shifts_r: np.ndarray, i0: int, count: int, grid=None, baker=True):
    """Points and weights for one (sector, shift): lattice -> tent -> Vegas map."""
    u = lattice_u(z, m, shifts_r, i0, count)
    if baker:
        u = tent(u)
    if grid is None:
        return u, np.ones(count), None
    x, w, b = vegas_map(grid, u)
    return x, w, b
