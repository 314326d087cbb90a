"""Pins of the oracle's lattice construction, Vegas refit and error estimate.

Each compares the oracle with an independent route:
* the CBC generating vector against the weighted P_2 figure computed on the
  dual lattice (sum over h != 0 with h.z = 0 mod N of prod_j gamma_j / h_j^2,
  residues summed in closed form by the cosecant identity), which shares no
  formula with the Bernoulli-polynomial form the search uses;
* the Vegas refit against the fixed point of the grid, found by an independent
  shooting solver, and against one-step predictions that follow from the
  refit's definition without re-typing it (a single occupied bin, a flat
  histogram);
* the shift-to-shift error against the t distribution it must follow, over
  many seeds, two-sided.
"""
import math

import mpmath as mp
import numpy as np
import pytest
from scipy import stats

import sectorgen
from oracle import integrate, points, vegas


# ------------------------------------------------------------------ CBC vector

def residue_sums(N: int) -> np.ndarray:
    """c[r] = sum over integers h = r (mod N), h != 0, of 1 / h^2.

    For r != 0 this is pi^2 / (N^2 sin^2(pi r / N)) (partial fractions of
    1/sin^2), for r = 0 it is zeta(2) / N^2."""
    r = np.arange(N)
    c = np.empty(N)
    c[0] = math.pi ** 2 / 6.0 / N ** 2
    c[1:] = math.pi ** 2 / (N ** 2 * np.sin(math.pi * r[1:] / N) ** 2)
    return c


def dual_p2(z, N: int) -> float:
    """sum_{h != 0, h.z = 0 mod N} prod_j r_j(h_j)^-1, r_j(0) = 1, r_j(h) = h^2 j^2.

    Summing h_j over each residue class rho_j mod N first leaves a finite sum
    over rho in Z_N^d with rho.z = 0 mod N."""
    c = residue_sums(N)
    d = len(z)
    # per dimension: the factor of residue rho (the h_j = 0 term counts in class 0)
    fac = [np.where(np.arange(N) == 0, 1.0, 0.0) + c / (j + 1) ** 2 for j in range(d)]
    # convolve over dimensions: acc[s] = sum over rho_1..rho_j with sum rho_i z_i = s mod N
    acc = np.zeros(N)
    acc[0] = 1.0
    for j in range(d):
        nxt = np.zeros(N)
        step = (np.arange(N) * z[j]) % N
        for rho in range(N):
            nxt += fac[j][rho] * np.roll(acc, step[rho])
        acc = nxt
    return float(acc[0] - 1.0)


def test_dual_p2_matches_brute_force_truncation():
    # the residue-class route against a direct (truncated) sum over h
    N, z = 8, (1, 3)
    H = 400
    h = np.arange(-H, H + 1)
    r = np.where(h == 0, 1.0, 0.0) + np.where(h == 0, 0.0, 1.0 / np.maximum(h, 1) ** 2)
    r = np.where(h == 0, 1.0, 1.0 / np.where(h == 0, 1, h) ** 2)
    r2 = np.where(h == 0, 1.0, 1.0 / (4.0 * np.where(h == 0, 1, h) ** 2))
    tot = 0.0
    for i, h1 in enumerate(h):
        ok = ((h1 * z[0] + h * z[1]) % N) == 0
        tot += r[i] * np.sum(r2[ok])
    tail = 2 * (2.0 / H) * (1 + math.pi ** 2 / 3)   # both dimensions' tails, generously
    assert abs((tot - 1.0) - dual_p2(z, N)) < tail


@pytest.mark.parametrize("m", [4, 5, 6, 7])
def test_cbc_vector_is_the_componentwise_minimum(m):
    """Every component z_j minimises the dual-lattice P_2 of (z_1..z_{j-1}, c)
    over all odd c < N (all candidates for N <= 128); z_1 = 1."""
    N = 1 << m
    d = 3
    z = points.cbc_vector(m, d)
    assert z[0] == 1
    for j in range(1, d):
        vals = {c: dual_p2(list(z[:j]) + [c], N) for c in range(1, N, 2)}
        best = min(vals.values())
        assert vals[z[j]] <= best * (1 + 1e-9), (m, j, z[j], min(vals, key=vals.get))


@pytest.mark.parametrize("m", [8, 9])
def test_cbc_vector_minimises_over_hashed_candidates(m):
    N = 1 << m
    z = points.cbc_vector(m, 3)
    cands = points.cbc_candidates(m)
    assert len(cands) == points.CBC_CANDIDATES and all(c % 2 == 1 and 0 < c < N for c in cands)
    for j in range(1, 3):
        vals = [dual_p2(list(z[:j]) + [c], N) for c in cands]
        assert dual_p2(list(z[:j + 1]), N) <= min(vals) * (1 + 1e-9)


def test_cbc_error_figure_decays_with_n():
    # P_2 of the chosen vectors falls close to the N^-2 rate (up to logs) of a good lattice
    p = [dual_p2(points.cbc_vector(m, 2), 1 << m) for m in (5, 7, 9)]
    assert p[1] < p[0] / 8 and p[2] < p[1] / 8


# ------------------------------------------------------------------ Vegas refit

def poly_bin_integrals(grid: np.ndarray, coef) -> np.ndarray:
    """Exact int over each bin of h(x)^2 for the polynomial h = sum coef_k x^k."""
    h2 = np.polynomial.polynomial.polymul(coef, coef)
    prim = np.polynomial.polynomial.polyint(h2)
    v = np.polynomial.polynomial.polyval(grid, prim)
    return np.diff(v)


def exact_importance(grid: np.ndarray, coef) -> np.ndarray:
    """Expected histogram of one dimension for N uniform latent points mapped by
    the grid and f = h: each bin holds N/NB points of weight NB dg_b, so
    d_b = N NB dg_b int_bin h^2 (N = 1 here: only ratios matter)."""
    nb = grid.shape[0] - 1
    return nb * np.diff(grid) * poly_bin_integrals(grid, coef)


def fixed_point_grid(coef, nb: int) -> np.ndarray:
    """Edges with dg_b * int_bin h^2 equal for every bin: shooting on the common
    value c (bisection), each edge from the previous one by bisection."""
    def edges_for(c):
        g = [0.0]
        for _ in range(nb):
            a = g[-1]
            if poly_bin_integrals(np.array([a, 1.0]), coef)[0] * (1.0 - a) < c:
                return None
            lo, hi = a, 1.0
            for _ in range(56):
                mid = 0.5 * (lo + hi)
                if (mid - a) * poly_bin_integrals(np.array([a, mid]), coef)[0] < c:
                    lo = mid
                else:
                    hi = mid
            g.append(0.5 * (lo + hi))
        return g
    lo, hi = 0.0, 1.0
    for _ in range(60):
        c = 0.5 * (lo + hi)
        g = edges_for(c)
        if g is None or g[-1] < 1.0 - 1e-15:
            if g is None:
                hi = c
            else:
                lo = c
        else:
            lo = c
    g = np.array(edges_for(lo)[:-1] + [1.0])
    return g


@pytest.mark.parametrize("coef", [(0.0, 0.0, 1.0), (0.2, 1.0), (1.0, 0.0, 0.0, 3.0)])
def test_refit_fixed_point_is_the_equal_importance_grid(coef):
    nb = 16
    target = fixed_point_grid(coef, nb)
    d = exact_importance(target, coef)
    assert np.ptp(d) < 1e-9 * d.mean()                      # the solver's grid equalises
    same = vegas.refit(target[None, :], d[None, :])[0]
    assert np.max(np.abs(same - target)) < 1e-9             # and refit leaves it in place
    # from the identity the first refits approach it (in the noise-free limit
    # the 3-point smoothing amplifies an odd-even mode of the widths, so later
    # iterations drift away again: that is a property of the method, not of
    # this implementation)
    g = points.identity_grid(1, nb)[0]
    dist = [np.max(np.abs(g - target))]
    for _ in range(4):
        g = vegas.refit(g[None, :], exact_importance(g, coef)[None, :])[0]
        dist.append(np.max(np.abs(g - target)))
    assert all(b < a for a, b in zip(dist, dist[1:])), dist
    assert dist[-1] < 0.25 * dist[0]


@pytest.mark.parametrize("coef", [(0.0, 0.0, 1.0), (0.2, 1.0)])
def test_histogram_importance_matches_exact_bin_integrals(coef):
    """The oracle's histogram of |w f|^2 over a 1-D lattice mapped by a
    non-uniform grid equals N NB dg_b int_bin h^2 up to the quadrature error
    of N/NB equispaced latent points per bin."""
    nb, m = 16, 14
    N = 1 << m
    g = np.sort(np.concatenate([[0.0, 1.0], np.random.default_rng(5).uniform(size=nb - 1)]))
    sh = points.shift_table(3, 0, 1, 1, m)[0]
    x, w, b = points.sector_points((1,), m, sh, 0, N, g[None, :], baker=False)
    f = np.polynomial.polynomial.polyval(x[:, 0], coef)
    h = vegas.histogram(b, (f * w)[None, :], nb)[0, :, 0]
    ex = N * exact_importance(g, coef)
    assert np.allclose(h, ex, rtol=2e-3, atol=1e-9 * ex.max())
    d = vegas.importance(vegas.histogram(b, np.stack([f * w, 3 * f * w]), nb))[0]
    assert np.allclose(d, 2 * ex / ex.sum(), rtol=2e-3)    # orders normalised to equal weight


def test_refit_single_occupied_bin_spreads_over_its_smoothing_window():
    """Only bin b has weight: smoothing gives bins b-1, b, b+1 one third each and
    the rest zero, so every new bin lies inside those three old bins, uniformly."""
    nb = 32
    g = np.sort(np.concatenate([[0.0, 1.0], np.random.default_rng(3).uniform(size=nb - 1)]))
    for b in (5, 17):
        d = np.zeros(nb)
        d[b] = 7.0
        new = vegas.refit(g[None, :], d[None, :])[0]
        # the three old bins have equal importance, so each holds nb/3 new bins,
        # spread linearly inside it
        lo, hi = g[b - 1], g[b + 2]
        assert new[0] == 0.0 and new[-1] == 1.0
        assert np.all(new[1:-1] >= lo) and np.all(new[1:-1] <= hi)
        for k in range(1, nb):
            t = 3.0 * k / nb                     # position in units of old bins from b-1
            i = min(int(t), 2)
            exp = g[b - 1 + i] + (t - i) * (g[b + i] - g[b - 1 + i])
            assert new[k] == pytest.approx(exp, abs=1e-12)


def test_refit_compression_exponent_from_two_level_histogram():
    """Two levels in halves of an identity grid: far from the step, new bin
    widths are inversely proportional to the compressed importance m(r), whose
    ratio between the halves is ((r2-1)/ln r2 / ((r1-1)/ln r1))^alpha; the
    ratio must change with alpha as that power and be 1 at alpha = 0."""
    nb = 64
    g = points.identity_grid(1, nb)
    d = np.ones((1, nb))
    d[0, nb // 2:] = 9.0
    widths = {}
    for alpha in (0.0, 0.75, 1.5):
        new = vegas.refit(g, d, alpha=alpha)[0]
        w = np.diff(new)
        widths[alpha] = w[4] / w[nb - 5]
    assert widths[0.0] == pytest.approx(1.0, rel=1e-12)
    # log width ratio is linear in alpha
    assert math.log(widths[1.5]) == pytest.approx(2.0 * math.log(widths[0.75]), rel=1e-9)
    assert widths[1.5] > 1.0                                  # light half gets the wider bins


# ------------------------------------------------------------------ error estimate

def smooth_sector():
    """Two variables, no singular variable and b = 0, so every order
    f_k = G0 Lambda^k / k! is smooth on the closed cube: the shift-to-shift
    errors of the lattice rule then behave like sample means.  (A log-singular
    integrand such as the bubble's higher orders has a skewed estimator: the
    rare shifts that put a point near the face carry the mean, so its
    t statistic is biased low although the estimator is unbiased.)"""
    from sectorgen import Factor, Sector
    U = Factor(-2.0, 1.0, np.array([1.0, 0.6, 0.3, 0.8]),
               np.array([[0, 0], [1, 0], [0, 1], [1, 1]], dtype=np.uint8))
    F = Factor(-1.0, -2.0, np.array([0.5, 1.0, 0.7]), np.array([[0, 0], [2, 0], [0, 2]], dtype=np.uint8))
    return Sector(a=np.array([0.0, 0.0]), b=np.array([0.0, 0.0]), factors=[U, F])


def test_shift_errors_follow_student_t_over_many_seeds():
    """(estimate - exact) / sigma over 150 seeds and three orders of a smooth
    sector follows the t distribution with R - 1 degrees of freedom: two-sided
    coverage of the central 68 % and 95 % bands and the second moment
    (R-1)/(R-3).  A sigma off by 2x in either direction fails."""
    from oracle import integrand
    sec = smooth_sector()
    prob = sectorgen.Problem(sectors=[sec], order_min=0, order_max=2)
    x1, w1 = np.polynomial.legendre.leggauss(40)
    x1, w1 = 0.5 * (x1 + 1), 0.5 * w1
    gx = np.stack([a.ravel() for a in np.meshgrid(x1, x1, indexing="ij")], axis=1)
    gw = np.outer(w1, w1).ravel()
    f, _, _ = integrand.sector_f(sec, gx, 2)
    exact = f @ gw                                        # Gauss-Legendre, exact to rounding here
    R = 8
    zs = []
    for seed in range(1, 151):
        _, val, er, _ = integrate.integrate(prob, 6, R, seed)
        zs.append((val.real - exact.real) / er)
    zs = np.array(zs).ravel()
    t68, t95 = stats.t.ppf(0.84, R - 1), stats.t.ppf(0.975, R - 1)
    c68, c95 = np.mean(np.abs(zs) < t68), np.mean(np.abs(zs) < t95)
    assert 0.56 < c68 < 0.82, c68
    assert 0.89 < c95 < 0.995, c95
    m2 = np.mean(zs ** 2)
    assert 0.8 < m2 < 2.4, m2      # t_7: 1.4; sigma 2x too large gives 0.35, 2x too small 5.6
    assert abs(np.mean(zs)) < 0.25


def test_monte_carlo_points():
    """Monte Carlo points: strictly inside (0, 1), distinct per shift and sector,
    uniform (moments within 5 sigma) and uncorrelated across variables."""
    from oracle import points as PT
    u = PT.mc_u(7, 3, 1, 0, 4096, 2)
    assert np.all((u > 0.0) & (u < 1.0))
    assert np.all(u * 2.0 ** 52 - 0.5 == np.floor(u * 2.0 ** 52))             # (b + 1/2) 2^-52
    n = u.shape[0]
    assert abs(u.mean() - 0.5) < 5 * math.sqrt(1 / 12 / (2 * n))
    assert abs((u ** 2).mean() - 1 / 3) < 5 * math.sqrt((1 / 5 - 1 / 9) / (2 * n))
    c = np.corrcoef(u[:, 0], u[:, 1])[0, 1]
    assert abs(c) < 5 / math.sqrt(n)
    assert not np.array_equal(PT.mc_u(7, 3, 2, 0, 8, 2), PT.mc_u(7, 3, 1, 0, 8, 2))
    assert not np.array_equal(PT.mc_u(7, 4, 1, 0, 8, 2), PT.mc_u(7, 3, 1, 0, 8, 2))
    assert np.array_equal(PT.mc_u(7, 3, 1, 5, 3, 2), u[5:8])                  # counter-based: any index range


def test_vectorised_philox_equals_the_scalar_one():
    from oracle import points as PT
    rng = np.random.default_rng(3)
    ctr = rng.integers(0, 2 ** 32, size=(4, 64), dtype=np.uint64)
    key = (0x12345678, 0x9ABCDEF0)
    v = PT.philox4x32_10_np(*ctr, key)
    for i in range(64):
        assert [int(w[i]) for w in v] == PT.philox4x32_10([int(c[i]) for c in ctr], key)
