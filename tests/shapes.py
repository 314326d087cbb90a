"""Seeded sectors at the largest shapes the library accepts (shared by the
GPU parity tests and the CPU pins of the multiprecision oracle).

Real mode: 16 variables, 4 singular variables, 4 factors with exponents up to
3, 8 orders (eps^-4 .. eps^3).  Complex mode: 8 variables with 4 singular
ones and a sign-changing F (the deformation factor)."""
import numpy as np

from sectorgen import Factor, Problem, Sector, SplitMix64


def poly(rng, n, nterms, emax=3, signs=False):
    exps = {tuple([0] * n)}
    rows = [tuple([0] * n)]
    while len(rows) < nterms:
        e = tuple(rng.randint(0, emax) if rng.uniform() < 0.3 else 0 for _ in range(n))
        if e not in exps:
            exps.add(e)
            rows.append(e)
    coef = [1.0] + [(0.1 + 0.9 * rng.uniform()) * (-1.0 if signs and rng.uniform() < 0.4 else 1.0)
                    for _ in rows[1:]]
    return np.array(coef), np.array(rows, dtype=np.uint8)


def max_real_problem():
    """Three 16-variable sectors with 4 singular variables and 4 factors."""
    rng = SplitMix64(1601)
    secs = []
    for kind in ("integer", "general", "mixed"):
        n = 16
        a = np.zeros(n)
        b = np.array([float(rng.randint(-2, 2)) for _ in range(n)])
        a[:4] = -1.0
        b[:4] = [1.0, -2.0, 2.0, -1.0]
        if kind != "integer":
            a[4:8] = [0.5, 0.25, 1.0, 2.0]
            b[4:8] = [0.5, -1.5, 1.0, 0.0]
        facs = []
        for fm in range(4):
            c, e = poly(rng, n, 8 + 6 * fm)
            if kind == "integer" or (kind == "mixed" and fm % 2 == 0):
                g, d = float(rng.choice([-3, -2, -1, 1, 2])), float(rng.choice([-2, -1, 1, 2]))
            else:
                g, d = rng.choice([-1.5, -0.5, 0.5, 1.25]), rng.choice([-1.0, -0.5, 0.75])
            facs.append(Factor(g, d, c, e))
        secs.append(Sector(a=a, b=b, factors=facs, coeff=1.0 + 0.5j * (kind == "mixed")))
    return Problem(sectors=secs, order_min=-4, order_max=3, name="max16")


def max_complex_problem():
    """Two 8-variable deformed sectors with 4 singular variables."""
    rng = SplitMix64(802)
    secs = []
    for s in range(2):
        n = 8
        a = np.zeros(n)
        b = np.array([float(rng.randint(-2, 2)) for _ in range(n)])
        a[:4] = -1.0
        b[:4] = [1.0, -1.0, 2.0, -2.0]
        cu, eu = poly(rng, n, 10)
        cf, ef = poly(rng, n, 14, signs=True)
        cg, eg = poly(rng, n, 6)
        facs = [Factor(-2.0 + s, 3.0, cu, eu), Factor(-1.0 - s, -2.0, cf, ef), Factor(1.0, 1.0, cg, eg)]
        secs.append(Sector(a=a, b=b, factors=facs, deform_factor=1, deform_mono=np.zeros(n, np.int32)))
    return Problem(sectors=secs, order_min=-4, order_max=3, complex_mode=True, lam=0.2, name="max8c")
