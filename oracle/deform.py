"""Oracle: automatic choice of the contour-deformation size per sector.

TEST INFRASTRUCTURE ONLY (see the package docstring).

In complex mode the deformation z = y - i lam y (1 - y) dF/dy must keep
Im F(z) <= 0 (the F - i0 prescription); the paper's ComplexMode option
(section 4.4) either takes lam as given or tunes it automatically in
(0, MaxComplexShift], with LambdaSplit controlling the fineness of the search,
LambdaIterations the number of test points, and ConservativeComplexShift
halving the result.  Reading taken (the paper gives no formula):

* test points: the first 2^m points of the tent-transformed rank-1 lattice of
  sector s with the Philox shift of row TUNE_ROW (the pass shifts use rows
  below it, training rows lie above it);
* a point fails lam when Im F(z) > 0 at some corner x_W = 0 of the pole
  subtraction (the same corners the integrand evaluates);
* round r tries lam_k = top * k / split for k = split .. 1 and keeps the
  largest lam_k at which no test point fails; if none passes, top /= split and
  the next round starts (at most ROUNDS rounds, then lam = 0);
* conservative: the chosen lam is halved.
"""
from __future__ import annotations

import numpy as np

from . import points
from .integrand import f_derivatives, full_f_terms, singular_set

TUNE_ROW = 65535
ROUNDS = 4


def imf_positive(sector, x: np.ndarray, lam: float) -> np.ndarray:
    """Per point: Im F(z) > 0 at some corner of the singular set."""
    if sector.deform_factor < 0:
        return np.zeros(x.shape[0], dtype=bool)
    S = singular_set(sector)
    coef, exps = full_f_terms(sector)
    out = np.zeros(x.shape[0], dtype=bool)
    for wmask in range(1 << len(S)):
        y = x.copy()
        for i, j in enumerate(S):
            if wmask >> i & 1:
                y[:, j] = 0.0
        grad, _ = f_derivatives(sector, y)
        z = (y - 1j * lam * y * (1.0 - y) * grad).astype(np.complex128)
        fz = np.zeros(x.shape[0], dtype=np.complex128)
        for t in range(coef.shape[0]):
            mono = np.full(x.shape[0], coef[t], dtype=np.complex128)
            for j in range(sector.n):
                if exps[t, j]:
                    mono = mono * z[:, j] ** int(exps[t, j])
            fz = fz + mono
        out |= fz.imag > 0.0
    return out


def test_points(sector, s: int, m: int, seed: int) -> np.ndarray:
    z = points.cbc_vector(m, sector.n)
    sh = np.array([points.shift_int(seed, s, TUNE_ROW, j, m) for j in range(sector.n)], dtype=np.uint64)
    x, _, _ = points.sector_points(z, m, sh, 0, 1 << m, None, True)
    return x


def tune_lambda(sector, s: int, lam_max: float, split: int, m: int, seed: int,
                conservative: bool = False) -> float:
    """The deformation size chosen for sector s (index s keys its test points)."""
    x = test_points(sector, s, m, seed)
    top = lam_max
    for _ in range(ROUNDS):
        for k in range(split, 0, -1):
            lam = top * k / split
            if not imf_positive(sector, x, lam).any():
                return lam / 2.0 if conservative else lam
        top = top / split
    return 0.0
