"""Oracle: the Feynman prefactor series of eq. (2).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Eq. (2) writes a Feynman integral as (i pi^(d/2))^l Gamma(A - l d/2) / prod_j
Gamma(a_j) times the Feynman-parameter integral; section 4.3 states that results
are given with (i pi^(d/2))^l and exp(-l gamma_E eps) pulled out.  The series
that multiplies the sector sum is therefore

    Pi(eps) = exp(l gamma_E eps) Gamma(A - l d0/2 + l eps) / prod_j Gamma(a_j),

d = d0 - 2 eps.  It is expanded here with textbook identities, in mpmath
multiprecision, and rounded to fp64 at the end:

    ln Gamma(1 + x) = -gamma_E x + sum_{k>=2} (-1)^k zeta(k) x^k / k,
    Gamma(N + x)    = Gamma(1 + x) prod_{k=1}^{N-1} (k + x)            (N >= 1),
    Gamma(N + x)    = Gamma(1 + x) / prod_{k=N}^{0} (k + x)             (N <= 0).
"""
from __future__ import annotations

from typing import List, Sequence, Tuple

import mpmath as mp


def _mul(a, b, n):
    out = [mp.mpf(0)] * n
    for i, ai in enumerate(a[:n]):
        if ai == 0:
            continue
        for j, bj in enumerate(b[: n - i]):
            out[i + j] += ai * bj
    return out


def _exp_series(c, n):
    """exp of a power series c (c[0] must be 0), truncated to n terms."""
    assert c[0] == 0
    out = [mp.mpf(0)] * n
    out[0] = mp.mpf(1)
    term = out[:]
    for k in range(1, n):
        term = _mul(term, c, n)
        term = [t / k for t in term]
        out = [o + t for o, t in zip(out, term)]
    return out


def _inv_series(a, n):
    """1/a for a power series with a[0] != 0."""
    out = [mp.mpf(0)] * n
    out[0] = 1 / a[0]
    for k in range(1, n):
        s = mp.mpf(0)
        for j in range(1, k + 1):
            if j < len(a):
                s += a[j] * out[k - j]
        out[k] = -s / a[0]
    return out


def feynman_prefactor(loops: int, indices: Sequence[int], d0: int, length: int,
                      dps: int = 40) -> Tuple[int, List[float]]:
    """Return (lead, coeffs): Pi(eps) = sum_i coeffs[i] eps^(lead + i), ``length`` terms."""
    if loops < 1 or any(int(a) != a or a < 1 for a in indices):
        raise ValueError("loops >= 1 and integer indices >= 1 required")
    if (loops * d0) % 2:
        raise ValueError("l*d0 must be even for an integer Gamma argument")
    with mp.workdps(dps):
        A = sum(indices)
        N0 = A - loops * d0 // 2           # Gamma(N0 + l eps)
        n = length + 2
        # series in eps of ln Gamma(1 + l eps) + l gamma_E eps
        c = [mp.mpf(0)] * n
        for k in range(2, n):
            c[k] = (-1) ** k * mp.zeta(k) * mp.mpf(loops) ** k / k
        ser = _exp_series(c, n)                    # exp(l gamma eps) Gamma(1 + l eps)
        lead = 0
        if N0 >= 1:
            for k in range(1, N0):
                ser = _mul(ser, [mp.mpf(k), mp.mpf(loops)], n)
        else:
            den = [mp.mpf(1)]
            for k in range(N0, 0):
                den = _mul(den + [mp.mpf(0)] * n, [mp.mpf(k), mp.mpf(loops)], n)
            ser = _mul(ser, _inv_series(den, n), n)
            ser = [s / loops for s in ser]         # the k = 0 factor (l eps)
            lead = -1
        norm = mp.mpf(1)
        for a in indices:
            norm *= mp.gamma(a)
        ser = [s / norm for s in ser]
        return lead, [float(s) for s in ser[:length]]


def explicit_or_feynman(problem, length: int) -> Tuple[int, list]:
    """The prefactor series of a ``sectorgen.Problem``: explicit, or expanded here."""
    if problem.feynman is not None:
        f = problem.feynman
        return feynman_prefactor(f.loops, f.indices, f.d0, length)
    return problem.pref_lead, [complex(p) for p in problem.pref]


__all__ = ["feynman_prefactor", "explicit_or_feynman"]
