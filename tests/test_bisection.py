"""Bisection of variables (the BisectionVariables option of section 4.4): the
two parts of a bisected sector integrate to the sector's integral, order by
order (oracle, shifted-lattice estimates within 5 standard errors), for a
regular variable, a singular one (a_j = -1) and a variable with a non-integer
exponent, and the GPU integrates the bisected problem to the same values."""
import numpy as np
import pytest

import sectorgen
from sectorgen import Factor, Problem, Sector
from sectorgen.feynman import bisect_problem, bisect_sector
from oracle import integrate


def cases():
    prob = sectorgen.config2()
    picks = []
    for s in prob.sectors[:40]:
        S = [j for j in range(s.n) if s.a[j] == -1]
        R = [j for j in range(s.n) if s.a[j] != -1]
        if S and R:
            picks.append((s, S[0]))
            picks.append((s, R[0]))
        if len(picks) >= 4:
            break
    frac = Sector(a=np.array([0.5, -1.0]), b=np.array([-1.0, 2.0]),
                  factors=[Factor(-1.5, 0.5, np.array([1.0, 0.7, 0.3]),
                                  np.array([[0, 0], [1, 0], [1, 1]], dtype=np.uint8))])
    picks.append((frac, 0))
    return picks


@pytest.mark.parametrize("case", range(5))
def test_parts_add_up_to_the_sector(case):
    sec, j = cases()[case]
    whole = Problem(sectors=[sec], order_min=-2, order_max=0)
    parts = Problem(sectors=bisect_sector(sec, j, 0.5), order_min=-2, order_max=0)
    _, va, ra, ia = integrate.integrate(whole, 12, 16, 5)
    _, vb, rb, ib = integrate.integrate(parts, 12, 16, 6)
    err = np.sqrt(ra ** 2 + ia ** 2 + rb ** 2 + ib ** 2)
    assert np.all(np.abs(va - vb) <= 5 * err + 1e-12 * np.abs(va)), (va, vb, err)


def test_bisection_keeps_the_input_format():
    sec, j = cases()[0]
    lo, up = bisect_sector(sec, j, 0.3)
    for part in (lo, up):
        assert part.n == sec.n
        for f in part.factors:
            assert f.exps.max() <= 3 and np.any(np.all(f.exps == 0, axis=1))   # a constant term
    assert complex(lo.coeff) == pytest.approx(0.3 * complex(sec.coeff))
    assert complex(up.coeff) == pytest.approx(0.7 * complex(sec.coeff))
    two = bisect_problem(Problem(sectors=[sec], order_min=-2, order_max=0), [j, (j + 1) % sec.n])
    assert len(two.sectors) == 4


@pytest.mark.gpu
def test_gpu_bisected_problem_parity_and_invariance():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1511_03614_amd as P
    from test_gpu_parity import assert_close_shift, oracle_shift_values, set_params

    prob = sectorgen.config2()
    prob.sectors = prob.sectors[:8]
    parts = bisect_problem(prob, [0], 0.5)
    ctx = P.sdi_ctx_create(0)
    try:
        res = []
        for pr in (prob, parts):
            set_params(ctx, lattice_log2=14, shifts=16, seed=3)
            h = P.sdi_problem_create(ctx, pr)
            try:
                res.append(P.sdi_integrate(ctx, h))
                if pr is parts:
                    # the bisected sectors (negative coefficients, constant factors) at the parity bar
                    set_params(ctx, lattice_log2=10, shifts=4, seed=3)
                    P.sdi_integrate(ctx, h)
                    for s in (0, 1, 5):
                        _, _, per, _ = P.sdi_sector_results(ctx, h, s, 4)
                        oq, scale = oracle_shift_values(parts, s, 10, 4, 3)
                        assert_close_shift(per, oq, scale, f"bisected sector {s}")
            finally:
                P.sdi_problem_destroy(h)
        a, b = res
        err = np.sqrt(a["err_re"] ** 2 + a["err_im"] ** 2 + b["err_re"] ** 2 + b["err_im"] ** 2)
        assert np.all(np.abs(a["value"] - b["value"]) <= 5 * err + 1e-12 * np.abs(a["value"]))
    finally:
        set_params(ctx)
        P.sdi_ctx_destroy(ctx)
