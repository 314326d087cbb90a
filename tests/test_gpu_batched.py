"""The batched, uneven configuration at its real shape: 2000 synthetic sectors
(4-9 variables, 5-40 terms, |S| <= 3) in one persistent launch per pass, with
per-sector lattice sizes reallocated from a pilot pass (Neyman).

Checks: the allocation equals the rule applied to the pilot's own per-sector
errors (the pilot is reproduced by a plain pass with the same seed and size);
the allocation spans several sizes; sampled sectors of the final pass agree
with the oracle on identical points at the 1e-10 bar."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1511_03614_amd as P  # noqa: E402
import sectorgen  # noqa: E402
from oracle import integrate  # noqa: E402

from test_gpu_parity import assert_close_shift, log, oracle_shift_values, set_params  # noqa: E402


def oracle_shift_mean_chunked(problem, s, m, R, seed, r, chunk_log2=16):
    """One shift's mean of a long lattice from the oracle, summed over index
    ranges of 2^chunk_log2 points (each range summed exactly, math.fsum over
    every value), and mean |w F| per order."""
    import math
    from oracle import integrand, points
    lead, pref = integrate.prefactor_for(problem)
    sec = problem.sectors[s]
    z = points.cbc_vector(m, sec.n)
    sh = points.shift_table(seed, s, R, sec.n, m)[r]
    N = 1 << m
    K = problem.norders
    parts = [[[], []] for _ in range(K)]
    absum = np.zeros(K)
    for i0 in range(0, N, 1 << chunk_log2):
        x, w, _ = points.sector_points(z, m, sh, i0, min(1 << chunk_log2, N - i0))
        vals, _, _ = integrand.sector_orders(sec, x, problem.order_min, problem.order_max, lead, pref)
        wf = vals * w[None, :]
        for k in range(K):
            parts[k][0].extend(wf[k].real.tolist())
            parts[k][1].extend(wf[k].imag.tolist())
            absum[k] += float(np.sum(np.abs(wf[k])))
    q = np.array([complex(math.fsum(parts[k][0]), math.fsum(parts[k][1])) / N for k in range(K)])
    return q, absum / N


@pytest.fixture(scope="module")
def ctx():
    c = P.sdi_ctx_create(0)
    yield c
    P.sdi_ctx_destroy(c)


def test_config4_allocation_at_scale(ctx):
    prob = sectorgen.config4()
    ns = len(prob.sectors)
    assert ns == 2000
    R, pilot, lo, hi = 16, 10, 8, 16
    budget = 1 << 28
    h = P.sdi_problem_create(ctx, prob)
    try:
        # the pilot pass alone (a plain pass with the pilot's size and seed)
        set_params(ctx, lattice_log2=pilot, shifts=R, seed=41)
        P.sdi_integrate(ctx, h)
        est = []
        for s in range(ns):
            mean, err, _, _ = P.sdi_sector_results(ctx, h, s, R)
            est.append(integrate.SectorEstimate(q=None, mean=mean, err_re=err[:, 0],
                                                err_im=err[:, 1], n_nonfinite=0, n_imf_positive=0, grid=None))
        m_rule = integrate.neyman_allocation(est, budget, R, lo, hi)
        set_params(ctx, shifts=R, seed=41, budget=budget, pilot_log2=pilot, alloc_min_log2=lo, alloc_max_log2=hi)
        res = P.sdi_integrate(ctx, h)
        m_gpu = []
        for s in range(ns):
            _, _, _, nev = P.sdi_sector_results(ctx, h, s, R)
            m_gpu.append(int(nev // R).bit_length() - 1)
        assert m_gpu == m_rule
        assert len(set(m_gpu)) >= 3
        log(f"config4: sizes {sorted(set(m_gpu))}, final evals {sum(R << m for m in m_gpu):.3e}, "
            f"pass {res['ms_total']:.1f} ms, kernel {res['ms_eval_kernel']:.1f} ms")
        # sampled sectors: the smallest, a middle and the largest allocation;
        # lattices above 2^14 points are compared on two shifts, the oracle
        # summing the shift in index ranges of 2^16 points
        order = np.argsort(m_gpu, kind="stable")
        for s in (int(order[0]), int(order[ns // 2]), int(order[-1])):
            _, _, per, _ = P.sdi_sector_results(ctx, h, s, R)
            if m_gpu[s] <= 14:
                oq, scale = oracle_shift_values(prob, s, m_gpu[s], R, 41)
                assert_close_shift(per, oq, scale, f"config4 sector {s} (m={m_gpu[s]})")
            else:
                for r in (0, R - 1):
                    oq, scale = oracle_shift_mean_chunked(prob, s, m_gpu[s], R, 41, r)
                    assert_close_shift(per[r:r + 1], oq[None, :], scale, f"config4 sector {s} (m={m_gpu[s]}) shift {r}")
    finally:
        P.sdi_problem_destroy(h)
        set_params(ctx)
