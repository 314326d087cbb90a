"""Large lattices: the one-loop bubble (two one-variable sectors) at 2^22 points
per shift against the oracle on every point, and at the largest accepted size,
2^30 points per shift (8 shifts), through the points at the end of the index
range (bit for bit) and the closed form of the integral (within 5 standard
errors)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1511_03614_amd as P  # noqa: E402
import sectorgen  # noqa: E402
from oracle import points  # noqa: E402

from test_gpu_parity import assert_close_shift, log, oracle_shift_values, set_params  # noqa: E402

# e^(gamma eps) Gamma(eps) Gamma(1-eps)^2 / Gamma(2-2eps): 1/eps + 2 + (4 - pi^2/12) eps + ...
BUBBLE = [1.0, 2.0, 4.0 - np.pi ** 2 / 12.0, 8.0 - np.pi ** 2 / 6.0 - 7.0 * 1.2020569031595942 / 3.0]


@pytest.fixture(scope="module")
def ctx():
    c = P.sdi_ctx_create(0)
    yield c
    P.sdi_ctx_destroy(c)


def test_lattice_2_22_parity(ctx):
    prob = sectorgen.config1()
    m, R, seed = 22, 2, 13
    set_params(ctx, lattice_log2=m, shifts=R, seed=seed, tile_log2=0)
    h = P.sdi_problem_create(ctx, prob)
    try:
        res = P.sdi_integrate(ctx, h)
        for s in range(2):
            _, _, per, nev = P.sdi_sector_results(ctx, h, s, R)
            assert nev == R << m
            oq, scale = oracle_shift_values(prob, s, m, R, seed)
            assert_close_shift(per, oq, scale, f"bubble sector {s} at 2^22")
        log(f"2^22: {res['value'].real} +- {res['err_re']}")
    finally:
        P.sdi_problem_destroy(h)
        set_params(ctx)


def test_largest_lattice(ctx):
    prob = sectorgen.config1()
    m, R, seed = 30, 8, 17
    set_params(ctx, lattice_log2=m, shifts=R, seed=seed, tile_log2=14, ppt=2)   # a fixed launch: no tuning at this size
    h = P.sdi_problem_create(ctx, prob)
    try:
        # the last 4096 points of shift 1 of sector 1, bit for bit
        i0, cnt = (1 << m) - 4096, 4096
        x, w = P.sdi_sample_points(ctx, h, 1, 1, i0, cnt, 1)
        z = points.cbc_vector(m, 1)
        sh = points.shift_table(seed, 1, R, 1, m)
        xo, wo, _ = points.sector_points(z, m, sh[1], i0, cnt, None, True)
        assert np.array_equal(x.cpu().numpy(), xo) and np.array_equal(w.cpu().numpy(), wo)
        res = P.sdi_integrate(ctx, h)
        assert res["n_evals"] == 2 * R << m and res["n_nonfinite"] == 0
        v, e = res["value"].real, res["err_re"]
        log(f"2^30: {v} +- {e}, {res['ms_total']:.1f} ms")
        assert np.all(np.abs(v - np.array(BUBBLE)) <= 5 * e + 1e-7)
    finally:
        P.sdi_problem_destroy(h)
        set_params(ctx)
