"""Integrator parameters under the names of the SetCurrentIntegratorParameter
command's vocabulary (section 4.6): points, budget_total, budget_min,
budget_max, iterations and sampler = lattice | vegas | flow map onto the
library's own keys; malformed values are refused; the result reports the
flow training time that went into it."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1511_03614_amd as P  # noqa: E402
import sectorgen  # noqa: E402

from test_gpu_parity import set_params  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    c = P.sdi_ctx_create(0)
    yield c
    P.sdi_ctx_destroy(c)


def test_aliases_map_onto_the_library_keys(ctx):
    set_params(ctx, shifts=8)
    P.sdi_set_param(ctx, "points", 8 << 12)
    assert P.sdi_get_param(ctx, "lattice_log2") == "12"
    assert P.sdi_get_param(ctx, "points") == str(8 << 12)
    P.sdi_set_param(ctx, "budget_total", 1 << 24)
    assert P.sdi_get_param(ctx, "budget") == str(1 << 24)
    P.sdi_set_param(ctx, "budget_min", 8 << 10)
    P.sdi_set_param(ctx, "budget_max", 8 << 18)
    assert (P.sdi_get_param(ctx, "alloc_min_log2"), P.sdi_get_param(ctx, "alloc_max_log2")) == ("10", "18")
    P.sdi_set_param(ctx, "iterations", 3)
    assert P.sdi_get_param(ctx, "warmup") == "3"
    P.sdi_set_param(ctx, "warmup", 0)
    P.sdi_set_param(ctx, "sampler", "vegas")
    assert P.sdi_get_param(ctx, "sampler") == "0" and P.sdi_get_param(ctx, "warmup") == "5"
    P.sdi_set_param(ctx, "sampler", "flow")
    assert P.sdi_get_param(ctx, "sampler") == "1"
    P.sdi_set_param(ctx, "sampler", "lattice")
    assert P.sdi_get_param(ctx, "sampler") == "0"
    for key, val in (("points", 8 * 3 << 10), ("points", 7), ("budget_min", 8 << 30), ("sampler", "mc"),
                     ("iterations", 65)):
        with pytest.raises(P.SdiError):
            P.sdi_set_param(ctx, key, val)
    set_params(ctx)


def test_vegas_alias_runs_the_warmup(ctx):
    """sampler = vegas equals five warm-up iterations (fresh problems: grids persist with a problem)."""
    prob = sectorgen.config2()
    res = []
    for alias in (True, False):
        h = P.sdi_problem_create(ctx, prob)
        try:
            set_params(ctx, lattice_log2=10, shifts=4, warmup=0 if alias else 5)
            if alias:
                P.sdi_set_param(ctx, "sampler", "vegas")
            res.append(P.sdi_integrate(ctx, h))
            assert res[-1]["ms_warmup"] > 0.0
        finally:
            P.sdi_problem_destroy(h)
            set_params(ctx)
    # the warm-up histograms are summed with atomics, so grids agree to rounding only
    assert np.allclose(res[0]["value"], res[1]["value"], rtol=1e-12, atol=0.0)


def test_result_reports_the_training_time(ctx):
    prob = sectorgen.config2()
    h = P.sdi_problem_create(ctx, prob)
    try:
        set_params(ctx, lattice_log2=10, shifts=4)
        assert P.sdi_integrate(ctx, h)["ms_flow_train"] == 0.0
        P.sdi_flow_init(ctx, h, 3)
        ms = P.sdi_flow_train(ctx, h, 2, 8, 3e-3, sectors=[0, 1])
        ms += P.sdi_flow_train(ctx, h, 2, 8, 3e-3, sectors=[2])
        r = P.sdi_integrate(ctx, h)
        assert r["ms_flow_train"] == pytest.approx(ms, rel=1e-6)
        assert P.sdi_integrate(ctx, h)["ms_flow_train"] == 0.0
    finally:
        P.sdi_problem_destroy(h)
        set_params(ctx)
