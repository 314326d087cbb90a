"""The autotuner of the final-pass launch: tile size and launch variant chosen by
timing the kernel on the problem's own tiles, reported with the result,
reproduced when requested explicitly, kept across contexts by sdi_tune_save /
sdi_tune_load (and ignored when saved by another build of the kernels), and
built on a caller workspace of sdi_workspace_bytes."""
import json

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1511_03614_amd as P  # noqa: E402
import sectorgen  # noqa: E402

from test_gpu_parity import assert_close_shift, log, oracle_shift_values, set_params  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    c = P.sdi_ctx_create(0)
    yield c
    P.sdi_ctx_destroy(c)


def small_problem(nsec=16):
    prob = sectorgen.config2()
    prob.sectors = prob.sectors[:nsec]
    return prob


def run(ctx, prob, workspace=None):
    h = P.sdi_problem_create(ctx, prob)
    try:
        res = P.sdi_integrate(ctx, h, workspace)
        R = int(P.sdi_get_param(ctx, "shifts"))
        per = [P.sdi_sector_results(ctx, h, s, R)[2] for s in range(len(prob.sectors))]
        return res, per
    finally:
        P.sdi_problem_destroy(h)


def test_tuned_tile_is_reported_and_reproducible(ctx):
    prob = small_problem(64)
    m, R = 14, 4
    try:
        set_params(ctx, lattice_log2=m, shifts=R, seed=7, tile_log2=0, ppt=0)
        P.sdi_set_param(ctx, "tune", "search")
        a, per_a = run(ctx, prob)
        log(f"tuned: tile 2^{a['tile_log2']}, {a['ppt']} points/thread, {a['waves_per_simd']} waves/SIMD")
        assert 10 <= a["tile_log2"] <= 14
        assert a["ppt"] in (1, 2, 4) and 1 <= a["waves_per_simd"] <= 4
        # the chosen tile and points per thread, requested explicitly: the same sums in the same order
        set_params(ctx, lattice_log2=m, shifts=R, seed=7, tile_log2=a["tile_log2"], ppt=a["ppt"])
        b, per_b = run(ctx, prob)
        assert b["tile_log2"] == a["tile_log2"] and b["ppt"] == a["ppt"]
        np.testing.assert_allclose(b["value"], a["value"], rtol=1e-13, atol=0)
        for s in (0, 37):
            oq, scale = oracle_shift_values(prob, s, m, R, 7)
            assert_close_shift(per_a[s], oq, scale, f"tuned tile, sector {s}")
    finally:
        P.sdi_set_param(ctx, "tune", "cached")
        set_params(ctx)


def test_tune_cache_save_and_load(ctx, tmp_path):
    prob = small_problem()
    path = tmp_path / "tune.json"
    c2 = None
    try:
        set_params(ctx, lattice_log2=12, shifts=4, seed=7, tile_log2=0, ppt=0)
        P.sdi_set_param(ctx, "tune", "search")
        a, _ = run(ctx, prob)
        P.sdi_tune_save(ctx, str(path))
        doc = json.loads(path.read_text())
        assert doc["format"] == "sdint-autotune-1" and doc["entries"]
        # plant a decision timing would not necessarily make; a fresh context must use it
        mine = doc["entries"][-1]     # the newest decision: this problem's
        assert (mine["tile_log2"], mine["points_per_thread"], mine["waves_per_simd"]) == \
            (a["tile_log2"], a["ppt"], a["waves_per_simd"])
        mine.update(tile_log2=10, points_per_thread=1, waves_per_simd=4)
        path.write_text(json.dumps(doc))
        c2 = P.sdi_ctx_create(0)
        assert P.sdi_tune_load(c2, str(path)) == len(doc["entries"])
        set_params(c2, lattice_log2=12, shifts=4, seed=7, tile_log2=0, ppt=0)
        b, _ = run(c2, prob)
        assert (b["tile_log2"], b["ppt"], b["waves_per_simd"]) == (10, 1, 4)
        np.testing.assert_allclose(b["value"], a["value"], rtol=1e-10, atol=0)
        # saved by another build of the kernels: nothing is loaded
        doc["kernel_hash"] = "0" * 16
        other = tmp_path / "other.json"
        other.write_text(json.dumps(doc))
        assert P.sdi_tune_load(c2, str(other)) == 0
        # malformed files are rejected
        for bad in ('{"format": "sdint-autotune-1", "kernel_hash": "x", "entries": [{"key": "k"}]}',
                    '{"format": "something-else", "entries": []}', '[1, 2]', ''):
            other.write_text(bad)
            with pytest.raises(P.SdiError) as ei:
                P.sdi_tune_load(c2, str(other))
            assert ei.value.code == -1
        with pytest.raises(P.SdiError):
            P.sdi_tune_load(c2, str(tmp_path / "missing.json"))
    finally:
        if c2 is not None:
            P.sdi_ctx_destroy(c2)
        P.sdi_set_param(ctx, "tune", "cached")
        set_params(ctx)


def test_tuning_on_caller_workspace(ctx):
    prob = small_problem()
    try:
        set_params(ctx, lattice_log2=13, shifts=4, seed=11, tile_log2=0, ppt=0)
        P.sdi_set_param(ctx, "tune", "search")
        h = P.sdi_problem_create(ctx, prob)
        try:
            nb = P.sdi_workspace_bytes(ctx, h)
            ws = torch.full((nb,), 255, dtype=torch.uint8, device="cuda")
            a = P.sdi_integrate(ctx, h, ws)
            assert 10 <= a["tile_log2"] <= 13
        finally:
            P.sdi_problem_destroy(h)
        set_params(ctx, lattice_log2=13, shifts=4, seed=11, tile_log2=a["tile_log2"], ppt=a["ppt"])
        b, _ = run(ctx, prob)
        np.testing.assert_allclose(b["value"], a["value"], rtol=1e-13, atol=0)
    finally:
        P.sdi_set_param(ctx, "tune", "cached")
        set_params(ctx)
