"""Resumable lattice passes (the -continue option and the saved partial
results of sections 2.5 and 4.5): a pass split into slices of 2^slice_log2
points per shift, with its sums moved between contexts by
sdi_checkpoint_export / sdi_checkpoint_import.

Checks: once the lattice is complete a split run equals one run over the
whole lattice bit for bit (per shift, per sector and in total), also across
an export into a fresh context; a partial pass equals the oracle's mean over
the same leading lattice indices; settings that would break the sums are
rejected."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1511_03614_amd as P  # noqa: E402
import sectorgen  # noqa: E402
from sectorgen import feynman  # noqa: E402
from oracle import integrand, integrate, points  # noqa: E402

from test_gpu_parity import assert_close_shift, log, set_params  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    c = P.sdi_ctx_create(0)
    yield c
    P.sdi_ctx_destroy(c)


def snapshot(ctx, h, res, ns, R):
    per = [P.sdi_sector_results(ctx, h, s, R) for s in range(ns)]
    return res, per


def assert_same(a, b, what):
    ra, pa = a
    rb, pb = b
    for key in ("value", "err_re", "err_im"):
        assert np.array_equal(ra[key], rb[key]), (what, key, ra[key], rb[key])
    assert ra["n_nonfinite"] == rb["n_nonfinite"] and ra["n_imf_positive"] == rb["n_imf_positive"], what
    for s, (x, y) in enumerate(zip(pa, pb)):
        for i in range(3):
            assert np.array_equal(x[i], y[i]), (what, s, i)
        assert x[3] == y[3], (what, s)


CASES = {
    # 64 synthetic real sectors: 2^14 points per shift in slices of 2^12, tiles of 2^10
    "synthetic64": (sectorgen.config2, dict(lattice_log2=14, shifts=8, seed=5, tile_log2=10, ppt=2, slice_log2=12)),
    # the physical-region double box in complex mode: 2^12 points in slices of 2^10, tiles of 2^9
    "doublebox_complex": (lambda: feynman.double_box_problem(5.0, -2.0, 1.0, order_max=0, complex_mode=True, lam=0.5),
                    dict(lattice_log2=12, shifts=4, seed=9, tile_log2=9, ppt=1, slice_log2=10)),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_split_run_equals_one_run(ctx, name):
    make, prm = CASES[name]
    prob = make()
    ns, R, m, sl = len(prob.sectors), prm["shifts"], prm["lattice_log2"], prm["slice_log2"]
    h = P.sdi_problem_create(ctx, prob)
    try:
        set_params(ctx, **{**prm, "slice_log2": 0})
        whole = snapshot(ctx, h, P.sdi_integrate(ctx, h), ns, R)
        assert whole[0]["lattice_done"] == 1 << m
        set_params(ctx, **prm)
        nslices = 1 << (m - sl)
        for i in range(nslices):
            res = P.sdi_integrate(ctx, h)
            assert res["lattice_done"] == (i + 1) << sl
            assert res["n_evals"] == ns * R << sl
        split = snapshot(ctx, h, res, ns, R)
        assert_same(whole, split, name)
        # a call after the last slice starts a new pass
        res = P.sdi_integrate(ctx, h)
        assert res["lattice_done"] == 1 << sl
        log(f"{name}: {nslices} slices equal one pass bit for bit")
    finally:
        P.sdi_problem_destroy(h)
        set_params(ctx)


def test_partial_pass_matches_oracle(ctx):
    """After 3 of 4 slices the estimates are the means over lattice indices
    [0, 3 * 2^12) of each shift's 2^14-point lattice."""
    prob = sectorgen.config2()
    prm = CASES["synthetic64"][1]
    R, m, sl, seed = prm["shifts"], prm["lattice_log2"], prm["slice_log2"], prm["seed"]
    done = 3 << sl
    h = P.sdi_problem_create(ctx, prob)
    try:
        set_params(ctx, **prm)
        for _ in range(3):
            res = P.sdi_integrate(ctx, h)
        assert res["lattice_done"] == done
        lead, pref = integrate.prefactor_for(prob)
        K = prob.norders
        for s in (0, 17, 63):
            sec = prob.sectors[s]
            z = points.cbc_vector(m, sec.n)
            sh = points.shift_table(seed, s, R, sec.n, m)
            q = np.zeros((R, K), dtype=complex)
            scale = np.zeros(K)
            for r in range(R):
                x, w, _ = points.sector_points(z, m, sh[r], 0, done)
                vals, _, _ = integrand.sector_orders(sec, x, prob.order_min, prob.order_max, lead, pref)
                wf = vals * w[None, :]
                for k in range(K):
                    q[r, k] = integrate.fsum_c(wf[k]) / done
                    scale[k] = max(scale[k], float(np.mean(np.abs(wf[k]))))
            _, _, per, nev = P.sdi_sector_results(ctx, h, s, R)
            assert nev == R * done
            assert_close_shift(per, q, scale, f"partial pass sector {s}")
    finally:
        P.sdi_problem_destroy(h)
        set_params(ctx)


def test_checkpoint_into_fresh_context(ctx):
    prob = sectorgen.config2()
    prm = CASES["synthetic64"][1]
    ns, R = len(prob.sectors), prm["shifts"]
    h = P.sdi_problem_create(ctx, prob)
    try:
        set_params(ctx, **{**prm, "slice_log2": 0})
        whole = snapshot(ctx, h, P.sdi_integrate(ctx, h), ns, R)
        set_params(ctx, **prm)
        with pytest.raises(P.SdiError):
            P.sdi_checkpoint_export(ctx, h)              # no pass in progress
        P.sdi_integrate(ctx, h)
        P.sdi_integrate(ctx, h)
        blob = P.sdi_checkpoint_export(ctx, h)
    finally:
        P.sdi_problem_destroy(h)
        set_params(ctx)
    c2 = P.sdi_ctx_create(0)
    try:
        h2 = P.sdi_problem_create(c2, prob)
        set_params(c2, **{**prm, "seed": prm["seed"] + 1})
        with pytest.raises(P.SdiError):
            P.sdi_checkpoint_import(c2, h2, blob)      # other seed
        set_params(c2, **prm)
        with pytest.raises(P.SdiError):
            P.sdi_checkpoint_import(c2, h2, blob[:-8])  # truncated
        bad = bytearray(blob)
        bad[0] ^= 0xFF
        with pytest.raises(P.SdiError):
            P.sdi_checkpoint_import(c2, h2, bytes(bad))  # not a checkpoint
        P.sdi_checkpoint_import(c2, h2, blob)
        assert P.sdi_integrate(c2, h2)["lattice_done"] == 3 << prm["slice_log2"]
        res = P.sdi_integrate(c2, h2)
        assert res["lattice_done"] == 1 << prm["lattice_log2"]
        assert_same(whole, snapshot(c2, h2, res, ns, R), "checkpoint")
        # a checkpoint of another problem is refused
        h3 = P.sdi_problem_create(c2, sectorgen.config1())
        with pytest.raises(P.SdiError):
            P.sdi_checkpoint_import(c2, h3, blob)
        P.sdi_problem_destroy(h3)
        P.sdi_problem_destroy(h2)
    finally:
        P.sdi_ctx_destroy(c2)


def test_slices_need_a_uniform_pass(ctx):
    prob = sectorgen.config2()
    h = P.sdi_problem_create(ctx, prob)
    try:
        for extra in (dict(budget=1 << 20, pilot_log2=8), dict(warmup=2)):
            set_params(ctx, lattice_log2=12, slice_log2=10, **extra)
            with pytest.raises(P.SdiError):
                P.sdi_integrate(ctx, h)
    finally:
        P.sdi_problem_destroy(h)
        set_params(ctx)
