"""GPU parity of integrands given as text (sdi_problem_from_text) against the
text oracle (oracle/expr.py) on identical points.

Bars: per point |gpu - oracle| <= 1e-12 |oracle| + 8 u cond (cond: the
oracle's running rounding bound, u = 2^-53); per (shift) mean <= 1e-10 of
max(|mean|, mean |w f|), widened to the shift's mean rounding bound where that
is larger; closed-form integrals within 5 standard errors.  The same for
complex integrands (the text uses I), real and imaginary parts together."""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1511_03614_amd as P  # noqa: E402
import sectorgen  # noqa: E402
from sectorgen import textgen  # noqa: E402
from oracle import expr as E  # noqa: E402
from oracle import points  # noqa: E402

from test_gpu_parity import log, set_params  # noqa: E402

U = 2.0 ** -53


@pytest.fixture(scope="module")
def ctx():
    c = P.sdi_ctx_create(0)
    yield c
    P.sdi_ctx_destroy(c)


def texts():
    out = [("paper example", textgen.PAPER_EXAMPLE),
           ("functions", "2;2;x[1]*x[2]+0.5;p[f[1],3]-l[f[1]];f[2]/(f[1]+x[2])+PolyGamma[2,3]*G-P;|"),
           ("constant", "1;0;2.5;|"), ("variable", "4;0;x[4];|"),
           ("signs", "3;0;-(-x[1])+ -x[2]*-x[3]-p[x[1],-0.5];|")]
    for seed in range(12):
        n = 1 + (5 * seed) % 16
        out.append((f"random {seed} (n={n})", textgen.random_text(100 + seed, n, nfuncs=seed % 4, depth=3,
                                                                  terms=1 + seed % 4)))
    out.append(("3000 terms", textgen.random_text(999, 6, nfuncs=8, depth=3, terms=3000)))
    return out


def test_pointwise_matches_oracle(ctx):
    rng = np.random.default_rng(7)
    fr = []
    for name, text in texts():
        e = E.parse(text)
        x = rng.uniform(1e-4, 1.0, size=(1000, e.n))
        h = P.sdi_problem_from_text(ctx, text)
        try:
            assert P.sdi_problem_nsectors(h) == 1 and P.sdi_problem_norders(h) == 1
            g, gc = P.sdi_evaluate(ctx, h, 0, torch.from_numpy(x).cuda(), with_cond=True)
            g = g.cpu().numpy()
            assert torch.all(gc == 0.0)
        finally:
            P.sdi_problem_destroy(h)
        v, c = E.evaluate(e, x)
        d = np.abs(g[:, 0, 0] - v)
        assert np.all(g[:, 0, 1] == 0.0)
        ok = d <= 1e-12 * np.abs(v) + 8 * U * c
        assert ok.all(), f"{name}: {np.argwhere(~ok)[:5].ravel()} max rel {np.max(d / np.abs(v))}"
        fr.append((d <= 1e-12 * np.abs(v)).mean())
    log(f"text integrands: strict-clause fraction min {min(fr):.4f}")


def oracle_shifts(text, m, R, seed, grid=None):
    e = E.parse(text)
    z = points.cbc_vector(m, e.n)
    sh = points.shift_table(seed, 0, R, e.n, m)
    q, scale, bound = np.zeros(R), 0.0, np.zeros(R)
    for r in range(R):
        x, w, _ = points.sector_points(z, m, sh[r], 0, 1 << m, grid, True)
        v, c = E.evaluate(e, x)
        q[r] = math.fsum(v * w) / (1 << m)
        scale = max(scale, float(np.mean(np.abs(v * w))))
        bound[r] = 8 * U * float(np.mean(c * w))
    return q, scale, bound


@pytest.mark.parametrize("case", [0, 1, 5, 9, 17])
def test_integrate_matches_oracle(ctx, case):
    name, text = texts()[case]
    m, R, seed = 12, 8, 4
    set_params(ctx, lattice_log2=m, shifts=R, seed=seed, tile_log2=0)
    h = P.sdi_problem_from_text(ctx, text)
    try:
        res = P.sdi_integrate(ctx, h)
        _, _, per, nev = P.sdi_sector_results(ctx, h, 0, R)
    finally:
        P.sdi_problem_destroy(h)
        set_params(ctx)
    assert nev == R << m and res["n_nonfinite"] == 0
    q, scale, bound = oracle_shifts(text, m, R, seed)
    tol = np.maximum(1e-10 * np.maximum(np.abs(q), scale), bound)
    d = np.abs(per[:, 0].real - q)
    assert np.all(d <= tol), f"{name}: max d/tol {np.max(d / tol)}"
    mean = q.mean()
    assert abs(res["value"][0].real - mean) <= max(1e-10 * max(abs(mean), scale), bound.mean())
    assert res["value"][0].imag == 0.0


@pytest.mark.parametrize("text,exact", [
    (textgen.PAPER_EXAMPLE, 0.7),
    ("2;0;1/(1+x[1]*x[2]);|", math.pi ** 2 / 12.0),
    ("1;0;l[x[1]];|", -1.0),
    ("3;1;x[1]+x[2]+x[3];p[f[1],2];|", 2.5),
])
def test_closed_form_integrals(ctx, text, exact):
    set_params(ctx, lattice_log2=14, shifts=16, seed=9)
    h = P.sdi_problem_from_text(ctx, text)
    try:
        res = P.sdi_integrate(ctx, h)
    finally:
        P.sdi_problem_destroy(h)
        set_params(ctx)
    err = res["err_re"][0]
    assert abs(res["value"][0].real - exact) <= 5 * err + 1e-12, (res["value"][0], err)


def test_bubble_text_equals_the_sector_path(ctx):
    """The eps^k coefficients of t^(-eps) (1+t)^(-2+2eps) written out as text
    give, shift by shift, what the sector path computes for the same sector."""
    sec = sectorgen.Sector(a=np.array([0.0]), b=np.array([-1.0]),
                           factors=[sectorgen.Factor(-2.0, 2.0, np.array([1.0, 1.0]),
                                                     np.array([[0], [1]], dtype=np.uint8))])
    prob = sectorgen.Problem(sectors=[sec], order_min=0, order_max=2)
    m, R = 12, 8
    set_params(ctx, lattice_log2=m, shifts=R, seed=2)
    try:
        h = P.sdi_problem_create(ctx, prob)
        try:
            P.sdi_integrate(ctx, h)
            _, _, per_s, _ = P.sdi_sector_results(ctx, h, 0, R)
        finally:
            P.sdi_problem_destroy(h)
        for k in range(3):
            body = "p[1+x[1],-2]" if k == 0 else f"p[1+x[1],-2]*p[2*l[1+x[1]]-l[x[1]],{k}]/{math.factorial(k)}"
            h = P.sdi_problem_from_text(ctx, f"1;\n0;\n{body};\n|\n")
            try:
                P.sdi_integrate(ctx, h)
                _, _, per_t, _ = P.sdi_sector_results(ctx, h, 0, R)
            finally:
                P.sdi_problem_destroy(h)
            np.testing.assert_allclose(per_t[:, 0].real, per_s[:, k].real, rtol=1e-11, atol=0)
    finally:
        set_params(ctx)


def test_vegas_warmup_on_text(ctx):
    """A peaked integrand: int_0^1 dx/(x + 0.01) = ln 101.  The warm-up adapts the
    grid (smaller error than the plain lattice) and the result stays within 5 sigma."""
    text = "1;0;1/(x[1]+0.01);|"
    exact = math.log(101.0)
    errs = []
    try:
        for warm in (0, 4):
            set_params(ctx, lattice_log2=12, shifts=8, seed=6, warmup=warm, warmup_log2=12, nbins=64)
            h = P.sdi_problem_from_text(ctx, text)
            try:
                res = P.sdi_integrate(ctx, h)
            finally:
                P.sdi_problem_destroy(h)
            err = res["err_re"][0]
            assert abs(res["value"][0].real - exact) <= 5 * err + 1e-12
            errs.append(err)
    finally:
        set_params(ctx)
    log(f"ln 101: error {errs[0]:.3e} plain, {errs[1]:.3e} after warm-up")
    assert errs[1] < errs[0]


def test_sample_points_and_determinism(ctx):
    text = texts()[6][1]
    e = E.parse(text)
    m, R, seed = 10, 4, 12
    set_params(ctx, lattice_log2=m, shifts=R, seed=seed)
    h = P.sdi_problem_from_text(ctx, text)
    try:
        x, w = P.sdi_sample_points(ctx, h, 0, 2, 0, 1 << m, e.n)
        z = points.cbc_vector(m, e.n)
        sh = points.shift_table(seed, 0, R, e.n, m)
        xo, wo, _ = points.sector_points(z, m, sh[2], 0, 1 << m, None, True)
        assert np.array_equal(x.cpu().numpy(), xo) and np.array_equal(w.cpu().numpy(), wo)
        a = P.sdi_integrate(ctx, h)
        b = P.sdi_integrate(ctx, h)
        assert a["value"][0] == b["value"][0] and a["err_re"][0] == b["err_re"][0]
    finally:
        P.sdi_problem_destroy(h)
        set_params(ctx)


def test_text_errors_are_reported(ctx):
    for bad in ("1;0;x[2];|", "1;0;x[1]+0.2;", "1;0;(x[1];|", "1;0;y;|"):
        with pytest.raises(P.SdiError) as ei:
            P.sdi_problem_from_text(ctx, bad)
        assert ei.value.code == -1 and "problem_from_text" in str(ei.value)
    with pytest.raises(P.SdiError) as ei:
        P.sdi_problem_from_text(ctx, "1;0;PolyGamma[4,1]*x[1];|")
    assert ei.value.code == -4
    h = P.sdi_problem_from_text(ctx, textgen.PAPER_EXAMPLE)
    try:
        with pytest.raises(P.SdiError) as ei:
            P.sdi_flow_init(ctx, h, 1)
        assert ei.value.code == -4
    finally:
        P.sdi_problem_destroy(h)



# ---------------------------------------------------------------- complex integrands

def complex_texts():
    out = [("branch", "1;0;l[x[1]-2]+p[x[1]-3,0.5]+0*I;|"),
           ("constant log", "1;0;l[-1]*x[1]+p[-4,0.5]+I;|"),
           ("quotient", "2;1;x[1]+I*x[2];p[f[1],3]/(f[1]+2*I)-l[f[1]];|")]
    for seed in range(8):
        n = 1 + (3 * seed) % 12
        out.append((f"random complex {seed} (n={n})",
                    textgen.random_text(300 + seed, n, nfuncs=seed % 3, depth=2 + seed % 2, terms=1 + seed % 3,
                                        complex_=True)))
    out.append(("1000 complex terms", textgen.random_text(777, 5, nfuncs=4, depth=2, terms=1000, complex_=True)))
    return out


def test_complex_pointwise_matches_oracle(ctx):
    rng = np.random.default_rng(17)
    fr = []
    for name, text in complex_texts():
        e = E.parse(text)
        assert e.complex, name
        x = rng.uniform(1e-4, 1.0, size=(1000, e.n))
        h = P.sdi_problem_from_text(ctx, text)
        try:
            g = P.sdi_evaluate(ctx, h, 0, torch.from_numpy(x).cuda()).cpu().numpy()
        finally:
            P.sdi_problem_destroy(h)
        v, c = E.evaluate(e, x)
        gv = g[:, 0, 0] + 1j * g[:, 0, 1]
        d = np.abs(gv - v)
        ok = d <= 1e-12 * np.abs(v) + 8 * U * c
        assert ok.all(), f"{name}: {np.argwhere(~ok)[:5].ravel()} max rel {np.max(d / np.abs(v))}"
        fr.append((d <= 1e-12 * np.abs(v)).mean())
    log(f"complex text integrands: strict-clause fraction min {min(fr):.4f}")


def oracle_shifts_c(text, m, R, seed):
    e = E.parse(text)
    z = points.cbc_vector(m, e.n)
    sh = points.shift_table(seed, 0, R, e.n, m)
    q, scale, bound = np.zeros(R, complex), 0.0, np.zeros(R)
    for r in range(R):
        x, w, _ = points.sector_points(z, m, sh[r], 0, 1 << m, None, True)
        v, c = E.evaluate(e, x)
        q[r] = complex(math.fsum((v * w).real), math.fsum((v * w).imag)) / (1 << m)
        scale = max(scale, float(np.mean(np.abs(v * w))))
        bound[r] = 8 * U * float(np.mean(c * w))
    return q, scale, bound


@pytest.mark.parametrize("case", [0, 2, 5, 9])
def test_complex_integrate_matches_oracle(ctx, case):
    name, text = complex_texts()[case]
    m, R, seed = 12, 8, 4
    set_params(ctx, lattice_log2=m, shifts=R, seed=seed, tile_log2=0)
    h = P.sdi_problem_from_text(ctx, text)
    try:
        res = P.sdi_integrate(ctx, h)
        _, _, per, nev = P.sdi_sector_results(ctx, h, 0, R)
    finally:
        P.sdi_problem_destroy(h)
        set_params(ctx)
    assert nev == R << m and res["n_nonfinite"] == 0
    q, scale, bound = oracle_shifts_c(text, m, R, seed)
    tol = np.maximum(1e-10 * np.maximum(np.abs(q), scale), bound)
    d = np.abs(per[:, 0] - q)
    assert np.all(d <= tol), f"{name}: max d/tol {np.max(d / tol)}"
    mean = q.mean()
    assert abs(res["value"][0] - mean) <= max(1e-10 * max(abs(mean), scale), bound.mean())


@pytest.mark.parametrize("text,exact", [
    ("1;0;1/(x[1]+I);|", 0.5 * math.log(2.0) - 0.25j * math.pi),
    ("1;0;l[x[1]-2]+0*I;|", 2.0 * math.log(2.0) - 1.0 - 1j * math.pi),
    ("2;1;x[1]*I-x[2];p[f[1],2];|", -0.5j),
])
def test_complex_closed_form_integrals(ctx, text, exact):
    set_params(ctx, lattice_log2=14, shifts=16, seed=9, warmup=1)
    h = P.sdi_problem_from_text(ctx, text)
    try:
        res = P.sdi_integrate(ctx, h)
    finally:
        P.sdi_problem_destroy(h)
        set_params(ctx)
    v, er, ei = res["value"][0], res["err_re"][0], res["err_im"][0]
    assert abs(v.real - exact.real) <= 5 * er + 1e-12 and abs(v.imag - exact.imag) <= 5 * ei + 1e-12, (v, er, ei)
