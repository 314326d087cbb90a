"""Pins of the text-integrand oracle (oracle/expr.py) against values fixed by the
paper's format and by mathematics: literal arithmetic, the built-in constants,
closed-form integrals (the paper's own example among them) and the sector
oracle's eps expansion of the massless bubble; complex integrands (the text
uses I) against closed-form integrals that fix the branch of the logarithm
and of non-integer powers on the negative real axis, and their rounding bound
against a reordered evaluation."""
import math

import numpy as np
import pytest

from oracle import expr as E
from oracle import integrand, points
import sectorgen
from sectorgen import textgen


def value(body, n=1, x=None):
    e = E.parse(f"{n};0;{body};|")
    X = np.full((1, n), 0.5) if x is None else np.array([x], dtype=float)
    return float(E.evaluate(e, X)[0][0])


@pytest.mark.parametrize("body,want", [
    ("2+3*4", 14.0), ("2-3-4", -5.0), ("8/4/2", 1.0), ("-2*3", -6.0), ("2*-3", -6.0), ("-(2+3)*4", -20.0),
    ("((1))", 1.0), ("p[2,10]", 1024.0), ("p[4,0.5]", 2.0), ("p[2,-2]", 0.25), ("p[-2,3]", -8.0),
    ("1.5e1+.5", 15.5), ("2.", 2.0),
    ("P", 3.141592653589793), ("G", 0.5772156649015329), ("l[P]", 1.1447298858494002),
    # psi_1(1) = pi^2/6, psi_2(1) = -2 zeta(3), psi_3(2) = pi^4/15 - 6
    ("PolyGamma[1,1]", 1.6449340668482264), ("PolyGamma[2,1]", -2.4041138063191885),
    ("PolyGamma[2,4]", -2.4041138063191885 + 2.0 * (1.0 + 1.0 / 8.0 + 1.0 / 27.0)),
    ("PolyGamma[3,2]", 0.4939394022668291),
])
def test_literal_values(body, want):
    assert value(body) == pytest.approx(want, rel=1e-15, abs=1e-15)


def test_variables_and_intermediate_functions():
    e = E.parse("2;2;x[1]+x[2];f[1]*f[1];f[2]-f[1];|")
    v, _ = E.evaluate(e, np.array([[0.25, 0.5], [1.0, 2.0]]))
    assert v.tolist() == [0.5625 - 0.75, 9.0 - 3.0]
    e = E.parse("Integrate\n3;\n0;\nx[3]*10+x[2]*100+x[1];\n|\n")
    assert E.evaluate(e, np.array([[1.0, 2.0, 3.0]]))[0].tolist() == [231.0]


def test_real_powers_and_logs_of_negative_values_are_nan():
    assert math.isnan(value("p[-2,0.5]")) and math.isnan(value("l[-1]"))
    assert value("l[0]") == -math.inf


@pytest.mark.parametrize("text", [
    "1;0;x[1]+0.2;",            # no '|'
    "1;0;x[1]+0.2;|extra",
    "1;0;x[2];|", "1;0;x[0];|",
    "1;1;f[1];x[1];|",          # f[1] used in its own definition
    "1;0;q[1];|", "1;0;(x[1];|", "1;0;x[1]+;|", "1;0;p[x[1]];|",
    "0;0;1;|", "17;0;1;|", "1.5;0;1;|", "1;2;x[1];|",
])
def test_malformed_text_is_rejected(text):
    with pytest.raises(E.ParseError) as ei:
        E.parse(text)
    assert not ei.value.unsupported


def test_polygamma_outside_the_built_in_list_is_unsupported():
    with pytest.raises(E.ParseError) as ei:
        E.parse("1;0;PolyGamma[4,1];|")
    assert ei.value.unsupported


def lattice_estimate(text, m=14, R=16, seed=3):
    """Per-shift means of the oracle's shifted-lattice estimate (tent transform)."""
    e = E.parse(text)
    z = points.cbc_vector(m, e.n)
    sh = points.shift_table(seed, 0, R, e.n, m)
    means = []
    for r in range(R):
        x, w, _ = points.sector_points(z, m, sh[r], 0, 1 << m, None, True)
        v, _ = E.evaluate(e, x)
        means.append(float(np.mean(v * w)))
    means = np.array(means)
    return means.mean(), means.std(ddof=1) / math.sqrt(R)


@pytest.mark.parametrize("text,exact", [
    (textgen.PAPER_EXAMPLE, 0.7),                        # the paper's example: int_0^1 (x + 0.2) dx
    ("2;0;x[1]*p[x[2],2];|", 1.0 / 6.0),
    ("1;0;l[x[1]];|", -1.0),
    ("1;0;p[x[1],-0.5];|", 2.0),
    ("3;1;x[1]+x[2]+x[3];p[f[1],2];|", 2.5),            # E[(X1+X2+X3)^2] = 3/3 + 6/4
    ("2;0;1/(1+x[1]*x[2]);|", math.pi ** 2 / 12.0),     # int int 1/(1+xy) = pi^2/12
])
def test_closed_form_integrals(text, exact):
    mean, err = lattice_estimate(text)
    assert abs(mean - exact) <= 5 * err + 1e-9, (mean, err)


def test_bubble_orders_match_the_sector_oracle():
    """t^(-eps) (1+t)^(-2+2eps): its eps^k coefficient written out as text,
    against the sector oracle's expansion of the same sector."""
    sec = sectorgen.Sector(a=np.array([0.0]), b=np.array([-1.0]),
                           factors=[sectorgen.Factor(-2.0, 2.0, np.array([1.0, 1.0]),
                                                     np.array([[0], [1]], dtype=np.uint8))])
    rng = np.random.default_rng(5)
    x = rng.uniform(1e-6, 1.0, size=(4096, 1))
    vals, _, _ = integrand.sector_orders(sec, x, 0, 3, 0, np.ones(1, dtype=complex))
    for k in range(4):
        body = "p[1+x[1],-2]" if k == 0 else f"p[1+x[1],-2]*p[2*l[1+x[1]]-l[x[1]],{k}]/{math.factorial(k)}"
        v, _ = E.evaluate(E.parse(f"1;0;{body};|"), x)
        np.testing.assert_allclose(v, vals[k].real, rtol=1e-13, atol=0)


def test_rounding_bound_covers_a_reordered_evaluation():
    """The same sums in another order differ by less than 2 u cond."""
    rng = np.random.default_rng(2)
    x = rng.uniform(0.01, 1.0, size=(256, 3))
    a = E.parse("3;0;(x[1]+x[2]+x[3])*(x[1]-x[2])/(1+x[3]);|")
    b = E.parse("3;0;(x[3]+(x[2]+x[1]))*(x[1]-x[2])/(x[3]+1);|")
    va, ca = E.evaluate(a, x)
    vb, _ = E.evaluate(b, x)
    assert np.all(np.abs(va - vb) <= 2 * 2.0 ** -53 * ca)


# ---------------------------------------------------------------- complex integrands

def gl_integral(text, nodes=40):
    """Integral over [0,1]^n of the oracle's values by tensor Gauss-Legendre quadrature."""
    e = E.parse(text)
    t, w = np.polynomial.legendre.leggauss(nodes)
    t, w = 0.5 * (t + 1.0), 0.5 * w
    grids = np.meshgrid(*([t] * e.n), indexing="ij")
    wts = np.meshgrid(*([w] * e.n), indexing="ij")
    x = np.stack([g.ravel() for g in grids], axis=1)
    ww = np.prod(np.stack([g.ravel() for g in wts], axis=1), axis=1)
    v, _ = E.evaluate(e, x)
    return e, complex(np.sum(v * ww))


@pytest.mark.parametrize("text,exact", [
    ("1;0;p[x[1]+I,2];|", -2.0 / 3.0 + 1j),                                   # (x + i)^2
    ("1;0;1/(x[1]+I);|", 0.5 * math.log(2.0) - 0.25j * math.pi),              # Log(1 + i) - Log(i)
    ("1;0;p[x[1]+I,0.5];|", 2.0 / 3.0 * ((1 + 1j) ** 1.5 - 1j ** 1.5)),       # principal square root
    ("1;0;l[x[1]-2]+0*I;|", 2.0 * math.log(2.0) - 1.0 - 1j * math.pi),        # negative argument: arg -pi
    ("1;0;p[x[1]-2,-0.5]*I;|", 1j * 2.0 * (math.sqrt(2.0) - 1.0) * 1j),        # (x-2)^(-1/2) = i |x-2|^(-1/2)
    ("2;1;x[1]*I-x[2];p[f[1],2];|", -0.5j),                                   # (i x - y)^2
    # Log(-1 - i x) = ln(1 + x^2)/2 + i (atan x - pi): third quadrant, arg -pi at x = 0
    ("2;0;x[2]*l[-1-x[1]*I];|", 0.5 * (0.5 * (math.log(2.0) - 2.0 + math.pi / 2.0)
                                        - 1j * (0.75 * math.pi + 0.5 * math.log(2.0)))),
])
def test_complex_closed_form_integrals(text, exact):
    e, got = gl_integral(text)
    assert e.complex
    assert abs(got - exact) <= 1e-12 * max(1.0, abs(exact)), (got, exact)


def test_complex_rounding_bound_covers_a_reordered_evaluation():
    rng = np.random.default_rng(4)
    x = rng.uniform(0.01, 1.0, size=(256, 3))
    a = E.parse("3;0;(x[1]+I*x[2]+x[3])*(x[1]-I*x[2])/(1+I*x[3])*l[x[2]-x[1]-I*x[3]];|")
    b = E.parse("3;0;(x[3]+(x[2]*I+x[1]))*(x[1]-x[2]*I)/(x[3]*I+1)*l[(x[2]-x[1])-x[3]*I];|")
    va, ca = E.evaluate(a, x)
    vb, _ = E.evaluate(b, x)
    assert np.all(np.abs(va - vb) <= 2 * 2.0 ** -53 * ca)
