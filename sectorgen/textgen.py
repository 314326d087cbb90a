"""Seeded integrands in the integration workers' text format (inputs only).

The format (section 4.6 of the paper): the number of variables, the number of
intermediate functions, one line per intermediate function, the integrand,
each line ended by ';', then a line '|'.  ``random_text`` builds expressions
whose subexpressions stay positive on (0, 1]^n (sums, products, quotients and
powers of positive terms, logarithms of 1 + positive), with a few signed
differences at the top, so that values are finite at every lattice point.
It performs none of the method's arithmetic: it writes text.
"""
from __future__ import annotations

from typing import List

from . import SplitMix64

__all__ = ["random_text", "PAPER_EXAMPLE"]

# the worker-format example of the paper: the integral of x + 0.2 over [0, 1]
PAPER_EXAMPLE = "1;\n0;\nx[1]+0.2;\n|\n"


def _num(rng: SplitMix64) -> str:
    return f"{0.1 + 1.9 * rng.uniform():.4f}"


def _pos(rng: SplitMix64, n: int, nf: int, depth: int) -> str:
    """A positive expression on (0, 1]^n."""
    if depth <= 0:
        k = rng.randint(0, 5)
        if k <= 2:
            return f"x[{rng.randint(1, n)}]"
        if k == 3 and nf:
            return f"f[{rng.randint(1, nf)}]"
        if k == 4:
            return rng.choice(["P", "G", "PolyGamma[1,1]", "PolyGamma[3,2]"])
        return _num(rng)
    a = _pos(rng, n, nf, depth - 1)
    b = _pos(rng, n, nf, depth - 1)
    k = rng.randint(0, 7)
    if k == 0:
        return f"({a}+{b})"
    if k == 1:
        return f"{a}*{b}"
    if k == 2:
        return f"{a}/({b}+{_num(rng)})"
    if k == 3:
        return f"p[{a}+{_num(rng)},{rng.randint(-3, 4)}]"
    if k == 4:
        return f"p[{a}+{_num(rng)},{rng.choice(['0.5', '-1.5', '0.25', '1.75'])}]"
    if k == 5:
        return f"l[1+{a}]"
    if k == 6:
        return f"({a}*{_num(rng)}+{b})"
    return f"({a}+{b})/{_num(rng)}"


def _complex_term(rng: SplitMix64, e: str) -> str:
    """A complex expression around e (a real positive or a complex expression
    whose real part stays positive): the imaginary unit I, logarithms and a
    power of a real negative argument (the branch below the cut), and
    arguments kept off the negative real axis otherwise."""
    c = _num(rng)
    k = rng.randint(0, 5)
    if k == 0:
        return f"{c}*I*{e}"
    if k == 1:
        return f"p[{e}+{c}*I,{rng.choice(['2', '-1', '0.5', '-1.5'])}]"
    if k == 2:
        return f"l[{e}-{c}-2]"                 # real and negative: arg -pi
    if k == 3:
        return f"l[{e}+{c}*I]"
    if k == 4:
        return f"p[-{e}-{c},0.5]*{e}"          # the square root of a negative real value
    return f"{e}/({e}+{c}*I)"


def random_text(seed: int, n: int, nfuncs: int = 2, depth: int = 4, terms: int = 3, complex_: bool = False) -> str:
    """n variables, nfuncs intermediate functions, an integrand of ``terms``
    signed terms of positive subexpressions of the given depth; with complex_,
    every other intermediate function gets an imaginary part c*I, every term a
    complex form (the imaginary unit, logarithms and powers on or off the
    negative real axis) and the integrand a last term c*I."""
    rng = SplitMix64(seed)
    lines: List[str] = [f"{n};", f"{nfuncs};"]
    for i in range(nfuncs):
        e = _pos(rng, n, i, depth)
        lines.append((f"{e}+{_num(rng)}*I" if complex_ and i % 2 == 0 else e) + ";")
    parts = []
    for t in range(terms):
        e = _pos(rng, n, nfuncs, depth)
        if complex_:
            e = _complex_term(rng, e)
        parts.append(("-" if t and rng.uniform() < 0.3 else "+" if t else "") + e)
    if complex_:
        parts.append(f"+{_num(rng)}*I")       # the text names I even where no term does
    lines.append("".join(parts) + ";")
    lines.append("|")
    return "\n".join(lines) + "\n"
