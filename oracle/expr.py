"""Oracle: integrands given as text, evaluated point by point in fp64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The integration workers read an integrand as text (section 4.6, CIntegrate
options): a line with the number of variables, a line with the number of
intermediate functions, one line per intermediate function, then the
integrand, every line ended by ';', and a last line '|'.  Expressions are
built from + - * /, round brackets, decimal numbers, the variables x[1] ..
x[n], earlier intermediate functions f[1], f[2], ..., powers p[base,exponent],
natural logarithms l[arg], the constants P (pi) and G (Euler's gamma), and the
PolyGamma values the paper lists as built in: PolyGamma[1,1], PolyGamma[2,1..4]
and PolyGamma[3,1..2].  The paper's example is ``1; 0; x[1]+0.2; |``, the
integral of x + 0.2 over [0, 1].

Readings (the paper gives the grammar only by example):
* usual precedence: unary sign binds tighter than * and /, which bind tighter
  than + and -; binary operators associate to the left;
* p[a, b] is a real power: NaN for a < 0 unless b is a whole number, and l[a]
  is NaN for a < 0 (a real worker has no other value to give);
* an optional first line ``Integrate`` (the worker command) is skipped;
* complex integrands (the complex workers of section 4.2): the text names the
  imaginary unit as ``I`` (as the Mathematica side writes it).  Such an
  integrand is complex throughout: l[a] is the principal logarithm with
  arg = -pi on the negative real axis (the side an F - i0 prescription
  approaches), p[a, b] is a^k by repeated products for a whole number
  |b| <= 64 and exp(b l[a]) otherwise.  Without ``I`` nothing changes.

``evaluate`` returns the values at the given points and, per point, a
rounding bound ``cond``: the sum over every operation of the magnitude its
rounding can contribute to the result (first-order running error analysis,
Higham, Accuracy and Stability of Numerical Algorithms, section 3.3), in
units of the unit roundoff.  Two evaluations that round each operation once
differ by at most about 2 u cond.
"""
from __future__ import annotations

import math
import re

import mpmath as mp
import numpy as np

__all__ = ["ParseError", "Expression", "parse", "evaluate"]


class ParseError(ValueError):
    """Malformed text; ``unsupported`` is set for valid input the workers cannot evaluate."""

    def __init__(self, msg, unsupported=False):
        super().__init__(msg)
        self.unsupported = unsupported


_TOKEN = re.compile(r"\s*(?:(\d+\.?\d*(?:[eE][+-]?\d+)?|\.\d+(?:[eE][+-]?\d+)?)|(PolyGamma|EulerGamma|Pi|[A-Za-z]+)|(.))")

_POLYGAMMA_BUILTIN = {(1, 1), (2, 1), (2, 2), (2, 3), (2, 4), (3, 1), (3, 2)}


def _tokens(s):
    out = []
    pos = 0
    while pos < len(s):
        m = _TOKEN.match(s, pos)
        if m is None or m.end() == pos:
            if s[pos:].strip() == "":
                break
            raise ParseError(f"cannot read {s[pos:pos + 10]!r}")
        pos = m.end()
        num, name, ch = m.groups()
        if num is not None:
            out.append(("num", float(num)))
        elif name is not None:
            out.append(("name", name))
        elif ch is not None and not ch.isspace():
            out.append(("op", ch))
    return out


class _Parser:
    """Recursive descent over one expression; produces a nested tuple tree."""

    def __init__(self, text, nvars, nfuncs):
        self.t = _tokens(text)
        self.i = 0
        self.n = nvars
        self.nf = nfuncs
        self.complex = False

    def peek(self):
        return self.t[self.i] if self.i < len(self.t) else (None, None)

    def take(self, kind=None, val=None):
        k, v = self.peek()
        if k is None or (kind and k != kind) or (val is not None and v != val):
            raise ParseError(f"expected {val or kind}, found {v!r}")
        self.i += 1
        return v

    def accept(self, val):
        if self.peek() == ("op", val):
            self.i += 1
            return True
        return False

    def parse(self):
        e = self.sum()
        if self.i != len(self.t):
            raise ParseError(f"unexpected {self.peek()[1]!r}")
        return e

    def sum(self):
        e = self.product()
        while True:
            if self.accept("+"):
                e = ("+", e, self.product())
            elif self.accept("-"):
                e = ("-", e, self.product())
            else:
                return e

    def product(self):
        e = self.signed()
        while True:
            if self.accept("*"):
                e = ("*", e, self.signed())
            elif self.accept("/"):
                e = ("/", e, self.signed())
            else:
                return e

    def signed(self):
        if self.accept("-"):
            return ("neg", self.signed())
        if self.accept("+"):
            return self.signed()
        return self.atom()

    def index(self):
        self.take("op", "[")
        sign = -1 if self.accept("-") else 1
        v = self.take("num")
        if v != int(v):
            raise ParseError("index must be an integer")
        self.take("op", "]")
        return sign * int(v)

    def atom(self):
        k, v = self.peek()
        if k == "num":
            self.i += 1
            return ("const", v)
        if self.accept("("):
            e = self.sum()
            self.take("op", ")")
            return e
        if k != "name":
            raise ParseError(f"unexpected {v!r}")
        self.i += 1
        if v == "x":
            j = self.index()
            if not 1 <= j <= self.n:
                raise ParseError(f"x[{j}] outside x[1]..x[{self.n}]")
            return ("x", j - 1)
        if v == "f":
            j = self.index()
            if not 1 <= j <= self.nf:
                raise ParseError(f"f[{j}] is not an earlier intermediate function")
            return ("f", j - 1)
        if v in ("p", "l"):
            self.take("op", "[")
            a = self.sum()
            if v == "p":
                self.take("op", ",")
                b = self.sum()
                self.take("op", "]")
                return ("pow", a, b)
            self.take("op", "]")
            return ("log", a)
        if v == "I":
            self.complex = True
            return ("const", 1j)
        if v in ("P", "Pi"):
            return ("const", math.pi)
        if v in ("G", "EulerGamma"):
            return ("const", 0.5772156649015329)
        if v == "PolyGamma":
            self.take("op", "[")
            m = self.take("num")
            self.take("op", ",")
            z = self.take("num")
            self.take("op", "]")
            if (m, z) not in _POLYGAMMA_BUILTIN:
                raise ParseError(f"PolyGamma[{m:g},{z:g}] is not built in", unsupported=True)
            return ("const", float(mp.polygamma(int(m), int(z))))
        raise ParseError(f"unknown symbol {v!r}")


class Expression:
    """A parsed integrand: ``n`` variables, intermediate functions, the integrand tree."""

    def __init__(self, n, funcs, body, complex_=False):
        self.n = n
        self.funcs = funcs
        self.body = body
        self.complex = complex_


def parse(text: str) -> Expression:
    s = text.strip()
    if s.startswith("Integrate"):
        s = s[len("Integrate"):]
    if "|" not in s:
        raise ParseError("missing the final '|' line")
    head, tail = s.split("|", 1)
    if tail.strip():
        raise ParseError("text after the final '|'")
    parts = head.split(";")
    if parts[-1].strip():
        raise ParseError("line without ';'")
    lines = [p for p in parts[:-1]]

    def count(line, lo, hi, what):
        tree = _Parser(line, 0, 0).parse()
        if tree[0] != "const" or tree[1] != int(tree[1]) or not lo <= tree[1] <= hi:
            raise ParseError(f"{what} must be an integer in {lo}..{hi}")
        return int(tree[1])

    if len(lines) < 3:
        raise ParseError("need the variable count, the function count and the integrand")
    n = count(lines[0], 1, 16, "the number of variables")
    m = count(lines[1], 0, 1 << 20, "the number of intermediate functions")
    if len(lines) != 3 + m:
        raise ParseError(f"expected {m} intermediate functions and one integrand, found {len(lines) - 2} lines")
    parsers = [_Parser(lines[2 + i], n, i) for i in range(m)] + [_Parser(lines[2 + m], n, m)]
    trees = [q.parse() for q in parsers]
    return Expression(n, trees[:-1], trees[-1], any(q.complex for q in parsers))


def _log_mi0(a):
    """Principal complex logarithm, arg = -pi where a is real and negative."""
    ang = np.where((a.imag == 0.0) & (a.real < 0.0), -np.pi, np.angle(a))
    return np.log(np.abs(a)) + 1j * ang


def _apply_c(node, args, x, fvals):
    """(value, cond) of one node of a complex integrand (first-order bounds in
    units of u: the operands' bounds carried through, plus each operation's own
    rounding - a complex product about 3 |a||b|, a quotient 5 |v|, a logarithm
    |v| + 4, exp(b l[a]) |v| (3 + 3 |b l[a]|) and products |v| (3 |b| + 1))."""
    op = node[0]
    if op == "const":
        v = np.full(x.shape[0], complex(node[1]))
        return v, np.zeros(x.shape[0])
    if op == "x":
        v = x[:, node[1]].astype(np.complex128)
        return v, np.zeros(x.shape[0])
    if op == "f":
        return fvals[node[1]]
    if op == "neg":
        a, ca = args[0]
        return -a, ca
    if op == "log":
        a, ca = args[0]
        v = _log_mi0(a)
        return v, ca / np.abs(a) + np.abs(v) + 4.0
    (a, ca), (b, cb) = args
    if op == "+":
        v = a + b
        return v, ca + cb + np.abs(v)
    if op == "-":
        v = a - b
        return v, ca + cb + np.abs(v)
    if op == "*":
        v = a * b
        return v, ca * np.abs(b) + np.abs(a) * cb + 3.0 * np.abs(a) * np.abs(b)
    if op == "/":
        v = a / b
        return v, ca / np.abs(b) + np.abs(a) * cb / np.abs(b) ** 2 + 5.0 * np.abs(v)
    if op == "pow":
        la = _log_mi0(a)
        whole = bool(np.all(b.imag == 0.0) and np.all(b.real == np.round(b.real)) and np.all(np.abs(b) <= 64))
        if whole:
            k = int(b.real[0]) if b.size else 0
            if not np.all(b.real == k):
                whole = False
        if whole:
            v = np.ones_like(a)
            for _ in range(abs(k)):
                v = v * a
            if k < 0:
                v = 1.0 / v
        else:
            v = np.exp(b * la)
        own = np.abs(v) * (3.0 * np.abs(b) + 1.0 + 3.0 + 3.0 * np.abs(b * la))
        return v, np.abs(v) * (np.abs(b) * ca / np.abs(a) + np.abs(la) * cb) + own
    raise AssertionError(op)


def _apply(node, args, x, fvals):
    """(value, cond) of one node from its operands' (value, cond)."""
    op = node[0]
    if op == "const":
        v = np.full(x.shape[0], node[1])
        return v, np.zeros_like(v)
    if op == "x":
        v = x[:, node[1]].astype(np.float64)
        return v, np.zeros_like(v)
    if op == "f":
        return fvals[node[1]]
    if op == "neg":
        a, ca = args[0]
        return -a, ca
    if op == "log":
        a, ca = args[0]
        v = np.log(a)
        return v, ca / np.abs(a) + np.abs(v)
    (a, ca), (b, cb) = args
    if op == "+":
        v = a + b
        return v, ca + cb + np.abs(v)
    if op == "-":
        v = a - b
        return v, ca + cb + np.abs(v)
    if op == "*":
        v = a * b
        return v, ca * np.abs(b) + np.abs(a) * cb + np.abs(v)
    if op == "/":
        v = a / b
        return v, ca / np.abs(b) + np.abs(a) * cb / (b * b) + np.abs(v)
    if op == "pow":
        v = np.power(a, b)
        la = np.log(np.abs(a))
        # a whole-number exponent is evaluated by products: about one rounding per factor
        whole = bool(np.all(b == np.round(b)) and np.all(np.abs(b) <= 64))
        own = np.abs(v) * (np.abs(b) + 1.0) if whole else np.abs(v) * (1.0 + np.abs(b * la))
        return v, np.abs(v) * (np.abs(b) * ca / np.abs(a) + np.abs(la) * cb) + own
    raise AssertionError(op)


def _eval(tree, x, fvals, apply=None):
    """(value, cond) arrays of a tree at the points x (npts, n), without recursion
    (left-nested sums of long integrands are deeper than Python's stack)."""
    apply = apply or _apply
    out = []
    stack = [(tree, False)]
    while stack:
        node, done = stack.pop()
        nargs = {"const": 0, "x": 0, "f": 0, "neg": 1, "log": 1}.get(node[0], 2)
        if done or nargs == 0:
            args = out[len(out) - nargs:] if nargs else []
            if nargs:
                del out[len(out) - nargs:]
            out.append(apply(node, args, x, fvals))
            continue
        stack.append((node, True))
        for child in reversed(node[1:1 + nargs]):
            stack.append((child, False))
    return out[0]


def evaluate(expr: Expression, x: np.ndarray):
    """Integrand values (complex for a complex integrand) and rounding bounds
    (units of u) at points x (npts, n)."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    if x.ndim != 2 or x.shape[1] != expr.n:
        raise ValueError("x must be (npts, n)")
    apply = _apply_c if expr.complex else _apply
    with np.errstate(all="ignore"):
        fvals = []
        for f in expr.funcs:
            fvals.append(_eval(f, x, fvals, apply))
        v, c = _eval(expr.body, x, fvals, apply)
    return v, c
