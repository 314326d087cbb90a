"""Host logic of the text-integrand compiler (sdi_text_info: no context, no
device): acceptance and rejection agree with the text oracle, errors carry the
parser's message, constants fold, repeated operations merge, and an integrand
of the paper's size class fits the slot budget."""
import numpy as np
import pytest

import paper_1511_03614_amd as P
from oracle import expr as E
from sectorgen import textgen

MALFORMED = [
    "1;0;x[1]+0.2;", "1;0;x[1]+0.2;|extra", "1;0;x[2];|", "1;0;x[0];|", "1;1;f[1];x[1];|",
    "1;0;q[1];|", "1;0;(x[1];|", "1;0;x[1]+;|", "1;0;p[x[1]];|", "0;0;1;|", "17;0;1;|", "1.5;0;1;|", "1;2;x[1];|",
]


def test_paper_example_compiles():
    info = P.sdi_text_info(textgen.PAPER_EXAMPLE)
    assert info == {"nvars": 1, "ninstructions": 8, "nslots": 2}   # one add (x[1] + 0.2), padded to a fetch


@pytest.mark.parametrize("text", MALFORMED)
def test_malformed_text_is_rejected_like_the_oracle(text):
    with pytest.raises(E.ParseError):
        E.parse(text)
    with pytest.raises(P.SdiError) as ei:
        P.sdi_text_info(text)
    assert ei.value.code == -1 and len(str(ei.value)) > 20


def test_syntax_errors_name_the_offset():
    with pytest.raises(P.SdiError) as ei:
        P.sdi_text_info("1;0;(x[1]*2;|")
    assert "offset" in str(ei.value)


def test_unsupported_polygamma():
    with pytest.raises(P.SdiError) as ei:
        P.sdi_text_info("1;0;PolyGamma[4,1]*x[1];|")
    assert ei.value.code == -4


def test_constants_fold_and_operations_merge():
    assert P.sdi_text_info("1;0;2*3+p[2,3]-l[P];|")["ninstructions"] == 8          # a single constant
    # (x+1)*(x+1): the sum is computed once, then one product; (x+1)*(x+2): three operations
    assert P.sdi_text_info("1;0;(x[1]+1)*(x[1]+1);|")["ninstructions"] == 8
    assert P.sdi_text_info("1;0;(x[1]+1)*(x[1]+2)+x[1]*x[1]*x[1]*x[1]*x[1]*x[1]*x[1];|")["ninstructions"] == 16
    assert P.sdi_text_info("1;0;x[1];|")["ninstructions"] == 0                         # the variable itself


@pytest.mark.parametrize("seed", range(8))
def test_random_integrands_agree_with_the_oracle_on_shape(seed):
    n = 1 + 3 * seed % 16
    text = textgen.random_text(300 + seed, n, nfuncs=seed % 4, depth=3, terms=1 + seed % 3)
    assert P.sdi_text_info(text)["nvars"] == E.parse(text).n == n


def test_paper_sized_integrand_fits_the_slot_budget():
    text = textgen.random_text(999, 6, nfuncs=8, depth=3, terms=3000)
    assert len(text) > 150_000
    info = P.sdi_text_info(text)
    assert info["nvars"] == 6 and info["nslots"] <= 96 and info["ninstructions"] % 8 == 0
    assert 20_000 < info["ninstructions"] < 40_000


def test_complex_integrands_compile_within_the_complex_slot_budget():
    """A text that names I compiles to a complex tape: at most 48 complex slots
    (the LDS of 96 real ones); I is one operation, shared; logarithms and
    powers of negative constants fold into re + im I."""
    info = P.sdi_text_info("1;0;x[1]+I;|")
    assert info["nvars"] == 1 and info["ninstructions"] == 8 and info["nslots"] == 2   # i, then x + i in its slot
    assert P.sdi_text_info("1;0;I*x[1]+I*I;|")["ninstructions"] == 8                  # i once: 4 operations
    assert P.sdi_text_info("1;0;l[-1]*x[1]+I;|")["ninstructions"] == 8
    text = textgen.random_text(777, 5, nfuncs=4, depth=2, terms=1000, complex_=True)
    info = P.sdi_text_info(text)
    assert info["nslots"] <= 48 and E.parse(text).complex
    # a right-nested product of 60 distinct complex factors keeps all of them live
    body = "x[1]"
    for k in range(60, 0, -1):
        body = f"(x[1]+{k}*I)*({body})"
    with pytest.raises(P.SdiError) as ei:
        P.sdi_text_info(f"1;0;{body};|")
    assert ei.value.code == -4 and "48 live complex temporaries" in str(ei.value)
    assert P.sdi_text_info(f"1;0;{body.replace('*I', '')};|")["nslots"] > 48     # real: 96 slots suffice
    # the same text without I compiles as a real tape
    assert P.sdi_text_info("1;0;x[1]+2;|")["nslots"] == 2
