"""Problems built by the library's front end (sdi_problem_from_feynman,
SDEvaluate[{U, F, l}, indices, order] of section 4.3) integrate to the same
values as the same integrals decomposed by the input tool (sectorgen.feynman)
and compiled sector by sector: the section 4.3 box, the Euclidean double box
the physical (massive, complex-mode) double box and the bubble with a
complex mass (complex F coefficients), bit for bit; and the box lands on its
textbook value."""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1511_03614_amd as P  # noqa: E402
from sectorgen import feynman  # noqa: E402

from test_gpu_parity import log, set_params  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    c = P.sdi_ctx_create(0)
    yield c
    P.sdi_ctx_destroy(c)


def complex_mass_bubble_case():
    """Equal-mass bubble at p^2 = 5 with m^2 = 1 - i/4 (complex F coefficients)."""
    import sectorgen
    m2, s = 1.0 - 0.25j, 5.0
    U = {(1, 0): 1.0, (0, 1): 1.0}
    F = {(2, 0): m2, (1, 1): 2.0 * m2 - s, (0, 2): m2}
    prob = sectorgen.Problem(sectors=feynman.feynman_sectors(U, F, (1, 1), 1), order_min=-1, order_max=0,
                             feynman=sectorgen.FeynmanPrefactor(1, (1, 1), 4), complex_mode=True, lam=0.3)
    return (U, F), 1, (1, 1), prob, True, 0.3


CASES = {
    "bubble, complex mass": complex_mass_bubble_case,
    "box": lambda: (feynman.box_uf(3.0, 1.0), 1, (1, 1, 1, 1), feynman.box_problem(3.0, 1.0), False, 0.0),
    "double box": lambda: (feynman.double_box_uf(-3.0, -1.0, 0.0), 2, (1,) * 7,
                           feynman.double_box_problem(-3.0, -1.0, 0.0), False, 0.0),
    "double box, physical": lambda: (feynman.double_box_uf(5.0, -2.0, 1.0), 2, (1,) * 7,
                                     feynman.double_box_problem(5.0, -2.0, 1.0, complex_mode=True, lam=0.5),
                                     True, 0.5),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_front_end_equals_input_tool(ctx, name):
    (U, F), loops, idx, prob, cplx, lam = CASES[name]()
    h_tool = P.sdi_problem_create(ctx, prob)
    h_lib = P.sdi_problem_from_feynman(ctx, U, F, loops, idx, 0, complex_mode=cplx, lam=lam)
    try:
        ns = P.sdi_problem_nsectors(h_tool)
        assert P.sdi_problem_nsectors(h_lib) == ns
        for s in range(ns):
            assert P.sdi_problem_nvars(h_lib, s) == P.sdi_problem_nvars(h_tool, s)
        set_params(ctx, lattice_log2=12, shifts=8, seed=3, tile_log2=10, ppt=1)
        a = P.sdi_integrate(ctx, h_tool)
        b = P.sdi_integrate(ctx, h_lib)
        K = len(b["value"])
        off = b["order_min"] - a["order_min"]
        assert off >= 0
        assert np.array_equal(a["value"][off:off + K], b["value"]), (a["value"], b["value"])
        assert np.array_equal(a["err_re"][off:off + K], b["err_re"])
        assert np.all(a["value"][:off] == 0)      # orders below the library's leading pole vanish
        log(f"{name}: {ns} sectors, orders from {b['order_min']}, values equal bit for bit")
        if name == "box":
            exact = [4 / 3, -2 * math.log(3) / 3, -4 * math.pi ** 2 / 9]
            assert np.all(np.abs(b["value"].real - exact) <= 5 * b["err_re"] + 1e-9)
    finally:
        P.sdi_problem_destroy(h_tool)
        P.sdi_problem_destroy(h_lib)
        set_params(ctx)


def test_front_end_errors(ctx):
    U, F = feynman.box_uf(3.0, 1.0)
    with pytest.raises(P.SdiError) as e:
        P.sdi_problem_from_feynman(ctx, U, F, 1, (1, 1, 1, 1), 0, d0=2,     # a_j < -1, reduced in real mode only
                                   complex_mode=True, lam=0.1)
    assert e.value.code == -4
    with pytest.raises(P.SdiError):
        P.sdi_problem_from_feynman(ctx, U, F, 1, (1, 1, 1, 1), 9)           # beyond 8 orders
    with pytest.raises(P.SdiError):
        P.sdi_problem_from_feynman(ctx, U, F, 1, (1, 1, 0, 1), 0)           # index 0
