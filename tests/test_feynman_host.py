"""The library's front end for Feynman integrals (sdi_problem_from_feynman /
sdi_feynman_sectors, SDEvaluate[{U, F, l}, indices, order] of section 4.3)
against the input tool's decomposition (sectorgen.feynman), on the host: the
number of sectors and the lowest result order of the bubble, the massive
bubble, the section 4.3 box and both double boxes; inputs with a_j < -1 are
refused by both."""
import numpy as np
import pytest

import paper_1511_03614_amd as P
from sectorgen import feynman


def cases():
    return {
        "bubble": (feynman.symanzik([[1], [1]], [[0], [1]], [[-1.0]], [0, 0]), 1, (1, 1), -1),
        "massive bubble": (feynman.symanzik([[1], [1]], [[0], [1]], [[5.0]], [1, 1]), 1, (1, 1), -1),
        "box": (feynman.box_uf(3.0, 1.0), 1, (1, 1, 1, 1), -2),
        "double box": (feynman.double_box_uf(-3.0, -1.0, 0.0), 2, (1,) * 7, -4),
        "double box, massive": (feynman.double_box_uf(5.0, -2.0, 1.0), 2, (1,) * 7, 0),   # finite: no poles
    }


@pytest.mark.parametrize("name", sorted(cases()))
def test_sector_counts_and_lowest_order(name):
    try:
        P.load_library()
    except Exception as e:                       # noqa: BLE001
        pytest.skip(f"library not built: {e}")
    (U, F), loops, idx, om = cases()[name]
    ns, got_om, nv = P.sdi_feynman_sectors(U, F, loops, idx)
    assert ns == len(feynman.feynman_sectors(U, F, idx, loops))
    assert got_om == om
    assert nv == len(idx) - 1


def test_sectors_with_a_below_minus_one_are_kept_by_both():
    """The box in d = 2 - 2 eps has sectors with a_j = -2: both decompositions
    keep them (the library reduces them when it compiles the problem) and
    count one more singular variable for the leading pole."""
    try:
        P.load_library()
    except Exception as e:                       # noqa: BLE001
        pytest.skip(f"library not built: {e}")
    U, F = feynman.box_uf(3.0, 1.0)
    secs = feynman.feynman_sectors(U, F, (1, 1, 1, 1), 1, d0=2)
    assert min(float(s.a.min()) for s in secs) == -2.0
    ns, om, nv = P.sdi_feynman_sectors(U, F, 1, (1, 1, 1, 1), d0=2)
    assert ns == len(secs) and nv == 3
    lead = P.sdi_prefactor_feynman(1, (1, 1, 1, 1), 2, 1)[0]
    most = max(int(sum((s.a <= -1.0) & (s.a == np.floor(s.a)))) for s in secs)
    assert om == lead - most


def test_complex_masses_decompose_like_real_ones():
    """F with complex coefficients (m^2 - i m Gamma) decomposes into the same sectors as with real ones."""
    U = {(1, 0): 1.0, (0, 1): 1.0}
    Fr = {(2, 0): 1.0, (1, 1): 2.0 - 5.0, (0, 2): 1.0}
    Fc = {(2, 0): 1.0 - 0.25j, (1, 1): 2.0 * (1.0 - 0.25j) - 5.0, (0, 2): 1.0 - 0.25j}
    assert P.sdi_feynman_sectors(U, Fc, 1, (1, 1)) == P.sdi_feynman_sectors(U, Fr, 1, (1, 1))
    with pytest.raises(P.SdiError):
        P.sdi_feynman_sectors({(1, 0): 1.0 + 1j, (0, 1): 1.0}, Fr, 1, (1, 1))
