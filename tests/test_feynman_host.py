"""The library's front end for Feynman integrals (sdi_problem_from_feynman /
sdi_feynman_sectors, SDEvaluate[{U, F, l}, indices, order] of section 4.3)
against the input tool's decomposition (sectorgen.feynman), on the host: the
number of sectors and the lowest result order of the bubble, the massive
bubble, the section 4.3 box and both double boxes; inputs with a_j < -1 are
refused by both."""
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


def test_second_order_poles_are_refused_by_both():
    try:
        P.load_library()
    except Exception as e:                       # noqa: BLE001
        pytest.skip(f"library not built: {e}")
    U, F = feynman.box_uf(3.0, 1.0)
    with pytest.raises(NotImplementedError):
        feynman.feynman_sectors(U, F, (1, 1, 1, 1), 1, d0=2)
    with pytest.raises(P.SdiError) as e:
        P.sdi_feynman_sectors(U, F, 1, (1, 1, 1, 1), d0=2)
    assert e.value.code == -4
