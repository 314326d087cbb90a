"""CPU-only checks of the C ABI library: it loads, exports every declared symbol,
and its host-side helpers (prefactor series, CBC lattice vectors) agree with the
oracle's independent implementations.  No device work is issued."""
import os

import numpy as np
import pytest

import paper_1511_03614_amd as P
from oracle import points, prefactor

pytestmark = pytest.mark.skipif(not os.path.exists(P.library_path()), reason="libsdint.so not built")


def test_library_exports_every_declared_symbol():
    lib = P.load_library()
    names = P.declared_functions()
    assert len(names) >= 16
    missing = [n for n in names if not hasattr(lib, n)]
    assert missing == []


@pytest.mark.parametrize("loops,indices,d0", [
    (1, (1, 1), 4), (1, (1, 1, 1, 1), 4), (2, (1,) * 7, 4), (1, (1,), 4), (2, (1, 1, 1), 4),
    (3, (1, 1, 1, 1), 4), (2, (1, 1, 1, 1, 2), 4), (1, (2, 1), 6), (2, (3, 1, 1), 6),
])
def test_prefactor_matches_oracle(loops, indices, d0):
    lead, ser = P.sdi_prefactor_feynman(loops, indices, d0, 7)
    olead, oser = prefactor.feynman_prefactor(loops, indices, d0, 7)
    assert lead == olead
    assert np.allclose(ser, oser, rtol=1e-14, atol=1e-14)


def test_prefactor_rejects_bad_input():
    with pytest.raises(P.SdiError):
        P.sdi_prefactor_feynman(0, (1, 1), 4, 3)
    with pytest.raises(P.SdiError):
        P.sdi_prefactor_feynman(1, (0, 1), 4, 3)


@pytest.mark.parametrize("m", [4, 5, 6, 7, 8, 10, 12, 14, 16])
def test_lattice_vector_matches_oracle(m):
    z = P.sdi_lattice_vector(m, 16)
    assert tuple(int(v) for v in z) == points.cbc_vector(m, 16)


def test_lattice_vector_prefix_property():
    z16 = P.sdi_lattice_vector(12, 16)
    z5 = P.sdi_lattice_vector(12, 5)
    assert np.array_equal(z16[:5], z5)
    with pytest.raises(P.SdiError):
        P.sdi_lattice_vector(3, 4)


def test_context_creation_without_device_fails_cleanly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    lib = P.load_library()
    import ctypes
    h = ctypes.c_void_p()
    rc = lib.sdi_ctx_create(0, None, ctypes.byref(h))
    assert rc in (-3, -1)
