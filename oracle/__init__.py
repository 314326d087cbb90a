"""Plain, slow, fp64 CPU oracle of the sector-integrand hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, links or runs
this package; only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` do.  It shares no code with the HIP
library: the two meet only in the seeded inputs of ``sectorgen``.

What it computes (paper: FIESTA 4, arXiv:1511.03614):

* ``integrand``  - the eps-expanded sector integrand of eq. (2) after sector
  decomposition: subtraction of the x_j^(-1+b eps) poles, expansion of
  x^(b eps) and P^(delta eps) into log powers, the optional contour
  deformation (section 4.4, ComplexMode) and the prefactor fold.
* ``prefactor``  - exp(l gamma_E eps) Gamma(A - l d/2)/prod Gamma(a_i) as a
  Laurent series (eq. (2), normalisation of section 4.3).
* ``points``     - rank-1 lattice points (CBC generating vector, Philox4x32-10
  random shifts), the tent (baker) transform and the Vegas map.
* ``vegas``      - Lepage's grid refit from per-bin histograms.
* ``integrate``  - per-sector, per-shift means, the shift-to-shift error and
  the root-sum-square combination of section 4.3.

Where the paper is silent, each function's docstring states the reading it
takes and names the passage it follows.
"""
from . import integrand, points, prefactor, vegas, integrate  # noqa: F401
