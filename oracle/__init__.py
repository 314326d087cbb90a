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

* ``integrand_mp`` - the real sector integrand in multiprecision (the
  reference of the endpoint-precision mode).
* ``deform``     - the automatic deformation size (ComplexMode tuning).
* ``flow``       - the learned importance-sampling map (sampling, log q,
  gradient, Adam, training loss weights).
* ``expr``       - integrands in the workers' text format (section 4.6).
* ``poles``      - sectors with a_j < -1 reduced to a_j >= -1 by integration
  by parts (analytic continuation in eps), with coefficient series.
* ``cubature``   - globally adaptive deterministic cubature (the Cuhre
  option of CurrentIntegrator, section 4.4): the Genz-Malik degree-7/5 rule
  pair on dyadic regions, split along the largest fourth difference.
* ``suave``      - subregion-adaptive Monte Carlo (the Suave option):
  sampled dyadic regions halved where the samples spread most.
* ``divonne``    - partition by spreads, then a lattice rule per region (the
  Divonne option): stratified sampling with one refinement.
* ``separate``   - SeparateTerms (section 4.4): a sector as the sum of the
  integrable terms of its subtraction, each a sector of its own.

Where the paper is silent, each function's docstring states the reading it
takes and names the passage it follows.

Pins (each function checked against something other than itself; tests in
``tests/test_oracle_*.py``):

* integrand: hypergeometric closed forms in one variable, separable products,
  a direct integral at finite eps, the bubble's Gamma-function expansion, the
  paper's box example (section 4.3), the massive bubble above threshold and
  lambda invariance (Cauchy) in complex mode, the deformation Jacobian by
  finite differences;
* prefactor: mpmath Taylor series of the Gamma functions;
* points: Philox known-answer vectors, exact lattice projections and shift
  means, the exactness of the tent map; the CBC vector as the componentwise
  minimum of the P_2 figure computed on the dual lattice;
* vegas: the refit's fixed point against an independent shooting solver, a
  single occupied bin, the compression exponent, the histogram against exact
  bin integrals;
* integrate: shift-to-shift errors calibrated against Student's t over many
  seeds; the allocation's proportionality and clamps;
* integrand_mp: closed forms that stay exact at the faces;
* deform: Im F flags against plain complex arithmetic, the chosen lambda
  against a direct scan of the candidates, small lambda never failing;
* flow: finite-difference gradients, invertibility, unit mean weight,
  torch's Adam, convergence to the chi^2-optimal density;
* expr: hand-evaluated expressions and closed-form integrals;
* poles: hypergeometric closed forms for a = -2, -3, -1.5, a separable
  two-variable product, an elementary polynomial case and the expansion's
  structure;
* cubature: the rule pair's degrees (every monomial of degree <= 7 exact,
  degree 5 exactly for the embedded rule), polynomials on dyadic boxes of a
  sector, the split axis of one-axis integrands, the dyadic tiling, one split
  per round taking the largest priority, and whole runs against the bubble's
  and the section 4.3 box's closed forms.
"""
from . import integrand, points, prefactor, vegas, integrate  # noqa: F401
