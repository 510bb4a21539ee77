"""CPU oracle for weighted-quadrature (WQ) formation of isogeometric Galerkin
matrices (Calabro, Sangalli, Tani, arXiv:1605.01238).

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously correct
reference written from the paper.  Only ``tests/``, the smoke check in
``__graft_entry__`` and the CPU-baseline leg of ``bench.py`` may import it.
The HIP library never imports, links or calls it, and it shares no code,
tables or helpers with the HIP path.

Precision: the univariate WQ weights and the exact 1D integrals are computed
in exact rational arithmetic (``fractions.Fraction``) and rounded once to
FP64; everything downstream (geometry, assembly) is plain FP64 numpy.

Modules
-------
splines   Cox-de Boor B-spline values/derivatives, index sets.
rules     Quadrature-point layout (Remark 4.1), exact integrals (eq. 4.2),
          WQ weights by minimum-norm solves (Algorithm 2).
geometry  Spline map F, Jacobian, det J and the stiffness coefficient
          c_lm = det(J) (J^{-1} J^{-T})_lm (Section 3) at given points.
assembly  Row formation: direct WQ sum (eq. massquadrature and its stiffness
          analogue), sum-factorized rows (Algorithm 3), CSR pattern, and
          element-wise standard Gauss quadrature (SGQ) for exactness tests.

Parity status: every function is pinned by tests under tests/ against values
printed in the paper, closed forms or invariants (see each module header).
"""
