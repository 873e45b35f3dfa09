"""FP64 CPU oracle for the full-space Gauss-Newton KKT step (arXiv 2204.06489).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only the tests, the smoke check and the benchmark's
CPU-baseline leg use it.  It shares no code with the HIP implementation; the
only common module is ``synthetic`` (seeded inputs, no method arithmetic).

It is a plain, slow, obviously correct restatement of the paper's mathematics
in numpy/scipy complex128:

* ``pml``        grid coordinates and PML stretch factors X(x), Z(z)  (Section 2)
* ``helmholtz``  the assembled 5-point Helmholtz matrix A with PML and a banded
                 LU of it (Section 2, the discrete forward problem A u = f)
* ``kkt``        sources, observation Q, weights W, the KKT matrix M, right-hand
                 side b, the block-triangular preconditioner, exact KKT solutions
                 (dense and Schur/normal-equation routes), right-preconditioned
                 GMRES, the reduced gradient and the Newton update
                 (Sections 3-5)

Every function cites the passage of the paper it follows.  Pins (tests that
tie each function to something other than itself) live in
``tests/test_oracle_*.py``.  Readings taken where the paper is silent:

* time convention e^{-i w t}: outgoing field behaves like e^{+ikr} and the PML
  factor is X = 1 + i sigma(x)/w;
* quadratic PML profile with reflection coefficient R0 and reference speed
  c_ref, on all four sides, inside the listed grid;
* the control s (squared slowness) lives on the core (non-PML) nodes only, so
  P = w^2 diag(u) E with E the extension from core to full grid;
* ``*`` is the conjugate transpose; the complex-linear KKT system is solved as
  printed and the real model takes Re(ds);
* the source is a unit discrete delta f_k = e_src / h^2.
"""

from . import pml, helmholtz, kkt  # noqa: F401
