"""Plain, slow FP64 CPU oracle for the MGCNN solver -- TEST INFRASTRUCTURE ONLY.

Only the test-suite, the smoke check and the CPU-baseline leg of the benchmark
may import this package.  The GPU library never calls it, links it or reads
anything it produces; the two implementations share no code.  Its inputs come
from the neutral seeded generators in ``datagen`` (float32 values promoted to
float64 here).

Modules:
  operator  -- the discrete operator A(a, b), its transpose, diagonal, sparse
               assembly and the setup features (Sec. 2.5; Sec. 3.2 remark).
  network   -- convolutions, setup phase (Alg. 2) and solve phase (Alg. 3).
  solve     -- stationary iteration with relative-residual stop (Eq. (1),
               Sec. 4.1) and the residual loss (Eq. (19)).
  adjoint   -- reverse mode of the unrolled iteration and of the setup network.
  gmg       -- the geometric multigrid baseline (Sec. 2.3, Alg. 1 as a V-cycle; Sec. 4.1
               GMG settings).

Parity pinning: every function here is checked by the "not gpu" tests against
closed forms, library routines (scipy.signal, scipy.sparse, numpy.linalg),
textbook special cases (weighted Jacobi, full weighting / bilinear transfer),
invariants (linearity, adjoint identities) or central finite differences.
The learned setup network with general weights has no closed form; it is pinned
only through special cases (zero, diagonal and bias-only layers).
"""
from . import operator, network, solve, adjoint, gmg  # noqa: F401
