"""FP64 reference for the geometric multigrid (GMG) baseline -- TEST INFRASTRUCTURE ONLY.

The classical solver the paper measures MGCNN against (Sec. 2.3: the two-grid method of
Alg. 1 applied recursively as a V-cycle, with the settings listed at the end of Sec. 2.3 and
the "GMG settings" paragraph of Sec. 4.1):

* coarse grid: half the points per side, n_{l+1} = (n_l - 1) / 2; coarse node (I, J) sits on
  fine node (2I + 1, 2J + 1);
* coarse operator: the same PDE discretised again on the coarse grid (the operator of
  ``operator.apply_A`` with h_{l+1} = 2 h_l), its coefficient a sampled at the coarse nodes
  (injection: the paper does not say how a is carried to the coarse grid);
* transfers: P = bilinear interpolation, R = P^T / 4 (full weighting);
* smoother: weighted Jacobi, e <- e + omega (r - A e) / D, `sweeps` times before and `sweeps`
  times after the coarse-grid correction; omega = 0.67 and three sweeps (Sec. 4.1);
* coarsest level: solved exactly (the "coarse grid solver" of Alg. 1, step 4; with the
  smoother alone on a 15 x 15 coarsest grid the cycle contracts Poisson errors only by about
  0.9, against the 17 iterations to 1e-8 that Sec. 4.1 reports at 31 x 31);
* levels: log2(n + 1) - 3, at least 1 (Sec. 4.1 uses fewer levels for GMG than for MGCNN:
  two at 31 x 31, three at 63 x 63), so the coarsest grid is 15 x 15 (or the whole grid
  below 31 x 31); at most log2(n + 1) (coarsest 1 x 1).

The cycle V maps a residual r to a correction e ~ A^{-1} r with zero initial guess on every
level; the stationary solve is u <- u + V(f - A u) with the stopping rule of ``solve``.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse.linalg as spla

from . import operator as op
from . import solve as sv

OMEGA = 0.67
SWEEPS = 3

# bilinear interpolation weights of a coarse value onto the 3 x 3 fine nodes around it
_W = np.outer([0.5, 1.0, 0.5], [0.5, 1.0, 0.5])


def default_levels(n: int) -> int:
    """Levels of the paper's GMG runs: log2(n + 1) - 3, at least one."""
    k = int(round(math.log2(n + 1)))
    return max(1, k - 3)


def inject(a: np.ndarray) -> np.ndarray:
    """Coefficient on the coarse grid: its values at the fine nodes the coarse nodes sit on."""
    return np.asarray(a, dtype=np.float64)[1::2, 1::2].copy()


def prolong(ec: np.ndarray) -> np.ndarray:
    """Bilinear interpolation P: coarse (nc x nc) -> fine (2 nc + 1 x 2 nc + 1), zero values
    outside the coarse grid (the Dirichlet boundary)."""
    nc = ec.shape[0]
    n = 2 * nc + 1
    e = np.zeros((n, n))
    for p in range(3):
        for q in range(3):
            e[p:p + 2 * nc:2, q:q + 2 * nc:2] += _W[p, q] * ec
    return e


def restrict(r: np.ndarray) -> np.ndarray:
    """Full weighting R = P^T / 4: fine (n x n) -> coarse ((n - 1)/2 x (n - 1)/2)."""
    n = r.shape[0]
    nc = (n - 1) // 2
    rc = np.zeros((nc, nc))
    for p in range(3):
        for q in range(3):
            rc += 0.25 * _W[p, q] * r[p:p + 2 * nc:2, q:q + 2 * nc:2]
    return rc


def jacobi(a, b, D, e, r, omega: float, sweeps: int, form: str = "div") -> np.ndarray:
    """`sweeps` weighted-Jacobi steps on A e = r from e."""
    for _ in range(sweeps):
        e = e + omega * (r - op.apply_A(a, b, e, form)) / D
    return e


class GMG:
    """Hierarchy of rediscretised operators for one problem (a, b) and its V-cycle."""

    def __init__(self, a, b, levels: int | None = None, omega: float = OMEGA, sweeps: int = SWEEPS,
                 form: str = "div"):
        a = np.asarray(a, dtype=np.float64)
        self.b = np.asarray(b, dtype=np.float64)
        self.n = a.shape[0]
        full = int(round(math.log2(self.n + 1)))
        self.levels = default_levels(self.n) if levels is None or levels == 0 else int(levels)
        if not 1 <= self.levels <= full:
            raise ValueError("levels must lie in [1, log2(n + 1)]")
        self.omega = float(omega)
        self.sweeps = int(sweeps)
        self.a = [a]
        for _ in range(self.levels - 1):
            self.a.append(inject(self.a[-1]))
        self.form = form
        self.D = [op.diagonal(al, self.b, form) for al in self.a]

    def A(self, l: int, e):
        return op.apply_A(self.a[l], self.b, e, self.form)

    def _cycle(self, l: int, r):
        a, D = self.a[l], self.D[l]
        if l + 1 == self.levels:
            A = op.assemble_A(a, self.b, self.form).tocsc()
            return spla.spsolve(A, r.ravel()).reshape(r.shape)
        e = jacobi(a, self.b, D, np.zeros_like(r), r, self.omega, self.sweeps, self.form)
        rc = restrict(r - self.A(l, e))
        e = e + prolong(self._cycle(l + 1, rc))
        return jacobi(a, self.b, D, e, r, self.omega, self.sweeps, self.form)

    def cycle(self, r) -> np.ndarray:
        """One V-cycle: a correction e ~ A^{-1} r from a zero initial guess."""
        return self._cycle(0, np.asarray(r, dtype=np.float64))

    # the stationary iteration u <- u + V(f - A u), stopped as in ``solve``
    def residual(self, f, u):
        return np.asarray(f, dtype=np.float64) - self.A(0, u)

    def correction(self, r):
        return self.cycle(r)

    def solve(self, f, tol: float, maxit: int, u0=None):
        """Returns (u, status, iters, relres, history) with the semantics of solve.Solver."""
        return sv.stationary(self, f, tol, maxit, u0)
