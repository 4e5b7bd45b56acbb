"""FP64 reference for the solver loop (test infrastructure).

The solve is the stationary iteration of Sec. 2.2, Eq. (1),
    u_{k+1} = u_k + B (f - A u_k),
with B the solve network applied to the diagonally scaled residual
r / D (D = diag A), stopped on the relative residual ||f - A u_k||_2 / ||f||_2
(Sec. 4.1, "Iterative method settings").  The training loss is the residual
loss of Sec. 3.4, Eq. (19), here normalised per problem by ||f||^2 and taken
after K unrolled iterations.

Status codes (same meaning as the C library's):
    OK = 0, NOT_CONVERGED = 1, DIVERGED = -6.
"""
from __future__ import annotations

import math

import numpy as np

from . import network as net
from . import operator as op

OK, NOT_CONVERGED, DIVERGED = 0, 1, -6
DIVERGENCE_LIMIT = 1e10


class Solver:
    """Setup once for one problem (a, b), then iterate (Sec. 3.1, network phases)."""

    def __init__(self, weights: np.ndarray, a: np.ndarray, b, levels: int | None = None,
                 form: str = "div", up_post: bool = False):
        self.C = net.channels_of(np.asarray(weights).size)
        self.P = net.unpack_weights(weights, self.C)
        self.a = np.asarray(a, dtype=np.float64)
        self.b = np.asarray(b, dtype=np.float64)
        self.n = self.a.shape[0]
        self.L = levels if levels is not None else net.num_levels(self.n)
        self.form = form
        self.up_post = up_post            # up smoother in adjoint form (symmetric variant)
        self.D = op.diagonal(self.a, self.b, form)
        self.F = op.features(self.a, self.b, form)
        self.s = net.setup(self.P, self.F, self.L)

    def residual(self, f, u):
        return np.asarray(f, dtype=np.float64) - op.apply_A(self.a, self.b, u, self.form)

    def correction(self, r):
        return net.vcycle(self.P, self.s, r / self.D, up_post=self.up_post)

    def pcg_correction(self, r):
        """The network as a symmetric preconditioner: D^-1/2 B(D^-1/2 r).  With B symmetric (the
        symmetric variant of Sec. 3.3) this map is symmetric; for a constant diagonal it equals
        the correction B(r / D) of Eq. (1)."""
        h = 1.0 / np.sqrt(self.D)
        return h * net.vcycle(self.P, self.s, h * r, up_post=self.up_post)

    def step(self, f, u):
        """One iteration u + B((f - A u)/D)."""
        return u + self.correction(self.residual(f, u))

    def forward(self, f, K: int, u0=None):
        """K unrolled iterations from u0 (default 0); returns u_K."""
        u = np.zeros((self.n, self.n)) if u0 is None else np.asarray(u0, dtype=np.float64).copy()
        for _ in range(K):
            u = self.step(f, u)
        return u

    def solve(self, f, tol: float, maxit: int, u0=None):
        """Tolerance-driven solve; see ``stationary``."""
        return stationary(self, f, tol, maxit, u0)


def stationary(it, f, tol: float, maxit: int, u0=None):
    """Tolerance-driven stationary iteration u <- u + it.correction(f - A u) for any object
    with ``residual(f, u)`` and ``correction(r)``.  Returns (u, status, iters, relres, history).

    At iterate k: r_k = f - A u_k, rho_k = ||r_k|| / ||f||; stop with OK if rho_k <= tol
    (iters = k), with NOT_CONVERGED if k == maxit, with DIVERGED if rho_k is not finite or
    exceeds 1e10; otherwise apply one more correction.  A zero right-hand side returns u = 0,
    iters = 0, OK."""
    f = np.asarray(f, dtype=np.float64)
    nf = math.sqrt(float(np.sum(f * f)))
    if nf == 0.0:
        return np.zeros_like(f), OK, 0, 0.0, [0.0]
    u = np.zeros_like(f) if u0 is None else np.asarray(u0, dtype=np.float64).copy()
    hist = []
    k = 0
    while True:
        r = it.residual(f, u)
        rho = math.sqrt(float(np.sum(r * r))) / nf
        hist.append(rho)
        if rho <= tol:
            return u, OK, k, rho, hist
        if k == maxit:
            return u, NOT_CONVERGED, k, rho, hist
        if not math.isfinite(rho) or rho > DIVERGENCE_LIMIT:
            return u, DIVERGED, k, rho, hist
        u = u + it.correction(r)
        k += 1


def pcg(apply_A, precond, f, tol: float, maxit: int, u0=None):
    """Preconditioned conjugate gradients for a symmetric positive definite A with a symmetric
    positive definite preconditioner M (the network or a V-cycle as preconditioner of a Krylov
    method, Sec. 2.2; the short recurrence that a symmetric network allows, Sec. 3.3), in f64:

        r_0 = f - A u_0,  z_0 = M r_0,  p_0 = z_0,
        alpha_k = (r_k, z_k) / (p_k, A p_k),  u_{k+1} = u_k + alpha_k p_k,
        r_{k+1} = r_k - alpha_k A p_k,  z_{k+1} = M r_{k+1},
        beta_k = (r_{k+1}, z_{k+1}) / (r_k, z_k),  p_{k+1} = z_{k+1} + beta_k p_k.

    ``apply_A(x)`` and ``precond(r)`` are callables.  The stopping rule is that of
    ``stationary`` on the true residual f - A u_k (iters = k preconditioner applications
    before u_k); (p, A p) <= 0 or (r, z) <= 0 is a breakdown and returns DIVERGED.  Returns
    (u, status, iters, relres, history)."""
    f = np.asarray(f, dtype=np.float64)
    nf = math.sqrt(float(np.sum(f * f)))
    if nf == 0.0:
        return np.zeros_like(f), OK, 0, 0.0, [0.0]
    u = np.zeros_like(f) if u0 is None else np.asarray(u0, dtype=np.float64).copy()
    r = f - apply_A(u)
    hist = []
    k = 0
    p = rz = None
    while True:
        rho = math.sqrt(float(np.sum((f - apply_A(u)) ** 2))) / nf
        hist.append(rho)
        if rho <= tol:
            return u, OK, k, rho, hist
        if k == maxit:
            return u, NOT_CONVERGED, k, rho, hist
        if not math.isfinite(rho) or rho > DIVERGENCE_LIMIT:
            return u, DIVERGED, k, rho, hist
        z = precond(r)
        rz_new = float(np.sum(r * z))
        if not rz_new > 0.0:
            return u, DIVERGED, k, rho, hist
        p = z.copy() if p is None else z + (rz_new / rz) * p
        rz = rz_new
        q = apply_A(p)
        pq = float(np.sum(p * q))
        if not pq > 0.0:
            return u, DIVERGED, k, rho, hist
        alpha = rz / pq
        u = u + alpha * p
        r = r - alpha * q
        k += 1


def relres(a, b, f, u, form: str = "div") -> float:
    f = np.asarray(f, dtype=np.float64)
    r = f - op.apply_A(np.asarray(a, dtype=np.float64), b, u, form)
    return math.sqrt(float(np.sum(r * r))) / math.sqrt(float(np.sum(f * f)))


def loss(a_batch, b_batch, f_batch, u_batch, form: str = "div") -> float:
    """Mean over the batch of ||f_i - A_i u_i||^2 / ||f_i||^2."""
    N = len(f_batch)
    tot = 0.0
    for i in range(N):
        f = np.asarray(f_batch[i], dtype=np.float64)
        r = f - op.apply_A(np.asarray(a_batch[i], dtype=np.float64), b_batch[i], u_batch[i], form)
        tot += float(np.sum(r * r)) / float(np.sum(f * f))
    return tot / N
