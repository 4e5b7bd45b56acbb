"""Pins of the oracle's preconditioned conjugate gradients and of the symmetry of its
preconditioners (the short-recurrence Krylov method that a symmetric network allows).

* CG optimality: the k-th PCG iterate minimises the energy norm of the error over
  u_0 + span{M r_0, (M A) M r_0, ..., (M A)^{k-1} M r_0}; checked against a brute-force
  projection for the identity, Jacobi and V-cycle preconditioners.  A wrong alpha, beta or
  update order gives a non-optimal iterate.
* An exact preconditioner M = A^-1 solves in one step; plain CG on 9 unknowns terminates in 9.
* The V-cycle (b = 0) and the symmetric variant of the network with the D^-1/2 scaling are
  symmetric positive definite; the network's plain scaling B(r / D) is not symmetric.
"""
import numpy as np
import pytest

import datagen
from oracle import gmg as ogmg
from oracle import network as net
from oracle import operator as op
from oracle import solve as osv


def _problem(n, seed, b=(0.0, 0.0)):
    rng = np.random.default_rng(seed)
    a = np.exp(rng.standard_normal((n, n)))
    f = rng.standard_normal((n, n))
    return a, np.asarray(b, dtype=np.float64), f


def _energy_optimal(A, M, r0, k):
    """argmin over x in span{M r0, (MA) M r0, ...} (k vectors) of ||A^-1 r0 - x||_A."""
    N = r0.size
    V = np.zeros((N, k))
    v = M @ r0
    for j in range(k):
        for i in range(j):                      # orthogonalise twice: the span is what counts
            v = v - (V[:, i] @ v) * V[:, i]
        for i in range(j):
            v = v - (V[:, i] @ v) * V[:, i]
        V[:, j] = v / np.linalg.norm(v)
        v = M @ (A @ V[:, j])
    y = np.linalg.solve(V.T @ A @ V, V.T @ r0)
    return V @ y


@pytest.mark.parametrize("precond", ["identity", "jacobi", "vcycle"])
def test_pcg_iterates_minimise_the_energy_error(precond):
    n = 7
    a, b, f = _problem(n, 3)
    A = op.assemble_A(a, b).toarray()
    N = n * n
    if precond == "identity":
        M = np.eye(N)
    elif precond == "jacobi":
        M = np.diag(1.0 / op.diagonal(a, b).ravel())
    else:
        G = ogmg.GMG(a, b, levels=2)
        M = np.stack([G.cycle(e.reshape(n, n)).ravel() for e in np.eye(N)], axis=1)
    ustar = np.linalg.solve(A, f.ravel())
    u0 = np.random.default_rng(9).standard_normal(N)
    r0 = f.ravel() - A @ u0
    for k in range(1, 7):
        u, st, it, _, _ = osv.pcg(lambda x: (A @ x.ravel()).reshape(n, n),
                                  lambda r: (M @ r.ravel()).reshape(n, n), f, 0.0, k,
                                  u0=u0.reshape(n, n))
        assert st == osv.NOT_CONVERGED and it == k
        e = u.ravel() - (u0 + _energy_optimal(A, M, r0, k))
        enorm = lambda x: np.sqrt(x @ A @ x)
        assert enorm(e) <= 1e-9 * enorm(ustar - u0), (precond, k)


def test_pcg_exact_preconditioner_and_finite_termination():
    n = 7
    a, b, f = _problem(n, 4)
    A = op.assemble_A(a, b).toarray()
    Ainv = np.linalg.inv(A)
    Aop = lambda x: (A @ x.ravel()).reshape(n, n)
    u, st, it, rr, _ = osv.pcg(Aop, lambda r: (Ainv @ r.ravel()).reshape(n, n), f, 1e-12, 5)
    assert st == osv.OK and it == 1 and rr <= 1e-12
    n = 3
    a, b, f = _problem(n, 5)
    A3 = op.assemble_A(a, b).toarray()
    u, st, it, rr, hist = osv.pcg(lambda x: (A3 @ x.ravel()).reshape(n, n), lambda r: r.copy(),
                                  f, 0.0, 9)
    assert hist[-1] <= 1e-12 and it == 9


def test_pcg_zero_rhs_and_breakdown():
    n = 7
    a, b, f = _problem(n, 6)
    Aop = lambda x: op.apply_A(a, b, x)
    u, st, it, rr, _ = osv.pcg(Aop, lambda r: r.copy(), np.zeros((n, n)), 1e-8, 10)
    assert st == osv.OK and it == 0 and not u.any()
    # an indefinite preconditioner (-I) gives (r, z) < 0: a breakdown, reported as DIVERGED
    u, st, it, rr, _ = osv.pcg(Aop, lambda r: -r, f, 1e-8, 10)
    assert st == osv.DIVERGED and it == 0


def test_vcycle_is_symmetric_positive_definite_for_b_zero():
    """Equal pre- and post-sweeps, full weighting = bilinear interpolation transposed / 4 and
    symmetric rediscretised coarse operators: the V-cycle is an SPD map when b = 0."""
    n = 15
    a, b, _ = _problem(n, 7)
    N = n * n
    G = ogmg.GMG(a, b)
    M = np.stack([G.cycle(e.reshape(n, n)).ravel() for e in np.eye(N)], axis=1)
    assert np.linalg.norm(M - M.T) <= 1e-12 * np.linalg.norm(M)
    assert np.linalg.eigvalsh(0.5 * (M + M.T)).min() > 0.0
    Gb = ogmg.GMG(a, np.array([1.0, 0.5]))
    Mb = np.stack([Gb.cycle(e.reshape(n, n)).ravel() for e in np.eye(N)], axis=1)
    assert np.linalg.norm(Mb - Mb.T) >= 1e-3 * np.linalg.norm(Mb)


def _tied_weights(C, seed):
    P = net.unpack_weights(datagen.xavier_weights(C, seed).astype(np.float64), C)
    adj = lambda W: np.flip(W, (2, 3)).transpose(1, 0, 2, 3).copy()
    P["W_up"] = adj(P["W_dn"])
    P["W_T"] = P["W_R"].copy()
    P["W_out"] = adj(P["W_in"])
    return net.pack_weights(P, C)


def test_symmetric_variant_is_spd_with_the_half_scaling():
    """Adjoint-tied weights and the up smoother x + s . (W_up * x): every level maps x to
    G^T (I + R^T M_coarse R) G x with G = I + W_dn * (s . .), so the network is positive
    semi-definite for any weights and setup tensors, and D^-1/2 B(D^-1/2 r) is SPD.  The
    scaling B(r / D) of the stationary iteration is not symmetric when D varies."""
    C, n = 4, 7
    a, b, _ = _problem(n, 8)
    w = _tied_weights(C, 11)
    S = osv.Solver(w, a, b, up_post=True)
    N = n * n
    Mh = np.stack([S.pcg_correction(e.reshape(n, n)).ravel() for e in np.eye(N)], axis=1)
    assert np.linalg.norm(Mh - Mh.T) <= 1e-12 * np.linalg.norm(Mh)
    ev = np.linalg.eigvalsh(0.5 * (Mh + Mh.T))
    assert ev.min() > -1e-12 * ev.max()
    Md = np.stack([S.correction(e.reshape(n, n)).ravel() for e in np.eye(N)], axis=1)
    assert np.linalg.norm(Md - Md.T) >= 1e-3 * np.linalg.norm(Md)


def test_pcg_with_the_vcycle_beats_the_stationary_cycle():
    n = 31
    a, b, f = _problem(n, 12)
    G = ogmg.GMG(a, b)
    u, st, it, rr, _ = osv.pcg(lambda x: op.apply_A(a, b, x), G.cycle, f, 1e-10, 100)
    _, st2, it2, _, _ = G.solve(f, 1e-10, 100)
    assert st == osv.OK and st2 == osv.OK and it < it2
    assert osv.relres(a, b, f, u) <= 1e-10
