"""Pins of the oracle's geometric multigrid baseline (Sec. 2.3, Alg. 1 as a V-cycle; the GMG
settings of Sec. 4.1) against closed forms and invariants -- CPU only.

* bilinear interpolation is exact on bilinear functions, full weighting keeps constants and is
  P^T / 4 (adjoint identity);
* injection samples the coefficient at the coarse nodes' coordinates;
* the rediscretised coarse operator approximates -Laplace on the coarse grid (h_c = 2 h);
* one sweep from zero is omega r / D; the error propagator of k Jacobi sweeps has the closed-form
  spectrum (1 - omega mu)^k, mu the eigenvalues of D^-1 A for Poisson;
* with exact coarse solves the cycle is linear, symmetric for a symmetric A, exact on a single
  level, and contracts Poisson errors by a factor independent of n (textbook multigrid).
"""
import math

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import datagen
from oracle import gmg
from oracle import operator as op
from oracle import solve as sv


def coords(n):
    h = 1.0 / (n + 1)
    x = (np.arange(n) + 1) * h
    return np.meshgrid(x, x)      # X varies along j (+x), Y along i (+y)


def test_default_levels_follow_the_paper():
    # Sec. 4.1: two levels at 31 x 31, three at 63 x 63; the coarsest grid is 15 x 15
    assert gmg.default_levels(31) == 2 and gmg.default_levels(63) == 3
    assert [gmg.default_levels(n) for n in (3, 7, 15)] == [1, 1, 1]
    for n in (31, 63, 127):
        assert gmg.GMG(np.ones((n, n)), (0, 0)).a[-1].shape == (15, 15)


def test_prolong_exact_on_bilinear_functions():
    nc = 15
    n = 2 * nc + 1
    g = lambda X, Y: 0.3 + 1.7 * X - 0.9 * Y + 2.3 * X * Y
    e = gmg.prolong(g(*coords(nc)))
    ref = g(*coords(n))
    # fine nodes whose interpolation stencil stays inside the coarse grid
    assert np.allclose(e[1:-1, 1:-1], ref[1:-1, 1:-1], rtol=0, atol=1e-14)
    # coarse nodes are copied
    assert np.array_equal(e[1::2, 1::2], g(*coords(nc)))


def test_restrict_keeps_constants_and_is_scaled_transpose():
    n = 31
    assert np.allclose(gmg.restrict(np.ones((n, n))), 1.0, atol=1e-15)
    rng = np.random.default_rng(0)
    x = rng.standard_normal((n, n))
    y = rng.standard_normal(((n - 1) // 2, (n - 1) // 2))
    lhs = float(np.sum(gmg.restrict(x) * y))
    rhs = 0.25 * float(np.sum(x * gmg.prolong(y)))
    assert lhs == pytest.approx(rhs, rel=1e-13)


def test_injection_samples_coarse_node_coordinates():
    n = 63
    g = lambda X, Y: np.exp(X - 2 * Y) + X * Y
    ac = gmg.inject(g(*coords(n)))
    assert np.allclose(ac, g(*coords((n - 1) // 2)), rtol=1e-14, atol=0)


def test_rediscretised_coarse_operator_is_laplacian_on_coarse_grid():
    # a = 1, b = 0: A_c g ~ 2 pi^2 g for g = sin(pi x) sin(pi y), second order in h_c
    n = 63
    G = gmg.GMG(np.ones((n, n)), (0.0, 0.0), levels=2)
    X, Y = coords((n - 1) // 2)
    g = np.sin(np.pi * X) * np.sin(np.pi * Y)
    Ag = G.A(1, g)
    hc = 1.0 / 32
    err = np.max(np.abs(Ag - 2 * np.pi ** 2 * g)) / (2 * np.pi ** 2)
    assert err < (np.pi * hc) ** 2 / 4                      # truncation error O(h_c^2)
    assert err > (np.pi * hc) ** 2 / 100                    # (and not the fine grid's)


def test_one_sweep_from_zero():
    rng = np.random.default_rng(1)
    n = 15
    a = np.exp(rng.standard_normal((n, n)))
    b = (1.5, -0.5)
    r = rng.standard_normal((n, n))
    e = gmg.jacobi(a, b, op.diagonal(a, b), np.zeros((n, n)), r, 0.67, 1)
    assert np.allclose(e, 0.67 * r / op.diagonal(a, b), rtol=1e-15, atol=0)


def test_jacobi_error_propagator_closed_form_spectrum():
    # Poisson: D^-1 A has eigenvalues mu_kl = 1 - (cos(k pi h) + cos(l pi h)) / 2, so k sweeps
    # multiply the error by (1 - omega mu)^k
    n, omega, k = 7, 0.67, 3
    a = np.ones((n, n))
    D = op.diagonal(a, (0, 0))
    cols = []
    for idx in range(n * n):
        e0 = np.zeros(n * n); e0[idx] = 1.0
        e0 = e0.reshape(n, n)
        cols.append(gmg.jacobi(a, (0, 0), D, e0, np.zeros((n, n)), omega, k).ravel())
    E = np.array(cols).T
    got = np.sort(np.linalg.eigvalsh((E + E.T) / 2))
    h = 1.0 / (n + 1)
    c = np.cos(np.arange(1, n + 1) * np.pi * h)
    mu = 1 - (c[:, None] + c[None, :]) / 2
    want = np.sort(((1 - omega * mu) ** k).ravel())
    assert np.allclose(E, E.T, atol=1e-14)
    assert np.allclose(got, want, atol=1e-13)


def test_single_level_is_exact_solve():
    rng = np.random.default_rng(2)
    n = 15
    a = np.exp(rng.standard_normal((n, n)))
    G = gmg.GMG(a, (0.7, 1.3))
    assert G.levels == 1
    r = rng.standard_normal((n, n))
    assert np.allclose(op.apply_A(a, (0.7, 1.3), G.cycle(r)), r, rtol=0, atol=1e-10 * np.abs(r).max())


def cycle_matrix(G, n):
    cols = []
    for idx in range(n * n):
        r = np.zeros(n * n); r[idx] = 1.0
        cols.append(G.cycle(r.reshape(n, n)).ravel())
    return np.array(cols).T


def test_cycle_linear_and_symmetric_for_symmetric_operator():
    rng = np.random.default_rng(3)
    n = 15
    a = np.exp(1.5 * rng.standard_normal((n, n)))
    G = gmg.GMG(a, (0.0, 0.0), levels=3)
    V = cycle_matrix(G, n)
    assert np.allclose(V, V.T, rtol=0, atol=1e-12 * np.abs(V).max())
    r1, r2 = rng.standard_normal((2, n, n))
    assert np.allclose(G.cycle(2.5 * r1 - r2), 2.5 * G.cycle(r1) - G.cycle(r2), atol=1e-12)
    # with convection the cycle is no longer symmetric
    Gc = gmg.GMG(a, (40.0, -25.0), levels=3)
    Vc = cycle_matrix(Gc, n)
    assert not np.allclose(Vc, Vc.T, rtol=0, atol=1e-6 * np.abs(Vc).max())


def contraction(G, n, its=40, seed=0):
    """Power iteration on the error propagator I - V A."""
    rng = np.random.default_rng(seed)
    e = rng.standard_normal((n, n))
    rate = 0.0
    for _ in range(its):
        e2 = e - G.cycle(G.A(0, e))
        rate = np.linalg.norm(e2) / np.linalg.norm(e)
        e = e2 / np.linalg.norm(e2)
    return rate


def test_poisson_contraction_is_grid_independent():
    rates = []
    for n in (15, 31, 63):
        rates.append(contraction(gmg.GMG(np.ones((n, n)), (0, 0), levels=int(math.log2(n + 1))), n))
    assert max(rates) < 0.2
    assert max(rates) - min(rates) < 0.02
    # the paper's level count (exact solve on 15 x 15) contracts no worse
    assert contraction(gmg.GMG(np.ones((63, 63)), (0, 0)), 63) < 0.2


def test_stationary_solve_convection_diffusion():
    a, b, f = datagen.make_batch("grf31", 31, 1, seed=4)
    G = gmg.GMG(a[0], b[0])
    u, st, it, rho, hist = G.solve(f[0], 1e-10, 100)
    assert st == sv.OK and it < 30
    assert sv.relres(a[0], b[0], f[0], u) <= 1e-10
    uex = spla.spsolve(op.assemble_A(a[0], b[0]).tocsc(), f[0].astype(np.float64).ravel())
    assert np.allclose(u.ravel(), uex, rtol=0, atol=1e-8 * np.abs(uex).max())
