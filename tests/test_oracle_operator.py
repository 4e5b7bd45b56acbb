"""Pins of the oracle's discrete operator against closed forms, the paper's printed
kernels, textbook properties and library routines (CPU only)."""
import json
import os

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import operator as op

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _grid(n):
    h = 1.0 / (n + 1)
    x = (np.arange(n) + 1) * h
    X, Y = np.meshgrid(x, x)          # X varies along j (columns), Y along i (rows)
    return h, X, Y


@pytest.mark.parametrize("n", [7, 15, 31])
@pytest.mark.parametrize("b", [(0.0, 0.0), (1.0, 1.0), (-2.5, 0.7), (3.0, -4.0)])
def test_polynomial_closed_form(n, b):
    """Constant a, p = x(1-x) y(1-y) vanishes on the boundary, so the 5-point
    second differences are exact and the upwind differences have a closed form."""
    a0 = 1.7
    h, X, Y = _grid(n)
    p = X * (1 - X) * Y * (1 - Y)
    bx, by = b
    bxp, bxm, byp, bym = max(bx, 0), min(bx, 0), max(by, 0), min(by, 0)
    exact = (2 * a0 * (X * (1 - X) + Y * (1 - Y))
             + Y * (1 - Y) * (bxp * (1 - 2 * X + h) + bxm * (1 - 2 * X - h))
             + X * (1 - X) * (byp * (1 - 2 * Y + h) + bym * (1 - 2 * Y - h)))
    got = op.apply_A(np.full((n, n), a0), b, p)
    np.testing.assert_allclose(got, exact, rtol=1e-11, atol=1e-11)


def test_layered_medium_harmonic_flux():
    """a = a(x) layered, b = 0: the potential with constant flux through cells of
    constant a (u' = q / a piecewise, u(0) = 0) is annihilated by A on every row
    whose east neighbour is interior and whose north/south neighbours are
    interior -- the exact-flux property of harmonic face averaging."""
    n = 15
    h = 1.0 / (n + 1)
    rng = np.random.default_rng(3)
    acol = 10.0 ** rng.uniform(-2, 2, n)
    q = 1.0
    # node 0 at x = h, its cell of constant a_0 extends back to x = 0
    ucol = np.zeros(n)
    ucol[0] = q * h / acol[0]
    for j in range(1, n):
        ucol[j] = ucol[j - 1] + q * (0.5 * h / acol[j - 1] + 0.5 * h / acol[j])
    a = np.tile(acol, (n, 1))
    u = np.tile(ucol, (n, 1))
    Au = op.apply_A(a, (0.0, 0.0), u)
    inner = Au[1:-1, :-1]
    scale = np.abs(a).max() * np.abs(u).max() / h ** 2
    assert np.abs(inner).max() < 1e-12 * scale
    # negative control: arithmetic face averages do not conserve the flux
    am = 0.5 * (acol[:-1] + acol[1:])
    flux_arith = am * np.diff(ucol) / h
    assert np.abs(flux_arith - q).max() > 1e-2


def test_matches_paper_kernels():
    """With constant a = mu, h * A reproduces the paper's kernel
    (mu/h) * 5-point + v . K_upwind (velocity applied once); the paper's kernels
    put +y on the top row, this grid puts +y at row index i+1, so rows flip."""
    g = json.load(open(os.path.join(GOLDEN, "paper_kernels.json")))
    lap = np.array(g["laplace5"], float)
    dxp, dxm = np.array(g["dx_plus"], float), np.array(g["dx_minus"], float)
    dyp, dym = np.array(g["dy_plus"], float), np.array(g["dy_minus"], float)
    n = 9
    h = 1.0 / (n + 1)
    mu = 0.37
    for vx, vy in [(np.sin(0.5), np.cos(0.5)), (-0.8, 0.3), (0.2, -0.9)]:
        K = (mu / h) * lap + (max(vx, 0) * dxm + min(vx, 0) * dxp + max(vy, 0) * dym + min(vy, 0) * dyp)
        K = K / h
        K_ours = K[::-1, :]
        # read our 3x3 stencil at an interior node by applying A to unit vectors
        ic, jc = 4, 4
        got = np.zeros((3, 3))
        for p in range(3):
            for qq in range(3):
                e = np.zeros((n, n)); e[ic + p - 1, jc + qq - 1] = 1.0
                got[p, qq] = op.apply_A(np.full((n, n), mu), (vx, vy), e)[ic, jc]
        np.testing.assert_allclose(got, K_ours, rtol=1e-12, atol=1e-9)


@pytest.mark.parametrize("seed", [0, 1])
def test_invariants(seed):
    n = 15
    rng = np.random.default_rng(seed)
    a = 10.0 ** rng.uniform(-2, 2, (n, n))
    b = rng.uniform(-5, 5, 2)
    A = op.assemble_A(a, b).toarray()
    # symmetric without convection
    A0 = op.assemble_A(a, (0.0, 0.0)).toarray()
    np.testing.assert_allclose(A0, A0.T, rtol=1e-13, atol=0)
    # M-matrix sign pattern
    off = A - np.diag(np.diag(A))
    assert (off <= 0).all() and (np.diag(A) > 0).all()
    # weak row and column diagonal dominance, strict on boundary rows
    rows = np.diag(A) + off.sum(axis=1)
    cols = np.diag(A) + off.sum(axis=0)
    assert (rows >= -1e-9 * np.diag(A)).all() and (cols >= -1e-9 * np.diag(A)).all()
    # A 1 = 0 on nodes whose four neighbours are interior
    ones = np.ones((n, n))
    A1 = op.apply_A(a, b, ones)
    assert np.abs(A1[1:-1, 1:-1]).max() < 1e-9 * np.abs(A).max()
    # diagonal helper
    np.testing.assert_allclose(op.diagonal(a, b).ravel(), np.diag(A), rtol=1e-14)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_matrix_free_vs_sparse_and_transpose(seed):
    n = 31
    rng = np.random.default_rng(seed)
    a = np.exp(rng.standard_normal((n, n)))
    b = rng.uniform(-3, 3, 2)
    u = rng.standard_normal((n, n))
    v = rng.standard_normal((n, n))
    A = op.assemble_A(a, b)
    np.testing.assert_allclose(op.apply_A(a, b, u).ravel(), A @ u.ravel(), rtol=1e-12, atol=1e-9)
    np.testing.assert_allclose(op.apply_AT(a, b, v).ravel(), A.T @ v.ravel(), rtol=1e-12, atol=1e-9)
    lhs = np.sum(op.apply_A(a, b, u) * v)
    rhs = np.sum(u * op.apply_AT(a, b, v))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs) + 1e-9


def test_direct_solve_dense_vs_sparse():
    n = 15
    rng = np.random.default_rng(5)
    a = np.exp(rng.standard_normal((n, n)))
    b = (1.0, 1.0)
    f = rng.uniform(-1, 1, (n, n))
    A = op.assemble_A(a, b)
    u_sp = spla.spsolve(A.tocsc(), f.ravel())
    u_de = np.linalg.solve(A.toarray(), f.ravel())
    np.testing.assert_allclose(u_sp, u_de, rtol=1e-10, atol=1e-12)
    r = f - op.apply_A(a, b, u_sp.reshape(n, n))
    assert np.linalg.norm(r) / np.linalg.norm(f) < 1e-12


def test_features():
    n = 15
    rng = np.random.default_rng(7)
    a = 10.0 ** rng.uniform(-2, 2, (n, n))
    b = (2.0, -3.0)
    F = op.features(a, b)
    assert F.shape == (4, n, n)
    assert (F >= 0).all() and (F <= 1).all()
    # interior nodes: the four couplings of D^-1 A sum to one (zero row sum of A)
    np.testing.assert_allclose(F.sum(axis=0)[1:-1, 1:-1], 1.0, rtol=1e-13)
    # absent neighbours give zero channels
    assert (F[0][:, 0] == 0).all() and (F[1][:, -1] == 0).all()
    assert (F[2][0, :] == 0).all() and (F[3][-1, :] == 0).all()
    # constant a, no convection: each interior coupling is 1/4
    F0 = op.features(np.ones((n, n)), (0.0, 0.0))
    np.testing.assert_allclose(F0[:, 1:-1, 1:-1], 0.25, rtol=1e-14)
    # constant a, convection along +x then -y: the upwind side carries |b| h / a extra
    h = 1.0 / (n + 1)
    for (bx, by), (upw, other) in [((3.0, 0.0), (0, 1)), ((0.0, -2.0), (3, 2))]:
        Fb = op.features(np.ones((n, n)), (bx, by))
        D = 4 / h ** 2 + (abs(bx) + abs(by)) / h
        np.testing.assert_allclose(Fb[upw][1:-1, 1:-1], (1 / h ** 2 + (abs(bx) + abs(by)) / h) / D, rtol=1e-13)
        np.testing.assert_allclose(Fb[other][1:-1, 1:-1], (1 / h ** 2) / D, rtol=1e-13)
