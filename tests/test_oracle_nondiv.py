"""Pins of the oracle's non-divergence operator (Eq. (7), the form the paper computes with)
and of the GMG baseline on the paper's own test problems -- CPU only.

* -a (u_xx + u_yy) on a polynomial the 5-point Laplacian differentiates exactly: closed form;
* equal to the divergence form for a constant coefficient; zero row sums without convection;
  not symmetric for a variable coefficient; transpose and sparse assembly agree;
* every interior stencil feature is 1/4 without convection;
* the GMG V-cycle with the paper's settings needs the iteration counts the paper prints for
  GMG on these problems (golden fixture, cited in the file).
"""
import json
import os

import numpy as np
import pytest

import datagen
from oracle import gmg
from oracle import operator as op

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_gmg_iterations.json")


def coords(n):
    h = 1.0 / (n + 1)
    x = (np.arange(n) + 1) * h
    return np.meshgrid(x, x)


def test_closed_form_on_quadratic_product():
    n = 31
    X, Y = coords(n)
    a = 1.0 + X + Y ** 2
    u = X * (1 - X) * Y * (1 - Y)
    Au = op.apply_A(a, (0.0, 0.0), u, form="nondiv")
    exact = a * 2.0 * (X * (1 - X) + Y * (1 - Y))
    assert np.allclose(Au, exact, rtol=1e-10, atol=0)
    # the divergence form differs by the a_x u_x + a_y u_y term (here O(1))
    assert not np.allclose(op.apply_A(a, (0.0, 0.0), u), exact, rtol=1e-3, atol=0)


def test_constant_coefficient_forms_agree_and_row_sums():
    rng = np.random.default_rng(0)
    n = 15
    u = rng.standard_normal((n, n))
    b = (0.7, -1.9)
    a = np.full((n, n), 2.5)
    assert np.allclose(op.apply_A(a, b, u, "nondiv"), op.apply_A(a, b, u, "div"), rtol=1e-14)
    av = np.exp(rng.standard_normal((n, n)))
    A = op.assemble_A(av, (0.0, 0.0), "nondiv").toarray()
    inner = np.zeros((n, n), bool)
    inner[1:-1, 1:-1] = True
    assert np.allclose(A.sum(axis=1).reshape(n, n)[inner], 0.0, atol=1e-9 * np.abs(A).max())
    assert not np.allclose(A, A.T, atol=1e-6 * np.abs(A).max())
    Ab = op.assemble_A(av, b, "nondiv")
    v = rng.standard_normal((n, n))
    assert np.allclose(op.apply_AT(av, b, v, "nondiv").ravel(), Ab.T @ v.ravel(), rtol=1e-13)
    assert np.allclose(op.apply_A(av, b, v, "nondiv").ravel(), Ab @ v.ravel(), rtol=1e-13)


def test_features_quarter_without_convection():
    rng = np.random.default_rng(1)
    n = 15
    F = op.features(np.exp(2 * rng.standard_normal((n, n))), (0.0, 0.0), "nondiv")
    assert np.allclose(F[:, 1:-1, 1:-1], 0.25, rtol=1e-14)


def test_paper_workload_recipe():
    p = datagen.make_problem("paper_re1e3", 63, 0, 0)
    coef = p.a.astype(np.float64) * 64
    assert coef.min() == pytest.approx(1e-3, rel=1e-5) and coef.max() == pytest.approx(1.0, rel=1e-6)
    assert np.allclose(p.b, [np.sin(0.5), np.cos(0.5)]) and np.all(p.f == 1.0)


@pytest.mark.parametrize("workload", ["paper_re1e3", "paper_mldata", "paper_re10", "paper_re1e5"])
@pytest.mark.parametrize("n", [127, 255])
def test_gmg_iterations_match_the_paper(n, workload):
    """GMG (levels log2(n+1) - 3, exact 15 x 15 coarsest solve, 3 + 3 sweeps of weight 0.67)
    on the paper's problems, for the coefficient distributions of Appendix B.1 (white noise with
    Re = 1000, 10, 1e5, and the multi-level data of Alg. 4): within 15 % of the printed mean
    iteration count.  (At 31 and 63 the oracle needs 12 and 15 iterations on white noise
    against the printed 16.7 and 19.2.)"""
    tab = json.load(open(GOLDEN))["appendix_b1"]
    want = tab["gmg_iterations"][tab["workload_column"][workload]][str(n)]
    p = datagen.make_problem(workload, n, 0, 0)
    G = gmg.GMG(p.a, p.b, omega=0.67, form="nondiv")
    u, st, it, rho, _ = G.solve(p.f, 1e-8, 200)
    assert st == 0
    assert abs(it - want) <= 0.15 * want, (it, want)
