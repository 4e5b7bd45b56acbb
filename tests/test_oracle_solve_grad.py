"""Pins of the oracle's solver loop, status semantics, loss and reverse mode
(central finite differences, adjoint identities) -- CPU only."""
import numpy as np
import pytest

import datagen
from oracle import adjoint as adj
from oracle import network as net
from oracle import operator as op
from oracle import solve as sv


def _problem(n, seed, contrast=1.0):
    rng = np.random.default_rng(seed)
    a = np.exp(contrast * rng.standard_normal((n, n)))
    b = rng.uniform(-2, 2, 2)
    f = rng.standard_normal((n, n))
    return a, b, f


def _jacobi(C, omega):
    P = {k: np.zeros_like(v) for k, v in net.unpack_weights(np.zeros(81 * C * C + 58 * C), C).items()}
    P["W_in"][0, 0, 1, 1] = 1.0
    P["W_out"][0, 0, 1, 1] = omega
    return net.pack_weights(P, C)


def test_status_zero_rhs():
    a, b, f = _problem(7, 0)
    S = sv.Solver(datagen.xavier_weights(4, 0), a, b)
    u, st, it, rho, _ = S.solve(np.zeros_like(f), 1e-8, 10, u0=np.ones_like(f))
    assert st == sv.OK and it == 0 and np.all(u == 0)


def test_status_maxit_zero_and_loose_tol():
    a, b, f = _problem(7, 1)
    S = sv.Solver(_jacobi(2, 1.0), a, b)
    u, st, it, rho, _ = S.solve(f, 1e-8, 0)
    assert st == sv.NOT_CONVERGED and it == 0 and rho == pytest.approx(1.0)
    u, st, it, rho, _ = S.solve(f, 2.0, 10)
    assert st == sv.OK and it == 0


def test_status_nonfinite_and_divergence():
    a, b, f = _problem(7, 2)
    S = sv.Solver(_jacobi(2, 1.0), a, b)
    fn = f.copy(); fn[3, 3] = np.nan
    _, st, it, _, _ = S.solve(fn, 1e-8, 10)
    assert st == sv.DIVERGED and it == 0
    # omega = 100 makes weighted Jacobi blow up
    S = sv.Solver(_jacobi(2, 100.0), a, b)
    _, st, it, rho, hist = S.solve(f, 1e-8, 200)
    assert st == sv.DIVERGED and rho > sv.DIVERGENCE_LIMIT and it < 200
    assert all(h <= sv.DIVERGENCE_LIMIT for h in hist[:-1])


def test_iteration_counts_follow_history():
    a, b, f = _problem(7, 3)
    S = sv.Solver(_jacobi(2, 1.0), a, b)
    u, st, it, rho, hist = S.solve(f, 1e-6, 1000)
    assert st == sv.OK and len(hist) == it + 1
    assert hist[-1] <= 1e-6 < hist[-2]
    assert rho == pytest.approx(sv.relres(a, b, f, u), rel=1e-12)


# ----------------------------------------------------------------------------------------------
# reverse mode
# ----------------------------------------------------------------------------------------------

def _loss(w, batch, K):
    a_b, b_b, f_b = batch
    us = [sv.Solver(w, a, b).forward(f, K) for a, b, f in zip(a_b, b_b, f_b)]
    return sv.loss(a_b, b_b, f_b, us)


@pytest.fixture(scope="module")
def grad_case():
    C, n, K = 4, 7, 3
    rng = np.random.default_rng(21)
    w = datagen.xavier_weights(C, 3).astype(np.float64) * 0.6
    w[-(9 * C):] *= 1.0
    # non-zero biases so that every parameter tensor has a non-trivial gradient
    P = net.unpack_weights(w, C)
    for k in range(4):
        P[f"beta_k{k}"] = 0.3 * rng.standard_normal(C)
    w = net.pack_weights(P, C)
    batch = ([np.exp(rng.standard_normal((n, n))) for _ in range(2)],
             [rng.uniform(-2, 2, 2) for _ in range(2)],
             [rng.standard_normal((n, n)) for _ in range(2)])
    L0, g = adj.loss_and_grad(w, *batch, K)
    return C, K, w, batch, L0, g


def test_loss_value(grad_case):
    C, K, w, batch, L0, g = grad_case
    assert L0 == pytest.approx(_loss(w, batch, K), rel=1e-13)


def test_gradient_vs_central_differences_every_tensor(grad_case):
    """Central differences in FP64 (h = 1e-3) on at least two coordinates of
    every parameter tensor (>= 32 coordinates in total)."""
    C, K, w, batch, L0, g = grad_case
    names = list(net.unpack_weights(w, C).keys())
    offsets, off = {}, 0
    for nm in names:
        size = net.unpack_weights(w, C)[nm].size
        offsets[nm] = (off, size)
        off += size
    rng = np.random.default_rng(0)
    h = 1e-3
    checked = 0
    for nm in names:
        o, size = offsets[nm]
        for i in rng.choice(size, 2, replace=False):
            idx = o + i
            wp, wm = w.copy(), w.copy()
            wp[idx] += h; wm[idx] -= h
            fd = (_loss(wp, batch, K) - _loss(wm, batch, K)) / (2 * h)
            assert abs(g[idx] - fd) <= 1e-5 * max(abs(fd), 1e-3 * np.abs(g).max()), (nm, i, g[idx], fd)
            checked += 1
    assert checked >= 32


def test_gradient_directional(grad_case):
    C, K, w, batch, L0, g = grad_case
    rng = np.random.default_rng(1)
    h = 1e-3
    for _ in range(8):
        d = rng.standard_normal(w.size)
        d /= np.linalg.norm(d)
        fd = (_loss(w + h * d, batch, K) - _loss(w - h * d, batch, K)) / (2 * h)
        assert abs(g @ d - fd) <= 1e-5 * max(abs(fd), 1e-6)


def test_gradient_wrt_rhs():
    C, n, K = 3, 7, 2
    rng = np.random.default_rng(5)
    w = datagen.xavier_weights(C, 4).astype(np.float64) * 0.5
    batch = ([np.exp(rng.standard_normal((n, n)))], [np.array([1.0, -1.0])], [rng.standard_normal((n, n))])
    L0, g, dfs = adj.loss_and_grad(w, *batch, K, want_df=True)
    h = 1e-4
    for _ in range(6):
        i, j = rng.integers(n, size=2)
        fp = batch[2][0].copy(); fp[i, j] += h
        fm = batch[2][0].copy(); fm[i, j] -= h
        fd = (_loss(w, (batch[0], batch[1], [fp]), K) - _loss(w, (batch[0], batch[1], [fm]), K)) / (2 * h)
        assert abs(dfs[0][i, j] - fd) <= 1e-6 * max(abs(fd), 1e-4)


def test_gradient_nondiv_form():
    """The reverse mode with the non-divergence operator (Eq. (7)): loss value and
    directional central differences."""
    C, n, K = 3, 7, 2
    rng = np.random.default_rng(8)
    w = datagen.xavier_weights(C, 5).astype(np.float64) * 0.5
    batch = ([np.exp(rng.standard_normal((n, n)))], [np.array([0.4, 0.9])],
             [rng.standard_normal((n, n))])
    L0, g = adj.loss_and_grad(w, *batch, K, form="nondiv")

    def loss(wv):
        us = [sv.Solver(wv, a, b, form="nondiv").forward(f, K) for a, b, f in zip(*batch)]
        return sv.loss(*batch, us, form="nondiv")

    assert L0 == pytest.approx(loss(w), rel=1e-13)
    assert L0 != pytest.approx(_loss(w, batch, K), rel=1e-6)     # the form matters here
    h = 1e-3
    for _ in range(6):
        d = rng.standard_normal(w.size)
        d /= np.linalg.norm(d)
        fd = (loss(w + h * d) - loss(w - h * d)) / (2 * h)
        assert abs(g @ d - fd) <= 1e-5 * max(abs(fd), 1e-6)


def test_solve_network_adjoint_identity():
    """<B x, y> = <x, B^T y> for the reverse of one solve-network application."""
    C, n = 4, 15
    rng = np.random.default_rng(6)
    w = datagen.xavier_weights(C, 5)
    a = np.exp(rng.standard_normal((n, n)))
    S = sv.Solver(w, a, (1.0, 1.0))
    x = rng.standard_normal((n, n))
    y = rng.standard_normal((n, n))
    Bx, tape = net.vcycle(S.P, S.s, x, keep=True)
    dP = {k: np.zeros_like(v) for k, v in S.P.items()}
    BTy, _ = adj.vcycle_backward(S.P, S.s, tape, y, dP)
    lhs, rhs = np.sum(Bx * y), np.sum(x * BTy)
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), 1.0)


def test_conv_same_adjoint_identity():
    rng = np.random.default_rng(7)
    W = rng.standard_normal((3, 5, 3, 3))
    x = rng.standard_normal((5, 9, 9))
    y = rng.standard_normal((3, 9, 9))
    assert abs(np.sum(net.conv_same(W, x) * y) - np.sum(x * adj.conv_same_dx(W, y))) < 1e-11
