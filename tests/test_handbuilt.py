"""CPU: the hand-set cycle weights do what their construction states, checked through the
FP64 oracle against the operator itself (not against a retyped formula): the first down
smoother is one weighted-Jacobi sweep (E = omega r/D, R = the scaled residual after it), the
setup state carries the D-normalised couplings, and the cycle converges on Poisson."""
import numpy as np

import datagen
from oracle import network as onet
from oracle import operator as oop
from oracle import solve as osv
from paper_2312_11093_amd.handbuilt import DC, DE, E, FCH, R, RC, parameter_shapes, vcycle_weights

OMEGA, ALPHA = float(np.float32(0.9)), 0.05          # the weights are stored as float32


def test_layout_matches_oracle_order():
    assert [s for _, s in parameter_shapes(16)] == [s for _, s in datagen.weight_shapes(16)]
    assert vcycle_weights().size == datagen.num_weights(16)


def _problem(n, seed):
    rng = np.random.default_rng(seed)
    a = np.exp(datagen.grf(n, rng, 0.1, 1.0)).astype(np.float32).astype(np.float64)
    return a, (2.0, -1.0), rng.standard_normal((n, n))


def test_setup_state_carries_couplings():
    n = 15
    a, b, _ = _problem(n, 1)
    P = onet.unpack_weights(vcycle_weights().astype(np.float64), 16)
    F = oop.features(a, b)
    s = onet.setup(P, F, onet.num_levels(n))
    for ch in (R, E, DE):
        assert np.allclose(s[0][ch], 1.0, atol=1e-6)
    # s_RC[d](i) = tanh(alpha F_d(i - dir_d)), i.e. F_d of the neighbour opposite to d
    shift = [(0, -1), (0, 1), (-1, 0), (1, 0)]          # W, E, S, N as (di, dj)
    for d in range(4):
        di, dj = shift[d]
        src = np.zeros((n, n))
        ii, jj = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
        ok = (ii - di >= 0) & (ii - di < n) & (jj - dj >= 0) & (jj - dj < n)
        src[ok] = F[d][(ii - di)[ok], (jj - dj)[ok]]
        assert np.allclose(s[0][RC[d]], np.tanh(ALPHA * src), atol=1e-12)
        assert np.allclose(s[0][DC[d]], np.tanh(ALPHA * src), atol=1e-12)
        assert np.allclose(s[0][FCH[d]], F[d], atol=1e-12)


def test_first_down_smoother_is_jacobi_sweep():
    n = 15
    a, b, r = _problem(n, 2)
    P = onet.unpack_weights(vcycle_weights().astype(np.float64), 16)
    s = onet.setup(P, oop.features(a, b), onet.num_levels(n))
    D = oop.diagonal(a, b)
    _, tape = onet.vcycle(P, s, r / D, keep=True)
    x = tape["xdn"][0]
    e = OMEGA * r / D
    # s_E = 4 tanh(beta) with beta = atanh(1/4) rounded to float32: 1 within 1e-6
    assert np.allclose(x[E], e, rtol=0, atol=1e-6 * np.abs(e).max())
    r_after = (r - oop.apply_A(a, b, e)) / D
    # tanh(alpha F) / alpha = F (1 - (alpha F)^2 / 3 + ...): relative error <= alpha^2 / 3
    err = np.abs(x[R] - r_after).max() / np.abs(r / D).max()
    assert err <= ALPHA ** 2 / 3 * OMEGA * 1.01


def test_cycle_converges_on_poisson():
    n = 31
    a = np.ones((n, n))
    f = np.random.default_rng(3).standard_normal((n, n))
    # omega = 0.8 is the classical choice for this cycle on Poisson (the default, 0.9, was
    # chosen for the Krylov-wrapped block workload)
    u, st, it, rho, hist = osv.Solver(vcycle_weights(omega=0.8), a, (0.0, 0.0)).solve(f, 1e-8, 60)
    assert st == osv.OK and it <= 25
    assert osv.relres(a, (0.0, 0.0), f, u) <= 1e-8
