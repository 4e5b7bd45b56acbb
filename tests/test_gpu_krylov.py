"""GPU: the stationary solve with the hand-set cycle weights against the FP64 oracle, and the
batched FGMRES solve (the network as right preconditioner, Sec. 2.2) checked by the property
that defines a solution: the oracle recomputes ||f - A u|| / ||f|| in FP64 and it must be at
most tol, for every problem of the batch; zero right-hand sides give u = 0."""
import sys

import numpy as np
import pytest

import datagen
from parity_util import assert_close
from oracle import solve as osv

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2312_11093_amd import Solver  # noqa: E402
from paper_2312_11093_amd import mgcnn as M  # noqa: E402
from paper_2312_11093_amd.handbuilt import vcycle_weights  # noqa: E402


def say(*a):
    print("[gpu-test]", *a, flush=True)
    sys.stdout.flush()


def dev(x, dtype=torch.float32):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda", dtype)


def test_stationary_handbuilt_matches_oracle():
    """A convergent learned-layout cycle (hand-set weights): same iteration count as the
    oracle's stationary iteration (within one check), solution within 1e-6 of the oracle's."""
    say("stationary hand-set cycle grf31")
    n, B = 31, 3
    a, b, f = datagen.make_batch("grf31", n, B, seed=11)
    w = vcycle_weights()
    S = Solver(w, state="f32", u="f64", check_every=1)
    S.setup(dev(a), b)
    u = torch.zeros((B, n, n), dtype=torch.float64, device="cuda")
    st, it, rr, ps = S.solve(dev(f), u, 1e-8, 200)
    assert st == M.OK, (it, rr, ps)
    for p in range(B):
        ou, ost, oit, orho, _ = osv.Solver(w, a[p], b[p]).solve(f[p], 1e-8, 200)
        assert ost == osv.OK
        assert abs(int(it[p]) - oit) <= 1, (p, it[p], oit)
        up = u[p].cpu().numpy()
        assert_close(up, ou, 1e-6, f"solution {p}")
        assert osv.relres(a[p], b[p], f[p], up) <= 1e-8
    S.close()


# bf16 state only at small n: its rounding noise, amplified ~n^2 by A, stalls the solve at
# larger sizes (the 1e-8 runs use f32 state)
@pytest.mark.parametrize("workload,n,B,state,restart,gs,omega", [
    ("grf31", 31, 3, "f32", 30, 2, 0.9),
    ("mixture127", 127, 4, "bf16", 20, 2, 0.8),
    ("blocks1023", 63, 4, "bf16", 30, 2, 0.8),
    ("blocks1023", 255, 2, "f32", 8, 2, 0.9),
    ("blocks1023", 255, 3, "f32", 63, 1, 0.9),
])
def test_fgmres_converges_to_tol(workload, n, B, state, restart, gs, omega):
    say("fgmres", workload, n, B, state, restart, "gs passes", gs, "omega", omega)
    a, b, f = datagen.make_batch(workload, n, B, seed=12)
    f[B - 1] = 0.0                                   # a zero right-hand side in the batch
    S = Solver(vcycle_weights(omega=omega), state=state, u="f64", method="fgmres", restart=restart,
               gs_passes=gs)
    S.setup(dev(a), b)
    u = torch.full((B, n, n), 0.5, dtype=torch.float64, device="cuda")
    tol = 1e-8
    st, it, rr, ps = S.solve(dev(f), u, tol, 2000)
    say("  iters", list(it), "relres", list(rr))
    assert st == M.OK and (ps == 0).all()
    assert int(it[B - 1]) == 0 and (u[B - 1] == 0).all()
    for p in range(B - 1):
        rho = osv.relres(a[p], b[p], f[p], u[p].cpu().numpy())
        assert rho <= tol * (1 + 1e-6), (p, rho)
        assert abs(rho - rr[p]) <= 1e-3 * tol + 1e-6 * rho, (p, rho, rr[p])
    S.close()


def test_fgmres_maxit_and_args():
    say("fgmres maxit / args")
    n, B = 63, 2
    a, b, f = datagen.make_batch("blocks1023", n, B, seed=13)
    S = Solver(vcycle_weights(), state="f32", u="f64", method="fgmres", restart=4)
    S.setup(dev(a), b)
    u = torch.zeros((B, n, n), dtype=torch.float64, device="cuda")
    st, it, rr, ps = S.solve(dev(f), u, 1e-12, 6)
    assert st == M.NOT_CONVERGED and (ps == M.NOT_CONVERGED).all()
    assert (it <= 6).all() and (it >= 1).all()
    for p in range(B):   # the reported residual is that of the returned u
        rho = osv.relres(a[p], b[p], f[p], u[p].cpu().numpy())
        assert abs(rho - rr[p]) <= 1e-5 * rho
    S.close()
    with pytest.raises(M.MGCNNError):
        Solver(vcycle_weights(), method="fgmres", restart=64)


def test_single_4095_to_1e10():
    """One 4095^2 problem (lognormal GRF, length 0.05, variance 2, b = (1, 1)) to relative
    residual 1e-10 with FGMRES and f32 state; the oracle recomputes the residual in f64."""
    say("4095^2 to 1e-10")
    p = datagen.make_problem("grf4095", 4095, 0, 0)
    S = Solver(vcycle_weights(), state="f32", u="f64", method="fgmres", restart=30)
    S.setup(dev(p.a).view(1, 4095, 4095), p.b.reshape(1, 2))
    u = torch.zeros((1, 4095, 4095), dtype=torch.float64, device="cuda")
    st, it, rr, ps = S.solve(dev(p.f).view(1, 4095, 4095), u, 1e-10, 1000)
    say("  iters", int(it[0]), "relres", float(rr[0]))
    assert st == M.OK
    rho = osv.relres(p.a, p.b, p.f, u[0].cpu().numpy())
    say("  oracle relres", rho)
    assert rho <= 1e-10 * (1 + 1e-5)
    S.close()


def test_bf16_setup_tensors_option():
    """opts.s_bf16: the setup tensors are the f32 ones rounded once to bf16 (round to nearest
    even), and an FGMRES solve still reaches the tolerance (the oracle re-checks)."""
    say("s_bf16")
    n, B = 127, 3
    a, b, f = datagen.make_batch("blocks1023", n, B, seed=14)
    w = vcycle_weights()
    S32 = Solver(w, state="f32", u="f64")
    S16 = Solver(w, state="f32", u="f64", s_bf16=True, method="fgmres", restart=30)
    S32.setup(dev(a), b)
    S16.setup(dev(a), b)
    for lvl in (1, 2, S32.levels):
        ref = S32.get_setup_tensor(lvl).cpu().numpy().astype(np.float32)
        bits = ref.view(np.uint32).astype(np.uint64)
        rnd = ((bits + 0x7FFF + ((bits >> 16) & 1)) >> 16 << 16).astype(np.uint32).view(np.float32)
        got = S16.get_setup_tensor(lvl).cpu().numpy()
        assert np.array_equal(got, rnd), lvl
    u = torch.zeros((B, n, n), dtype=torch.float64, device="cuda")
    st, it, rr, ps = S16.solve(dev(f), u, 1e-8, 3000)
    say("  iters", list(it))
    assert st == M.OK
    for p in range(B):
        assert osv.relres(a[p], b[p], f[p], u[p].cpu().numpy()) <= 1e-8 * (1 + 1e-6)
    S32.close()
    S16.close()


@pytest.mark.parametrize("precond,n,B,restart,kd", [
    ("network", 255, 3, 63, 16),
    ("network", 127, 4, 30, 8),
    ("gmg", 255, 3, 30, 8),
])
def test_fgmres_deflated_restarts(precond, n, B, restart, kd):
    """opts.deflate: restarts keep the kd smallest singular directions of the cycle.  Every
    problem still reaches the tolerance (the oracle re-checks; a zero right-hand side stays
    zero), in fewer Arnoldi steps in total than plain restarts."""
    say("fgmres deflated restarts", precond, n, B, restart, kd)
    a, b, f = datagen.make_batch("blocks1023", n, B, seed=16)
    f[B - 1] = 0.0
    w = vcycle_weights() if precond == "network" else None
    its = {}
    for k in (0, kd):
        S = Solver(w, precond=precond, state="f32", u="f64", method="fgmres", restart=restart,
                   gs_passes=1, deflate=k)
        S.setup(dev(a), b)
        u = torch.zeros((B, n, n), dtype=torch.float64, device="cuda")
        st, it, rr, ps = S.solve(dev(f), u, 1e-8, 4000)
        say("  deflate", k, "iters", list(it))
        assert st == M.OK and (ps == 0).all()
        assert int(it[B - 1]) == 0 and (u[B - 1] == 0).all()
        for p in range(B - 1):
            rho = osv.relres(a[p], b[p], f[p], u[p].cpu().numpy())
            assert rho <= 1e-8 * (1 + 1e-6), (k, p, rho)
            assert abs(rho - rr[p]) <= 1e-3 * 1e-8 + 1e-6 * rho
        its[k] = int(it.sum())
        S.close()
    assert its[kd] < its[0], its
    with pytest.raises(M.MGCNNError):
        Solver(w, precond=precond, method="fgmres", restart=8, deflate=8)
    with pytest.raises(M.MGCNNError):
        Solver(w, precond=precond, method="fgmres", restart=9, deflate=5)


@pytest.mark.parametrize("precond", ["network", "gmg"])
@pytest.mark.parametrize("n", [3, 7, 15, 31])
def test_deflation_edge_sizes(n, precond):
    """Deflated restarts at the edge of their range: k = restart / 2 (the largest k the options
    allow) on tiny grids (3^2 has only 9 unknowns, fewer than the basis), where cycles end early
    on an exact solution or a numerically dependent basis; every problem still reaches 1e-10
    and the oracle agrees."""
    say("deflation edge", n, precond)
    B = 3
    a, b, f = datagen.make_batch("mixture127", n, B, seed=23)
    w = vcycle_weights() if precond == "network" else None
    S = Solver(w, precond=precond, state="f32", u="f64", method="fgmres", restart=9, gs_passes=1,
               deflate=4)
    S.setup(dev(a), b)
    u = torch.zeros((B, n, n), dtype=torch.float64, device="cuda")
    st, it, rr, ps = S.solve(dev(f), u, 1e-10, 2000)
    say("  iters", list(it))
    assert st == M.OK and (ps == 0).all()
    for p in range(B):
        assert osv.relres(a[p], b[p], f[p], u[p].cpu().numpy()) <= 1e-10 * (1 + 1e-5)
    S.close()
