"""GPU: batched preconditioned conjugate gradients (method "pcg": symmetric problems, b = 0) with
the V-cycle and with the symmetric variant of the network as preconditioner, against the FP64
oracle's PCG on the same inputs: the iterate after a fixed number of steps element by element,
and tolerance-driven solves by the property that defines a solution (the oracle's FP64 residual
of the returned u is at most tol) and by their iteration counts."""
import sys

import numpy as np
import pytest

import datagen
from parity_util import assert_close
from oracle import gmg as ogmg
from oracle import operator as oop
from oracle import solve as osv

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2312_11093_amd import Solver  # noqa: E402
from paper_2312_11093_amd import mgcnn as M  # noqa: E402
from paper_2312_11093_amd.weights import symmetric_variant  # noqa: E402


def say(*a):
    print("[gpu-test]", *a, flush=True)
    sys.stdout.flush()


def dev(x, dtype=torch.float32):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda", dtype)


def tied_weights(C=16, seed=6):
    """Xavier weights with W_up, W_T, W_out the adjoints of W_dn, W_R, W_in (the library's
    helper; checked against the oracle-side construction in test_weights_symmetric): with the
    up smoother x + s . (W_up * x) the network is symmetric positive semi-definite."""
    return symmetric_variant(datagen.xavier_weights(C, seed))


def symmetric_batch(workload, n, B, seed):
    a, b, f = datagen.make_batch(workload, n, B, seed=seed)
    return a, np.zeros_like(b), f


def oracle_pcg(precond, w, a, f, tol, maxit):
    a64 = a.astype(np.float64)
    b0 = np.zeros(2)
    if precond == "gmg":
        M_ = ogmg.GMG(a64, b0).cycle
    else:
        M_ = osv.Solver(w.astype(np.float64), a64, b0, up_post=True).pcg_correction
    return osv.pcg(lambda x: oop.apply_A(a64, b0, x), M_, f.astype(np.float64), tol, maxit)


def make_solver(precond, w, u="f64"):
    if precond == "gmg":
        return Solver(None, precond="gmg", state="f32", u=u, method="pcg")
    return Solver(w, state="f32", u=u, method="pcg", up_post=True)


@pytest.mark.parametrize("precond,n", [("gmg", 31), ("gmg", 63), ("network", 15), ("network", 31)])
def test_pcg_fixed_steps_match_oracle(precond, n):
    """maxit = K steps and an unreachable tolerance: u_K of the batched float32 recurrence equals
    the oracle's FP64 u_K to float32-level accuracy, and the reported residual is the true one."""
    say("pcg fixed steps", precond, n)
    B, K = 3, 3
    a, b, f = symmetric_batch("mixture127", n, B, seed=31)
    w = tied_weights() if precond == "network" else None
    S = make_solver(precond, w)
    S.setup(dev(a), b)
    u = torch.zeros((B, n, n), dtype=torch.float64, device="cuda")
    st, it, rr, ps = S.solve(dev(f), u, 1e-30, K)
    S.close()
    assert st == M.NOT_CONVERGED and (it == K).all() and (ps == M.NOT_CONVERGED).all()
    for p in range(B):
        uo, sto, ito, rro, _ = oracle_pcg(precond, w, a[p], f[p], 1e-30, K)
        assert ito == K
        ug = u[p].cpu().numpy()
        say("  problem", p, "relres", rr[p], rro)
        assert_close(ug, uo, 1e-5 if precond == "gmg" else 1e-4, f"problem {p}", say)
        assert abs(rr[p] - osv.relres(a[p], b[p], f[p], ug)) <= 1e-6 * rr[p]


@pytest.mark.parametrize("precond,n,tol", [
    ("gmg", 63, 1e-10), ("gmg", 127, 1e-8), ("network", 15, 1e-8), ("network", 31, 1e-8)])
def test_pcg_solves_to_tolerance(precond, n, tol):
    """Every problem of a mixed batch (one zero right-hand side) reaches tol on the oracle's FP64
    residual.  The float32 recurrence restarts from the true residual after each 1e-5 drop,
    where the oracle runs one FP64 recurrence: the step counts may differ by the Krylov
    information a restart discards, at most 50 % here."""
    say("pcg to tolerance", precond, n, tol)
    B = 4
    a, b, f = symmetric_batch("mixture127", n, B, seed=32)
    f[2] = 0.0
    w = tied_weights() if precond == "network" else None
    S = make_solver(precond, w)
    S.setup(dev(a), b)
    u = torch.zeros((B, n, n), dtype=torch.float64, device="cuda")
    st, it, rr, ps = S.solve(dev(f), u, tol, 3000)
    S.close()
    say("  iters", list(it), "relres", list(rr))
    assert st == M.OK and (ps == M.OK).all()
    assert it[2] == 0 and (u[2] == 0).all()
    for p in range(B):
        if p == 2:
            continue
        ug = u[p].cpu().numpy()
        rho = osv.relres(a[p], b[p], f[p], ug)
        assert rho <= tol * (1 + 1e-5), (p, rho)
        assert abs(rho - rr[p]) <= 1e-3 * tol
        if n <= 63:
            _, sto, ito, _, _ = oracle_pcg(precond, w, a[p], f[p], tol, 3000)
            say("  problem", p, "oracle iters", ito)
            assert sto == osv.OK and ito - 3 <= int(it[p]) <= 1.5 * ito + 3, (p, it[p], ito)


def test_pcg_float32_u_and_rejections():
    """u in float32 works the same way (a looser tolerance); b != 0 is refused at solve time
    (the operator is not symmetric) and the network without its symmetric form at create."""
    say("pcg f32 u and rejections")
    n, B = 31, 2
    a, b, f = symmetric_batch("grf31", n, B, seed=33)
    S = make_solver("gmg", None, u="f32")
    S.setup(dev(a), b)
    u = torch.zeros((B, n, n), dtype=torch.float32, device="cuda")
    st, it, rr, ps = S.solve(dev(f), u, 1e-5, 500)
    assert st == M.OK
    for p in range(B):
        assert osv.relres(a[p], b[p], f[p], u[p].cpu().numpy().astype(np.float64)) <= 1e-5 * (1 + 1e-3)
    b1 = b.copy()
    b1[1] = (1.0, 0.5)
    S.setup(dev(a), b1)
    with pytest.raises(M.MGCNNError):
        S.solve(dev(f), u, 1e-5, 500)
    S.close()
    with pytest.raises(M.MGCNNError):
        Solver(tied_weights(), state="f32", method="pcg")


@pytest.mark.parametrize("precond", ["gmg", "network"])
@pytest.mark.parametrize("n", [3, 7])
def test_pcg_edge_sizes(n, precond):
    """Tiny grids (9 and 49 unknowns: the recurrence terminates within n^2 steps in exact
    arithmetic), a batch of one, and maxit = 0 (no step: the true residual of u = 0 is 1)."""
    say("pcg edge", n, precond)
    a, b, f = symmetric_batch("mixture127", n, 1, seed=34)
    w = tied_weights() if precond == "network" else None
    S = make_solver(precond, w)
    S.setup(dev(a), b)
    u = torch.zeros((1, n, n), dtype=torch.float64, device="cuda")
    st, it, rr, ps = S.solve(dev(f), u, 1e-10, 0)
    assert st == M.NOT_CONVERGED and it[0] == 0 and abs(rr[0] - 1.0) <= 1e-12 and not u.any()
    st, it, rr, ps = S.solve(dev(f), u, 1e-10, 500)
    S.close()
    say("  iters", int(it[0]), "relres", float(rr[0]))
    assert st == M.OK and it[0] <= 3 * n * n
    assert osv.relres(a[0], b[0], f[0], u[0].cpu().numpy()) <= 1e-10 * (1 + 1e-5)


def test_pcg_group_of_uneven_sizes():
    """The group API (one batched problem set per size, concurrent streams) with conjugate
    gradients: problems of 31^2, 63^2 and 127^2 with b = 0 all reach 1e-9 on the oracle's
    FP64 residual."""
    from paper_2312_11093_amd import GroupSolver
    say("pcg group")
    sizes = [31, 63, 127, 31, 63]
    probs = [datagen.make_problem("mixture127", n, i, 35) for i, n in enumerate(sizes)]
    a = [dev(p.a) for p in probs]
    f = [dev(p.f) for p in probs]
    b = np.zeros((len(sizes), 2), np.float32)
    u = [torch.zeros((n, n), dtype=torch.float64, device="cuda") for n in sizes]
    G = GroupSolver(None, precond="gmg", state="f32", u="f64", method="pcg")
    G.setup(a, b)
    st, it, rr, ps = G.solve(f, u, 1e-9, 1000)
    G.close()
    say("  iters", list(it))
    assert st == M.OK and (np.asarray(ps) == 0).all()
    for i, p in enumerate(probs):
        assert osv.relres(p.a, b[i], p.f, u[i].cpu().numpy()) <= 1e-9 * (1 + 1e-5)
