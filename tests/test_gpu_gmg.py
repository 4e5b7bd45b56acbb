"""GPU: the geometric multigrid preconditioner (Sec. 2.3 V-cycle with the GMG settings of
Sec. 4.1) through the C-ABI against the FP64 oracle ``oracle.gmg``.

* one cycle z = V(r) (mgcnn_apply) element by element against the oracle's cycle, at sizes that
  span several 32 x 32 tiles with a ragged edge, for every sweep count, the default and the full
  level count, the single-level case (exact solve) and convection;
* the stationary solve against the oracle's iteration count and solution;
* FGMRES with the GMG preconditioner on high-contrast blocks, and at the full 64 x 1023^2 size:
  the oracle recomputes ||f - A u|| / ||f|| in FP64;
* option errors.

Tolerance of one cycle: the kernels run in float32 and the coarsest solve in float64 from a
float32 right-hand side; each level adds a few float32 roundings (relative 6e-8) that the
coarse solve can amplify by the condition number of the coarsest operator.  Measured on these
inputs: max|z - z_ref| / max|z_ref| between 3e-8 and 4e-7 (the 10^4-contrast cases at the top).
The bound used, TOL = 2e-6, leaves a factor of 5 over that; a wrong weight, index or sign
gives errors of order 1.
"""
import sys

import numpy as np
import pytest

import datagen
from parity_util import assert_close
from oracle import gmg as ogmg
from oracle import solve as osv

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2312_11093_amd import GroupSolver, Solver  # noqa: E402
from paper_2312_11093_amd import mgcnn as M  # noqa: E402


def say(*a):
    print("[gpu-test]", *a, flush=True)
    sys.stdout.flush()


def dev(x, dtype=torch.float32):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda", dtype)


@pytest.mark.parametrize("workload,n,B,levels,sweeps,omega,tol", [
    ("grf31", 31, 3, 0, 3, 0.67, 2e-6),          # paper levels: 2 (coarsest 15 x 15)
    ("grf31", 63, 2, 0, 1, 0.67, 2e-6),
    ("grf31", 63, 2, 6, 2, 0.8, 2e-6),           # full depth: coarsest 1 x 1
    ("mixture127", 127, 3, 0, 3, 0.67, 2e-6),
    ("mixture127", 127, 2, 7, 4, 0.67, 2e-6),
    ("blocks1023", 255, 2, 0, 3, 0.67, 2e-6),
    ("grf31", 15, 2, 0, 3, 0.67, 2e-6),          # one level: exact solve of the whole grid
    ("grf31", 7, 2, 0, 3, 0.67, 2e-6),
    ("grf31", 3, 2, 2, 2, 0.67, 2e-6),
])
def test_cycle_matches_oracle(workload, n, B, levels, sweeps, omega, tol):
    say("gmg cycle", workload, n, B, "levels", levels, "sweeps", sweeps, "omega", omega)
    a, b, _ = datagen.make_batch(workload, n, B, seed=31)
    rng = np.random.default_rng(32)
    r = rng.standard_normal((B, n, n)).astype(np.float32)
    S = Solver(None, precond="gmg", gmg_levels=levels, gmg_sweeps=sweeps, gmg_omega=omega)
    S.setup(dev(a), b)
    z = S.apply(dev(r)).cpu().numpy()
    for p in range(B):
        G = ogmg.GMG(a[p], b[p], levels=levels, omega=np.float32(omega), sweeps=sweeps)
        assert S.gmg_levels == G.levels
        ref = G.cycle(r[p])
        err = np.abs(z[p] - ref).max() / np.abs(ref).max()
        say("  problem", p, "levels", G.levels, "rel max err", err)
        assert err <= tol, (p, err)
    S.close()


def test_stationary_matches_oracle():
    n, B = 63, 3
    say("gmg stationary", n, B)
    a, b, f = datagen.make_batch("grf31", n, B, seed=33)
    f[1] = 0.0
    S = Solver(None, precond="gmg", state="f32", u="f64", check_every=1)
    S.setup(dev(a), b)
    u = torch.zeros((B, n, n), dtype=torch.float64, device="cuda")
    st, it, rr, ps = S.solve(dev(f), u, 1e-8, 100)
    say("  iters", list(it), "relres", list(rr))
    assert st == M.OK
    assert int(it[1]) == 0 and (u[1] == 0).all()
    for p in (0, 2):
        ou, ost, oit, orho, _ = ogmg.GMG(a[p], b[p], omega=np.float32(0.67)).solve(f[p], 1e-8, 100)
        assert ost == osv.OK
        assert abs(int(it[p]) - oit) <= 1, (p, it[p], oit)
        up = u[p].cpu().numpy()
        assert osv.relres(a[p], b[p], f[p], up) <= 1e-8 * (1 + 1e-6)
        assert_close(up, ou, 1e-6, f"solution {p}")
    S.close()


@pytest.mark.parametrize("n,B,restart,gs", [(255, 3, 30, 2), (127, 4, 63, 1)])
def test_fgmres_blocks_converges(n, B, restart, gs):
    say("gmg fgmres blocks", n, B, restart, gs)
    a, b, f = datagen.make_batch("blocks1023", n, B, seed=34)
    f[B - 1] = 0.0
    S = Solver(None, precond="gmg", u="f64", method="fgmres", restart=restart, gs_passes=gs)
    S.setup(dev(a), b)
    u = torch.full((B, n, n), 0.25, dtype=torch.float64, device="cuda")
    st, it, rr, ps = S.solve(dev(f), u, 1e-8, 1000)
    say("  iters", list(it), "relres", list(rr))
    assert st == M.OK and (ps == 0).all()
    assert int(it[B - 1]) == 0 and (u[B - 1] == 0).all()
    for p in range(B - 1):
        rho = osv.relres(a[p], b[p], f[p], u[p].cpu().numpy())
        assert rho <= 1e-8 * (1 + 1e-6), (p, rho)
    S.close()


def test_fgmres_full_size_64x1023():
    """The benchmark workload (64 problems of 1023^2, random 16 x 16 blocks of contrast 10^4)
    solved to 1e-8 with FGMRES(63) and the GMG preconditioner; the oracle checks the residual
    of four sampled problems."""
    n, B = 1023, 64
    say("gmg fgmres 64 x 1023^2")
    a, b, f = datagen.make_batch("blocks1023", n, B, seed=0)
    S = Solver(None, precond="gmg", u="f64", method="fgmres", restart=63, gs_passes=1)
    S.setup(dev(a), b)
    u = torch.zeros((B, n, n), dtype=torch.float64, device="cuda")
    st, it, rr, ps = S.solve(dev(f), u, 1e-8, 2000)
    say("  iters mean", float(np.mean(it)), "max", int(np.max(it)))
    assert st == M.OK
    for p in (0, 21, 42, 63):
        rho = osv.relres(a[p], b[p], f[p], u[p].cpu().numpy())
        say("  problem", p, "oracle relres", rho)
        assert rho <= 1e-8 * (1 + 1e-6)
    S.close()


def test_group_gmg_matches_individual():
    sizes = [31, 63, 15, 63, 127]
    say("gmg group", sizes)
    ps = [datagen.make_problem("mixture_var", n, i, 35) for i, n in enumerate(sizes)]
    G = GroupSolver(None, precond="gmg", u="f64", method="fgmres", restart=20)
    a = [dev(p.a) for p in ps]
    f = [dev(p.f) for p in ps]
    b = np.stack([p.b for p in ps])
    G.setup(a, b)
    u = [torch.zeros((p.n, p.n), dtype=torch.float64, device="cuda") for p in ps]
    st, it, rr, stat = G.solve(f, u, 1e-8, 500)
    assert st == M.OK
    for i, p in enumerate(ps):
        S = Solver(None, precond="gmg", u="f64", method="fgmres", restart=20)
        S.setup(a[i].view(1, p.n, p.n), b[i:i + 1])
        ui = torch.zeros((1, p.n, p.n), dtype=torch.float64, device="cuda")
        _, it1, rr1, _ = S.solve(f[i].view(1, p.n, p.n), ui, 1e-8, 500)
        S.close()
        assert int(it1[0]) == int(it[i]) and torch.equal(ui[0], u[i]), i
        assert osv.relres(p.a, p.b, p.f, u[i].cpu().numpy()) <= 1e-8 * (1 + 1e-6)
    G.close()


def test_gmg_option_errors():
    say("gmg option errors")
    a, b, f = datagen.make_batch("grf31", 63, 1, seed=36)
    S = Solver(None, precond="gmg", gmg_levels=2)      # coarsest 31 x 31: too large
    with pytest.raises(M.MGCNNError) as e:
        S.setup(dev(a), b)
    assert e.value.status == M.E_ARG
    S.close()
    S = Solver(None, precond="gmg", u="f32")
    S.setup(dev(a), b)
    with pytest.raises(M.MGCNNError) as e:
        S.get_setup_tensor(1)
    assert e.value.status == M.E_STATE
    u = torch.zeros((1, 63, 63), dtype=torch.float32, device="cuda")
    with pytest.raises(M.MGCNNError) as e:
        S.forward(dev(f), u, 2, record=True)
    assert e.value.status == M.E_STATE
    S.forward(dev(f), u, 2)                              # unrecorded iterations are allowed
    rho = osv.relres(a[0], b[0], f[0], u[0].cpu().numpy().astype(np.float64))
    G = ogmg.GMG(a[0], b[0], omega=np.float32(0.67))
    uo = G.correction(G.residual(f[0], np.zeros((63, 63))))
    uo = uo + G.correction(G.residual(f[0], uo))
    assert abs(rho - osv.relres(a[0], b[0], f[0], uo)) <= 1e-3 * rho
    S.close()
    with pytest.raises(M.MGCNNError):
        Solver(None, precond="gmg", gmg_sweeps=5)


def test_graph_replay_matches_eager():
    """Stationary GMG solves with hipGraph-captured blocks of iterations give the same iterates
    as eager launches, bitwise, over several solves (replays with eager work in between)."""
    n, B = 63, 3
    say("gmg graph vs eager")
    a, b, f = datagen.make_batch("grf31", n, B, seed=37)
    Se = Solver(None, precond="gmg", u="f64", check_every=3, use_graph=False)
    Sg = Solver(None, precond="gmg", u="f64", check_every=3, use_graph=True)
    Se.setup(dev(a), b)
    Sg.setup(dev(a), b)
    for rep in range(3):
        ue = torch.zeros((B, n, n), dtype=torch.float64, device="cuda")
        ug = torch.zeros((B, n, n), dtype=torch.float64, device="cuda")
        ste, ite, rre, _ = Se.solve(dev(f), ue, 1e-9, 60)
        stg, itg, rrg, _ = Sg.solve(dev(f), ug, 1e-9, 60)
        assert ste == stg == M.OK
        assert np.array_equal(ite, itg) and np.array_equal(rre, rrg), rep
        assert torch.equal(ue, ug), rep
    Se.close()
    Sg.close()


def test_fgmres_inner_steps():
    """Two GMG cycles per preconditioner application (z = V(v), z += V(v - A z)): still a
    solve to the tolerance, in fewer Arnoldi steps than one cycle.  On smooth coefficients,
    where the stationary GMG iteration contracts; on the 10^4-contrast blocks it diverges, and
    a second cycle then amplifies the divergent modes instead of damping them."""
    n, B = 127, 2
    say("gmg fgmres inner steps")
    a, b, f = datagen.make_batch("grf31", n, B, seed=38)
    its = {}
    for inner in (1, 2):
        S = Solver(None, precond="gmg", u="f64", method="fgmres", restart=30, inner_steps=inner)
        S.setup(dev(a), b)
        u = torch.zeros((B, n, n), dtype=torch.float64, device="cuda")
        st, it, rr, ps = S.solve(dev(f), u, 1e-8, 1000)
        say("  inner", inner, "iters", list(it))
        assert st == M.OK
        for p in range(B):
            assert osv.relres(a[p], b[p], f[p], u[p].cpu().numpy()) <= 1e-8 * (1 + 1e-6)
        its[inner] = int(it.sum())
        S.close()
    assert its[2] < its[1]
