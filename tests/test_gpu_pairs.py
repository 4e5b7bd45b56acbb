"""GPU: packed pairs (opts.pack_pairs) for networks of at most 8 hidden channels.  Two problems
share one 16-channel state slot with block-diagonal 16 -> 16 weights; per problem the network
must stay the C-channel network of the oracle (the same operator as its zero-padded 16-channel
form), including the empty half of an odd batch's last slot.  f32 state is held to the f32
tolerance element by element; solves are checked on the oracle's residual and against the
unpacked library's iteration counts."""
import os
import sys

import numpy as np
import pytest

import datagen
from oracle import network as onet
from oracle import solve as osv
from parity_util import assert_close

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2312_11093_amd import Solver  # noqa: E402
from paper_2312_11093_amd import mgcnn as M  # noqa: E402
from paper_2312_11093_amd.weights import embed_channels  # noqa: E402

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TRAINED = os.path.join(ROOT, "paper_2312_11093_amd", "trained", "t5_c8.npy")
F32_TOL = 1e-5
SPLIT2_TOL = 1e-4
U_BF16 = 2.0 ** -8


def say(*a):
    print("[gpu-test]", *a, flush=True)
    sys.stdout.flush()


def dev(x, dtype=torch.float32):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda", dtype)


def weights(kind):
    if kind == "xavier8":
        return embed_channels(datagen.xavier_weights(8, 2))
    if kind == "xavier4":
        return embed_channels(datagen.xavier_weights(4, 3))
    return embed_channels(np.load(TRAINED, allow_pickle=False))


@pytest.mark.parametrize("kind,workload,form,levels", [
    ("xavier8", "mixture127", "div", 0), ("xavier4", "mixture127", "div", 0),
    ("trained", "paper_re1e3", "nondiv", -1)])
@pytest.mark.parametrize("n,B", [(15, 3), (63, 4), (127, 5)])
@pytest.mark.parametrize("split", [0, 1, 2])
def test_pairs_apply_matches_oracle(kind, workload, form, levels, n, B, split):
    """z = B(r / D) per problem with packed pairs against the oracle (f32 state: f32 matrix
    instructions, the three-way split, the two-way split in the finest down smoother)."""
    say("pairs apply", kind, n, B, "split", split)
    w = weights(kind)
    a, b, f = datagen.make_batch(workload, n, B, seed=7)
    r = np.random.default_rng(n + B).standard_normal((B, n, n)).astype(np.float32)
    S = Solver(w, state="f32", f32_split=split, form=form, levels=levels, pack_pairs=True)
    S.setup(dev(a), b)
    L = S.levels
    z = S.apply(dev(r)).cpu().numpy()
    S.close()
    tol = SPLIT2_TOL if split == 2 else F32_TOL
    for p in range(B):
        exp = osv.Solver(w, a[p], b[p], levels=L, form=form).correction(r[p].astype(np.float64))
        assert_close(z[p], exp, tol, f"problem {p}", say)


@pytest.mark.parametrize("n,B", [(63, 3), (127, 4)])
def test_pairs_bf16_apply_within_derived_bound(n, B):
    """bf16 state in packed pairs: per problem, |z - z_oracle| <= gamma_N |B|(|r / D|) element by
    element, with N = 12 L + 3 bf16 roundings along the longest path and u = 2^-8 (the bound of
    the unpacked bf16 test; |B| is the oracle's network with every weight and setup tensor
    replaced by its absolute value)."""
    say("pairs bf16 apply vs derived bound", n, B)
    w = weights("trained")
    a, b, f = datagen.make_batch("paper_re1e3", n, B, seed=5)
    r = np.random.default_rng(3 * n + B).standard_normal((B, n, n)).astype(np.float32)
    S = Solver(w, state="bf16", form="nondiv", levels=-1, pack_pairs=True)
    S.setup(dev(a), b)
    L = S.levels
    z = S.apply(dev(r)).cpu().numpy().astype(np.float64)
    S.close()
    for p in range(B):
        O = osv.Solver(w, a[p], b[p], levels=L, form="nondiv")
        rp = r[p].astype(np.float64)
        exp = O.correction(rp)
        mag = onet.vcycle({k: np.abs(v) for k, v in O.P.items()}, [np.abs(x) for x in O.s], np.abs(rp / O.D))
        N = 12 * O.L + 3
        bound = N * U_BF16 / (1.0 - N * U_BF16) * mag
        err = np.abs(z[p] - exp)
        say(f"  problem {p}: max |err| / bound {float(np.max(err / np.maximum(bound, 1e-300))):.3e}")
        assert np.all(err <= bound + 1e-6 * np.max(np.abs(exp)))


@pytest.mark.parametrize("state,udt", [("f32", "f64"), ("bf16", "f64"), ("f32", "f32"), ("bf16", "f32")])
def test_pairs_forward_matches_unpacked(state, udt):
    """Three fixed iterations u += B((f - A u) / D) on a ragged batch (odd B, n = 127), u in f64 and
    in f32: the packed library against the unpacked one with the same weights, per problem.  The two add the same
    products in another order on the matrix cores (the other problem's weights are exact zeros
    in the block-diagonal convs).  f32: the f32 tolerance.  bf16: an ulp of difference in an f32
    sum can flip the bf16 rounding of a stored value (2^-8 relative) that later layers carry;
    1e-2 of the largest value bounds a few such flips."""
    say("pairs forward vs unpacked", state, "u", udt)
    n, B, K = 127, 5, 3
    w = weights("trained")
    a, b, f = datagen.make_batch("paper_re1e3", n, B, seed=11)
    out = {}
    for pack in (False, True):
        S = Solver(w, state=state, u=udt, form="nondiv", levels=-1, pack_pairs=pack)
        S.setup(dev(a), b)
        u = torch.zeros((B, n, n), dtype=S.u_dtype, device="cuda")
        S.forward(dev(f), u, K)
        out[pack] = u.cpu().numpy().astype(np.float64)
        S.close()
    tol = F32_TOL if state == "f32" else 1e-2
    for p in range(B):
        assert_close(out[True][p], out[False][p], tol, f"problem {p}", say)


@pytest.mark.parametrize("state,graph", [("f32", False), ("f32", True), ("bf16", True)])
def test_pairs_solve_paper_problems(state, graph):
    """Stationary solves of five 63^2 paper problems (odd batch, one with f = 0) to 1e-8 with the
    trained network: the oracle's f64 residual of every returned solution is <= tol, u = 0 for
    the zero right-hand side, and the iteration counts are those of the unpacked library within
    one (the summation order of the block-diagonal products differs)."""
    say("pairs solve", state, "graph" if graph else "eager")
    n, B, tol = 63, 5, 1e-8
    w = weights("trained")
    a, b, f = datagen.make_batch("paper_re1e3", n, B, seed=3)
    f[3] = 0.0
    its = {}
    for pack in (False, True):
        S = Solver(w, state=state, u="f64", form="nondiv", levels=-1, use_graph=graph, check_every=1,
                   pack_pairs=pack)
        S.setup(dev(a), b)
        u = torch.zeros((B, n, n), dtype=torch.float64, device="cuda")
        st, it, rr, ps = S.solve(dev(f), u, tol, 100)
        S.close()
        say("  pack" if pack else "  unpacked", "iters", list(map(int, it)))
        assert st == M.OK and (ps == 0).all()
        un = u.cpu().numpy()
        for p in range(B):
            if p == 3:
                assert not un[p].any() and int(it[p]) == 0
                continue
            assert osv.relres(a[p], b[p], f[p], un[p], "nondiv") <= tol * (1 + 1e-6)
        its[pack] = np.asarray(it)
    assert (np.abs(its[True] - its[False]) <= 1).all()


def test_pairs_reject_wider_networks_and_training():
    """A network that uses channels 8..15 cannot be packed (E_ARG when the weights are set);
    the recorded forward and the setup-tensor read-out report E_STATE."""
    say("pairs rejections")
    with pytest.raises(M.MGCNNError) as e:
        Solver(datagen.xavier_weights(16, 0), pack_pairs=True)
    assert e.value.status == M.E_ARG
    n, B = 15, 2
    a, b, f = datagen.make_batch("mixture127", n, B, seed=1)
    S = Solver(weights("xavier8"), state="f32", u="f32", pack_pairs=True)
    S.setup(dev(a), b)
    u = torch.zeros((B, n, n), dtype=torch.float32, device="cuda")
    with pytest.raises(M.MGCNNError) as e:
        S.forward(dev(f), u, 1, record=True)
    assert e.value.status == M.E_STATE
    with pytest.raises(M.MGCNNError) as e:
        S.get_setup_tensor(1)
    assert e.value.status == M.E_STATE
    S.close()


@pytest.mark.parametrize("state", ["f32", "bf16"])
def test_pairs_group_on_aligned_levels(state):
    """Uneven sizes in one group call with packed pairs: every size group of odd count gets a
    phantom partner, so that pairs never mix sizes.  Nine paper problems (three of 127^2, one
    each of 15^2 and 7^2, one with f = 0) solved to 1e-8 with the trained network: the oracle's
    residual of every returned solution is <= tol, u = 0 for the zero right-hand side, the
    iteration counts are those of the unpacked group within one, and the device completion times
    are positive for the problems that iterated."""
    from paper_2312_11093_amd import GroupSolver
    sizes = [31, 127, 15, 63, 127, 7, 31, 63, 127]
    say("pairs group", state, sizes)
    ps = [datagen.make_problem("paper_re1e3", n, i, 8) for i, n in enumerate(sizes)]
    ps[4].f[:] = 0.0
    w = weights("trained")
    a = [dev(p.a) for p in ps]
    f = [dev(p.f) for p in ps]
    b = np.stack([p.b for p in ps])
    its = {}
    for pack in (False, True):
        G = GroupSolver(w, state=state, u="f64", method="stationary", check_every=2, levels=-1, form="nondiv",
                        use_graph=True, pack_pairs=pack)
        assert G.aligned
        G.setup(a, b)
        u = [torch.zeros((p.n, p.n), dtype=torch.float64, device="cuda") for p in ps]
        st, it, rr, stat = G.solve(f, u, 1e-8, 60)
        ct = G.completion_times()
        G.close()
        say("  pack" if pack else "  unpacked", "iters", list(map(int, it)))
        assert st == M.OK and (stat == 0).all()
        for i, p in enumerate(ps):
            x = u[i].cpu().numpy()
            if i == 4:
                assert not x.any() and int(it[i]) == 0 and ct[i] == 0.0
                continue
            assert osv.relres(p.a, p.b, p.f, x, "nondiv") <= 1e-8 * (1 + 1e-6), i
            assert ct[i] > 0.0
        its[pack] = np.asarray(it)
    assert (np.abs(its[True] - its[False]) <= 1).all()


def test_pairs_full_size_paper_batch_sampled():
    """The benchmark's packed-pair launch at its real size: 64 paper problems at 1023^2 (32 state
    slots), f32 state with the two-way split in the finest down smoother, one application of the
    trained network to a random residual.  Both halves of the first and the last slot (problems
    0, 1, 62, 63) against the oracle element by element (the two-way split's tolerance)."""
    n, B = 1023, 64
    say("pairs full size", n, B)
    w = weights("trained")
    a, b, _ = datagen.make_batch("paper_re1e3", n, B, seed=2)
    r = np.random.default_rng(17).standard_normal((B, n, n)).astype(np.float32)
    S = Solver(w, state="f32", f32_split=2, form="nondiv", levels=-1, pack_pairs=True)
    S.setup(dev(a), b)
    L = S.levels
    z = S.apply(dev(r))
    picks = [0, 1, B - 2, B - 1]
    got = {p: z[p].cpu().numpy() for p in picks}
    S.close()
    del z
    for p in picks:
        exp = osv.Solver(w, a[p], b[p], levels=L, form="nondiv").correction(r[p].astype(np.float64))
        assert_close(got[p], exp, SPLIT2_TOL, f"problem {p}", say)


def test_pairs_uneven_full_sizes_converge():
    """Uneven sizes at their real range (63..2047) in one group call with packed pairs and bf16
    state: 24 paper problems solved to 1e-8 by the stationary iteration with the trained
    network; every problem converges, and the oracle's residual of one problem of each size is
    <= tol."""
    from paper_2312_11093_amd import GroupSolver
    sizes = datagen.var_sizes(24, seed=1, workload="paper_re1e3")
    say("pairs uneven full sizes", sizes)
    ps = [datagen.make_problem("paper_re1e3", n, i, 4) for i, n in enumerate(sizes)]
    G = GroupSolver(weights("trained"), state="bf16", u="f64", method="stationary", check_every=2,
                    levels=-1, form="nondiv", use_graph=True, pack_pairs=True)
    assert G.aligned
    G.setup([dev(p.a) for p in ps], np.stack([p.b for p in ps]))
    u = [torch.zeros((p.n, p.n), dtype=torch.float64, device="cuda") for p in ps]
    st, it, rr, stat = G.solve([dev(p.f) for p in ps], u, 1e-8, 60)
    G.close()
    say("  iters", list(map(int, it)))
    assert st == M.OK and (stat == 0).all()
    for n in sorted(set(sizes)):
        i = sizes.index(n)
        rho = osv.relres(ps[i].a, ps[i].b, ps[i].f, u[i].cpu().numpy(), "nondiv")
        say("  n", n, "oracle relres", rho)
        assert rho <= 1e-8 * (1 + 1e-6)


@pytest.mark.parametrize("sizes", [[63], [7, 15, 31, 63], [31, 31]])
def test_pairs_group_edge_layouts(sizes):
    """Pair groups whose every size group needs a phantom partner (one problem; four distinct
    sizes) and one without any (two problems of one size): bf16 state, the trained network, every
    problem to 1e-8 on the oracle's residual, iteration counts of the unpacked group within one."""
    from paper_2312_11093_amd import GroupSolver
    say("pairs group edge layout", sizes)
    ps = [datagen.make_problem("paper_re1e3", n, i, 12) for i, n in enumerate(sizes)]
    w = weights("trained")
    its = {}
    for pack in (False, True):
        G = GroupSolver(w, state="bf16", u="f64", method="stationary", check_every=1, levels=-1, form="nondiv",
                        use_graph=True, pack_pairs=pack)
        assert G.aligned
        G.setup([dev(p.a) for p in ps], np.stack([p.b for p in ps]))
        u = [torch.zeros((p.n, p.n), dtype=torch.float64, device="cuda") for p in ps]
        st, it, rr, stat = G.solve([dev(p.f) for p in ps], u, 1e-8, 60)
        G.close()
        assert st == M.OK and (stat == 0).all()
        for i, p in enumerate(ps):
            assert osv.relres(p.a, p.b, p.f, u[i].cpu().numpy(), "nondiv") <= 1e-8 * (1 + 1e-6), (pack, i)
        its[pack] = np.asarray(it)
    say("  iters", list(map(int, its[False])), list(map(int, its[True])))
    assert (np.abs(its[True] - its[False]) <= 1).all()


def test_pairs_largest_grid_solve():
    """Packed pairs at the largest grid (two 4095^2 paper problems in one state slot, bf16 state,
    the paper's level count) solved to 1e-10: the oracle's residual of both solutions <= tol and
    the unpacked library's iteration counts within one."""
    n, B, tol = 4095, 2, 1e-10
    say("pairs 4095^2 x 2 to", tol)
    w = weights("trained")
    a, b, f = datagen.make_batch("paper_re1e3", n, B, seed=13)
    its = {}
    for pack in (False, True):
        S = Solver(w, state="bf16", u="f64", form="nondiv", levels=-1, use_graph=True, check_every=1,
                   pack_pairs=pack)
        S.setup(dev(a), b)
        u = torch.zeros((B, n, n), dtype=torch.float64, device="cuda")
        st, it, rr, ps = S.solve(dev(f), u, tol, 100)
        S.close()
        assert st == M.OK and (ps == 0).all()
        un = u.cpu().numpy()
        del u
        for p in range(B):
            rho = osv.relres(a[p], b[p], f[p], un[p], "nondiv")
            say("  pack" if pack else "  unpacked", "problem", p, "iters", int(it[p]), "oracle relres", rho)
            assert rho <= tol * (1 + 1e-6)
        its[pack] = np.asarray(it)
    assert (np.abs(its[True] - its[False]) <= 1).all()
