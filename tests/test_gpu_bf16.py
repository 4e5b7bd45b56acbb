"""bf16 state (bf16 storage of the network state, the setup tensors and the 16 -> 16 weights;
products accumulated in f32) against the FP64 oracle, with a bound derived from the arithmetic.

Forward error bound.  One application z = B(r / D) of the solve network is linear in its input
and a sum over paths through the layers (Alg. 3).  In bf16 storage every value on a path is
rounded to 8 significant bits a bounded number of times: each stored state, each s . x product
staged for the matrix cores, the setup tensor s and each weight of a 16 -> 16 convolution, each a
relative perturbation of at most u = 2^-8 (round to nearest).  Along the longest path (down to
the coarsest level and back) there are at most N = 12 L + 3 such roundings (per level and
direction: state, product, s and weight of the smoother, weight and state of the transfer; plus
the reChannel-in state and the f32 input), so by the standard composition of relative errors
|z_bf16 - z| <= gamma_N |B|(|r / D|) element by element, gamma_N = N u / (1 - N u), where |B| is
the same network with every weight and setup tensor replaced by its absolute value (computed by
the oracle).  The f32 accumulation of the products adds at most about 2^-24 per term, far below.

Solves.  With the network trained by the paper's protocol, a stationary solve in bf16 state with
f64 u and residual reaches the tolerance on the oracle's residual, in at most one iteration more
than the f32 state (the refinement of Sec. 2.2, Eq. (1))."""
import os
import sys

import numpy as np
import pytest

import datagen
from oracle import network as onet
from oracle import solve as osv

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2312_11093_amd import Solver  # noqa: E402
from paper_2312_11093_amd import mgcnn as M  # noqa: E402
from paper_2312_11093_amd.weights import embed_channels  # noqa: E402

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TRAINED = os.path.join(ROOT, "paper_2312_11093_amd", "trained", "t5_c8.npy")
U_BF16 = 2.0 ** -8


def say(*a):
    print("[gpu-test]", *a, flush=True)
    sys.stdout.flush()


def dev(x, dtype=torch.float32):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda", dtype)


def abs_bound(O, r):
    """gamma_N |B|(|r / D|) for the oracle solver O (levels O.L)."""
    P = {k: np.abs(v) for k, v in O.P.items()}
    s = [np.abs(x) for x in O.s]
    mag = onet.vcycle(P, s, np.abs(r / O.D))
    N = 12 * O.L + 3
    return N * U_BF16 / (1.0 - N * U_BF16) * mag


@pytest.mark.parametrize("wname,workload,form,n,levels", [
    ("xavier", "mixture127", "div", 31, 0), ("xavier", "mixture127", "div", 63, 0),
    ("trained", "paper_re1e3", "nondiv", 63, -1), ("trained", "paper_re1e3", "nondiv", 127, -1)])
def test_bf16_apply_within_derived_bound(wname, workload, form, n, levels):
    say("bf16 apply vs derived bound", wname, n)
    B = 2
    a, b, f = datagen.make_batch(workload, n, B, seed=4)
    w = (datagen.xavier_weights(16, 5) if wname == "xavier"
         else embed_channels(np.load(TRAINED, allow_pickle=False)))
    r = np.random.default_rng(n).standard_normal((B, n, n)).astype(np.float32)
    S = Solver(w, state="bf16", form=form, levels=levels)
    S.setup(dev(a), b)
    L = S.levels
    z = S.apply(dev(r)).cpu().numpy().astype(np.float64)
    S.close()
    for p in range(B):
        O = osv.Solver(w, a[p], b[p], levels=L, form=form)
        exp = O.correction(r[p].astype(np.float64))
        bound = abs_bound(O, r[p].astype(np.float64))
        err = np.abs(z[p] - exp)
        ratio = float(np.max(err / np.maximum(bound, 1e-300)))
        say(f"  problem {p}: max |err| / bound {ratio:.3e}, max |err| / max |z| "
            f"{float(np.max(err) / np.max(np.abs(exp))):.3e}")
        assert np.all(err <= bound + 1e-6 * np.max(np.abs(exp))), ratio


def test_bf16_state_stationary_solve_with_trained_network():
    """Two 255^2 paper problems to 1e-8: bf16 state with f64 u / residual / norm converges, the
    oracle's f64 residual of the returned solutions is <= tol, and it needs at most one more
    iteration than f32 state."""
    say("bf16 state stationary solve, trained network")
    n, B, tol = 255, 2, 1e-8
    a, b, f = datagen.make_batch("paper_re1e3", n, B, seed=2)
    w = embed_channels(np.load(TRAINED, allow_pickle=False))
    its = {}
    for state in ("f32", "bf16"):
        S = Solver(w, state=state, u="f64", form="nondiv", levels=-1, check_every=1)
        S.setup(dev(a), b)
        u = torch.zeros((B, n, n), dtype=torch.float64, device="cuda")
        st, it, rr, ps = S.solve(dev(f), u, tol, 100)
        S.close()
        say("  ", state, "iters", list(it), "relres", list(rr))
        assert st == M.OK and (ps == 0).all()
        for p in range(B):
            assert osv.relres(a[p], b[p], f[p], u[p].cpu().numpy(), "nondiv") <= tol * (1 + 1e-6)
        its[state] = it
    assert (its["bf16"] <= its["f32"] + 1).all()
