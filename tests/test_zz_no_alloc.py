"""mgcnn_residual_norms_noalloc (no context, no device allocation: its scratch memory is one
fixed device array) against the context entry point mgcnn_residual_norms on the same inputs:
bit-for-bit equal (same kernels), and within 1e-12 of the oracle's f64 relative residual.  Two
calls in a row, the second with a smaller input, so the second reads a scratch array that still
holds the first call's larger contents."""
import sys

import numpy as np
import pytest

import datagen
from oracle import solve as osv

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2312_11093_amd import Solver  # noqa: E402
from paper_2312_11093_amd import mgcnn as M  # noqa: E402


def say(*a):
    print("[gpu-test]", *a, flush=True)
    sys.stdout.flush()


def dev(x, dtype=torch.float32):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda", dtype)


def case(workload, n, B, seed, udt, form):
    a, b, f = datagen.make_batch(workload, n, B, seed=seed)
    rng = np.random.default_rng(seed)
    u = rng.standard_normal((B, n, n)) * 1e-3
    f[B - 1] = 0.0 if B > 2 else f[B - 1]        # a zero right-hand side gives 0
    S = Solver(datagen.xavier_weights(16, 0), u=udt, form=form)
    S.setup(dev(a), b)
    ud = dev(u, S.u_dtype)
    fd = dev(f)
    ref = S.residual_norms(fd, ud)
    S.close()
    got = M.residual_norms_noalloc(dev(a), b, fd, ud, form=form)
    say(f"  {workload} n={n} B={B} u={udt} form={form}: noalloc {got[:2]} ctx {ref[:2]}")
    assert np.array_equal(got, ref)
    for p in range(B):
        if not f[p].any():
            assert got[p] == 0.0
            continue
        uu = u[p] if udt == "f64" else u[p].astype(np.float32).astype(np.float64)
        exp = osv.relres(a[p], b[p], f[p], uu, form)
        tol = 1e-12 if udt == "f64" else 1e-5
        assert abs(got[p] - exp) <= tol * max(exp, 1e-300), (p, got[p], exp)


def test_noalloc_matches_context_entry_point_twice_shrinking():
    say("noalloc residual norms: 127 x 5 then 31 x 2")
    case("mixture127", 127, 5, 3, "f64", "div")
    case("grf31", 31, 2, 4, "f64", "div")


def test_noalloc_f32_u_and_nondiv_form():
    say("noalloc residual norms: f32 u, non-divergence form")
    case("paper_re1e3", 63, 3, 5, "f32", "nondiv")
    case("paper_re1e3", 15, 1, 6, "f64", "nondiv")


def test_noalloc_rejects_oversize_before_launch():
    say("noalloc scratch bound")
    n, B = 4095, 200
    stand = torch.zeros((1, 3, 3), dtype=torch.float32, device="cuda")
    L = M.lib()
    out = np.zeros(B)
    bh = np.ones((B, 2), np.float32)
    st = L.mgcnn_residual_norms_noalloc(stand.data_ptr(), bh.ctypes.data, n, B, 0, stand.data_ptr(),
                                        stand.data_ptr(), 1, out.ctypes.data, None)
    assert st == M.E_SCRATCH
