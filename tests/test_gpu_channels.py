"""GPU: the paper's 4-, 8- and 12-channel networks (Sec. 4.2) run through the 16-channel
library by zero-padded weights (paper_2312_11093_amd.weights.embed_channels), against the FP64
oracle evaluated with the C-channel weights themselves: setup tensors (extra channels exactly
zero), one network application and K = 3 stationary iterations."""
import sys

import numpy as np
import pytest

import datagen
from parity_util import assert_close
from oracle import network as onet
from oracle import operator as oop
from oracle import solve as osv

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2312_11093_amd import Solver  # noqa: E402
from paper_2312_11093_amd.weights import embed_channels  # noqa: E402


def say(*a):
    print("[gpu-test]", *a, flush=True)
    sys.stdout.flush()


def dev(x, dtype=torch.float32):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda", dtype)


def small_weights(C):
    rng = np.random.default_rng(40 + C)
    P = onet.unpack_weights(datagen.xavier_weights(C, C), C)
    for k in range(4):
        P[f"beta_k{k}"] = 0.2 * rng.standard_normal(C)
    return onet.pack_weights(P, C).astype(np.float32)


@pytest.mark.parametrize("C", [4, 8, 12])
def test_small_network_through_the_library(C):
    n, B, K = 63, 2, 3
    say("channels", C, n, B)
    a, b, f = datagen.make_batch("mixture127", n, B, seed=41)
    w = small_weights(C)
    S = Solver(embed_channels(w), state="f32", u="f64")
    S.setup(dev(a), b)
    r = np.random.default_rng(42).standard_normal((B, n, n)).astype(np.float32)
    z = S.apply(dev(r)).cpu().numpy()
    u = torch.zeros((B, n, n), dtype=torch.float64, device="cuda")
    S.forward(dev(f), u, K)
    for p in range(B):
        O = osv.Solver(w, a[p], b[p])
        s_ref = onet.setup(O.P, oop.features(a[p], b[p]), onet.num_levels(n))
        for lvl in (1, 3):
            sg = S.get_setup_tensor(lvl).cpu().numpy()[p]          # [m][m][16]
            assert np.all(sg[..., C:] == 0)
            ref = np.moveaxis(s_ref[lvl - 1], 0, -1)
            assert np.max(np.abs(sg[..., :C] - ref)) <= 1e-5 * np.max(np.abs(ref))
        zr = O.correction(r[p].astype(np.float64))
        ez = np.max(np.abs(z[p] - zr)) / np.max(np.abs(zr))
        ur = O.forward(f[p], K)
        say("  problem", p, "apply err", ez)
        assert ez <= 1e-5
        assert_close(u[p].cpu().numpy(), ur, 1e-5, "forward", say)
    S.close()
