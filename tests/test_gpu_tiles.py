"""Tile variants of the 16 -> 16 convolutions (mgcnn_set_tile_variant, autotuning): every
variant computes the same per-pixel sums in the same order, so one application of the network,
a fixed-K forward and the setup tensors are bitwise the same for every variant and storage."""
import sys

import numpy as np
import pytest

import datagen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2312_11093_amd import Solver  # noqa: E402
from paper_2312_11093_amd import autotune as AT  # noqa: E402
from paper_2312_11093_amd import mgcnn as M  # noqa: E402


def say(*a):
    print("[gpu-test]", *a, flush=True)
    sys.stdout.flush()


def dev(x, dtype=torch.float32):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda", dtype)


def set_everything(state, v):
    """Variant v for every operation that has it, the default for the others."""
    for op in ("smoother", "restrict", "smooth_in", "prolong") + (("setup",) if state == "f32" else ()):
        AT.set_all(M.lib(), op, state, v if AT.has_variant(M.lib(), op, state, v) else 0)


@pytest.mark.parametrize("state", ["f32", "bf16"])
def test_tile_variants_are_bitwise_identical(state):
    say("tile variants", state)
    n, B = 127, 2
    a, b, f = datagen.make_batch("mixture127", n, B, seed=12)
    w = datagen.xavier_weights(16, 3)
    r = np.random.default_rng(5).standard_normal((B, n, n)).astype(np.float32)
    outs = []
    try:
        for v in range(AT.VARIANTS):
            set_everything(state, v)
            S = Solver(w, state=state, u="f64")
            S.setup(dev(a), b)
            z = S.apply(dev(r)).cpu()
            s2 = S.get_setup_tensor(2).cpu()
            u = torch.zeros((B, n, n), dtype=torch.float64, device="cuda")
            S.forward(dev(f), u, 2)
            outs.append((z, s2, u.cpu()))
            S.close()
    finally:
        set_everything(state, 0)
    for v in range(1, AT.VARIANTS):
        assert torch.equal(outs[0][0], outs[v][0]), v
        assert torch.equal(outs[0][1], outs[v][1]), v
        assert torch.equal(outs[0][2], outs[v][2]), v
    assert M.lib().mgcnn_tile_variant(0, 0, 127) == 0
