"""A C-channel network (C = 4, 8, 12: the paper's models, Sec. 4.2) embedded into the library's
16 channels by zero padding is the same linear operator: the oracle's setup tensors and network
applications with the C-channel weights and with the embedded weights agree -- CPU only."""
import numpy as np
import pytest

import datagen
from oracle import network as net
from oracle import operator as op
from oracle import solve as sv
from paper_2312_11093_amd.weights import channels_of, embed_channels


@pytest.mark.parametrize("C", [4, 8, 12])
def test_embedded_network_is_the_same_operator(C):
    rng = np.random.default_rng(C)
    w = datagen.xavier_weights(C, C)
    P = net.unpack_weights(w, C)
    for k in range(4):
        P[f"beta_k{k}"] = 0.3 * rng.standard_normal(C)
    w = net.pack_weights(P, C).astype(np.float32)
    w16 = embed_channels(w)
    assert w16.size == 81 * 256 + 58 * 16 and channels_of(w.size) == C
    n = 31
    a, b, _ = datagen.make_batch("mixture127", n, 1, seed=C)
    s_small = net.setup(net.unpack_weights(w, C), op.features(a[0], b[0]), net.num_levels(n))
    s_big = net.setup(net.unpack_weights(w16, 16), op.features(a[0], b[0]), net.num_levels(n))
    for sl, sb in zip(s_small, s_big):
        assert np.allclose(sb[:C], sl, rtol=0, atol=1e-14) and np.all(sb[C:] == 0)
    r = rng.standard_normal((n, n))
    z_small = sv.Solver(w, a[0], b[0]).correction(r)
    z_big = sv.Solver(w16, a[0], b[0]).correction(r)
    assert np.allclose(z_big, z_small, rtol=0, atol=1e-12 * np.abs(z_small).max())


def test_embed_rejects_wrong_sizes():
    with pytest.raises(ValueError):
        embed_channels(np.zeros(100, np.float32))
    with pytest.raises(ValueError):
        embed_channels(np.zeros(81 * 16 + 58 * 4, np.float32), C=5)
