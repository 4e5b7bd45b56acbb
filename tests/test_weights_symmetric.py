"""weights.symmetric_variant builds the adjoint-tied weights of the symmetric variant
(Sec. 3.3): checked element by element against the same construction on the oracle's unpacked
parameters, and by the property it exists for: with up_post the oracle's network is then a
symmetric operator."""
import numpy as np

import datagen
from oracle import network as onet
from oracle import solve as osv
from paper_2312_11093_amd.weights import symmetric_variant


def test_matches_the_oracle_side_construction():
    for C in (4, 16):
        w = datagen.xavier_weights(C, 7)
        P = onet.unpack_weights(w.astype(np.float64), C)
        adj = lambda W: np.flip(W, (2, 3)).transpose(1, 0, 2, 3)
        P["W_up"] = adj(P["W_dn"])
        P["W_T"] = P["W_R"].copy()
        P["W_out"] = adj(P["W_in"])
        exp = onet.pack_weights(P, C).astype(np.float32)
        got = symmetric_variant(w)
        assert got.dtype == np.float32 and got.shape == exp.shape
        assert np.array_equal(got, exp)


def test_the_network_becomes_symmetric():
    n, C = 7, 4
    rng = np.random.default_rng(3)
    a = np.exp(rng.standard_normal((n, n)))
    w = symmetric_variant(datagen.xavier_weights(C, 8)).astype(np.float64)
    S = osv.Solver(w, a, np.zeros(2), up_post=True)
    N = n * n
    M = np.stack([S.pcg_correction(e.reshape(n, n)).ravel() for e in np.eye(N)], axis=1)
    assert np.linalg.norm(M - M.T) <= 1e-12 * np.linalg.norm(M)
