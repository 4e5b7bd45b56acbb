"""The committed trained weights (paper's protocol, Appendix A.1, Table 5; 8 channels): the file
is a plain float32 vector (read with allow_pickle=False), and with the FP64 oracle the network is
a convergent stationary iteration on the paper's test problem (Sec. 4.1), in the iteration range
the paper reports for its 8-channel network (Sec. 4.2, Table 2: 7 at 31 x 31)."""
import os

import numpy as np

import datagen
from oracle import solve as osv

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
WEIGHTS = os.path.join(ROOT, "paper_2312_11093_amd", "trained", "t5_c8.npy")


def test_weights_file():
    w = np.load(WEIGHTS, allow_pickle=False)
    assert w.dtype == np.float32 and w.ndim == 1
    assert w.size == datagen.num_weights(8)
    assert np.all(np.isfinite(w))


def test_oracle_stationary_solve_with_trained_weights():
    w = np.load(WEIGHTS, allow_pickle=False)
    n = 31
    its = []
    for k in range(2):
        p = datagen.make_problem("paper_re1e3", n, k, 0)
        S = osv.Solver(w, p.a, p.b, levels=datagen.levels_for(n) - 1, form="nondiv")
        u, st, it, rho, hist = S.solve(p.f, 1e-8, 60)
        assert st == osv.OK and rho <= 1e-8
        assert osv.relres(p.a, p.b, p.f, u, "nondiv") <= 1e-8
        # every iteration reduces the residual by at least a factor 2 after the first
        assert all(h1 <= 0.5 * h0 for h0, h1 in zip(hist[1:], hist[2:]))
        its.append(it)
    assert max(its) <= 15, its
