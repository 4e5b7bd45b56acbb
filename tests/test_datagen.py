"""Seeded synthetic inputs: determinism, shapes and distribution checks (CPU)."""
import numpy as np
import pytest

import datagen


def test_determinism_and_independence():
    a1, b1, f1 = datagen.make_batch("blocks1023", 63, 3, seed=0)
    a2, b2, f2 = datagen.make_batch("blocks1023", 63, 3, seed=0)
    np.testing.assert_array_equal(a1, a2); np.testing.assert_array_equal(f1, f2)
    assert a1.dtype == np.float32 and b1.shape == (3, 2) and f1.shape == (3, 63, 63)
    assert not np.array_equal(f1[0], f1[1])
    a3, _, _ = datagen.make_batch("blocks1023", 63, 1, seed=1)
    assert not np.array_equal(a1[0], a3[0])
    # a sub-batch starting at problem k reproduces problem k
    a4, b4, f4 = datagen.make_batch("blocks1023", 63, 1, seed=0, first=2)
    np.testing.assert_array_equal(a4[0], a1[2]); np.testing.assert_array_equal(b4[0], b1[2])


def test_grf_covariance():
    """Empirical variance and correlation at distance l of the circulant-embedding
    sampler match the squared-exponential covariance."""
    n, ell, var = 63, 0.1, 2.0
    h = 1.0 / (n + 1)
    rng = np.random.default_rng(0)
    samples = np.stack([datagen.grf(n, rng, ell, var) for _ in range(400)])
    assert samples.var() == pytest.approx(var, rel=0.1)
    lag = int(round(ell / h))
    c = np.mean(samples[:, :, :-lag] * samples[:, :, lag:])
    assert c / var == pytest.approx(np.exp(-0.5 * (lag * h / ell) ** 2), abs=0.08)


def test_coefficient_families():
    n = 127
    rng = np.random.default_rng(1)
    bl = datagen.blocks_lognormal(n, rng)
    assert len(np.unique(bl)) <= 256 and bl.min() >= 1e-2 and bl.max() <= 1e2
    cb = datagen.checkerboard(n, rng)
    assert set(np.unique(cb)) == {1.0, 1e3}
    inc = datagen.inclusions(n, rng)
    assert set(np.unique(inc)) <= {1.0, 1e2} and (inc == 1e2).any()
    b = datagen.velocity(rng, "random")
    assert np.hypot(*b) <= 10
    ml = datagen.mldata(n, rng)
    assert ml.shape == (n, n) and np.isfinite(ml).all()


def test_xavier_bounds():
    C = 16
    w = datagen.xavier_weights(C, 0)
    off = 0
    for name, sh in datagen.weight_shapes(C):
        t = w[off:off + int(np.prod(sh))]
        off += t.size
        if len(sh) == 1:
            assert (t == 0).all()
        else:
            bound = np.sqrt(6.0 / (9 * (sh[0] + sh[1])))
            assert np.abs(t).max() <= bound and np.abs(t).max() > 0.8 * bound


def test_levels():
    assert datagen.levels_for(1023) == 10 and datagen.levels_for(31) == 5
    with pytest.raises(ValueError):
        datagen.levels_for(1000)


def test_var_sizes_seeded_and_in_range():
    s1 = datagen.var_sizes(256, seed=0)
    s2 = datagen.var_sizes(256, seed=0)
    assert s1 == s2 and set(s1) <= set(datagen.VAR_SIZES)
    assert len(set(s1)) == len(datagen.VAR_SIZES)          # 256 draws hit every size
    assert datagen.var_sizes(8, seed=1) != datagen.var_sizes(8, seed=0)


@pytest.mark.parametrize("workload", ["paper_re1e3", "paper_mldata"])
def test_paper_coefficients_span_the_reynolds_range(workload):
    """Sec. 4.1: coef = mu / h spans exactly [1/Re, 1] (the linear map sends the tensor's
    minimum to 1 and its maximum to 1/Re); the paper's velocity and a constant right-hand side."""
    n = 63
    p = datagen.make_problem(workload, n, 0)
    coef = p.a.astype(np.float64) * (n + 1)
    Re = datagen.WORKLOADS[workload].re
    assert np.isclose(coef.max(), 1.0, rtol=1e-6) and np.isclose(coef.min(), 1.0 / Re, rtol=1e-6)
    assert np.allclose(p.b, [np.sin(0.5), np.cos(0.5)]) and (p.f == 1).all()


def test_mldata_levels_and_smoothness():
    """Alg. 4: the doublings stop at the largest 5 * 2^k <= n, and the multi-level field is
    smoother than white noise (neighbouring values correlate strongly)."""
    assert [datagen.mldata_levels(n) for n in (7, 31, 63, 1023)] == [1, 2, 3, 7]
    rng = np.random.default_rng(3)
    ml = datagen.mldata(255, rng, levels=datagen.mldata_levels(255))
    d = ml - ml.mean()
    corr = float((d[:, 1:] * d[:, :-1]).sum() / np.sqrt((d[:, 1:] ** 2).sum() * (d[:, :-1] ** 2).sum()))
    assert corr > 0.9


@pytest.mark.parametrize("workload", sorted(datagen.WORKLOADS))
def test_problems_are_c_contiguous_float32(workload):
    """Every generated field is C-contiguous float32 (the binding takes device copies as is)."""
    if workload in ("grf4095",):
        pytest.skip("large")
    p = datagen.make_problem(workload, 31, 0)
    for x in (p.a, p.b, p.f):
        assert x.dtype == np.float32 and x.flags["C_CONTIGUOUS"]
