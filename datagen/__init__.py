"""Seeded synthetic inputs for the MGCNN solver: coefficient fields, velocities,
right-hand sides and initial weights.

This module is shared by the FP64 oracle and by the GPU path.  It holds random
number generation and geometry only, none of the solver's arithmetic: it never
builds the operator, the stencil, the setup network or the V-cycle.

Everything is drawn on the host in float64 and rounded to float32 exactly once,
so both sides consume identical float32 values.

Seeding: one ``numpy.random.Generator(PCG64(SeedSequence([seed, workload,
problem, stream])))`` per (problem, stream), stream 0 = diffusion coefficient
``a``, 1 = velocity ``b``, 2 = right-hand side ``f``.  Weights use their own
sequence ``SeedSequence([seed, WEIGHT_STREAM])``.

Grid convention: ``n`` interior points per side on the unit square,
``h = 1/(n+1)``, node ``(i, j)`` sits at ``x = (j+1) h``, ``y = (i+1) h``;
arrays are ``[i][j]`` (row = y, column = x).

The coefficient families follow the workloads this implementation is measured on:
lognormal Gaussian random fields, random block partitions, checkerboards and
circular inclusions; plus the paper's own test problems (Sec. 4.1 "Problem
settings"): white-noise coefficients mapped log-uniformly onto [1/Re, 1], velocity
(sin 0.5, cos 0.5), right-hand side 1, for the non-divergence operator.  The
paper's image datasets (Sec. 4.3) are not reproduced.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = [
    "rng_for", "grf", "blocks_lognormal", "checkerboard", "inclusions",
    "mixture", "velocity", "rhs", "mldata", "weight_shapes", "num_weights",
    "xavier_weights", "Problem", "make_batch", "WORKLOADS", "levels_for", "var_sizes", "VAR_SIZES",
    "white_noise_coef", "coef_from_tensor", "mldata_levels", "mldata_coef",
]

WEIGHT_STREAM = 0x5EED
STREAM_A, STREAM_B, STREAM_F, STREAM_N = 0, 1, 2, 3
VAR_SIZES = (63, 127, 255, 511, 1023, 2047)


def rng_for(seed: int, workload: int, problem: int, stream: int) -> np.random.Generator:
    """Counter-style generator for one (workload, problem, stream) triple."""
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, workload, problem, stream])))


def levels_for(n: int) -> int:
    """Number of grid levels for n = 2^L - 1 interior points (coarsest grid 1x1)."""
    L = int(round(math.log2(n + 1)))
    if (1 << L) - 1 != n:
        raise ValueError(f"n={n} is not of the form 2^L - 1")
    return L


# ----------------------------------------------------------------------------------------------
# coefficient fields a(x, y) > 0 on the n x n interior nodes
# ----------------------------------------------------------------------------------------------

def grf(n: int, rng: np.random.Generator, length: float, variance: float) -> np.ndarray:
    """Stationary Gaussian random field with squared-exponential covariance
    ``variance * exp(-r^2 / (2 length^2))`` sampled at the interior nodes.

    Circulant embedding on a periodic square of physical side 2 (M = 2(n+1)
    points per side, spacing h): eigenvalues of the block-circulant covariance
    are the 2-D FFT of its first row, negative ones (round-off) are clamped to
    zero, and the real part of ``fft2(sqrt(lambda) * xi) / M`` with complex
    standard normal ``xi`` has exactly the embedded covariance.
    """
    h = 1.0 / (n + 1)
    M = 2 * (n + 1)
    k = np.arange(M)
    d = np.minimum(k, M - k) * h                      # periodic distance along one axis
    c = variance * np.exp(-(d[:, None] ** 2 + d[None, :] ** 2) / (2.0 * length * length))
    lam = np.fft.fft2(c).real
    lam = np.maximum(lam, 0.0)
    xi = rng.standard_normal((M, M)) + 1j * rng.standard_normal((M, M))
    field = np.fft.fft2(np.sqrt(lam) * xi).real / M
    return field[:n, :n].copy()


def blocks_lognormal(n: int, rng: np.random.Generator, nblocks: int = 16,
                     log10_lo: float = -2.0, log10_hi: float = 2.0) -> np.ndarray:
    """Piecewise-constant field on an equal ``nblocks x nblocks`` partition;
    ``log10 a`` is uniform on ``[log10_lo, log10_hi]`` per block."""
    e = rng.uniform(log10_lo, log10_hi, size=(nblocks, nblocks))
    bi = (np.arange(n) * nblocks) // n
    return 10.0 ** e[bi[:, None], bi[None, :]]


def checkerboard(n: int, rng: np.random.Generator, cells: int = 8, contrast: float = 1e3) -> np.ndarray:
    """``cells x cells`` checkerboard with values {1, contrast}; the colour of the
    first cell is a fair coin."""
    phase = int(rng.integers(2))
    ci = (np.arange(n) * cells) // n
    par = (ci[:, None] + ci[None, :] + phase) % 2
    return np.where(par == 0, contrast, 1.0)


def inclusions(n: int, rng: np.random.Generator, count: int = 20, r_lo: float = 0.02,
               r_hi: float = 0.08, inside: float = 1e2) -> np.ndarray:
    """``count`` discs with centres uniform on the unit square and radii uniform
    on ``[r_lo, r_hi]`` (overlap allowed); a = ``inside`` in any disc, 1 elsewhere."""
    h = 1.0 / (n + 1)
    cx = rng.uniform(0.0, 1.0, count)
    cy = rng.uniform(0.0, 1.0, count)
    r = rng.uniform(r_lo, r_hi, count)
    x = (np.arange(n) + 1) * h
    a = np.ones((n, n))
    for k in range(count):
        mask = (x[None, :] - cx[k]) ** 2 + (x[:, None] - cy[k]) ** 2 <= r[k] ** 2
        a[mask] = inside
    return a


def mixture(n: int, rng: np.random.Generator) -> np.ndarray:
    """One of {lognormal GRF (length 0.1, variance 1), checkerboard 8x8 / 1e3,
    20 inclusions / 1e2}, chosen uniformly."""
    kind = int(rng.integers(3))
    if kind == 0:
        return np.exp(grf(n, rng, 0.1, 1.0))
    if kind == 1:
        return checkerboard(n, rng)
    return inclusions(n, rng)


def mldata(n: int, rng: np.random.Generator, levels: int = 4, init_size: int = 5) -> np.ndarray:
    """Multi-level random data (Appendix B.3, Alg. 4): white noise of side
    ``init_size``, repeatedly doubled by bilinear interpolation with added noise of
    amplitude 2^-i, finally interpolated to ``n x n``."""
    def interp(d, m):
        s = d.shape[0]
        t = np.linspace(0.0, s - 1.0, m)
        i0 = np.clip(np.floor(t).astype(int), 0, s - 2)
        w = t - i0
        rows = d[i0] * (1 - w)[:, None] + d[i0 + 1] * w[:, None]
        return rows[:, i0] * (1 - w)[None, :] + rows[:, i0 + 1] * w[None, :]
    d = rng.standard_normal((init_size, init_size))
    for i in range(1, levels + 1):
        d = interp(d, 2 * d.shape[0])
        d = d + 2.0 ** (-i) * rng.standard_normal(d.shape)
    return interp(d, n)


def coef_from_tensor(w: np.ndarray, Re: float) -> np.ndarray:
    """Sec. 4.1 "Problem settings": a random tensor mapped linearly onto [0, log10 Re] as a
    power p, then coef = 10^-p, so the mesh Reynolds number 1/coef spans [1, Re].  coef = mu / h
    is the diffusion coefficient in units of the mesh size; the returned field is
    mu = coef * h, the coefficient of the physically scaled operator, whose rows are the
    paper's (Eq. (8)) times 1/h."""
    n = w.shape[0]
    p = math.log10(Re) * (w - w.min()) / (w.max() - w.min())
    return 10.0 ** (-p) / (n + 1)


def white_noise_coef(n: int, rng: np.random.Generator, Re: float) -> np.ndarray:
    """The paper's test coefficients: white noise (i.i.d. N(0, 1)) through coef_from_tensor."""
    return coef_from_tensor(rng.standard_normal((n, n)), Re)


def mldata_levels(n: int, init_size: int = 5) -> int:
    """Doublings of Alg. 4 for a target side n: the most that keep init_size * 2^levels <= n,
    at least 1 (the noise then reaches down to the scale of a few mesh cells)."""
    levels = 0
    while init_size * 2 ** (levels + 1) <= n:
        levels += 1
    return max(1, levels)


def mldata_coef(n: int, rng: np.random.Generator, Re: float) -> np.ndarray:
    """The paper's "mldata" coefficients (Sec. 4.3, Alg. 4 with init_size 5) through
    coef_from_tensor."""
    return coef_from_tensor(mldata(n, rng, levels=mldata_levels(n)), Re)


def velocity(rng: np.random.Generator, kind: str) -> np.ndarray:
    """Constant convection velocity b = (bx, by): ``"unit"`` gives (1, 1);
    ``"random"`` gives |b| (cos t, sin t) with t ~ U(0, 2 pi), |b| ~ U(0, 10);
    ``"paper"`` gives the unit vector (sin 0.5, cos 0.5) of Sec. 4.1."""
    if kind == "unit":
        return np.array([1.0, 1.0])
    if kind == "paper":
        return np.array([math.sin(0.5), math.cos(0.5)])
    theta = rng.uniform(0.0, 2.0 * math.pi)
    mag = rng.uniform(0.0, 10.0)
    return np.array([mag * math.cos(theta), mag * math.sin(theta)])


def rhs(n: int, rng: np.random.Generator, kind: str) -> np.ndarray:
    """Right-hand side: ``"uniform"`` = U(-1, 1) i.i.d., ``"normal"`` = N(0, 1) i.i.d.,
    ``"ones"`` = constant 1 (the paper's test right-hand side, Sec. 4.1)."""
    if kind == "uniform":
        return rng.uniform(-1.0, 1.0, (n, n))
    if kind == "normal":
        return rng.standard_normal((n, n))
    if kind == "ones":
        return np.ones((n, n))
    raise ValueError(kind)


# ----------------------------------------------------------------------------------------------
# weights: flat float32 vector in the fixed parameter order of the network
# ----------------------------------------------------------------------------------------------

def weight_shapes(C: int) -> list[tuple[str, tuple[int, ...]]]:
    """Parameter order of the flat weight vector (float32, C-order per tensor):
    setup reChannel (C,4,3,3); four setup ResNet layers, each a conv (C,C,3,3)
    followed by its bias (C,); setup restriction (C,C,3,3); solve reChannel-in
    (C,1,3,3); down smoother, up smoother, restriction (C,C,3,3) each;
    transposed-conv prolongation (C_in=C, C_out=C, 3, 3); reChannel-out (1,C,3,3)."""
    s = [("setup_in", (C, 4, 3, 3))]
    for k in range(4):
        s += [(f"setup_res{k}_w", (C, C, 3, 3)), (f"setup_res{k}_b", (C,))]
    s += [("setup_restrict", (C, C, 3, 3)), ("solve_in", (C, 1, 3, 3)),
          ("smooth_down", (C, C, 3, 3)), ("smooth_up", (C, C, 3, 3)),
          ("restrict", (C, C, 3, 3)), ("prolong", (C, C, 3, 3)), ("solve_out", (1, C, 3, 3))]
    return s


def num_weights(C: int) -> int:
    return sum(int(np.prod(sh)) for _, sh in weight_shapes(C))


def xavier_weights(C: int = 16, seed: int = 0) -> np.ndarray:
    """Xavier-uniform (gain 1) conv weights, bound sqrt(6 / (9 C_in + 9 C_out)),
    zero biases; drawn tensor by tensor in parameter order.  Returns float32."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, WEIGHT_STREAM])))
    out = []
    for name, sh in weight_shapes(C):
        if len(sh) == 1:
            out.append(np.zeros(sh))
            continue
        fan = 9 * (sh[0] + sh[1])
        bound = math.sqrt(6.0 / fan)
        out.append(rng.uniform(-bound, bound, sh))
    return np.concatenate([t.ravel() for t in out]).astype(np.float32)


# ----------------------------------------------------------------------------------------------
# named workloads
# ----------------------------------------------------------------------------------------------

@dataclass(frozen=True)
class Workload:
    name: str
    wid: int
    coef: str          # "grf", "blocks", "mixture"
    grf_length: float
    grf_variance: float
    vel: str           # "unit" | "random" | "paper"
    f_kind: str        # "uniform" | "normal" | "ones"
    re: float = 0.0    # "white" coefficients: the range limit Re of the mesh Reynolds number
    form: str = "div"  # operator the workload is posed for: "div" or "nondiv"


WORKLOADS = {
    # single 31x31 problem, lognormal GRF (length 0.1, variance 1), b = (1,1), f ~ U(-1,1)
    "grf31": Workload("grf31", 1, "grf", 0.1, 1.0, "unit", "uniform"),
    # batched 1023x1023, 16x16 random blocks with log10 a ~ U(-2,2), random b, f ~ N(0,1)
    "blocks1023": Workload("blocks1023", 2, "blocks", 0.0, 0.0, "random", "normal"),
    # single 4095x4095, lognormal GRF (length 0.05, variance 2), b = (1,1), f ~ U(-1,1)
    "grf4095": Workload("grf4095", 3, "grf", 0.05, 2.0, "unit", "uniform"),
    # training mixture at 127x127: GRF / checkerboard / inclusions, random b, f ~ N(0,1)
    "mixture127": Workload("mixture127", 4, "mixture", 0.1, 1.0, "random", "normal"),
    # uneven-size mixture (sizes 63..2047)
    "mixture_var": Workload("mixture_var", 5, "mixture", 0.1, 1.0, "random", "normal"),
    # the paper's test problems (Sec. 4.1, Sec. 4.3): non-divergence operator, white-noise
    # coefficients with mesh Reynolds number in [1, Re], v = (sin 0.5, cos 0.5), rhs = 1
    "paper_re10": Workload("paper_re10", 6, "white", 0.0, 0.0, "paper", "ones", 10.0, "nondiv"),
    "paper_re1e3": Workload("paper_re1e3", 7, "white", 0.0, 0.0, "paper", "ones", 1e3, "nondiv"),
    "paper_re1e5": Workload("paper_re1e5", 8, "white", 0.0, 0.0, "paper", "ones", 1e5, "nondiv"),
    # the same problems with multi-level random coefficients (Sec. 4.3 "mldata", Alg. 4), Re = 1000
    "paper_mldata": Workload("paper_mldata", 9, "mldata", 0.0, 0.0, "paper", "ones", 1e3, "nondiv"),
}


@dataclass
class Problem:
    n: int
    a: np.ndarray      # (n, n) float32
    b: np.ndarray      # (2,) float32
    f: np.ndarray      # (n, n) float32


def make_problem(workload: str, n: int, index: int, seed: int = 0) -> Problem:
    w = WORKLOADS[workload]
    ra = rng_for(seed, w.wid, index, STREAM_A)
    if w.coef == "grf":
        a = np.exp(grf(n, ra, w.grf_length, w.grf_variance))
    elif w.coef == "blocks":
        a = blocks_lognormal(n, ra)
    elif w.coef == "mixture":
        a = mixture(n, ra)
    elif w.coef == "white":
        a = white_noise_coef(n, ra, w.re)
    elif w.coef == "mldata":
        a = mldata_coef(n, ra, w.re)
    else:
        raise ValueError(w.coef)
    b = velocity(rng_for(seed, w.wid, index, STREAM_B), w.vel)
    f = rhs(n, rng_for(seed, w.wid, index, STREAM_F), w.f_kind)
    # C-contiguous float32 (fancy indexing, as in the interpolation of mldata, can return
    # arrays in Fortran order, and astype keeps the order)
    c32 = lambda x: np.ascontiguousarray(x, dtype=np.float32)
    return Problem(n, c32(a), c32(b), c32(f))


def var_sizes(count: int, seed: int = 0, sizes=VAR_SIZES, workload: str = "mixture_var") -> list[int]:
    """Grid sizes of an uneven-size batch: problem i draws its n uniformly from `sizes` with the
    generator of (seed, workload, i, size stream)."""
    w = WORKLOADS[workload]
    return [int(sizes[rng_for(seed, w.wid, i, STREAM_N).integers(0, len(sizes))]) for i in range(count)]


def make_batch(workload: str, n: int, batch: int, seed: int = 0, first: int = 0):
    """Stacked float32 arrays ``a (B,n,n)``, ``b (B,2)``, ``f (B,n,n)``."""
    ps = [make_problem(workload, n, first + i, seed) for i in range(batch)]
    return (np.stack([p.a for p in ps]), np.stack([p.b for p in ps]), np.stack([p.f for p in ps]))
