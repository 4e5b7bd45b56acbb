"""Hand-set MGCNN weights that make the network a coefficient-aware V(1,1) multigrid cycle.

The MGCNN architecture (setup network, Alg. 2; solve network, Alg. 3) is expressive enough to
hold a classical cycle: a weighted-Jacobi smoother on the scaled residual, full-weighting
restriction and bilinear prolongation (the geometric multigrid that Sec. 2.3 relates MGCNN to).
This module sets the 81C^2 + 58C parameters by hand so that, in exact arithmetic,

* setup: s_l carries 1 on the channels R, E, DE and alpha * F_d(i - dir_d) on the copy channels
  RC[d], DC[d], where F_d are the four D-normalised neighbour couplings of the input features
  (tanh(alpha x) ~ alpha x for the small alpha used; the last three tanh layers add zero);
* down smoother on level l: E += omega * R (one Jacobi sweep on the correction) and
  R <- (1 - omega) R + omega * sum_d F_d R(i + dir_d), the scaled residual after that sweep;
* restriction: full weighting of R into R and its four copies RC[d];
* up smoother: E += omega * R + (1 - omega) DE + omega * sum_d F_d DE(i + dir_d), with DE the
  prolongated coarse correction;
* prolongation: bilinear interpolation of E into DE and its copies DC[d];
* output: u += E on the finest level.

The coarse levels use injected features (one stride-2 restriction of the setup state), not a
Galerkin operator, so the cycle is exact multigrid only for smooth coefficients.  It converges
for Poisson and smooth random fields; it needs the Krylov wrapper (FGMRES) for high-contrast
block coefficients.  These weights are a deterministic, data-free preconditioner for the
library; they are not the paper's trained network.

Channel roles (C >= 15): R = 0, E = 1, DE = 2, F_d = 3..6, RC[d] = 7..10, DC[d] = 11..14;
directions d = W, E, S, N.
"""
from __future__ import annotations

import numpy as np

R, E, DE = 0, 1, 2
FCH = (3, 4, 5, 6)
RC = (7, 8, 9, 10)
DC = (11, 12, 13, 14)
# 3x3 tap (p, q) that reads the neighbour in direction W, E, S, N of the output pixel
# (cross-correlation: tap (p, q) reads pixel (i + p - 1, j + q - 1); i grows towards N)
TAP = ((1, 0), (1, 2), (0, 1), (2, 1))
# tap that reads, at pixel j, the value of the pixel j - dir (the opposite neighbour)
OPP = ((1, 2), (1, 0), (2, 1), (0, 1))


def parameter_shapes(C: int) -> list[tuple[str, tuple[int, ...]]]:
    """Order and shapes of the flat weight vector (Alg. 2 then Alg. 3): setup reChannel,
    four setup ResNet layers (conv, bias), setup restriction, solve reChannel-in, down and up
    smoothers, restriction, transposed-conv prolongation [C_in][C_out], reChannel-out."""
    s = [("setup_in", (C, 4, 3, 3))]
    for k in range(4):
        s += [(f"setup_res{k}_w", (C, C, 3, 3)), (f"setup_res{k}_b", (C,))]
    s += [("setup_restrict", (C, C, 3, 3)), ("solve_in", (C, 1, 3, 3)),
          ("smooth_down", (C, C, 3, 3)), ("smooth_up", (C, C, 3, 3)),
          ("restrict", (C, C, 3, 3)), ("prolong", (C, C, 3, 3)), ("solve_out", (1, C, 3, 3))]
    return s


def vcycle_weights(C: int = 16, omega: float = 0.9, alpha: float = 0.05,
                   omega_up: float | None = None) -> np.ndarray:
    """Flat float32 weights of the hand-set V(1,1) cycle described in the module docstring.

    omega: Jacobi damping of both smoothers (0.9 measured best as an FGMRES preconditioner on
    the 10^4-contrast block workload; 0.8 converges faster as a stationary cycle on Poisson);
    omega_up: damping of the up smoother alone (default: omega);
    alpha: scale of the coupling features carried through the tanh layers (the smoother taps
    divide it out again)."""
    if C < 15:
        raise ValueError("the hand-set cycle needs at least 15 channels")
    P = {name: np.zeros(sh, dtype=np.float64) for name, sh in parameter_shapes(C)}
    for d in range(4):
        P["setup_in"][FCH[d], d, 1, 1] = 1.0
        P["setup_restrict"][FCH[d], FCH[d], 1, 1] = 1.0
    for k in range(4):
        P[f"setup_res{k}_b"][[R, E, DE]] = np.arctanh(0.25)   # four layers of tanh = 1/4 each
    for d in range(4):
        P["setup_res0_w"][RC[d], FCH[d], OPP[d][0], OPP[d][1]] = alpha
        P["setup_res0_w"][DC[d], FCH[d], OPP[d][0], OPP[d][1]] = alpha
    P["solve_in"][R, 0, 1, 1] = 1.0
    for d in range(4):
        P["solve_in"][RC[d], 0, 1, 1] = 1.0
    P["smooth_down"][E, R, 1, 1] = omega
    P["smooth_down"][R, R, 1, 1] = -omega
    for d in range(4):
        P["smooth_down"][R, RC[d], TAP[d][0], TAP[d][1]] = omega / alpha
    fw = np.outer([1.0, 2.0, 1.0], [1.0, 2.0, 1.0]) / 4.0
    P["restrict"][R, R] = fw
    for d in range(4):
        P["restrict"][RC[d], R] = fw
    P["prolong"][E, DE] = fw
    for d in range(4):
        P["prolong"][E, DC[d]] = fw
    wu = omega if omega_up is None else omega_up
    P["smooth_up"][E, R, 1, 1] = wu
    P["smooth_up"][E, DE, 1, 1] = 1.0 - wu
    for d in range(4):
        P["smooth_up"][E, DC[d], TAP[d][0], TAP[d][1]] = wu / alpha
    P["solve_out"][0, E, 1, 1] = 1.0
    return np.concatenate([P[name].ravel() for name, _ in parameter_shapes(C)]).astype(np.float32)
