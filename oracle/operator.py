"""FP64 reference for the discrete convection-diffusion operator (test infrastructure).

Operator of record: the divergence form  -div(a grad u) + b . grad u = f  (Sec. 2.5,
remark "Non-divergence form vs divergence form", Eq. (12)) on the unit square
with zero Dirichlet boundary values (Sec. 2.5: zero boundary condition, zero
padding).  Diffusion uses the 5-point flux stencil with the face coefficient
equal to the harmonic mean of the two nodal values (a boundary face takes the
interior node's value); convection uses the first-order upwind differences of
Sec. 2.5 (the dx+/dx-/dy+/dy- kernels, Eqs. (9)-(11)), with the velocity applied
once.  Physical scaling: 1/h^2 on diffusion and 1/h on convection.

form="nondiv" gives the non-divergence form -a (u_xx + u_yy) + b . grad u of Eq. (7),
the operator the paper computes with: the 5-point Laplacian of Eq. (8) times the
row's own a (every face of row (i, j) takes a[i, j]), the same upwind convection.

Grid: n x n interior nodes, h = 1/(n+1), array index [i, j] with i along +y and
j along +x, so "east" is j+1 and "north" is i+1.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def harmonic(p: np.ndarray, q: np.ndarray) -> np.ndarray:
    return 2.0 * p * q / (p + q)


def face_coefficients(a: np.ndarray, form: str = "div"):
    """Return (aE, aW, aN, aS), each (n, n) float64: the diffusion coefficient on
    the four faces of every node (harmonic means for the divergence form; the
    node's own value for the non-divergence form)."""
    a = np.asarray(a, dtype=np.float64)
    if form == "nondiv":
        return a.copy(), a.copy(), a.copy(), a.copy()
    if form != "div":
        raise ValueError(form)
    aE = a.copy(); aE[:, :-1] = harmonic(a[:, :-1], a[:, 1:])
    aW = a.copy(); aW[:, 1:] = harmonic(a[:, 1:], a[:, :-1])
    aN = a.copy(); aN[:-1, :] = harmonic(a[:-1, :], a[1:, :])
    aS = a.copy(); aS[1:, :] = harmonic(a[1:, :], a[:-1, :])
    return aE, aW, aN, aS


def upwind_split(b):
    bx, by = float(b[0]), float(b[1])
    return max(bx, 0.0), min(bx, 0.0), max(by, 0.0), min(by, 0.0)


def stencil(a: np.ndarray, b, form: str = "div") -> dict:
    """Matrix entries of every row: diagonal 'C' and couplings 'E','W','N','S'
    (the coefficient multiplying the neighbour's value; zero-Dirichlet
    neighbours outside the grid are simply not coupled)."""
    n = a.shape[0]
    h = 1.0 / (n + 1)
    aE, aW, aN, aS = face_coefficients(a, form)
    bxp, bxm, byp, bym = upwind_split(b)
    C = (aE + aW + aN + aS) / h ** 2 + (bxp - bxm + byp - bym) / h
    st = {
        "C": C,
        "E": -aE / h ** 2 + bxm / h,
        "W": -aW / h ** 2 - bxp / h,
        "N": -aN / h ** 2 + bym / h,
        "S": -aS / h ** 2 - byp / h,
    }
    return st


def apply_A(a: np.ndarray, b, u: np.ndarray, form: str = "div") -> np.ndarray:
    """Matrix-free A(a, b) u in float64."""
    n = a.shape[0]
    h = 1.0 / (n + 1)
    u = np.asarray(u, dtype=np.float64)
    up = np.zeros((n + 2, n + 2)); up[1:-1, 1:-1] = u
    uE, uW = up[1:-1, 2:], up[1:-1, :-2]
    uN, uS = up[2:, 1:-1], up[:-2, 1:-1]
    aE, aW, aN, aS = face_coefficients(a, form)
    bxp, bxm, byp, bym = upwind_split(b)
    diff = ((aE + aW + aN + aS) * u - aE * uE - aW * uW - aN * uN - aS * uS) / h ** 2
    conv = (bxp * (u - uW) + bxm * (uE - u) + byp * (u - uS) + bym * (uN - u)) / h
    return diff + conv


def apply_AT(a: np.ndarray, b, v: np.ndarray, form: str = "div") -> np.ndarray:
    """Transpose A(a, b)^T v in float64: every row's coupling scattered back to
    the neighbour it couples."""
    n = a.shape[0]
    st = stencil(a, b, form)
    v = np.asarray(v, dtype=np.float64)
    out = st["C"] * v
    # row (i,j) couples column (i,j+1) with E[i,j]  ->  out[i,j+1] += E[i,j] v[i,j]
    out[:, 1:] += st["E"][:, :-1] * v[:, :-1]
    out[:, :-1] += st["W"][:, 1:] * v[:, 1:]
    out[1:, :] += st["N"][:-1, :] * v[:-1, :]
    out[:-1, :] += st["S"][1:, :] * v[1:, :]
    return out


def diagonal(a: np.ndarray, b, form: str = "div") -> np.ndarray:
    """D = diag(A) = (aE+aW+aN+aS)/h^2 + (|bx|+|by|)/h."""
    return stencil(a, b, form)["C"]


def assemble_A(a: np.ndarray, b, form: str = "div") -> sp.csr_matrix:
    """Sparse A with row/column index i*n + j."""
    n = a.shape[0]
    st = stencil(a, b, form)
    idx = np.arange(n * n).reshape(n, n)
    rows, cols, vals = [idx.ravel()], [idx.ravel()], [st["C"].ravel()]
    rows.append(idx[:, :-1].ravel()); cols.append(idx[:, 1:].ravel()); vals.append(st["E"][:, :-1].ravel())
    rows.append(idx[:, 1:].ravel()); cols.append(idx[:, :-1].ravel()); vals.append(st["W"][:, 1:].ravel())
    rows.append(idx[:-1, :].ravel()); cols.append(idx[1:, :].ravel()); vals.append(st["N"][:-1, :].ravel())
    rows.append(idx[1:, :].ravel()); cols.append(idx[:-1, :].ravel()); vals.append(st["S"][1:, :].ravel())
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(n * n, n * n))


def features(a: np.ndarray, b, form: str = "div") -> np.ndarray:
    """Setup-network input: the four off-diagonal couplings of D^-1 A with the sign
    flipped, stacked as channels [W, E, S, N] (the remark "Matrix coefficients as
    input" of Sec. 3.2, Eqs. (15)-(16)); a channel is zero where that neighbour
    lies outside the grid.  Returns (4, n, n) float64 with values in [0, 1]."""
    st = stencil(a, b, form)
    D = st["C"]
    F = np.stack([-st["W"], -st["E"], -st["S"], -st["N"]]) / D
    F[0][:, 0] = 0.0
    F[1][:, -1] = 0.0
    F[2][0, :] = 0.0
    F[3][-1, :] = 0.0
    return F
