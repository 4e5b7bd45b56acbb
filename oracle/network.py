"""FP64 reference for the MGCNN setup and solve networks (test infrastructure).

Tensors are channel-first ``(channels, rows, cols)`` for one problem.  Weight
tensors follow the PyTorch conventions: convolution weights ``(C_out, C_in, 3, 3)``
applied as cross-correlation; transposed-convolution weights ``(C_in, C_out, 3, 3)``.

* Same-size 3x3 conv with zero padding 1 (Sec. 2.4, Eq. (2); zero padding, Sec. 2.5).
* Stride-2 restriction conv (RCNN, Sec. 2.4) with no padding, mapping 2m+1 -> m.
* Transposed stride-2 conv (TCNN, Sec. 2.4, Eq. (3)) with no padding, mapping m -> 2m+1.
* Setup phase (Sec. 3.2, Alg. 2, Eqs. (13)-(14)): reChannel of the coefficient
  features, then per level a four-layer tanh ResNet (Eq. (6)) and a stride-2
  restriction of the coefficient tensor, weights shared across levels (P3).
* Solve phase (Sec. 3.3, Alg. 3, Eqs. (17)-(18)): reChannel-in, down loop of
  multiplicative ResNet smoothers K (s * x) + x and restrictions, up loop of
  smoothers and transposed-conv additions, reChannel-out.  No bias, no activation.
"""
from __future__ import annotations

import numpy as np

NUM_SETUP_LAYERS = 4


def unpack_weights(w: np.ndarray, C: int) -> dict:
    """Split the flat weight vector into named float64 tensors.  Order: setup
    reChannel (C,4,3,3); 4 x [setup ResNet conv (C,C,3,3), bias (C,)]; setup
    restriction (C,C,3,3); solve reChannel-in (C,1,3,3); down smoother; up
    smoother; restriction (each (C,C,3,3)); prolongation (C_in,C_out,3,3);
    reChannel-out (1,C,3,3)."""
    w = np.asarray(w, dtype=np.float64).ravel()
    out, off = {}, 0

    def take(name, shape):
        nonlocal off
        size = int(np.prod(shape))
        out[name] = w[off:off + size].reshape(shape).copy()
        off += size

    take("W_sc", (C, 4, 3, 3))
    for k in range(NUM_SETUP_LAYERS):
        take(f"W_k{k}", (C, C, 3, 3))
        take(f"beta_k{k}", (C,))
    take("W_sr", (C, C, 3, 3))
    take("W_in", (C, 1, 3, 3))
    take("W_dn", (C, C, 3, 3))
    take("W_up", (C, C, 3, 3))
    take("W_R", (C, C, 3, 3))
    take("W_T", (C, C, 3, 3))
    take("W_out", (1, C, 3, 3))
    if off != w.size:
        raise ValueError(f"weight vector has {w.size} entries, expected {off} for C={C}")
    return out


def pack_weights(P: dict, C: int) -> np.ndarray:
    names = ["W_sc"]
    for k in range(NUM_SETUP_LAYERS):
        names += [f"W_k{k}", f"beta_k{k}"]
    names += ["W_sr", "W_in", "W_dn", "W_up", "W_R", "W_T", "W_out"]
    return np.concatenate([np.asarray(P[k], dtype=np.float64).ravel() for k in names])


def channels_of(w_size: int) -> int:
    for C in range(1, 257):
        if 81 * C * C + 58 * C == w_size:
            return C
    raise ValueError(f"no channel count matches {w_size} weights")


# ------------------------------------------------------------------------------------------
# convolution primitives
# ------------------------------------------------------------------------------------------

def conv_same(W: np.ndarray, x: np.ndarray) -> np.ndarray:
    """y[o,i,j] = sum_{c,p,q} W[o,c,p,q] x[c, i+p-1, j+q-1], x = 0 outside."""
    ci, n, m = x.shape
    xp = np.zeros((ci, n + 2, m + 2)); xp[:, 1:-1, 1:-1] = x
    y = np.zeros((W.shape[0], n, m))
    for p in range(3):
        for q in range(3):
            y += np.tensordot(W[:, :, p, q], xp[:, p:p + n, q:q + m], axes=(1, 0))
    return y


def conv_s2(W: np.ndarray, x: np.ndarray) -> np.ndarray:
    """y[o,I,J] = sum_{c,p,q} W[o,c,p,q] x[c, 2I+p, 2J+q] for 0 <= I,J < (m-1)/2."""
    ci, m, _ = x.shape
    mc = (m - 1) // 2
    y = np.zeros((W.shape[0], mc, mc))
    for p in range(3):
        for q in range(3):
            y += np.tensordot(W[:, :, p, q], x[:, p:p + 2 * mc - 1:2, q:q + 2 * mc - 1:2], axes=(1, 0))
    return y


def convT_s2(W: np.ndarray, x: np.ndarray) -> np.ndarray:
    """Transpose of conv_s2 with the same weight array read as (C_in, C_out, 3, 3):
    y[o, 2I+p, 2J+q] += W[c,o,p,q] x[c,I,J]; output side 2m+1."""
    ci, mc, _ = x.shape
    m = 2 * mc + 1
    y = np.zeros((W.shape[1], m, m))
    for p in range(3):
        for q in range(3):
            y[:, p:p + 2 * mc - 1:2, q:q + 2 * mc - 1:2] += np.tensordot(W[:, :, p, q], x, axes=(0, 0))
    return y


def num_levels(n: int) -> int:
    L, m = 1, n
    while m > 1:
        if m % 2 == 0:
            raise ValueError(f"n={n} is not of the form 2^L - 1")
        m = (m - 1) // 2
        L += 1
    return L


# ------------------------------------------------------------------------------------------
# setup phase (Alg. 2)
# ------------------------------------------------------------------------------------------

def setup(P: dict, F: np.ndarray, levels: int, keep: bool = False):
    """Return the per-level setup tensors s_1..s_L (each (C, n_l, n_l)).
    With ``keep`` also return the intermediates needed by the reverse pass."""
    c = conv_same(P["W_sc"], F)
    s, tape = [], []
    for l in range(levels):
        z = c
        layers = []
        for k in range(NUM_SETUP_LAYERS):
            t = np.tanh(conv_same(P[f"W_k{k}"], z) + P[f"beta_k{k}"][:, None, None])
            layers.append((z, t))
            z = z + t
        s.append(z)
        tape.append((c, layers))
        if l < levels - 1:
            c = conv_s2(P["W_sr"], c)
    return (s, tape) if keep else s


# ------------------------------------------------------------------------------------------
# solve phase (Alg. 3)
# ------------------------------------------------------------------------------------------

def vcycle(P: dict, s: list, r: np.ndarray, keep: bool = False, up_post: bool = False):
    """One application of the solve network B to a (n, n) input; returns (n, n).
    With ``keep`` also return the per-level states for the reverse pass.  ``up_post``: the up
    smoother in the form x + s * (W_up conv x), the adjoint form of the down smoother
    x + W_dn conv (s * x) (the symmetric variant of the remark in Sec. 3.3)."""
    L = len(s)
    xin = [None] * L
    xdn = [None] * L
    xup = [None] * L
    v = [None] * L
    xin[0] = conv_same(P["W_in"], r[None])
    for l in range(L):                                   # down cycle
        xdn[l] = xin[l] + conv_same(P["W_dn"], s[l] * xin[l])
        if l < L - 1:
            xin[l + 1] = conv_s2(P["W_R"], xdn[l])
    v[L - 1] = xdn[L - 1]
    for l in range(L - 1, -1, -1):                       # up cycle
        if up_post:
            xup[l] = v[l] + s[l] * conv_same(P["W_up"], v[l])
        else:
            xup[l] = v[l] + conv_same(P["W_up"], s[l] * v[l])
        if l > 0:
            v[l - 1] = xdn[l - 1] + convT_s2(P["W_T"], xup[l])
    out = conv_same(P["W_out"], xup[0])[0]
    if keep:
        return out, {"r": r, "xin": xin, "xdn": xdn, "v": v, "xup": xup}
    return out
