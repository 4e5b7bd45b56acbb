"""Layout helpers for the flat weight vector of the C-ABI (16 hidden channels).

The paper's networks use C = 4, 8 or 12 hidden channels (Sec. 4.2).  A network with C < 16
channels is exactly a 16-channel network whose extra channels are zero: every convolution maps
the zero channels to zero (their output rows are zero), the setup layers z + tanh(W z + beta)
keep them at tanh(0) = 0, and no extra channel feeds a real one (their input columns are zero).
``embed_channels`` therefore places each C-channel tensor in the leading channels of its
16-channel tensor and zeros the rest; the library then runs the C-channel network unchanged
(at the cost of 16 channels).
"""
from __future__ import annotations

import numpy as np

from .handbuilt import parameter_shapes

LIB_CHANNELS = 16


def channels_of(size: int) -> int:
    """Hidden channels of a flat weight vector of `size` entries (81 C^2 + 58 C)."""
    for C in range(1, LIB_CHANNELS + 1):
        if 81 * C * C + 58 * C == size:
            return C
    raise ValueError(f"{size} weights match no channel count in 1..{LIB_CHANNELS}")


def embed_channels(w, C: int | None = None) -> np.ndarray:
    """Flat float32 weights of a C-channel network -> the equivalent 16-channel flat vector."""
    w = np.asarray(w, dtype=np.float32).ravel()
    C = channels_of(w.size) if C is None else int(C)
    if 81 * C * C + 58 * C != w.size:
        raise ValueError(f"{w.size} weights do not describe a {C}-channel network")
    out = []
    off = 0
    for (name, small), (_, big) in zip(parameter_shapes(C), parameter_shapes(LIB_CHANNELS)):
        size = int(np.prod(small))
        t = np.zeros(big, dtype=np.float32)
        t[tuple(slice(0, d) for d in small)] = w[off:off + size].reshape(small)
        out.append(t.ravel())
        off += size
    return np.concatenate(out)


def symmetric_variant(w) -> np.ndarray:
    """Flat weights of the symmetric variant of the solve network (Sec. 3.3): the up smoother
    becomes the adjoint of the down smoother (3x3 taps flipped, channel axes swapped), the
    transposed-conv prolongation takes the restriction's array and reChannel-out the adjoint of
    reChannel-in; the setup network and the down path are kept.  With the up smoother applied
    in its adjoint form (opts.up_post = 1) the network is then symmetric positive semi-definite
    for any values, so it can precondition conjugate gradients (method PCG)."""
    w = np.asarray(w, dtype=np.float32).ravel()
    C = channels_of(w.size)
    parts, off = {}, 0
    for name, shape in parameter_shapes(C):
        size = int(np.prod(shape))
        parts[name] = w[off:off + size].reshape(shape).copy()
        off += size
    adj = lambda t: np.ascontiguousarray(np.flip(t, (2, 3)).transpose(1, 0, 2, 3))
    parts["smooth_up"] = adj(parts["smooth_down"])
    parts["prolong"] = parts["restrict"].copy()
    parts["solve_out"] = adj(parts["solve_in"])
    return np.concatenate([parts[name].ravel() for name, _ in parameter_shapes(C)]).astype(np.float32)
