"""FP64 reverse mode of the unrolled MGCNN iteration (test infrastructure).

Training minimises the residual loss of Sec. 3.4, Eq. (19), with the setup and
solve networks trained jointly (Sec. 3.4).  Here the loss is taken after K
unrolled iterations from u_0 = 0 and normalised per problem:

    L = (1/N) sum_i ||f_i - A_i u_{K,i}||^2 / ||f_i||^2 .

Reverse sweep, for the iteration u_{k+1} = u_k + B((f - A u_k)/D):

    lambda_K = dL/du_K = -2 A^T r_K / (N ||f||^2)
    for k = K-1 .. 0:   g = B^T lambda_{k+1}  (accumulating dL/dtheta_solve and dL/ds_l)
                        lambda_k = lambda_{k+1} - A^T (g / D)
    then the setup network is reversed with dL/ds_l (tanh' = 1 - tanh^2).

B^T is the exact reverse of Alg. 3: the transpose of a same-size conv is the
same-size conv with the kernel flipped and its channel axes swapped; the
transpose of the stride-2 conv is the stride-2 transposed conv with the same
array (Sec. 2.4, Eq. (3)) and vice versa.
"""
from __future__ import annotations

import numpy as np

from . import network as net
from . import operator as op


def conv_same_dx(W, g):
    Wf = np.ascontiguousarray(np.transpose(W[:, :, ::-1, ::-1], (1, 0, 2, 3)))
    return net.conv_same(Wf, g)


def conv_same_dW(g, x):
    ci, n, m = x.shape
    xp = np.zeros((ci, n + 2, m + 2)); xp[:, 1:-1, 1:-1] = x
    dW = np.zeros((g.shape[0], ci, 3, 3))
    for p in range(3):
        for q in range(3):
            dW[:, :, p, q] = np.tensordot(g, xp[:, p:p + n, q:q + m], axes=([1, 2], [1, 2]))
    return dW


def conv_s2_dW(g, x):
    mc = g.shape[1]
    dW = np.zeros((g.shape[0], x.shape[0], 3, 3))
    for p in range(3):
        for q in range(3):
            dW[:, :, p, q] = np.tensordot(g, x[:, p:p + 2 * mc - 1:2, q:q + 2 * mc - 1:2], axes=([1, 2], [1, 2]))
    return dW


def convT_s2_dW(g, x):
    mc = x.shape[1]
    dW = np.zeros((x.shape[0], g.shape[0], 3, 3))
    for p in range(3):
        for q in range(3):
            dW[:, :, p, q] = np.tensordot(x, g[:, p:p + 2 * mc - 1:2, q:q + 2 * mc - 1:2], axes=([1, 2], [1, 2]))
    return dW


def _zero_grads(P):
    return {k: np.zeros_like(v) for k, v in P.items()}


def vcycle_backward(P, s, tape, g_out, dP):
    """Reverse of one solve-network application.  ``g_out`` is dL/d(output),
    (n, n).  Accumulates weight gradients into ``dP``; returns (dL/d input,
    list of dL/ds_l)."""
    L = len(s)
    xin, xdn, v, xup = tape["xin"], tape["xdn"], tape["v"], tape["xup"]
    g_s = [np.zeros_like(sl) for sl in s]
    g_xdn = [np.zeros_like(x) for x in xdn]
    # reChannel-out
    g_out3 = g_out[None]
    dP["W_out"] += conv_same_dW(g_out3, xup[0])
    g_xup = conv_same_dx(P["W_out"], g_out3)
    # up cycle in reverse order: l = 0 .. L-1
    for l in range(L):
        z = s[l] * v[l]
        dP["W_up"] += conv_same_dW(g_xup, z)
        gz = conv_same_dx(P["W_up"], g_xup)
        g_s[l] += gz * v[l]
        g_v = g_xup + gz * s[l]
        g_xdn[l] += g_v
        if l < L - 1:
            # v[l] = xdn[l] + convT_s2(W_T, xup[l+1])
            dP["W_T"] += convT_s2_dW(g_v, xup[l + 1])
            g_xup = net.conv_s2(P["W_T"], g_v)
    # down cycle in reverse order: l = L-1 .. 0
    g_xin = None
    for l in range(L - 1, -1, -1):
        z = s[l] * xin[l]
        dP["W_dn"] += conv_same_dW(g_xdn[l], z)
        gz = conv_same_dx(P["W_dn"], g_xdn[l])
        g_s[l] += gz * xin[l]
        g_xin = g_xdn[l] + gz * s[l]
        if l > 0:
            # xin[l] = conv_s2(W_R, xdn[l-1])
            dP["W_R"] += conv_s2_dW(g_xin, xdn[l - 1])
            g_xdn[l - 1] += net.convT_s2(P["W_R"], g_xin)
    dP["W_in"] += conv_same_dW(g_xin, tape["r"][None])
    g_r = conv_same_dx(P["W_in"], g_xin)[0]
    return g_r, g_s


def setup_backward(P, F, stape, g_s, dP):
    """Reverse of Alg. 2 given dL/ds_l for every level; accumulates into dP."""
    L = len(stape)
    g_c = [None] * L
    for l in range(L - 1, -1, -1):
        c, layers = stape[l]
        gz = g_s[l].copy()
        for k in range(len(layers) - 1, -1, -1):
            z, t = layers[k]
            gp = gz * (1.0 - t * t)
            dP[f"W_k{k}"] += conv_same_dW(gp, z)
            dP[f"beta_k{k}"] += gp.sum(axis=(1, 2))
            gz = gz + conv_same_dx(P[f"W_k{k}"], gp)
        g_c[l] = gz if g_c[l] is None else g_c[l] + gz
        if l > 0:
            prev_c = stape[l - 1][0]
            dP["W_sr"] += conv_s2_dW(g_c[l], prev_c)
            back = net.convT_s2(P["W_sr"], g_c[l])
            g_c[l - 1] = back if g_c[l - 1] is None else g_c[l - 1] + back
    dP["W_sc"] += conv_same_dW(g_c[0], F)


def loss_terms(a, b, f, u, N: int, form: str = "div"):
    """Per-problem share of the loss and its partial derivatives:
    returns (||r||^2 / (N ||f||^2), dL/du, dL/df) with r = f - A u, where dL/df
    includes the dependence of the normalisation ||f||^2 on f."""
    f = np.asarray(f, dtype=np.float64)
    r = f - op.apply_A(a, b, u, form)
    nf2 = float(np.sum(f * f))
    rr = float(np.sum(r * r))
    dLdu = -2.0 * op.apply_AT(a, b, r, form) / (N * nf2)
    dLdf = 2.0 * r / (N * nf2) - 2.0 * rr * f / (N * nf2 * nf2)
    return rr / (N * nf2), dLdu, dLdf


def unrolled_backward(P, a, b, f, K: int, lam, dP, form: str = "div"):
    """Reverse of K iterations from u_0 = 0 given lam = dL/du_K.  Accumulates the
    weight gradient into dP and returns dL/df through the iteration."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    f = np.asarray(f, dtype=np.float64)
    n = a.shape[0]
    L = net.num_levels(n)
    D = op.diagonal(a, b, form)
    F = op.features(a, b, form)
    s, stape = net.setup(P, F, L, keep=True)
    u = np.zeros((n, n))
    tapes = []
    for _ in range(K):
        r = f - op.apply_A(a, b, u, form)
        corr, tape = net.vcycle(P, s, r / D, keep=True)
        tapes.append(tape)
        u = u + corr
    g_s_tot = [np.zeros_like(sl) for sl in s]
    df = np.zeros((n, n))
    for k in range(K - 1, -1, -1):
        g_rt, g_s = vcycle_backward(P, s, tapes[k], lam, dP)
        for l in range(L):
            g_s_tot[l] += g_s[l]
        g_r = g_rt / D
        df += g_r
        lam = lam - op.apply_AT(a, b, g_r, form)
    setup_backward(P, F, stape, g_s_tot, dP)
    return df, u


def loss_and_grad(weights, a_batch, b_batch, f_batch, K: int, want_df: bool = False,
                  form: str = "div"):
    """Loss after K unrolled iterations from zero and its gradient with respect to
    the flat weight vector (and optionally to every f_i).  Returns
    (loss, grad_flat[, df_list])."""
    weights = np.asarray(weights, dtype=np.float64)
    C = net.channels_of(weights.size)
    P = net.unpack_weights(weights, C)
    dP = _zero_grads(P)
    N = len(f_batch)
    total = 0.0
    dfs = []
    for i in range(N):
        a = np.asarray(a_batch[i], dtype=np.float64)
        b = np.asarray(b_batch[i], dtype=np.float64)
        f = np.asarray(f_batch[i], dtype=np.float64)
        s = net.setup(P, op.features(a, b, form), net.num_levels(a.shape[0]))
        u = np.zeros_like(f)
        D = op.diagonal(a, b, form)
        for _ in range(K):
            u = u + net.vcycle(P, s, (f - op.apply_A(a, b, u, form)) / D)
        li, dLdu, dLdf = loss_terms(a, b, f, u, N, form)
        total += li
        df_iter, _ = unrolled_backward(P, a, b, f, K, dLdu, dP, form)
        dfs.append(dLdf + df_iter)
    grad = net.pack_weights(dP, C)
    if want_df:
        return total, grad, dfs
    return total, grad
