"""ctypes binding of libmgcnn.so (argument marshalling only).

PyTorch supplies device memory and the HIP stream; every step of the solver runs in
the library's HIP kernels.  Importing this module without a built library raises.

Low-level: ``lib()`` returns the ctypes handle with the C signatures of
``include/mgcnn.h`` declared (``mgcnn_create``, ``mgcnn_setup``, ``mgcnn_solve``, ...).
High-level: ``Solver`` wraps one context; its methods carry the C names without the
``mgcnn_`` prefix.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmgcnn.so")

OK, NOT_CONVERGED = 0, 1
E_ARG, E_SIZE, E_STATE, E_NOMEM, E_HIP, E_DIVERGED, E_NORECORD, E_SCRATCH = -1, -2, -3, -4, -5, -6, -7, -8
NOALLOC_SCRATCH_BYTES = 8 << 20
F32, BF16 = 0, 1
U_F32, U_F64 = 0, 1

_lib = None


class mgcnn_opts(ctypes.Structure):
    _fields_ = [("channels", ctypes.c_int), ("state_dtype", ctypes.c_int), ("u_dtype", ctypes.c_int),
                ("use_graph", ctypes.c_int), ("check_every", ctypes.c_int),
                ("method", ctypes.c_int), ("restart", ctypes.c_int), ("f32_split", ctypes.c_int),
                ("s_bf16", ctypes.c_int), ("inner_steps", ctypes.c_int), ("gs_passes", ctypes.c_int),
                ("precond", ctypes.c_int), ("gmg_levels", ctypes.c_int), ("gmg_sweeps", ctypes.c_int),
                ("gmg_omega", ctypes.c_float), ("op_form", ctypes.c_int), ("deflate", ctypes.c_int),
                ("levels", ctypes.c_int), ("up_post", ctypes.c_int), ("pack_pairs", ctypes.c_int)]


class mgcnn_kernel_stat(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("level", ctypes.c_int), ("launches", ctypes.c_int),
                ("ms_total", ctypes.c_double), ("bytes_per_launch", ctypes.c_double),
                ("flops_per_launch", ctypes.c_double)]


KERNEL_KINDS = {0: "residual", 1: "finalize", 2: "conv_in", 3: "smooth_down", 4: "restrict",
                5: "smooth_up", 6: "prolong", 7: "out_update", 8: "smooth_in", 9: "smooth_out",
                10: "krylov_apply_A", 11: "krylov_dots", 12: "krylov_orth", 13: "krylov_scale",
                14: "krylov_combine", 15: "krylov_residual", 16: "scale_by_diag", 17: "zero",
                18: "gmg_down", 19: "gmg_up", 20: "gmg_coarse"}
PRECONDS = {"network": 0, "gmg": 1}
FORMS = {"div": 0, "nondiv": 1}

EXPORTS = {
    # name: (restype, argtypes)
    "mgcnn_default_opts": (None, [ctypes.POINTER(mgcnn_opts)]),
    "mgcnn_num_weights": (ctypes.c_size_t, [ctypes.c_int]),
    "mgcnn_gmg_levels": (ctypes.c_int, [ctypes.c_void_p]),
    "mgcnn_create": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(mgcnn_opts),
                                    ctypes.c_void_p, ctypes.c_void_p]),
    "mgcnn_set_weights": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "mgcnn_set_stream": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "mgcnn_setup": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                   ctypes.c_int]),
    "mgcnn_solve": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double,
                                   ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "mgcnn_forward": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                     ctypes.c_int]),
    "mgcnn_apply": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "mgcnn_residual_norms": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                            ctypes.c_void_p]),
    "mgcnn_get_setup_tensor": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p]),
    "mgcnn_levels": (ctypes.c_int, [ctypes.c_void_p]),
    "mgcnn_residual": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "mgcnn_loss": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                  ctypes.c_void_p, ctypes.c_void_p]),
    "mgcnn_backward": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "mgcnn_set_weights_device": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "mgcnn_profile_begin": (ctypes.c_int, [ctypes.c_void_p]),
    "mgcnn_profile_end": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                         ctypes.POINTER(ctypes.c_int)]),
    "mgcnn_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "mgcnn_last_error": (ctypes.c_char_p, [ctypes.c_void_p]),
    "mgcnn_destroy": (None, [ctypes.c_void_p]),
    "mgcnn_group_create": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(mgcnn_opts),
                                          ctypes.c_void_p, ctypes.c_void_p]),
    "mgcnn_group_setup": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_void_p, ctypes.c_int]),
    "mgcnn_group_solve": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_double, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_void_p]),
    "mgcnn_group_buckets": (ctypes.c_int, [ctypes.c_void_p]),
    "mgcnn_group_aligned": (ctypes.c_int, [ctypes.c_void_p]),
    "mgcnn_group_completion_times": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "mgcnn_group_last_error": (ctypes.c_char_p, [ctypes.c_void_p]),
    "mgcnn_group_destroy": (None, [ctypes.c_void_p]),
    "mgcnn_set_tile_variant": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int]),
    "mgcnn_tile_variant": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int]),
    "mgcnn_tile_rows": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int]),
    "mgcnn_residual_norms_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                                    ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                                    ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                                                    ctypes.c_void_p]),
}


def lib():
    """Load libmgcnn.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2312_11093_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in EXPORTS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


class MGCNNError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"mgcnn status {status}: {msg}")
        self.status = status


def _ptr(t) -> int:
    return t.data_ptr()


def _check_dev(t, dtype, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def _set_gmg(o, precond, levels, sweeps, omega):
    o.precond = PRECONDS[precond]
    o.gmg_levels = int(levels)
    o.gmg_sweeps = int(sweeps)
    o.gmg_omega = float(omega)


def _weights_ptr(owner, weights, count):
    """Host pointer to the flat float32 weights (kept alive on `owner`), or None (all zero;
    allowed for the GMG preconditioner, which has no weights)."""
    if weights is None:
        owner._w = None
        return None
    w = np.ascontiguousarray(np.asarray(weights, dtype=np.float32).ravel())
    if w.size != count:
        raise ValueError(f"expected {count} weights, got {w.size}")
    owner._w = w
    return w.ctypes.data


def residual_norms_noalloc(a, b, f, u, form: str = "div", stream=None):
    """mgcnn_residual_norms_noalloc: relative residuals ||f - A u|| / ||f|| per problem with no
    context and no device allocation (the library's fixed scratch array).  a, f: (B, n, n)
    float32 device tensors; u: (B, n, n) float32 or float64 device tensor; b: (B, 2) host
    array.  Returns a float64 numpy array (B,); raises MGCNNError on a non-zero status."""
    import torch
    L = lib()
    _check_dev(a, torch.float32, "a")
    _check_dev(f, torch.float32, "f")
    if not isinstance(u, torch.Tensor) or not u.is_cuda or u.dtype not in (torch.float32, torch.float64):
        raise TypeError("u must be a float32 or float64 device tensor")
    if not u.is_contiguous():
        raise ValueError("u must be contiguous")
    B, n, _ = a.shape
    if tuple(f.shape) != (B, n, n) or tuple(u.shape) != (B, n, n):
        raise ValueError("a, f and u must have the same (B, n, n) shape")
    bh = np.ascontiguousarray(np.asarray(b, dtype=np.float32).reshape(B, 2))
    out = np.zeros(B, np.float64)
    s = stream if stream is not None else torch.cuda.current_stream()
    st = L.mgcnn_residual_norms_noalloc(_ptr(a), bh.ctypes.data, n, B, FORMS[form], _ptr(f), _ptr(u),
                                        U_F64 if u.dtype == torch.float64 else U_F32,
                                        out.ctypes.data, ctypes.c_void_p(s.cuda_stream))
    if st != OK:
        raise MGCNNError(st, L.mgcnn_status_string(st).decode())
    return out


class Solver:
    """One library context (weights + workspace for one problem set)."""

    def __init__(self, weights, state: str = "f32", u: str = "f64", use_graph: bool = False,
                 check_every: int = 4, stream=None, method: str = "stationary", restart: int = 30,
                 f32_split: bool | int = True, s_bf16: bool = False, inner_steps: int = 1,
                 gs_passes: int = 2, precond: str = "network", gmg_levels: int = 0,
                 gmg_sweeps: int = 3, gmg_omega: float = 0.67, form: str = "div", deflate: int = 0,
                 levels: int = 0, up_post: bool = False, pack_pairs: bool = False):
        """weights: the flat network weights, or None with precond="gmg" (the geometric
        multigrid baseline has none).  form: "div" (divergence form, harmonic face
        coefficients) or "nondiv" (the non-divergence form -a Lap(u) + b . grad u).
        levels: network levels, 0 = log2(n+1), -d = log2(n+1) - d, > 0 = that many.
        up_post: up smoother in the adjoint form x + s . (W_up * x) (symmetric variant).
        pack_pairs: two problems per 16-channel state slot, for weights of at most 8 hidden
        channels in the 16-channel layout (stationary method, network preconditioner)."""
        import torch
        self._L = lib()
        o = mgcnn_opts()
        self._L.mgcnn_default_opts(ctypes.byref(o))
        o.channels = 16
        o.state_dtype = {"f32": F32, "bf16": BF16}[state]
        o.u_dtype = {"f32": U_F32, "f64": U_F64}[u]
        o.use_graph = int(bool(use_graph))
        o.check_every = int(check_every)
        o.method = {"stationary": 0, "fgmres": 1, "pcg": 2}[method]
        o.restart = int(restart)
        o.f32_split = 2 if f32_split == 2 else int(bool(f32_split))
        o.s_bf16 = int(bool(s_bf16))
        o.inner_steps = int(inner_steps)
        o.gs_passes = int(gs_passes)
        _set_gmg(o, precond, gmg_levels, gmg_sweeps, gmg_omega)
        o.op_form = FORMS[form]
        o.deflate = int(deflate)
        o.levels = int(levels)
        o.up_post = int(bool(up_post))
        o.pack_pairs = int(bool(pack_pairs))
        self.opts = o
        self.u_dtype = torch.float64 if o.u_dtype == U_F64 else torch.float32
        wp = _weights_ptr(self, weights, self._L.mgcnn_num_weights(16))
        self._stream = stream if stream is not None else torch.cuda.current_stream()
        h = ctypes.c_void_p()
        st = self._L.mgcnn_create(ctypes.byref(h), ctypes.byref(o), wp, ctypes.c_void_p(self._stream.cuda_stream))
        if st != OK:
            raise MGCNNError(st, self._L.mgcnn_status_string(st).decode())
        self._h = h
        self.n = 0
        self.batch = 0

    # -- helpers ---------------------------------------------------------------------------
    def _raise(self, st):
        if st not in (OK, NOT_CONVERGED):
            raise MGCNNError(st, self._L.mgcnn_last_error(self._h).decode())
        return st

    def close(self):
        if getattr(self, "_h", None):
            self._L.mgcnn_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- API (names of the C entry points without the prefix) --------------------------------
    def set_weights(self, weights):
        w = np.ascontiguousarray(np.asarray(weights, dtype=np.float32).ravel())
        return self._raise(self._L.mgcnn_set_weights(self._h, w.ctypes.data))

    def setup(self, a, b):
        """a: (B, n, n) float32 device tensor; b: (B, 2) host array."""
        import torch
        _check_dev(a, torch.float32, "a")
        B, n, n2 = a.shape
        bh = np.ascontiguousarray(np.asarray(b, dtype=np.float32).reshape(B, 2))
        self._raise(self._L.mgcnn_setup(self._h, _ptr(a), bh.ctypes.data, n, B))
        self.n, self.batch = n, B

    def solve(self, f, u, tol: float, maxit: int):
        """Returns (status, iters[B], relres[B], per-problem status[B]); u updated in place."""
        import torch
        _check_dev(f, torch.float32, "f")
        _check_dev(u, self.u_dtype, "u")
        it = np.zeros(self.batch, np.int32)
        rr = np.zeros(self.batch, np.float64)
        ps = np.zeros(self.batch, np.int32)
        st = self._L.mgcnn_solve(self._h, _ptr(f), _ptr(u), float(tol), int(maxit), it.ctypes.data,
                                 rr.ctypes.data, ps.ctypes.data)
        if st not in (OK, NOT_CONVERGED, E_DIVERGED):
            self._raise(st)
        return st, it, rr, ps

    def forward(self, f, u, K: int, record: bool = False):
        import torch
        _check_dev(f, torch.float32, "f")
        _check_dev(u, self.u_dtype, "u")
        return self._raise(self._L.mgcnn_forward(self._h, _ptr(f), _ptr(u), int(K), int(record)))

    def apply(self, r, z=None):
        import torch
        _check_dev(r, torch.float32, "r")
        if z is None:
            z = torch.empty_like(r)
        self._raise(self._L.mgcnn_apply(self._h, _ptr(r), _ptr(z)))
        return z

    def residual(self, f, u, r=None):
        """r = f - A u (float32 device tensor)."""
        import torch
        _check_dev(f, torch.float32, "f")
        _check_dev(u, self.u_dtype, "u")
        if r is None:
            r = torch.empty_like(f)
        self._raise(self._L.mgcnn_residual(self._h, _ptr(f), _ptr(u), _ptr(r)))
        return r

    def residual_norms(self, f, u):
        import torch
        _check_dev(f, torch.float32, "f")
        _check_dev(u, self.u_dtype, "u")
        rr = np.zeros(self.batch, np.float64)
        self._raise(self._L.mgcnn_residual_norms(self._h, _ptr(f), _ptr(u), rr.ctypes.data))
        return rr

    def get_setup_tensor(self, level: int):
        import torch
        m = self.n
        for _ in range(level - 1):
            m = (m - 1) // 2
        out = torch.empty((self.batch, m, m, 16), dtype=torch.float32, device="cuda")
        self._raise(self._L.mgcnn_get_setup_tensor(self._h, int(level), _ptr(out)))
        return out

    def set_weights_device(self, w):
        import torch
        _check_dev(w, torch.float32, "weights")
        return self._raise(self._L.mgcnn_set_weights_device(self._h, _ptr(w)))

    def loss(self, f, u, dloss_du=None, dloss_df=None):
        """Mean over the batch of ||f - A u||^2 / ||f||^2 (u float32); optionally its gradients."""
        import torch
        _check_dev(f, torch.float32, "f")
        _check_dev(u, torch.float32, "u")
        out = ctypes.c_double(0.0)
        self._raise(self._L.mgcnn_loss(self._h, _ptr(f), _ptr(u), ctypes.byref(out),
                                       _ptr(dloss_du) if dloss_du is not None else None,
                                       _ptr(dloss_df) if dloss_df is not None else None))
        return out.value

    def backward(self, dL_du, dL_dw=None, dL_df=None):
        """Reverse pass of the last recorded forward; returns dL/dweights (device tensor).
        dL_df, if given, is accumulated into."""
        import torch
        _check_dev(dL_du, torch.float32, "dL_du")
        if dL_dw is None:
            dL_dw = torch.empty(int(self._L.mgcnn_num_weights(16)), dtype=torch.float32, device="cuda")
        self._raise(self._L.mgcnn_backward(self._h, _ptr(dL_du), _ptr(dL_dw),
                                           _ptr(dL_df) if dL_df is not None else None))
        return dL_dw

    def profile_begin(self):
        return self._raise(self._L.mgcnn_profile_begin(self._h))

    def profile_end(self, max_stats: int = 256):
        arr = (mgcnn_kernel_stat * max_stats)()
        cnt = ctypes.c_int(0)
        self._raise(self._L.mgcnn_profile_end(self._h, arr, max_stats, ctypes.byref(cnt)))
        return [dict(kind=KERNEL_KINDS.get(arr[i].kind, str(arr[i].kind)), level=arr[i].level,
                     launches=arr[i].launches, ms_total=arr[i].ms_total,
                     bytes_per_launch=arr[i].bytes_per_launch, flops_per_launch=arr[i].flops_per_launch)
                for i in range(min(cnt.value, max_stats))]

    @property
    def levels(self) -> int:
        return self._L.mgcnn_levels(self._h)

    @property
    def gmg_levels(self) -> int:
        """Levels of the GMG cycle of the current problem set (0 with the network)."""
        return self._L.mgcnn_gmg_levels(self._h)


class GroupSolver:
    """Problems of different sizes in one call (mgcnn_group_*).  The stationary iteration with
    the network (levels <= 0) runs on aligned levels: one stream, one launch per operation and
    level size over the whole mixed batch, optionally hipGraph-captured (use_graph).  Other
    configurations bucket the problems by size, one batched problem set per size on its own
    stream, buckets solved concurrently."""

    def __init__(self, weights, state: str = "f32", u: str = "f64", method: str = "stationary",
                 restart: int = 30, check_every: int = 4, f32_split: bool | int = True, s_bf16: bool = False,
                 inner_steps: int = 1, gs_passes: int = 2, stream=None, precond: str = "network",
                 gmg_levels: int = 0, gmg_sweeps: int = 3, gmg_omega: float = 0.67,
                 form: str = "div", deflate: int = 0, levels: int = 0, up_post: bool = False,
                 use_graph: bool = False, pack_pairs: bool = False):
        import torch
        self._L = lib()
        o = mgcnn_opts()
        self._L.mgcnn_default_opts(ctypes.byref(o))
        o.state_dtype = {"f32": F32, "bf16": BF16}[state]
        o.u_dtype = {"f32": U_F32, "f64": U_F64}[u]
        o.method = {"stationary": 0, "fgmres": 1, "pcg": 2}[method]
        o.restart = int(restart)
        o.check_every = int(check_every)
        o.f32_split = 2 if f32_split == 2 else int(bool(f32_split))
        o.s_bf16 = int(bool(s_bf16))
        o.inner_steps = int(inner_steps)
        o.gs_passes = int(gs_passes)
        _set_gmg(o, precond, gmg_levels, gmg_sweeps, gmg_omega)
        o.op_form = FORMS[form]
        o.deflate = int(deflate)
        o.levels = int(levels)
        o.up_post = int(bool(up_post))
        o.use_graph = int(bool(use_graph))
        o.pack_pairs = int(bool(pack_pairs))
        self.u_dtype = torch.float64 if o.u_dtype == U_F64 else torch.float32
        wp = _weights_ptr(self, weights, self._L.mgcnn_num_weights(16))
        self._stream = stream if stream is not None else torch.cuda.current_stream()
        h = ctypes.c_void_p()
        st = self._L.mgcnn_group_create(ctypes.byref(h), ctypes.byref(o), wp,
                                        ctypes.c_void_p(self._stream.cuda_stream))
        if st != OK:
            raise MGCNNError(st, self._L.mgcnn_status_string(st).decode())
        self._h = h
        self.count = 0

    def _raise(self, st):
        if st not in (OK, NOT_CONVERGED):
            raise MGCNNError(st, self._L.mgcnn_group_last_error(self._h).decode())
        return st

    @staticmethod
    def _ptrs(ts):
        return (ctypes.c_void_p * len(ts))(*[t.data_ptr() for t in ts])

    def setup(self, a_list, b):
        """a_list: list of (n_i, n_i) float32 device tensors; b: (count, 2) host array."""
        import torch
        for t in a_list:
            _check_dev(t, torch.float32, "a")
        n = np.asarray([t.shape[-1] for t in a_list], dtype=np.int32)
        bh = np.ascontiguousarray(np.asarray(b, dtype=np.float32).reshape(len(a_list), 2))
        self._a = list(a_list)
        self._raise(self._L.mgcnn_group_setup(self._h, self._ptrs(self._a), bh.ctypes.data,
                                              n.ctypes.data, len(a_list)))
        self.count = len(a_list)

    def solve(self, f_list, u_list, tol: float, maxit: int):
        """Returns (status, iters[count], relres[count], per-problem status[count])."""
        import torch
        for t in f_list:
            _check_dev(t, torch.float32, "f")
        for t in u_list:
            _check_dev(t, self.u_dtype, "u")
        it = np.zeros(self.count, np.int32)
        rr = np.zeros(self.count, np.float64)
        ps = np.zeros(self.count, np.int32)
        st = self._L.mgcnn_group_solve(self._h, self._ptrs(f_list), self._ptrs(u_list), float(tol), int(maxit),
                                       it.ctypes.data, rr.ctypes.data, ps.ctypes.data)
        if st not in (OK, NOT_CONVERGED, E_DIVERGED):
            self._raise(st)
        return st, it, rr, ps

    @property
    def buckets(self) -> int:
        return self._L.mgcnn_group_buckets(self._h)

    @property
    def aligned(self) -> bool:
        """True when the group runs on aligned levels (one stream, one launch per operation and
        level size), False on per-size buckets."""
        return bool(self._L.mgcnn_group_aligned(self._h))

    def completion_times(self):
        """Seconds from the start of the last solve's iterations to each problem's stop (device
        wall clock); aligned levels only."""
        out = np.zeros(self.count, np.float64)
        self._raise(self._L.mgcnn_group_completion_times(self._h, out.ctypes.data))
        return out

    def close(self):
        if getattr(self, "_h", None):
            self._L.mgcnn_group_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
