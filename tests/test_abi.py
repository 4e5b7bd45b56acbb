"""The C-ABI library builds for gfx950, loads on the host and exports every entry point
declared in include/mgcnn.h (no compute calls: those need a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mgcnn.h")
LIB = os.path.join(ROOT, "paper_2312_11093_amd", "libmgcnn.so")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mgcnn_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2312_11093_amd import build
        build.build()
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = declared()
    for must in ("mgcnn_create", "mgcnn_setup", "mgcnn_solve", "mgcnn_forward", "mgcnn_apply",
                 "mgcnn_destroy", "mgcnn_num_weights"):
        assert must in names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_declares_every_export():
    from paper_2312_11093_amd import mgcnn
    assert set(declared()) <= set(mgcnn.EXPORTS), set(declared()) - set(mgcnn.EXPORTS)


def test_host_only_calls(lib):
    lib.mgcnn_num_weights.restype = ctypes.c_size_t
    assert lib.mgcnn_num_weights(16) == 21664
    assert lib.mgcnn_num_weights(8) == 81 * 64 + 58 * 8
    lib.mgcnn_status_string.restype = ctypes.c_char_p
    assert lib.mgcnn_status_string(-6) == b"diverged"
    assert lib.mgcnn_status_string(0) == b"ok"
    # argument checking before any device work
    assert lib.mgcnn_create(None, None, None, None) == -1


def test_noalloc_argument_errors_before_device_work(lib):
    """mgcnn_residual_norms_noalloc checks its arguments and its scratch bound on the host and
    returns before any HIP call: null pointers, a bad size, and an input larger than the fixed
    scratch array (MGCNN_E_SCRATCH: 200 problems at 4095^2 need 13 MB of partial sums)."""
    import numpy as np
    f = lib.mgcnn_residual_norms_noalloc
    f.restype = ctypes.c_int
    f.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                  ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]
    stand_in = np.zeros(16, np.float32)        # never dereferenced on these paths
    p = stand_in.ctypes.data
    out = np.zeros(200, np.float64)
    b = np.ones((200, 2), np.float32)
    assert f(None, b.ctypes.data, 31, 1, 0, p, p, 1, out.ctypes.data, None) == -1
    assert f(p, b.ctypes.data, 31, 1, 2, p, p, 1, out.ctypes.data, None) == -1      # form
    assert f(p, b.ctypes.data, 31, 1, 0, p, p, 2, out.ctypes.data, None) == -1      # u_dtype
    assert f(p, b.ctypes.data, 30, 1, 0, p, p, 1, out.ctypes.data, None) == -2      # n
    assert f(p, b.ctypes.data, 31, 0, 0, p, p, 1, out.ctypes.data, None) == -2      # batch
    assert f(p, b.ctypes.data, 4095, 200, 0, p, p, 1, out.ctypes.data, None) == -8  # scratch
    lib.mgcnn_status_string.restype = ctypes.c_char_p
    assert b"scratch" in lib.mgcnn_status_string(-8)


def test_tile_variant_table(lib):
    """Host-only: the tile-variant table (autotuning) accepts valid entries, rejects bad ones and
    reports the rows of every variant."""
    for fn in ("mgcnn_set_tile_variant", "mgcnn_tile_variant", "mgcnn_tile_rows"):
        getattr(lib, fn).restype = ctypes.c_int
    assert [lib.mgcnn_tile_rows(0, 0, v) for v in range(5)] == [8, 4, 16, 10, 12]
    assert [lib.mgcnn_tile_rows(3, 1, v) for v in range(5)] == [8, 4, 16, 10, 12]
    assert lib.mgcnn_tile_rows(1, 0, 0) == 4 and lib.mgcnn_tile_rows(1, 1, 0) == 8
    assert lib.mgcnn_tile_rows(1, 0, 3) == -1 and lib.mgcnn_tile_rows(4, 0, 4) == -1   # three variants
    assert lib.mgcnn_tile_rows(0, 0, 5) == -1 and lib.mgcnn_tile_rows(5, 0, 0) == -1
    assert lib.mgcnn_tile_variant(0, 0, 255) == 0
    assert lib.mgcnn_set_tile_variant(0, 0, 255, 2) == 0
    assert lib.mgcnn_tile_variant(0, 0, 255) == 2 and lib.mgcnn_tile_variant(0, 0, 511) == 0
    assert lib.mgcnn_set_tile_variant(0, 0, 255, 0) == 0
    assert lib.mgcnn_set_tile_variant(0, 0, 255, 5) == -1        # no such variant
    assert lib.mgcnn_set_tile_variant(1, 0, 255, 3) == -1        # the restriction has three
    assert lib.mgcnn_set_tile_variant(0, 0, 255, 4) == 0 and lib.mgcnn_tile_variant(0, 0, 255) == 4
    assert lib.mgcnn_set_tile_variant(0, 0, 255, 0) == 0
    assert lib.mgcnn_set_tile_variant(0, 2, 255, 0) == -1        # bad storage
    assert lib.mgcnn_set_tile_variant(2, 1, 255, 0) == -1        # the setup runs in f32
    assert lib.mgcnn_set_tile_variant(0, 0, 0, 0) == -1          # bad side


def test_no_oracle_in_product_path():
    """The product package never imports the oracle."""
    pkg = os.path.join(ROOT, "paper_2312_11093_amd")
    for dirpath, _, files in os.walk(pkg):
        for fn in files:
            if fn.endswith((".py", ".hip", ".h", ".cpp")):
                src = open(os.path.join(dirpath, fn)).read()
                assert "import oracle" not in src and "from oracle" not in src, fn


def test_default_options_and_option_checks(lib):
    """Defaults as documented in the header; invalid options are rejected by mgcnn_create
    before any device work."""
    from paper_2312_11093_amd import mgcnn
    o = mgcnn.mgcnn_opts()
    lib.mgcnn_default_opts(ctypes.byref(o))
    assert (o.channels, o.method, o.restart, o.gs_passes) == (16, 0, 30, 2)
    assert (o.precond, o.gmg_levels, o.gmg_sweeps, o.op_form, o.deflate, o.levels, o.up_post) == (0, 0, 3, 0, 0, 0, 0)
    assert o.pack_pairs == 0
    assert abs(o.gmg_omega - 0.67) < 1e-7
    h = ctypes.c_void_p()
    for field, value in (("precond", 2), ("gmg_sweeps", 0), ("gmg_sweeps", 5), ("gmg_levels", -1),
                         ("op_form", 2), ("deflate", -1), ("deflate", 33), ("levels", -12), ("levels", 13), ("up_post", 2),
                         ("gmg_omega", 0.0), ("gmg_omega", 2.0), ("gs_passes", 3), ("f32_split", 3),
                         ("f32_split", -1), ("pack_pairs", 2)):
        bad = mgcnn.mgcnn_opts()
        lib.mgcnn_default_opts(ctypes.byref(bad))
        setattr(bad, field, value)
        assert lib.mgcnn_create(ctypes.byref(h), ctypes.byref(bad), None, None) == -1, field


def test_create_checks_the_pack_pairs_options(lib):
    """Packed pairs run the stationary method with the network preconditioner and f32 or bf16
    setup tensors in the state's type: FGMRES, PCG, GMG and s_bf16 are rejected before any
    device call, for a context and for a group."""
    from paper_2312_11093_amd import mgcnn
    h = ctypes.c_void_p()
    for changes in ({"method": 1, "restart": 30}, {"method": 2, "up_post": 1}, {"precond": 1}, {"s_bf16": 1}):
        bad = mgcnn.mgcnn_opts()
        lib.mgcnn_default_opts(ctypes.byref(bad))
        bad.pack_pairs = 1
        for k, v in changes.items():
            setattr(bad, k, v)
        assert lib.mgcnn_create(ctypes.byref(h), ctypes.byref(bad), None, None) == -1, changes
    g = ctypes.c_void_p()
    for changes in ({"method": 1, "restart": 30}, {"precond": 1}, {"s_bf16": 1}):
        bad = mgcnn.mgcnn_opts()
        lib.mgcnn_default_opts(ctypes.byref(bad))
        bad.pack_pairs = 1
        for k, v in changes.items():
            setattr(bad, k, v)
        assert lib.mgcnn_group_create(ctypes.byref(g), ctypes.byref(bad), None, None) == -1, changes


def test_create_rejects_deflation_beyond_half_the_restart(lib):
    """Deflated FGMRES keeps k directions per restart and needs 2k <= restart (at least as many
    new Krylov vectors per cycle as kept ones); invalid options fail before any device call."""
    from paper_2312_11093_amd import mgcnn
    h = ctypes.c_void_p()
    for restart, k in ((9, 5), (8, 8), (20, 11), (63, 32)):
        bad = mgcnn.mgcnn_opts()
        lib.mgcnn_default_opts(ctypes.byref(bad))
        bad.method, bad.restart, bad.deflate = 1, restart, k
        assert lib.mgcnn_create(ctypes.byref(h), ctypes.byref(bad), None, None) == -1, (restart, k)


def test_create_checks_the_pcg_options(lib):
    """Conjugate gradients: the network preconditioner only in its symmetric form (up_post), the
    divergence form only, one preconditioner application per step."""
    from paper_2312_11093_amd import mgcnn
    h = ctypes.c_void_p()
    for changes in ({"up_post": 0}, {"op_form": 1}, {"inner_steps": 2}, {"method": 3}):
        bad = mgcnn.mgcnn_opts()
        lib.mgcnn_default_opts(ctypes.byref(bad))
        bad.method, bad.up_post = 2, 1
        for k, v in changes.items():
            setattr(bad, k, v)
        assert lib.mgcnn_create(ctypes.byref(h), ctypes.byref(bad), None, None) == -1, changes
