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
    assert abs(o.gmg_omega - 0.67) < 1e-7
    h = ctypes.c_void_p()
    for field, value in (("precond", 2), ("gmg_sweeps", 0), ("gmg_sweeps", 5), ("gmg_levels", -1),
                         ("op_form", 2), ("deflate", -1), ("deflate", 33), ("levels", -12), ("levels", 13), ("up_post", 2),
                         ("gmg_omega", 0.0), ("gmg_omega", 2.0), ("gs_passes", 3), ("f32_split", 3),
                         ("f32_split", -1)):
        bad = mgcnn.mgcnn_opts()
        lib.mgcnn_default_opts(ctypes.byref(bad))
        setattr(bad, field, value)
        assert lib.mgcnn_create(ctypes.byref(h), ctypes.byref(bad), None, None) == -1, field


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
