"""The C ABI library loads on the CPU and exports every entry point that
include/membed.h declares (no GPU call is made)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "membed.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(me_[a-z_0-9]+)\s*\(", text)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("me_build_graph_ops", "me_build_workspace_bytes", "me_embed",
                     "me_embed_workspace_bytes", "me_embed_batch_workspace_bytes",
                     "me_graph_ops_export", "me_graph_ops_destroy", "me_status_string"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_2112_07862_amd import _lib
    lib = _lib.load()
    for name in declared_functions():
        assert hasattr(lib, name), name
        assert name in _lib.SIGNATURES, f"{name} has no ctypes signature"


def test_host_only_entry_points():
    from paper_2112_07862_amd import _lib
    lib = _lib.load()
    o = _lib.MeOpts()
    lib.me_opts_default(ctypes.byref(o))
    assert o.precond == _lib.ME_PRECOND_CHEBYSHEV and o.max_iter > 0 and o.check_every > 0
    assert 0 < o.eps_tol <= 1e-6
    for st in list(_lib.STATUS_NAMES):
        assert lib.me_status_string(st).decode()
    assert lib.me_embed_workspace_bytes(None, 4, None) == 0
    assert lib.me_graph_ops_bytes(None) == 0


def test_invalid_options_rejected_before_device_work():
    """Option checks run on the host before any device call."""
    from paper_2112_07862_amd import _lib
    lib = _lib.load()
    W = _lib.MeCsr()
    h = ctypes.c_void_p()
    for field, val in [("cheb_degree", 1), ("cheb_degree", 257), ("precond", 3),
                       ("precision", 2), ("max_iter", 0), ("check_every", 0),
                       ("eps_tol", 0.0), ("cheb_op", 2), ("cheb_op", -1),
                       ("addressing", 2), ("addressing", -1),
                       ("cheb_iterates", 2), ("cheb_iterates", -1)]:
        o = _lib.MeOpts()
        lib.me_opts_default(ctypes.byref(o))
        setattr(o, field, val)
        st = lib.me_build_graph_ops(ctypes.byref(W), ctypes.byref(o), None, 0, None,
                                    ctypes.byref(h), None)
        assert _lib.STATUS_NAMES[st] == "ME_ERR_INVALID_ARG", (field, val, st)


def test_workspace_too_small_rejected_before_device_work():
    """A caller workspace smaller than any call can use is ME_ERR_WORKSPACE,
    decided on the host (no device call is made): the build, the batch and a
    server over a region."""
    from paper_2112_07862_amd import _lib
    lib = _lib.load()
    W = _lib.MeCsr()
    W.n = 4
    h = ctypes.c_void_p()
    buf = ctypes.create_string_buffer(64)  # any non-null address; never dereferenced
    ws = ctypes.cast(buf, ctypes.c_void_p)
    st = lib.me_build_graph_ops(ctypes.byref(W), None, ws, 16, None, ctypes.byref(h), None)
    assert _lib.STATUS_NAMES[st] == "ME_ERR_WORKSPACE"
    Ws = (_lib.MeCsr * 1)(W)
    Ks = (ctypes.c_int * 1)(4)
    Xs = (ctypes.c_void_p * 1)(ws.value)
    Ls = (ctypes.c_void_p * 1)(ws.value)
    st = lib.me_embed_batch(1, Ws, Ks, 1e-6, None, ws, 16, Xs, Ls, None, None)
    assert _lib.STATUS_NAMES[st] == "ME_ERR_WORKSPACE"
    so = _lib.MeServerOpts()
    lib.me_server_opts_default(ctypes.byref(so))
    assert so.workspace is None
    so.workspace = ws.value
    so.mem_budget = 1 << 20
    srv = ctypes.c_void_p()
    st = lib.me_server_create(ctypes.byref(so), None, ctypes.byref(srv))
    assert _lib.STATUS_NAMES[st] == "ME_ERR_WORKSPACE" and not srv.value
    so.mem_budget = 0
    st = lib.me_server_create(ctypes.byref(so), None, ctypes.byref(srv))
    assert _lib.STATUS_NAMES[st] == "ME_ERR_WORKSPACE" and not srv.value


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    from paper_2112_07862_amd import _lib
    monkeypatch.setattr(_lib, "_lib", None)
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "absent.so"))
    with pytest.raises(RuntimeError, match="not found"):
        _lib.load()


def test_product_path_does_not_import_the_oracle():
    pkg = os.path.join(ROOT, "paper_2112_07862_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".h")):
                src = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in src and "from oracle" not in src, f
                assert "synthgraphs" not in src, f
