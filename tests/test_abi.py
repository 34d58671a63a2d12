"""The C ABI library loads and exports every entry point that include/dass.h declares (no GPU
compute is called), and the product package and the oracle stay independent."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dass.h")
PKG = os.path.join(ROOT, "paper_2411_14847_amd")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^(?:const\s+)?(?:dass_status|void|const char\*|char\*)\s*\**\s*(\w+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_hot_path_entry_points():
    names = declared_functions()
    for required in ("render_fwd", "render_bwd", "shift_apply", "adam_step", "densify_append"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_2411_14847_amd import _ffi
    assert os.path.exists(_ffi.LIB_PATH), "libdass.so not built (run __graft_entry__.build())"
    lib = ctypes.CDLL(_ffi.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), f"{name} declared in include/dass.h but not exported"
    assert sorted(_ffi.EXPORTS) == declared_functions()


def test_binding_declares_every_symbol():
    from paper_2411_14847_amd import _ffi
    lib = _ffi.lib()
    for name in declared_functions():
        assert getattr(lib, name).argtypes is not None or getattr(lib, name).restype is None


def test_null_context_is_rejected_without_a_device():
    from paper_2411_14847_amd import _ffi
    lib = _ffi.lib()
    assert lib.render_fwd(None, None, None, 1, None, None, None, None) == _ffi.DASS_E_INVALID
    assert lib.adam_step(None, None, 0, 0.9, 0.999, 1e-15, 1, None) == _ffi.DASS_E_INVALID
    assert lib.dass_sync(None, None) == _ffi.DASS_E_INVALID
    out = ctypes.c_void_p()
    assert lib.dass_create(ctypes.byref(out), 0, None) == _ffi.DASS_E_INVALID


def test_missing_library_raises(monkeypatch, tmp_path):
    from paper_2411_14847_amd import _ffi
    monkeypatch.setattr(_ffi, "_lib", None)
    monkeypatch.setattr(_ffi, "LIB_PATH", str(tmp_path / "nope.so"))
    with pytest.raises(_ffi.MissingLibrary):
        _ffi.lib()


def _py_sources(d):
    for base, _, files in os.walk(d):
        if "_build" in base or "__pycache__" in base:
            continue
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".c", ".cpp")):
                yield os.path.join(base, f)


def test_product_never_touches_the_oracle():
    for path in _py_sources(PKG):
        text = open(path).read()
        assert not re.search(r"^\s*(import|from)\s+oracle\b", text, flags=re.M), path
        assert "liboracle" not in text and "dass_oracle" not in text, path


def test_oracle_never_touches_the_product():
    for path in _py_sources(os.path.join(ROOT, "oracle")):
        text = open(path).read()
        assert "paper_2411_14847_amd" not in text and "libdass" not in text, path
