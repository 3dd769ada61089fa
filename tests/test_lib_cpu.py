"""Host-only checks of the C-ABI library: it loads, exports every entry point
the header declares, and the binding refuses to run without it."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "polylla.h")
LIB = os.path.join(ROOT, "paper_2204_05438_amd", "libpolylla.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(polylla_[a-z_]+)\s*\(", src)))


def test_header_declares_entry_points():
    names = declared_functions()
    for n in ["polylla_label", "polylla_build", "polylla_repair", "polylla_mesh"]:
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_strerror_without_gpu():
    from paper_2204_05438_amd import lib
    assert lib.strerror(0) == "ok"
    assert "capacity" in lib.strerror(lib.ECAPACITY)


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    from paper_2204_05438_amd import lib
    monkeypatch.setattr(lib, "_lib", None)
    monkeypatch.setattr(lib, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError, match="no fallback"):
        lib.load()
