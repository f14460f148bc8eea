"""The C-ABI library loads on the CPU host and exports every declared symbol."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "st.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(st_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    syms = declared_symbols()
    for need in ("st_problem_create", "st_extend_batch", "st_check_edges", "st_nearest", "st_plan"):
        assert need in syms


def test_library_exports_every_declared_symbol():
    from paper_2609_30533_amd import lib
    if not os.path.exists(lib.LIB_PATH):
        pytest.skip("library not built")
    L = ctypes.CDLL(lib.LIB_PATH)
    missing = [s for s in declared_symbols() if not hasattr(L, s)]
    assert not missing, missing
    assert sorted(lib.EXPORTS) == declared_symbols()


def test_no_cpu_fallback_when_library_missing(monkeypatch, tmp_path):
    from paper_2609_30533_amd import lib
    monkeypatch.setattr(lib, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(lib, "_lib", None)
    with pytest.raises(lib.StError):
        lib.load()
