"""The C-ABI library loads and exports every entry point include/fca.h
declares (no compute calls: this runs without a GPU)."""
from __future__ import annotations

import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fca.h")
LIB = os.path.join(ROOT, "paper_1805_06572_amd", "libfca.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fca_[a-z_]+)\s*\(", src)))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for want in ("fca_init", "fca_em_step", "fca_separate", "fca_destroy", "fca_gevd"):
        assert want in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libfca.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for name in declared_functions():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (fca_[a-z_]+)\b", out))
    assert set(declared_functions()) <= exported


@pytest.mark.skipif(not os.path.exists(LIB), reason="libfca.so not built")
def test_binding_names_match_the_header():
    from paper_1805_06572_amd import fca
    assert sorted(fca.EXPORTED) == declared_functions()
    for name in fca.EXPORTED:
        assert callable(getattr(fca, name))


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    from paper_1805_06572_amd import fca
    monkeypatch.setattr(fca, "_lib", None)
    monkeypatch.setattr(fca, "_LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError, match="missing"):
        fca.lib()
