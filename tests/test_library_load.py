"""The C-ABI library loads and exports every symbol include/bpm_llg.h declares (no GPU calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            names |= set(re.findall(r"^\s*(?:int|void|const char\*)\s+(bpm_\w+)\s*\(", txt, re.M))
    return names


def test_library_exports_every_declared_symbol():
    from paper_1603_09493_amd import bpm
    if not os.path.exists(bpm.LIB_PATH):
        pytest.fail("libbpmllg.so is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(bpm.LIB_PATH)
    decl = _declared_symbols()
    assert len(decl) >= 15
    missing = [s for s in sorted(decl) if not hasattr(lib, s)]
    assert not missing, missing
    # the binding knows them all too
    assert decl <= set(bpm.SYMBOLS) | set(getattr(bpm, "EXTRA_SYMBOLS", []))


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    from paper_1603_09493_amd import bpm
    monkeypatch.setattr(bpm, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(bpm, "_lib", None)
    with pytest.raises(ImportError):
        bpm.lib()
