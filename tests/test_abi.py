"""CPU-side checks of the C ABI library: it loads, and it exports every entry
point that include/lss.h declares (no compute call: there is no GPU here)."""
import ctypes
import os
import re

import pytest

import paper_1909_13356_amd as lss

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "lss.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lss_[a-z_]+)\s*\(", src)))


def test_header_declarations_match_binding():
    assert declared_symbols() == sorted(lss.EXPORTED_SYMBOLS)


def test_library_exports_every_declared_symbol():
    if not os.path.exists(lss.library_path()):
        pytest.skip("liblss.so not built")
    L = ctypes.CDLL(lss.library_path())
    for name in declared_symbols():
        assert hasattr(L, name), name


def test_struct_layouts():
    from paper_1909_13356_amd._binding import Options, Stats
    # lss_options: 4 int32, 2 double, 2 int32, 1 double, 6 int32 reserved
    assert ctypes.sizeof(Options) == 4 * 4 + 2 * 8 + 2 * 4 + 8 + 6 * 4
    assert ctypes.sizeof(Stats) == 8 * 2 + 4 * 2 + 8 * 3 + 4 * 2 + 8 + 8 + 8 + 8 + 4 + 4 + 8 + 8


def test_missing_library_fails_loudly(monkeypatch):
    import paper_1909_13356_amd._binding as b
    monkeypatch.setattr(b, "_lib", None)
    monkeypatch.setattr(b, "_LIBPATH", "/nonexistent/liblss.so")
    with pytest.raises(ImportError):
        b.load_library()
