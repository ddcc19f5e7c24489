"""CPU-side checks of the C ABI library: it loads, and it exports every entry
point that include/lss.h declares (no compute call: there is no GPU here)."""
import ctypes
import os
import re

import numpy as np
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
    # lss_options: 4 int32, 2 double, 2 int32, 1 double, count_useful, admissibility, curved_charts,
    # sigma_interp, 2 int32 reserved
    assert ctypes.sizeof(Options) == 4 * 4 + 2 * 8 + 2 * 4 + 8 + 4 + 4 + 4 + 4 + 2 * 4
    assert ctypes.sizeof(Stats) == 8 * 2 + 4 * 2 + 8 * 3 + 4 * 2 + 8 + 8 + 8 + 8 + 4 + 4 + 8 + 8 + 8 + 8


def test_struct_offsets_match_the_c_header(tmp_path):
    """Every field offset of the ctypes structures equals offsetof() in a C
    program compiled against include/lss.h."""
    import shutil
    import subprocess
    from paper_1909_13356_amd._binding import Options, Stats
    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "lss.h"', 'int main(void) {']
    for cname, S in (("lss_options", Options), ("lss_stats", Stats)):
        lines.append('printf("%%s sizeof %%zu\\n", "%s", sizeof(%s));' % (cname, cname))
        for f, _ in S._fields_:
            lines.append('printf("%%s %%s %%zu\\n", "%s", "%s", offsetof(%s, %s));' % (cname, f, cname, f))
    lines.append("return 0; }")
    src = tmp_path / "off.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "off"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    got = {}
    for line in subprocess.check_output([str(exe)]).decode().splitlines():
        a, b, v = line.split()
        got[(a, b)] = int(v)
    for cname, S in (("lss_options", Options), ("lss_stats", Stats)):
        assert got[(cname, "sizeof")] == ctypes.sizeof(S), cname
        for f, _ in S._fields_:
            assert got[(cname, f)] == getattr(S, f).offset, (cname, f)


def test_missing_library_fails_loudly(monkeypatch):
    import paper_1909_13356_amd._binding as b
    monkeypatch.setattr(b, "_lib", None)
    monkeypatch.setattr(b, "_LIBPATH", "/nonexistent/liblss.so")
    with pytest.raises(ImportError):
        b.load_library()


def test_default_rule_is_dunavant6():
    """lss_default_rule (the rule that rule_uvw == NULL selects): host-only, no
    device.  The same 12 rows as the rule the tests pass explicitly, bit for
    bit (both are built from the published orbit parameters), and exact on
    every monomial u^i v^j of degree <= 6 over T0 (integral i! j! / (i+j+2)!)."""
    if not os.path.exists(lss.library_path()):
        pytest.skip("liblss.so not built")
    from math import factorial
    from workloads import dunavant6
    r = lss.default_rule()
    assert r.shape == (12, 3)
    assert np.array_equal(r, dunavant6())
    u, v, w = r.T
    for i in range(7):
        for j in range(7 - i):
            exact = factorial(i) * factorial(j) / factorial(i + j + 2)
            assert abs(np.sum(w * u ** i * v ** j) - exact) < 2e-16, (i, j)
    assert np.all(u > 0) and np.all(v > 0) and np.all(u + v < 1)
    L = lss.load_library()
    assert L.lss_default_rule(None, 0) == 12
