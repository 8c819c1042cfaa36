"""CPU-side checks of the C ABI library: it loads, exports every entry point
declared in include/qsym.h, and its host-only calls validate arguments."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    hdr = open(os.path.join(ROOT, "include", "qsym.h")).read()
    return re.findall(r"^\s*(?:int|void|const char \*)\s*(qsym_\w+)\s*\(", hdr, re.M)


def test_library_exports_every_declared_symbol():
    from paper_1007_3458_amd import qsym
    L = qsym.lib()
    names = declared()
    assert len(names) >= 18
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(qsym.SIGNATURES)


def test_workspace_bytes_and_validation():
    from paper_1007_3458_amd import qsym
    L = qsym.lib()
    p = qsym.make_params()
    off = np.array([0, 100, 100, 5000], np.int64)
    nb = C.c_int64()
    assert L.qsym_workspace_bytes(C.byref(p), 3, off.ctypes.data_as(qsym._lp), C.byref(nb)) == 0
    assert nb.value > 5000 * 8 * 17
    bad = np.array([0, 10, 5], np.int64)
    assert L.qsym_workspace_bytes(C.byref(p), 2, bad.ctypes.data_as(qsym._lp), C.byref(nb)) == -1
    p2 = qsym.make_params(crude_safety=0.5)
    assert L.qsym_workspace_bytes(C.byref(p2), 3, off.ctypes.data_as(qsym._lp), C.byref(nb)) == -1
    p3 = qsym.make_params(kepler_mode=7)
    assert L.qsym_workspace_bytes(C.byref(p3), 3, off.ctypes.data_as(qsym._lp), C.byref(nb)) == -1


def test_params_struct_layout_matches_header():
    from paper_1007_3458_amd import qsym
    assert C.sizeof(qsym.Params) == 7 * 8 + 4 * 4 + 8 + 8 + 2 * 4
    assert C.sizeof(qsym.Stats) == 10 * 8 + 32 * 8 + 8 + 12 * 8 + 12 * 8 + 8 + 4 * 8 + 3 * 12 * 8 + 8


def test_product_path_does_not_import_oracle():
    """The HIP binding and package never reach the oracle."""
    pkg = os.path.join(ROOT, "paper_1007_3458_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".h", ".cpp")):
                src = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in src and "from oracle" not in src, f
                assert "qsym_oracle" not in src and "liboracle" not in src, f


def test_params_and_stats_match_the_c_header(tmp_path):
    """Sizes and field offsets of the ctypes mirrors equal the C compiler's."""
    import shutil
    import subprocess
    from paper_1007_3458_amd import qsym
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no C compiler")
    fields = [f for f, _ in qsym.Params._fields_]
    sfields = [f for f, _ in qsym.Stats._fields_]
    src = tmp_path / "probe.c"
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "qsym.h"', 'int main(void) {',
             'printf("%zu %zu\\n", sizeof(qsym_params), sizeof(qsym_stats_t));']
    lines += [f'printf("%zu\\n", offsetof(qsym_params, {f}));' for f in fields]
    lines += [f'printf("%zu\\n", offsetof(qsym_stats_t, {f}));' for f in sfields]
    lines += ['return 0; }']
    src.write_text("\n".join(lines))
    exe = tmp_path / "probe"
    subprocess.check_call([gcc, "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)])
    out = subprocess.check_output([str(exe)]).decode().split()
    sp, ss = int(out[0]), int(out[1])
    assert sp == C.sizeof(qsym.Params) and ss == C.sizeof(qsym.Stats)
    offs = [int(x) for x in out[2:]]
    assert offs[:len(fields)] == [getattr(qsym.Params, f).offset for f in fields]
    assert offs[len(fields):] == [getattr(qsym.Stats, f).offset for f in sfields]
