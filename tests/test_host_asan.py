"""Host-side memory checks on the CPU: the oracle and the library's host code
built with AddressSanitizer (and UBSan for the oracle), driven in a child
process with the sanitizer runtime preloaded.  The oracle runs whole hybrid
steps with encounter sets and the Hermite, the energy and a Kepler batch;
the library's C ABI runs its host-only paths: the workspace layout of many
system mixes (empty systems, one body, thousands of systems) and argument
validation, and context creation failing cleanly without a GPU.  Any
sanitizer report fails the test.  (The device code is built as usual; only
the host side is instrumented.)"""
import glob
import os
import shutil
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
pytestmark = pytest.mark.slow


def _run(env_extra, code, tmp_path):
    script = tmp_path / "drive.py"
    script.write_text(textwrap.dedent(code))
    env = dict(os.environ)
    env.update(env_extra)
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=0:exitcode=42"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:exitcode=43"
    p = subprocess.run([sys.executable, str(script)], env=env, capture_output=True, text=True,
                       timeout=600)
    out = p.stdout + p.stderr
    assert p.returncode == 0, out[-4000:]
    assert "ERROR: AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    return out


def test_oracle_under_asan_and_ubsan(tmp_path):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no C compiler")
    lib = tmp_path / "liboracle_asan.so"
    srcs = [os.path.join(ROOT, "oracle", f) for f in ("qsym_oracle.c", "kepler_guess_oracle.c")]
    subprocess.check_call([gcc, "-O1", "-g", "-fPIC", "-shared", "-ffp-contract=off",
                           "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
                           "-fno-sanitize-recover=undefined", "-o", str(lib), *srcs, "-lm"])
    pre = subprocess.check_output([gcc, "-print-file-name=libasan.so"]).decode().strip()
    ub = subprocess.check_output([gcc, "-print-file-name=libubsan.so"]).decode().strip()
    out = _run({"LD_PRELOAD": pre + ":" + ub}, f"""
        import sys
        sys.path.insert(0, {ROOT!r})
        import numpy as np
        import oracle
        oracle.LIB = {str(lib)!r}
        oracle.build = lambda force=False: oracle.LIB
        from paper_1007_3458_amd import inputs
        p = oracle.make_params()
        s = inputs.make_disk("crowd", 5, 92, 1e-6, 4.5, 6.0, "uniform", "uniform", 0.05, 0.01)
        q, v = s.q, s.v
        npairs = 0
        for _ in range(6):
            q, v, r = oracle.step(p, 0.05, s.m, s.h, q, v)
            npairs += len(r.pairs)
        assert npairs > 0
        w = inputs.two_planet_encounter(6)
        q2, v2, r2 = oracle.step(oracle.make_params(planet_mass=1e-4), 0.05, w.m, w.h, w.q, w.v)
        assert r2.stats["whole_system"] == 1
        E = oracle.energy(s.G, s.m0, s.m, q, v)
        t = inputs.kepler_test(300, seed=3)
        x, it, fails = oracle.kepler_roots(1.0, t.q, t.v, 0.05, 0)
        assert fails == 0
        print("oracle asan ok", npairs, E)
    """, tmp_path)
    assert "oracle asan ok" in out


def test_library_host_code_under_asan(tmp_path):
    hipcc = "/opt/rocm/bin/hipcc"
    rt = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not os.path.exists(hipcc) or not rt:
        pytest.skip("no hipcc or no clang ASan runtime")
    lib = tmp_path / "libqsym_asan.so"
    csrc = os.path.join(ROOT, "paper_1007_3458_amd", "csrc")
    host_asan = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fno-omit-frame-pointer"]
    subprocess.check_call([hipcc, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC",
                           "-shared", "-ffp-contract=off", "-Xclang", "-target-feature", "-Xclang",
                           "-packed-fp32-ops", *host_asan, "-I", os.path.join(ROOT, "include"),
                           "-o", str(lib), os.path.join(csrc, "qsym.hip"),
                           os.path.join(csrc, "qsym_guess.hip")],
                          stderr=subprocess.DEVNULL)
    out = _run({"LD_PRELOAD": rt[-1]}, f"""
        import ctypes as C
        import numpy as np
        import sys
        sys.path.insert(0, {ROOT!r})
        from paper_1007_3458_amd import inputs
        L = C.CDLL({str(lib)!r})
        class P(C.Structure):
            _fields_ = [("G", C.c_double), ("aE", C.c_double), ("aH", C.c_double),
                        ("epsH", C.c_double), ("eta", C.c_double), ("eta_s", C.c_double),
                        ("crude_safety", C.c_double), ("hill_mode", C.c_int32),
                        ("kepler_mode", C.c_int32), ("precision", C.c_int32),
                        ("max_substeps", C.c_int32), ("pair_capacity", C.c_int64),
                        ("planet_mass", C.c_double), ("sweep", C.c_int32), ("pad2", C.c_int32)]
        lp = C.POINTER(C.c_int64)
        def ws(sizes, **kw):
            d = dict(G=1.0, aE=3.0, aH=1.0, epsH=1e-8, eta=0.02, eta_s=0.01, crude_safety=1.1,
                     hill_mode=0, kepler_mode=0, precision=0, max_substeps=1000, pair_capacity=0,
                     planet_mass=0.0, sweep=0, pad2=0)
            d.update(kw)
            p = P(**d)
            off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
            nb = C.c_int64()
            rc = L.qsym_workspace_bytes(C.byref(p), len(sizes), off.ctypes.data_as(lp), C.byref(nb))
            return rc, nb.value
        mixes = [[104], [16388], [0], [1], [0, 5, 0, 2], list(inputs.batch_sizes()),
                 [1] * 3000, [131076], [300, 70000, 2]]
        for sizes in mixes:
            for kw in ({{}}, {{"sweep": 1}}, {{"planet_mass": 1e-4}}, {{"pair_capacity": 3}}):
                rc, nb = ws(sizes, **kw)
                assert rc == 0 and nb > 0, (sizes[:4], kw, rc)
        assert ws([5, 3], crude_safety=0.5)[0] == -1
        assert ws([5, 3], kepler_mode=9)[0] == -1
        off = np.array([0, 10, 5], np.int64)
        p = P(1.0, 3.0, 1.0, 1e-8, 0.02, 0.01, 1.1, 0, 0, 0, 100, 0, 0.0, 0, 0)
        nb = C.c_int64()
        assert L.qsym_workspace_bytes(C.byref(p), 2, off.ctypes.data_as(lp), C.byref(nb)) == -1
        # creation with a host buffer and no GPU fails cleanly (no context leaks a pointer)
        m0 = np.ones(1)
        off = np.array([0, 100], np.int64)
        buf = (C.c_char * (8 << 20))()
        base = (C.addressof(buf) + 255) // 256 * 256
        h = C.c_void_p()
        m0p = m0.ctypes.data_as(C.POINTER(C.c_double))
        rc = L.qsym_create(C.byref(p), 1, off.ctypes.data_as(lp), m0p, C.c_void_p(base), 16, None,
                           C.byref(h))
        assert rc == -2 and not h.value
        rc = L.qsym_create(C.byref(p), 1, off.ctypes.data_as(lp), m0p, C.c_void_p(base),
                           (7 << 20), None, C.byref(h))
        assert rc != 0 and not h.value
        print("library host asan ok")
    """, tmp_path)
    assert "library host asan ok" in out
