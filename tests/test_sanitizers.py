"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer, on the CPU.

The C oracle (gcc instrumentation, gcc's libasan preloaded) and the library's host code
(argument checks, level planning, workspace layout, schedules; clang instrumentation of the
host side, clang's ASan runtime preloaded) run the workloads of tests/sanitize_child.py in a
child process.  Every sanitizer report ends the child with an error; its results must equal
those of the regular builds in this process.  The mesh closedness check has its own
sanitized build in test_mesh_check.py.  Leak detection is off in these children (the Python
interpreter keeps its own allocations to the end); the mesh-check executable runs with it.
"""
import os
import shutil
import subprocess
import sys

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CHILD = os.path.join(HERE, "sanitize_child.py")
SAN_ENV = {"ASAN_OPTIONS": "detect_leaks=0:halt_on_error=1:abort_on_error=0",
           "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"}


def _gcc_asan():
    if shutil.which("gcc") is None:
        pytest.skip("no gcc")
    path = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(path) or not os.path.exists(path):
        pytest.skip("gcc's libasan is not installed")
    return path


def _child(kind, out, env_extra, preload):
    env = dict(os.environ, **SAN_ENV, **env_extra, LD_PRELOAD=preload)
    r = subprocess.run([sys.executable, CHILD, kind, str(out)], env=env, capture_output=True, text=True,
                       timeout=600)
    assert r.returncode == 0, "sanitized %s run failed:\n%s" % (kind, r.stderr[-4000:])
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-4000:]
    return np.load(out)


def _same(ref, got):
    assert sorted(ref) == sorted(got.files)
    bad = [k for k in ref if not np.array_equal(ref[k], got[k], equal_nan=True)]
    assert not bad, bad


def test_sanitizer_harness_reports_a_planted_overflow(tmp_path):
    """The set-up catches what it is for: a C file with a one-past-the-end heap read, built
    and loaded the same way as the oracle, ends the child with an ASan report."""
    from oracle.oracle import build_oracle_sanitized
    src = tmp_path / "planted.c"
    src.write_text("#include <stdlib.h>\n"
                   "double planted(int n) { double *a = malloc(sizeof(double) * n);\n"
                   "  for (int i = 0; i < n; ++i) a[i] = i;\n"
                   "  double s = a[n]; free(a); return s; }\n")
    lib = build_oracle_sanitized(str(tmp_path / "planted.so"), src=str(src))
    code = ("import ctypes as C; L = C.CDLL(%r); L.planted.restype = C.c_double; "
            "L.planted.argtypes = [C.c_int]; print(L.planted(8))" % lib)
    env = dict(os.environ, **SAN_ENV, LD_PRELOAD=_gcc_asan())
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=120)
    assert r.returncode != 0 and "heap-buffer-overflow" in r.stderr


def test_oracle_under_asan_ubsan(tmp_path):
    from oracle.oracle import build_oracle_sanitized
    sys.path.insert(0, HERE)
    import sanitize_child
    ref = sanitize_child.oracle_case()
    lib = build_oracle_sanitized(str(tmp_path / "liboracle_san.so"))
    got = _child("oracle", tmp_path / "oracle.npz", {"ORACLE_LIB": lib}, _gcc_asan())
    _same(ref, got)


def test_library_host_code_under_asan_ubsan(tmp_path):
    from paper_2505_17287_amd.build import asan_runtime, build_host_sanitized
    try:
        rt = asan_runtime()
    except FileNotFoundError as e:
        pytest.skip(str(e))
    sys.path.insert(0, HERE)
    import sanitize_child
    ref = sanitize_child.library_case()
    lib = build_host_sanitized(str(tmp_path / "ibmsan"))
    got = _child("library", tmp_path / "library.npz", {"IBM_LIB": lib}, rt)
    _same(ref, got)
