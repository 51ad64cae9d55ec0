"""The library's host-side planner and validation under AddressSanitizer and UndefinedBehaviorSanitizer:
every source is compiled with the sanitizers on its host code (device code unchanged) and linked with
`tests/sanitize/planner_check.cpp`, which exercises geometry and per-view validation on valid and
invalid inputs and the out-of-core planner over every direction, storage type and a sweep of caps.
Nothing it calls touches a GPU.  CPU only (about a minute to build)."""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1905_03748_amd", "csrc")
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=undefined"]


def _hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc"):
        if c and os.path.exists(c):
            return c
    return shutil.which("hipcc")


@pytest.mark.skipif(_hipcc() is None, reason="hipcc not available")
def test_planner_and_validation_under_sanitizers():
    hipcc = _hipcc()
    out = tempfile.mkdtemp(prefix="ct_asan_")
    try:
        common = ["-O1", "-g", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-I", os.path.join(ROOT, "include")]
        procs, objs = [], []
        srcs = sorted(f for f in os.listdir(CSRC) if f.endswith((".cpp", ".hip")))
        srcs = [os.path.join(CSRC, f) for f in srcs] + [os.path.join(ROOT, "tests", "sanitize", "planner_check.cpp")]
        for src in srcs:
            obj = os.path.join(out, os.path.basename(src) + ".o")
            lang = ["-x", "hip", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"] if src.endswith(".hip") else []
            procs.append(subprocess.Popen([hipcc] + lang + ["-c", src, "-o", obj] + common + HOST_SAN,
                                          stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True))
            objs.append(obj)
        for p, src in zip(procs, srcs):
            log = p.communicate(timeout=600)[0]
            assert p.returncode == 0, f"{src}:\n{log[-3000:]}"
        exe = os.path.join(out, "planner_check")
        r = subprocess.run([hipcc, "-o", exe] + objs + ["--offload-arch=gfx950"] + HOST_SAN, capture_output=True,
                           text=True, timeout=600)
        assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-2000:]
        # the binary carries the sanitizers' runtime
        nm = subprocess.run(["nm", exe], capture_output=True, text=True).stdout
        assert "__asan_init" in nm and "__ubsan_handle" in nm
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1:abort_on_error=0",
                   UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
        r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
        assert r.returncode == 0 and "planner check: 0 failures" in r.stdout, (r.stdout[-3000:], r.stderr[-5000:])
        assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-5000:]
    finally:
        shutil.rmtree(out, ignore_errors=True)
