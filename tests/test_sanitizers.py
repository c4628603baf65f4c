"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU).

Two drivers in tests/sanitize/ are built with the sanitizers and run:
  * oracle_driver.c: every C routine of the oracle on a closed mesh with two
    vertices of valence 80;
  * host_driver.cpp: the library's host-side mesh preparation (mesh_prep.cpp,
    built host-only) on the same mesh, on a torus large enough for its
    threaded passes, and on malformed ones, which must be rejected with
    PB_E_MESH / PB_E_INVALID_ARG; also built with ThreadSanitizer.
Device code is not instrumented (GPU sanitizers are not used here)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = os.path.join(ROOT, "tests", "sanitize")
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout}\n{r.stderr}"
    return r


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_c_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    _run(["gcc", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
          "-fno-omit-frame-pointer", "-o", exe, os.path.join(ROOT, "oracle", "pbm_oracle.c"),
          os.path.join(SAN, "oracle_driver.c"), "-lm"])
    r = _run([exe], env=ENV)
    assert r.stdout.strip() == "ok"


HIPCC = "/opt/rocm/bin/hipcc"
CLANG = "/opt/rocm/llvm/bin/clang++"


def _host_driver(tmp_path, sanitizers):
    flags = ["-x", "hip", "--cuda-host-only", "-O1", "-g", "-std=c++17",
             "-Xarch_host", "-fno-omit-frame-pointer", "-I", os.path.join(ROOT, "include")]
    for s in sanitizers:
        flags += ["-Xarch_host", "-fsanitize=" + s]
    if "thread" not in sanitizers:
        flags += ["-Xarch_host", "-fno-sanitize-recover=all"]
    objs = []
    for src in (os.path.join(ROOT, "paper_2108_10481_amd", "csrc", "mesh_prep.cpp"),
                os.path.join(SAN, "host_driver.cpp")):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        _run([HIPCC] + flags + ["-c", src, "-o", obj])
        objs.append(obj)
    exe = str(tmp_path / "host_driver")
    _run([CLANG, "-fsanitize=" + ",".join(sanitizers), "-pthread", "-o", exe] + objs)
    env = dict(ENV, TSAN_OPTIONS="halt_on_error=1")
    r = _run([exe], env=env)
    assert r.stdout.strip() == "ok"


@pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANG)), reason="ROCm compilers not available")
def test_host_mesh_preparation_under_sanitizers(tmp_path):
    _host_driver(tmp_path, ["address", "undefined"])


@pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANG)), reason="ROCm compilers not available")
def test_host_mesh_preparation_under_thread_sanitizer(tmp_path):
    _host_driver(tmp_path, ["thread"])
