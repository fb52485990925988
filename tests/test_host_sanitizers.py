"""The C ABI's host code under AddressSanitizer and UndefinedBehaviorSanitizer.

Every library source is compiled with both sanitizers on its host code (the
device code is built as usual and never runs), linked with
tests/host/abi_driver.cpp, and run on the CPU:
the driver drives the argument validation and the size queries of every
entry point (invalid descriptors, null and aliasing pointers, short
workspaces, the batch tables, the study's limits) and checks the return
codes.  A sanitizer report or a wrong code fails the test."""
import hashlib
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2507_15464_amd", "csrc")
DRIVER = os.path.join(ROOT, "tests", "host", "abi_driver.cpp")
BUILD = os.path.join(ROOT, "tests", "host", "_build")
# sanitizers on the host pass only (each -fsanitize= behind -Xarch_host)
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=undefined"]
FLAGS = ["--offload-arch=gfx950", "-O1", "-g", "-fno-omit-frame-pointer", "-std=c++17", "-Wno-unused-command-line-argument",
         f"-I{os.path.join(ROOT, 'include')}"]


def _hipcc():
    for c in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if c and os.path.exists(c):
            return c
    return None


def _sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".hip", ".cpp")))


def _digest(paths):
    h = hashlib.sha256()
    for p in paths + [os.path.join(ROOT, "include", "tidas.h")]:
        with open(p, "rb") as f:
            h.update(f.read())
    h.update(" ".join(FLAGS + SAN).encode())
    return h.hexdigest()[:16]


def _build():
    hipcc = _hipcc()
    if hipcc is None:
        pytest.skip("hipcc not available")
    srcs = _sources() + [DRIVER]
    exe = os.path.join(BUILD, f"abi_driver_{_digest(srcs)}")
    if os.path.exists(exe):
        return exe
    os.makedirs(BUILD, exist_ok=True)
    objs, procs = [], []
    for src in srcs:
        obj = os.path.join(BUILD, os.path.basename(src) + ".o")
        objs.append(obj)
        procs.append(subprocess.Popen([hipcc] + FLAGS + SAN + ["-x", "hip", "-c", src, "-o", obj],
                                      stdout=subprocess.PIPE, stderr=subprocess.PIPE))
    for p, src in zip(procs, srcs):
        out, err = p.communicate()
        if p.returncode != 0:
            raise AssertionError(f"compile of {src} failed:\n{err.decode()[-3000:]}")
    r = subprocess.run([hipcc, "--offload-arch=gfx950"] + SAN + ["-o", exe] + objs, capture_output=True, text=True)
    if r.returncode != 0:
        raise AssertionError(f"link failed:\n{r.stderr[-3000:]}")
    return exe


def test_abi_validation_under_asan_and_ubsan():
    exe = _build()
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", HIP_VISIBLE_DEVICES="")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    report = r.stdout + r.stderr
    assert "ERROR: AddressSanitizer" not in report, report[-4000:]
    assert "runtime error" not in report, report[-4000:]
    assert r.returncode == 0, report[-4000:]
    assert "ok (0 failures)" in r.stdout
