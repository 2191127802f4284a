"""AddressSanitizer / UndefinedBehaviorSanitizer builds of the CPU oracle (gcc) and of the
library's host-only code (hipcc, host compilation only), each run over random inputs by a driver
in tests/sanitize/. A sanitizer finding aborts the driver; the test then fails with its report."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = os.path.join(ROOT, "tests", "sanitize")
CSRC = os.path.join(ROOT, "paper_2009_02823_amd", "csrc")
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
           UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", OMP_NUM_THREADS="2")


def run(cmd, cwd, timeout):
    r = subprocess.run(cmd, cwd=cwd, capture_output=True, text=True, timeout=timeout, env=ENV)
    assert r.returncode == 0, f"{' '.join(cmd[:3])} ...\n{r.stdout[-3000:]}\n{r.stderr[-6000:]}"
    return r.stdout


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc missing")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    run(["gcc", "-std=gnu11", "-O1", "-g", "-fopenmp", "-fsanitize=address,undefined",
         "-fno-sanitize-recover=all", "-o", exe, os.path.join(SAN, "oracle_driver.c"), "-lm"],
        str(tmp_path), 300)
    assert "ok" in run([exe], str(tmp_path), 300)


HIPCC = os.environ.get("HIPCC", shutil.which("hipcc") or "/opt/rocm/bin/hipcc")


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc missing")
def test_host_code_under_sanitizers(tmp_path):
    """The validators, both planners and the tuning-cache reader, with the sanitizers on the
    host code (-Xarch_host); the device code is built as usual but never runs."""
    exe = str(tmp_path / "host_driver")
    # the fused-pass kernels are replaced by launch stand-ins (their device code takes minutes
    # to build and no kernel runs here); everything else is the library's own source
    srcs = [os.path.join(CSRC, f) for f in sorted(os.listdir(CSRC))
            if f.endswith(".hip") and f != "fused_kernels.hip"]
    srcs += [os.path.join(SAN, "fused_launch_stubs.cpp"), os.path.join(SAN, "host_driver.cpp")]
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all"]
    flags = ["--offload-arch=gfx950", "-O1", "-Xarch_host", "-g", "-std=c++17", *san, "-I", CSRC,
             "-I", os.path.join(ROOT, "include")]
    objs, procs = [], []
    for src in srcs:
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        lang = ["-x", "hip"] if src.endswith(".cpp") else []
        procs.append(subprocess.Popen([HIPCC, *flags, *lang, "-c", src, "-o", obj],
                                      stdout=subprocess.PIPE, stderr=subprocess.STDOUT,
                                      text=True, env=ENV))
        objs.append(obj)
    for p in procs:
        out, _ = p.communicate(timeout=1200)
        assert p.returncode == 0, out[-4000:]
    run([HIPCC, "--offload-arch=gfx950", *san, *objs, "-o", exe], str(tmp_path), 300)
    assert "ok" in run([exe], str(tmp_path), 600)
