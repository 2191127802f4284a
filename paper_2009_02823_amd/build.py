"""Build ``libqsv.so`` (the HIP library behind ``include/qsv.h``) in-tree for gfx950.

Each ``csrc/*.hip`` file is compiled by hipcc to an object in ``_build/`` and the objects are
linked into ``paper_2009_02823_amd/libqsv.so``. Cross-compiles without a GPU.
"""
from __future__ import annotations

import glob
import hashlib
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libqsv.so")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")

ARCH = "gfx950"
HIPCC = os.environ.get("HIPCC", shutil.which("hipcc") or "/opt/rocm/bin/hipcc")
CFLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-fPIC", "-std=c++17", "-Wall",
    "-Wno-unused-function", "-Wno-unused-result",
    # packed-FP32 instructions stay off on these boxes
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # keep per-branch register-array code apart: sinking/hoisting the common arithmetic of the
    # per-register-position branches turns static array indices into address selects, which
    # forces the thread's amplitude arrays into scratch memory
    "-mllvm", "-simplifycfg-sink-common=false", "-mllvm", "-simplifycfg-hoist-common=false",
    # branches on wave-uniform values (the op dispatch of the fused passes) stay plain scalar
    # branches; structurizing them inserts flow blocks whose joins copy the amplitude registers
    "-mllvm", "-structurizecfg-skip-uniform-regions=true",
    "-I", CSRC, "-I", INCLUDE,
]


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


def _headers():
    return glob.glob(os.path.join(CSRC, "*.h")) + glob.glob(os.path.join(INCLUDE, "*.h"))


def source_id() -> str:
    """Hash of every library source and header: tags persisted tuning choices, so that choices
    timed on other kernel sources are not reused."""
    h = hashlib.sha256()
    for f in sorted(sources() + _headers()):
        h.update(os.path.basename(f).encode())
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def build(force: bool = False, verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    newest_header = max((os.path.getmtime(h) for h in _headers()), default=0)
    sid = source_id()
    sid_file = os.path.join(BUILD, "source_id")
    old_sid = open(sid_file).read().strip() if os.path.exists(sid_file) else ""
    procs, objs = [], []
    for src in sources():
        obj = os.path.join(BUILD, os.path.basename(src) + ".o")
        objs.append(obj)
        api = os.path.basename(src) == "qsv_api.hip"
        stale = (force or not os.path.exists(obj) or os.path.getmtime(obj) < os.path.getmtime(src)
                 or os.path.getmtime(obj) < newest_header or (api and old_sid != sid))
        if stale:
            cmd = [HIPCC, *CFLAGS, "-c", src, "-o", obj]
            if api:
                cmd.insert(1, f'-DQSV_SOURCE_ID="{sid}"')
            if verbose:
                print(" ".join(cmd), flush=True)
            procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE,
                                                stderr=subprocess.STDOUT, text=True)))
    failed = []
    for src, p in procs:
        out, _ = p.communicate()
        if p.returncode != 0:
            failed.append(f"{os.path.basename(src)}:\n{out}")
        elif verbose and out.strip():
            print(out)
    if failed:
        raise RuntimeError("hipcc failed:\n" + "\n".join(failed))
    with open(sid_file, "w") as f:
        f.write(sid + "\n")
    if procs or force or not os.path.exists(LIB):
        tmp = LIB + ".tmp%d" % os.getpid()
        cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
        subprocess.run(cmd, check=True)
        os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(force="--force" in sys.argv, verbose="-v" in sys.argv))
