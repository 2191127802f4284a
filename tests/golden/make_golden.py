"""Write oracle reference values for the measured workloads into ``tests/golden/``.

Every value written here comes from the CPU oracle (``oracle/``), i.e. Algorithm 1 in complex128
with plain loops, on the seeded synthetic inputs of ``paper_2009_02823_amd/workloads.py``. The
GPU parity tests read these files so that workloads whose oracle run takes minutes (26 qubits)
do not have to be recomputed on every test run.

Usage:  python tests/golden/make_golden.py 1 2 3     (configuration numbers)
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_2009_02823_amd import workloads as W  # noqa: E402


def golden_path(name: str) -> str:
    return os.path.join(HERE, f"{name}.txt")


def write(problem: W.Problem, cid: int):
    t0 = time.time()
    e, g = O.adjoint_gradient(problem.n_qubits, problem.gates, problem.theta, problem.codes,
                              problem.coeffs)
    dt = time.time() - t0
    path = golden_path(problem.name)
    with open(path, "w") as f:
        f.write(f"# oracle Algorithm 1 (complex128) on workload {problem.name}\n")
        f.write(f"# configuration {cid}: n_qubits={problem.n_qubits} gates={problem.n_gates} "
                f"params={problem.n_params} terms={len(problem.coeffs)}\n")
        f.write(f"# written by tests/golden/make_golden.py {cid} "
                f"(oracle threads={O.num_threads()}, {dt:.1f} s)\n")
        f.write(f"energy {float(e.real)!r} {float(e.imag)!r}\n")
        for p, v in enumerate(g):
            f.write(f"{p} {float(v)!r}\n")
    print(f"wrote {path} in {dt:.1f} s", flush=True)


def read(name: str):
    """(energy complex, gradient ndarray) of a golden file, or None if absent."""
    path = golden_path(name)
    if not os.path.exists(path):
        return None
    e, g = None, []
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        parts = line.split()
        if parts[0] == "energy":
            e = complex(float(parts[1]), float(parts[2]))
        else:
            g.append((int(parts[0]), float(parts[1])))
    grad = np.zeros(len(g))
    for p, v in g:
        grad[p] = v
    return e, grad


if __name__ == "__main__":
    for arg in sys.argv[1:]:
        cid = int(arg)
        write(W.CONFIGS[cid](), cid)
