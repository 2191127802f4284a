"""Write oracle reference values for the measured workloads into ``tests/golden/``.

Every value written here comes from the CPU oracle (``oracle/``), i.e. Algorithm 1 in complex128
with plain loops, on the seeded synthetic inputs of ``paper_2009_02823_amd/workloads.py``. The
GPU parity tests read these files so that workloads whose oracle run takes minutes or hours (26
and 30 qubits, the 512-circuit batch) do not have to be recomputed on every test run.

Usage:  python tests/golden/make_golden.py 1 2 3 4 5    (configuration numbers)

Configuration 4 (512 independent circuits) is written as ``batch512_hea12-18_L5-15_heis.npz``:
arrays ``energy`` [B], ``grad`` (all gradients concatenated in circuit order), ``offset`` [B + 1]
and ``seconds`` (oracle time per circuit).
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


BATCH_NAME = "batch512_hea12-18_L5-15_heis"


def write_batch(probs):
    t0 = time.time()
    energy = np.zeros(len(probs))
    secs = np.zeros(len(probs))
    grads, offset = [], [0]
    for b, p in enumerate(probs):
        t1 = time.time()
        e, g = O.adjoint_gradient(p.n_qubits, p.gates, p.theta, p.codes, p.coeffs)
        secs[b] = time.time() - t1
        energy[b] = e.real
        grads.append(np.asarray(g, dtype=np.float64))
        offset.append(offset[-1] + len(g))
    path = os.path.join(HERE, BATCH_NAME + ".npz")
    np.savez_compressed(path, energy=energy, grad=np.concatenate(grads),
                        offset=np.asarray(offset, dtype=np.int64), seconds=secs,
                        threads=np.int64(O.num_threads()))
    print(f"wrote {path} in {time.time() - t0:.1f} s", flush=True)


def read_batch():
    """(energy [B], list of per-circuit gradients) of the batch golden, or None if absent."""
    path = os.path.join(HERE, BATCH_NAME + ".npz")
    if not os.path.exists(path):
        return None
    z = np.load(path)
    off = z["offset"]
    return z["energy"], [z["grad"][off[b]:off[b + 1]] for b in range(len(off) - 1)]


if __name__ == "__main__":
    for arg in sys.argv[1:]:
        cid = int(arg)
        if cid == 4:
            write_batch(W.CONFIGS[4]())
        else:
            write(W.CONFIGS[cid](), cid)
