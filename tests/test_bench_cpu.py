"""bench.py host logic (no GPU): the gate-granular byte model and the one-GPU contract."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


@pytest.mark.parametrize("config,units", [(1, 653), (2, 6008), (5, 4568)])
def test_gate_granular_bytes(config, units):
    """One HBM pass per gate: the per-config totals in units of the state size S (HEA layers:
    rotations 6S, CNOTs 3S; H 2S + 3S per further x-mask group; clones and energy 6S)."""
    import bench
    from paper_2009_02823_amd import workloads as W
    p = W.CONFIGS[config]()
    S = 16 << p.n_qubits
    assert bench.gate_granular_bytes(p, S) == units * S


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)
