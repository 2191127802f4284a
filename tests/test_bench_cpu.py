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


def test_sweep_flops_model():
    """FP64 flops of the sweeps: 6 per amplitude per rotation forward, 16 in reverse (two
    state updates and the product), none for CNOT/CZ."""
    import bench
    from paper_2009_02823_amd import workloads as W
    p = W.config5()
    f, b = bench.sweep_flops(p, p.n_qubits)
    assert f == 6 * 600 * 2.0 ** 30 and b == 16 * 600 * 2.0 ** 30
    p3 = W.config3()
    f, b = bench.sweep_flops(p3, p3.n_qubits)
    assert f == 6 * 1560 * 2.0 ** 26 and b == 16 * 1560 * 2.0 ** 26


def test_grad_error_report(tmp_path, monkeypatch):
    """grad_error compares with the stored oracle values and reports the per-entry quantiles."""
    import numpy as np
    import bench
    import make_golden
    from paper_2009_02823_amd import workloads as W
    p = W.config1()
    ref = make_golden.read(p.name)
    e_ref, g_ref = ref
    d = bench.grad_error(p, e_ref.real, g_ref + 1e-12, "c128")
    assert d["ok"] and abs(d["max_abs_grad_err"] - 1e-12) < 1e-15
    assert d["per_entry"]["entries"] == p.n_params and len(d["per_entry"]["abs"]) == 4
    d = bench.grad_error(p, e_ref.real, g_ref + 2e-10, "c128")
    assert not d["ok"]
