"""GPU reference gradient (Algorithm 2) against the CPU oracle and the GPU adjoint gradient.

Covers single-tile states (all entries in parallel, one workgroup each, phantom tile bits), a
multi-tile state (entries one after another), every gate kind including multi-parameter and
two-qubit gates, repeated parameters, and the paper's benchmark workload under Hadamard^(x)n.
"""
import numpy as np
import pytest

from paper_2009_02823_amd import workloads as W

pytestmark = pytest.mark.gpu
ALL_KINDS = list(W.GATE_NAMES)


@pytest.fixture(scope="module")
def Q():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2009_02823_amd import qsv
    qsv.lib()
    return qsv


def reference(Q, n, gates, theta, codes, coeffs, dtype, geom=None):
    with Q.StateVector(n, dtype) as sv:
        if geom is not None:
            sv.set_fusion(1, *geom)
        e, g = sv.reference_gradient(gates, theta, codes, coeffs)
        sv.sync()
        return float(e.cpu()[0]), g.cpu().numpy()


def check(dtype, e, g, e_ref, g_ref, coeffs):
    if dtype == "c128":
        assert abs(e - e_ref.real) <= 1e-10
        assert np.max(np.abs(g - g_ref)) <= 1e-10
    else:
        assert abs(e - e_ref.real) <= 2e-4 * max(abs(e_ref), 1.0)
        scale = max(np.max(np.abs(g_ref)), 1e-5 * np.abs(coeffs).sum())
        assert np.max(np.abs(g - g_ref)) <= 2e-4 * scale


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("n,geom", [(1, None), (3, None), (5, (2, 6)), (9, (3, 8)),
                                    (13, (3, 8))])
def test_random_circuits(Q, orc, dtype, n, geom):
    rng = np.random.default_rng(700 + n)
    kinds = [k for k in ALL_KINDS if n >= 2 or W.N_QUBITS[k] == 1]
    n_gates = 60 if n >= 13 else 90
    gates, P = W.random_circuit(rng, n, n_gates, kinds, n_params=None if n != 5 else 20)
    theta = W.uniform_angles(rng, P)
    codes = W.random_pauli_strings(rng, n, 6)
    coeffs = rng.standard_normal(6)
    e_ref, g_ref = orc.adjoint_gradient(n, gates, theta, codes, coeffs)
    e, g = reference(Q, n, gates, theta, codes, coeffs, dtype, geom)
    check(dtype, e, g, e_ref, g_ref, coeffs)


def test_matches_adjoint_on_paper_workload(Q, orc):
    """The paper's regime: 5 qubits, 40 HEA layers (P = 400), Hadamard^(x)5."""
    p = W.paper_benchmark(5, 40)
    g_orc = orc.reference_gradient(p.n_qubits, p.gates, p.theta, p.codes, p.coeffs)
    with Q.StateVector(p.n_qubits) as sv:
        e1, g1 = sv.adjoint_gradient(p.gates, p.theta, p.codes, p.coeffs)
        e2, g2 = sv.reference_gradient(p.gates, p.theta, p.codes, p.coeffs)
        sv.sync()
        g1, g2 = g1.cpu().numpy(), g2.cpu().numpy()
        assert abs(float(e1.cpu()[0]) - float(e2.cpu()[0])) < 1e-13
    assert np.max(np.abs(g1 - g2)) < 1e-12
    assert np.max(np.abs(g2 - g_orc)) < 1e-12


def test_no_parameters(Q):
    gates = W.circuit_table([W.gate_row(W.H, 0), W.gate_row(W.CNOT, 0, 1)])
    codes = np.array([[W.PAULI_Z, W.PAULI_Z]], dtype=np.uint8)
    with Q.StateVector(2) as sv:
        e, g = sv.reference_gradient(gates, np.zeros(3), codes, np.array([1.0]))
        sv.sync()
        assert abs(float(e.cpu()[0]) - 1.0) < 1e-14
        assert np.all(g.cpu().numpy() == 0.0)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("n", [2, 4, 6])
def test_wave_reference(Q, orc, dtype, n):
    """Algorithm 2 in waves (states of up to 6 qubits): lambda in one wave, one wave per
    parameter occurrence; every gate kind including the non-unitary ones, repeated parameters,
    against the oracle's Algorithm 2."""
    rng = np.random.default_rng(900 + n)
    kinds = [k for k in ALL_KINDS + list(W.NONUNITARY_NAMES) if n >= 2 or W.N_QUBITS[k] == 1]
    gates, P = W.random_circuit(rng, n, 150, kinds, n_params=50)
    theta = rng.uniform(-0.6, 0.6, P)  # the non-unitary factors stay moderate
    codes = W.random_pauli_strings(rng, n, 6)
    coeffs = rng.standard_normal(6)
    g_ref = orc.reference_gradient(n, gates, theta, codes, coeffs)
    e_ref, _ = orc.adjoint_gradient(n, gates, theta, codes, coeffs)
    e, g = reference(Q, n, gates, theta, codes, coeffs, dtype)
    scale = max(1.0, abs(e_ref), float(np.max(np.abs(g_ref))))
    tol = 1e-10 if dtype == "c128" else 2e-4
    assert abs(e - e_ref.real) <= tol * scale
    assert np.max(np.abs(g - g_ref)) <= tol * scale
