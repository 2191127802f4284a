"""GPU parity: the HIP path (through the C-ABI) against the CPU oracle on the same seeded inputs.

Tolerances: complex128 storage max |dg| <= 1e-10 and |dE| <= 1e-10 (absolute); complex64
storage with FP64 reductions
max |dg| <= 2e-4 * max|g_oracle| and |dE| <= 2e-4 * max(|E|, 1).
"""
import math
import os
import sys

import numpy as np
import pytest

from paper_2009_02823_amd import workloads as W

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))


@pytest.fixture(scope="module")
def Q():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2009_02823_amd import qsv
    qsv.lib()
    return qsv


def gpu_adjoint(Q, n, gates, theta, codes, coeffs, dtype="c128", prep=None, geom=None):
    with Q.StateVector(n, dtype) as sv:
        if geom is not None:
            sv.set_fusion(1, *geom)
        if prep is not None:
            sv.apply_circuit(*prep)
        e, g = sv.adjoint_gradient(gates, theta, codes, coeffs)
        sv.sync()
        return float(e.cpu()[0]), g.cpu().numpy()


def assert_c128(e_gpu, g_gpu, e_ref, g_ref, coeffs):
    assert abs(e_gpu - e_ref.real) <= 1e-10, (e_gpu, e_ref)
    if g_ref.size:
        err = np.max(np.abs(g_gpu - g_ref))
        assert err <= 1e-10, err


def c64_grad_scale(g_ref, coeffs):
    """|g| scale of the complex64 bound: max|g_oracle|, floored at 1e-5 * ||c||_1 so that
    vanishing gradients are compared absolutely (2e-4 of the floor is 2e-9 ||c||_1, well
    below one complex64 rounding of the energy scale, eps_32 ||c||_1 ~ 6e-8 ||c||_1)."""
    return max(float(np.max(np.abs(g_ref))) if g_ref.size else 0.0,
               1e-5 * float(np.abs(coeffs).sum()))


def assert_c64(e_gpu, g_gpu, e_ref, g_ref, coeffs):
    assert abs(e_gpu - e_ref.real) <= 2e-4 * max(abs(e_ref), 1.0)
    if g_ref.size:
        err = np.max(np.abs(g_gpu - g_ref))
        assert err <= 2e-4 * c64_grad_scale(g_ref, coeffs), err


def test_config1_c128(Q, orc):
    p = W.config1()
    e_ref, g_ref = orc.adjoint_gradient(p.n_qubits, p.gates, p.theta, p.codes, p.coeffs)
    e, g = gpu_adjoint(Q, p.n_qubits, p.gates, p.theta, p.codes, p.coeffs)
    assert_c128(e, g, e_ref, g_ref, p.coeffs)


ALL_KINDS = list(W.GATE_NAMES)


@pytest.mark.parametrize("n,seed", [(1, 0), (2, 1), (3, 2), (5, 3), (7, 4), (9, 5), (11, 6),
                                    (12, 7), (13, 8), (14, 9)])
@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_random_circuits_every_kind(Q, orc, n, seed, dtype):
    """Random gate sequences over every kind, random Pauli sums, shared parameters."""
    rng = np.random.default_rng(1000 + seed)
    kinds = ALL_KINDS if n >= 2 else [k for k in ALL_KINDS if W.N_QUBITS[k] == 1]
    gates, P = W.random_circuit(rng, n, 40 + 4 * n, kinds, n_params=None if seed % 2 else 15)
    theta = W.uniform_angles(rng, P)
    codes = W.random_pauli_strings(rng, n, 11)
    coeffs = rng.standard_normal(11)
    e_ref, g_ref = orc.adjoint_gradient(n, gates, theta, codes, coeffs)
    e, g = gpu_adjoint(Q, n, gates, theta, codes, coeffs, dtype)
    if dtype == "c128":
        assert_c128(e, g, e_ref, g_ref, coeffs)
    else:
        assert_c64(e, g, e_ref, g_ref, coeffs)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_apply_circuit_and_expectation(Q, orc, dtype):
    import torch
    n = 11
    rng = np.random.default_rng(77)
    gates, P = W.random_circuit(rng, n, 120, ALL_KINDS)
    theta = W.uniform_angles(rng, P)
    codes = W.random_pauli_strings(rng, n, 9)
    coeffs = rng.standard_normal(9)
    psi_ref = orc.statevector(n, gates, theta)
    e_ref = orc.energy(n, gates, theta, codes, coeffs)
    with Q.StateVector(n, dtype) as sv:
        sv.apply_circuit(gates, theta)
        e = sv.expectation(codes, coeffs)
        sv.sync()
        psi = sv.state.cpu().numpy().astype(np.complex128)
    tol = 1e-12 if dtype == "c128" else 2e-5
    assert np.max(np.abs(psi - psi_ref)) <= tol
    assert abs(float(e.cpu()[0]) - e_ref.real) <= (1e-11 if dtype == "c128" else 1e-4)
    del torch


def test_input_state_is_preserved_and_used(Q, orc):
    """The handle's state is the immutable |in> of Algorithm 1: a prepared non-trivial input is
    used and left unchanged bit for bit."""
    n = 10
    rng = np.random.default_rng(5)
    prep_g, prep_P = W.random_circuit(rng, n, 50, ALL_KINDS)
    prep_t = W.uniform_angles(rng, prep_P)
    gates = W.hea_circuit(n, 3)
    theta = W.uniform_angles(rng, 6 * n)
    codes, coeffs = W.heisenberg_chain(n)
    psi_in = orc.statevector(n, prep_g, prep_t)
    e_ref, g_ref = orc.adjoint_gradient(n, gates, theta, codes, coeffs, psi_in=psi_in)
    with Q.StateVector(n) as sv:
        sv.apply_circuit(prep_g, prep_t)
        before = sv.state.clone()
        e, g = sv.adjoint_gradient(gates, theta, codes, coeffs)
        sv.sync()
        assert bool((sv.state == before).all())
        assert_c128(float(e.cpu()[0]), g.cpu().numpy(), e_ref, g_ref, coeffs)
        # Algorithm 1 leaves phi = U_1^dag ... U_G^dag psi = |in>
        phi, _ = sv.workspace_states()
        assert float((phi - before).abs().max()) < 1e-12


def test_degenerate_inputs(Q, orc):
    n = 4
    codes = np.array([[3, 0, 0, 0], [1, 1, 0, 0]], np.uint8)
    coeffs = np.array([0.5, -1.5])
    # empty circuit: E = <0|H|0>, empty gradient
    e, g = gpu_adjoint(Q, n, np.zeros((0, 6), np.int32), [], codes, coeffs)
    assert abs(e - 0.5) < 1e-15 and g.size == 0
    # fixed gates only
    gates = W.circuit_table([W.gate_row(W.H, 0), W.gate_row(W.CNOT, 0, 1), W.gate_row(W.S, 1)])
    e_ref, _ = orc.adjoint_gradient(n, gates, [], codes, coeffs)
    e, g = gpu_adjoint(Q, n, gates, [], codes, coeffs)
    assert abs(e - e_ref.real) < 1e-14 and g.size == 0
    # empty Hamiltonian: E = 0, gradient 0; unused parameters get 0
    gates = W.circuit_table([W.gate_row(W.RY, 0, -1, 2)])
    e, g = gpu_adjoint(Q, n, gates, [0.1, 0.2, 0.3], np.zeros((0, n), np.uint8), np.zeros(0))
    assert e == 0.0 and np.all(g == 0.0) and g.size == 3
    gates = W.circuit_table([W.gate_row(W.RY, 0, -1, 2)])
    e, g = gpu_adjoint(Q, n, gates, [0.1, 0.2, 0.3], codes, coeffs)
    assert g[0] == 0.0 and g[1] == 0.0 and abs(g[2] - (-0.5 * math.sin(0.3))) < 1e-14


def test_deterministic(Q):
    p = W.config1()
    runs = [gpu_adjoint(Q, p.n_qubits, p.gates, p.theta, p.codes, p.coeffs) for _ in range(3)]
    for e, g in runs[1:]:
        assert e == runs[0][0] and np.array_equal(g, runs[0][1])


def test_invalid_call_leaves_outputs_untouched(Q):
    import torch
    n = 5
    with Q.StateVector(n) as sv:
        e = torch.full((1,), 7.0, dtype=torch.float64, device=sv.device)
        g = torch.full((3,), 7.0, dtype=torch.float64, device=sv.device)
        bad = W.circuit_table([W.gate_row(W.RY, 9, -1, 0)])
        with pytest.raises(Q.QsvError):
            sv.adjoint_gradient(bad, [0.1, 0.2, 0.3], np.zeros((1, n), np.uint8), [1.0], e, g)
        sv.sync()
        assert float(e.cpu()[0]) == 7.0 and bool((g == 7.0).all())


@pytest.mark.parametrize("k", [1, 2, 3])
def test_failed_launch_leaves_outputs_untouched(Q, orc, k):
    """A launch failure forced from the host (the k-th launch of the call is refused) makes
    the call return QSV_ERR_HIP with the energy and gradient buffers as they were and |in>
    unchanged; the next call on the same handle gives the oracle's result."""
    import torch
    p = W.config1()
    with Q.StateVector(p.n_qubits) as sv:
        psi0 = sv.state.clone()
        e = torch.full((1,), 7.0, dtype=torch.float64, device=sv.device)
        g = torch.full((p.n_params,), 7.0, dtype=torch.float64, device=sv.device)
        Q.debug_fail_launch(k)
        try:
            with pytest.raises(Q.QsvError) as err:
                sv.adjoint_gradient(p.gates, p.theta, p.codes, p.coeffs, e, g)
        finally:
            Q.debug_fail_launch(0)
        assert err.value.status == Q.QSV_ERR_HIP
        sv.sync()
        assert float(e.cpu()[0]) == 7.0 and bool((g == 7.0).all())
        assert torch.equal(sv.state, psi0)
        sv.adjoint_gradient(p.gates, p.theta, p.codes, p.coeffs, e, g)
        sv.sync()
        e_ref, g_ref = orc.adjoint_gradient(p.n_qubits, p.gates, p.theta, p.codes, p.coeffs)
        assert_c128(float(e.cpu()[0]), g.cpu().numpy(), e_ref, g_ref, p.coeffs)


@pytest.mark.parametrize("dtype,geom", [("c128", None), ("c128", (3, 9)), ("c64", None),
                                        ("c64", (3, 9)), ("c64", (4, 9))])
def test_config2_full(Q, orc, dtype, geom):
    """20 qubits, 20 layers (P = 800), TFIM: the full gradient against the oracle, in the
    automatic geometry and in those the benchmark's tuning picks."""
    import make_golden as golden_io
    p = W.config2()
    ref = golden_io.read(p.name)
    if ref is None:
        ref = orc.adjoint_gradient(p.n_qubits, p.gates, p.theta, p.codes, p.coeffs)
    e_ref, g_ref = ref
    e, g = gpu_adjoint(Q, p.n_qubits, p.gates, p.theta, p.codes, p.coeffs, dtype, geom=geom)
    if dtype == "c128":
        assert_c128(e, g, e_ref, g_ref, p.coeffs)
    else:
        assert_c64(e, g, e_ref, g_ref, p.coeffs)


@pytest.mark.parametrize("n", [16, 22])
def test_scalable_closed_form(Q, n):
    """One RY/RZ layer under an Ising chain: E and every gradient entry in closed form at sizes
    the oracle is not needed for."""
    import test_oracle_pins as pins
    gates, theta, codes, coeffs, E, G = pins.tfim_product_layer(n, np.random.default_rng(n))
    e, g = gpu_adjoint(Q, n, gates, theta, codes, coeffs)
    assert abs(e - E) < 1e-12 * n
    assert np.max(np.abs(g - G)) < 1e-12 * n
