"""The paper's benchmark observable Hadamard^(x)n (Sec. 3) and workload, pinned on the CPU.

The Pauli expansion of the observable is checked against the Kronecker product of Hadamard
matrices built by numpy alone; the oracle's energy and gradient under it against closed forms
and the dense expm reference.
"""
import math

import numpy as np
import pytest

import dense_ref
from paper_2009_02823_amd import workloads as W

HAD = np.array([[1, 1], [1, -1]], dtype=np.complex128) / math.sqrt(2)


@pytest.mark.parametrize("n", [1, 2, 3, 4])
def test_expansion_equals_kron_of_hadamards(n):
    codes, coeffs = W.hadamard_product_observable(n)
    assert codes.shape == (1 << n, n)
    want = np.ones((1, 1), dtype=np.complex128)
    for _ in range(n):
        want = np.kron(HAD, want)
    got = dense_ref.hamiltonian(codes, coeffs, n)
    assert np.max(np.abs(got - want)) < 1e-14


def test_one_qubit_closed_form(orc):
    """RY(t)|0> = (cos t/2, sin t/2): <Had> = (sin t + cos t)/sqrt 2, derivative
    (cos t - sin t)/sqrt 2."""
    codes, coeffs = W.hadamard_product_observable(1)
    gates = W.circuit_table([W.gate_row(W.RY, 0, p0=0)])
    for t in (0.0, 0.3, 1.9, 4.4):
        e, g = orc.adjoint_gradient(1, gates, np.array([t]), codes, coeffs)
        assert abs(e.real - (math.sin(t) + math.cos(t)) / math.sqrt(2)) < 1e-15
        assert abs(g[0] - (math.cos(t) - math.sin(t)) / math.sqrt(2)) < 1e-15


@pytest.mark.parametrize("n", [2, 4, 5])
def test_zero_angles_energy(orc, n):
    """At theta = 0 the HEA leaves |0...0>: E = <0|Had^(x)n|0> = 2^(-n/2)."""
    p = W.paper_benchmark(n, 3)
    e, g = orc.adjoint_gradient(n, p.gates, np.zeros(p.n_params), p.codes, p.coeffs)
    assert abs(e.real - 2.0 ** (-0.5 * n)) < 1e-14


def test_paper_workload_against_dense(orc):
    p = W.paper_benchmark(3, 4)
    e, g = orc.adjoint_gradient(p.n_qubits, p.gates, p.theta, p.codes, p.coeffs)
    e_d = dense_ref.energy(p.gates, p.theta, p.codes, p.coeffs, p.n_qubits)
    g_d = dense_ref.gradient_fd5(p.gates, p.theta, p.codes, p.coeffs, p.n_qubits)
    assert abs(e - e_d) < 1e-13
    assert np.max(np.abs(g - g_d)) < 1e-8
    g_ref = orc.reference_gradient(p.n_qubits, p.gates, p.theta, p.codes, p.coeffs)
    assert np.max(np.abs(g - g_ref)) < 1e-13


def test_paper_workload_sizes():
    p = W.paper_benchmark()
    assert (p.n_qubits, p.n_params) == (5, 1290)
    assert p.coeffs.shape == (32,)
