"""Oracle pins for non-Hermitian operators (App. B.4): <A> = <psi|A|psi> for A = sum c_t P_t with
complex c, and its complex gradient.

The paper's combination conjugates the A^dag run; that gives the conjugate of the derivative.
The oracle conjugates the A run instead (<dpsi|A|psi> = conj(<psi|A^dag|dpsi>)). The worked
example below (RX under |0><1|) separates the two readings.
"""
import math

import numpy as np
import pytest

import dense_ref
from paper_2009_02823_amd import workloads as W


def test_worked_example_rx_under_lowering(orc):
    """|psi> = RX(t)|0> = (cos t/2, -i sin t/2); A = |0><1| = (X + iY)/2:
    <A> = -(i/2) sin t and d<A>/dt = -(i/2) cos t."""
    codes = np.array([[W.PAULI_X], [W.PAULI_Y]], dtype=np.uint8)
    coeffs = np.array([0.5, 0.5j])
    gates = W.circuit_table([W.gate_row(W.RX, 0, p0=0)])
    for t in (0.2, 1.1, 2.9, 5.0):
        e, g = orc.adjoint_gradient_nonhermitian(1, gates, np.array([t]), codes, coeffs)
        assert abs(e - (-0.5j * math.sin(t))) < 1e-15
        assert abs(g[0] - (-0.5j * math.cos(t))) < 1e-15


@pytest.mark.parametrize("seed", [0, 1])
def test_linear_in_the_operator(orc, seed):
    """For A = H1 + i H2 (H1, H2 Hermitian): <A> = <H1> + i<H2>, grad A = grad H1 + i grad H2."""
    rng = np.random.default_rng(50 + seed)
    n = 4
    gates, P = W.random_circuit(rng, n, 40, list(W.GATE_NAMES), n_params=12)
    theta = W.uniform_angles(rng, P)
    codes = W.random_pauli_strings(rng, n, 7)
    a, b = rng.standard_normal(7), rng.standard_normal(7)
    e, g = orc.adjoint_gradient_nonhermitian(n, gates, theta, codes, a + 1j * b)
    e1, g1 = orc.adjoint_gradient(n, gates, theta, codes, a)
    e2, g2 = orc.adjoint_gradient(n, gates, theta, codes, b)
    assert abs(e - (e1.real + 1j * e2.real)) < 1e-13
    assert np.max(np.abs(g - (g1 + 1j * g2))) < 1e-13


def test_against_dense_difference_quotient(orc):
    rng = np.random.default_rng(61)
    n = 3
    gates, P = W.random_circuit(rng, n, 25, list(W.GATE_NAMES))
    theta = W.uniform_angles(rng, P)
    codes = W.random_pauli_strings(rng, n, 5)
    c = rng.standard_normal(5) + 1j * rng.standard_normal(5)
    e, g = orc.adjoint_gradient_nonhermitian(n, gates, theta, codes, c)
    Am = dense_ref.hamiltonian(codes, c, n)

    def E(t):
        psi = dense_ref.circuit_operator(gates, t, n) @ dense_ref.zero_state(n)
        return complex(np.vdot(psi, Am @ psi))

    assert abs(e - E(theta)) < 1e-13
    h = 1e-3
    for p in range(P):
        vals = []
        for k in (-2, -1, 1, 2):
            t = theta.copy()
            t[p] += k * h
            vals.append(E(t))
        fd = (vals[0] - 8 * vals[1] + 8 * vals[2] - vals[3]) / (12 * h)
        assert abs(g[p] - fd) < 1e-8, p


def test_hermitian_operator_reduces_to_algorithm1(orc):
    p = W.config1()
    e, g = orc.adjoint_gradient_nonhermitian(p.n_qubits, p.gates, p.theta, p.codes,
                                             p.coeffs.astype(np.complex128))
    e1, g1 = orc.adjoint_gradient(p.n_qubits, p.gates, p.theta, p.codes, p.coeffs)
    assert abs(e - e1) < 1e-13
    assert np.max(np.abs(g.imag)) < 1e-13
    assert np.max(np.abs(g.real - g1)) < 1e-13
