"""Oracle pins for non-unitary, invertible gates (App. B.3): the imaginary-time rotations
M(t) = exp(-t G / 2), G = X, Y, Z. Algorithm 1 un-does phi by M^-1 and lambda by M^dag; the
energy <psi|H|psi> is not normalised.
"""
import math

import numpy as np
import pytest

import dense_ref as D
from paper_2009_02823_amd import workloads as W

NONUNITARY = list(W.NONUNITARY_NAMES)
MIXED = list(W.GATE_NAMES) + NONUNITARY


@pytest.mark.parametrize("kind", NONUNITARY)
def test_matrix_and_derivative_vs_expm(orc, kind):
    n = 2
    rng = np.random.default_rng(400 + kind)
    psi = rng.standard_normal(4) + 1j * rng.standard_normal(4)
    theta = np.array([1.3])
    for q in (0, 1):
        row = W.gate_row(kind, q, p0=0)
        got = orc.statevector(n, W.circuit_table([row]), theta, psi_in=psi)
        assert np.max(abs(got - D.gate_operator(row, theta, n) @ psi)) < 1e-14
        h = 1e-3
        ops = [D.gate_operator(row, theta + k * h, n) for k in (-2, -1, 1, 2)]
        fd = (ops[0] - 8 * ops[1] + 8 * ops[2] - ops[3]) / (12 * h)
        dpsi = orc.apply_derivative(n, row, theta, psi)
        assert np.max(abs(dpsi - fd @ psi)) < 1e-10


@pytest.mark.parametrize("t", [0.3, 1.7, -0.9])
def test_closed_forms(orc, t):
    """exp(-t Y/2)|0> = (cosh t/2, -i sinh t/2): <Y> = -sinh t, <1> = cosh t.
    exp(-t X/2)|0> = (cosh t/2, -sinh t/2): <X> = -sinh t. exp(-t Z/2)|0> = e^{-t/2}|0>: <1> = e^{-t}."""
    one = np.zeros((1, 1), dtype=np.uint8)
    cases = [
        (W.NRY, W.PAULI_Y, -math.sinh(t), -math.cosh(t)),
        (W.NRY, W.PAULI_I, math.cosh(t), math.sinh(t)),
        (W.NRX, W.PAULI_X, -math.sinh(t), -math.cosh(t)),
        (W.NRZ, W.PAULI_I, math.exp(-t), -math.exp(-t)),
    ]
    for kind, code, e_want, g_want in cases:
        gates = W.circuit_table([W.gate_row(kind, 0, p0=0)])
        codes = one.copy()
        codes[0, 0] = code
        e, g = orc.adjoint_gradient(1, gates, np.array([t]), codes, np.array([1.0]))
        assert abs(e.real - e_want) < 1e-14 and abs(g[0] - g_want) < 1e-14, (kind, code)


@pytest.mark.parametrize("seed", range(3))
def test_mixed_circuits_against_dense(orc, seed):
    rng = np.random.default_rng(410 + seed)
    n = 3
    gates, P = W.random_circuit(rng, n, 30, MIXED, n_params=None if seed != 2 else 9)
    theta = rng.uniform(-1.0, 1.0, P)   # moderate angles: M grows like e^{|t|/2}
    codes = W.random_pauli_strings(rng, n, 4)
    coeffs = rng.standard_normal(4)
    e, g = orc.adjoint_gradient(n, gates, theta, codes, coeffs)
    assert abs(e - D.energy(gates, theta, codes, coeffs, n)) < 1e-12
    fd = D.gradient_fd5(gates, theta, codes, coeffs, n)
    assert np.max(np.abs(g - fd)) < 1e-8 * max(1.0, np.max(np.abs(fd)))
    g2 = orc.reference_gradient(n, gates, theta, codes, coeffs)
    assert np.max(np.abs(g - g2)) < 1e-12 * max(1.0, np.max(np.abs(g)))


def test_nonhermitian_with_nonunitary(orc):
    """App. B.3 and B.4 together: the complex gradient of a non-Hermitian operator through
    non-unitary gates against the dense complex difference quotient."""
    rng = np.random.default_rng(430)
    n = 2
    gates, P = W.random_circuit(rng, n, 16, MIXED)
    theta = rng.uniform(-1.0, 1.0, P)
    codes = W.random_pauli_strings(rng, n, 3)
    c = rng.standard_normal(3) + 1j * rng.standard_normal(3)
    e, g = orc.adjoint_gradient_nonhermitian(n, gates, theta, codes, c)
    Am = D.hamiltonian(codes, c, n)

    def E(t):
        psi = D.circuit_operator(gates, t, n) @ D.zero_state(n)
        return complex(np.vdot(psi, Am @ psi))

    assert abs(e - E(theta)) < 1e-12
    h = 1e-3
    for p in range(P):
        vals = []
        for k in (-2, -1, 1, 2):
            t = theta.copy()
            t[p] += k * h
            vals.append(E(t))
        assert abs(g[p] - (vals[0] - 8 * vals[1] + 8 * vals[2] - vals[3]) / (12 * h)) < 1e-8
