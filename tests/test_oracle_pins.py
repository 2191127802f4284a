"""Pins of the CPU oracle against what the paper and the mathematics fix (no GPU).

Each test checks the oracle against something other than itself: closed forms, a dense
brute force built from matrix exponentials, the two differently ordered exact algorithms of the
paper (Algorithm 1 vs Algorithm 2), the exact parameter-shift rule, finite differences
(Sec. 1, in central form), unitarity, Hermiticity and linearity.
"""
import math

import numpy as np
import pytest

import dense_ref as D
from paper_2009_02823_amd import workloads as W

TOL = 1e-12


def one_q_problem(a, b, hx, hy, hz):
    gates = W.circuit_table([W.gate_row(W.RY, 0, -1, 0), W.gate_row(W.RZ, 0, -1, 1)])
    codes = np.array([[W.PAULI_X], [W.PAULI_Y], [W.PAULI_Z]], dtype=np.uint8)
    return gates, np.array([a, b]), codes, np.array([hx, hy, hz])


# --------------------------------------------------------------------------- closed forms
@pytest.mark.parametrize("seed", range(6))
def test_closed_form_single_qubit(orc, seed):
    """RY(a) then RZ(b) on |0>, H = hx X + hy Y + hz Z (Bloch vector of the state):
    E = hx sin a cos b + hy sin a sin b + hz cos a, with its analytic partial derivatives."""
    rng = np.random.default_rng(seed)
    a, b = rng.uniform(0, 2 * math.pi, 2)
    hx, hy, hz = rng.standard_normal(3)
    gates, theta, codes, coeffs = one_q_problem(a, b, hx, hy, hz)
    e, g = orc.adjoint_gradient(1, gates, theta, codes, coeffs)
    E = hx * math.sin(a) * math.cos(b) + hy * math.sin(a) * math.sin(b) + hz * math.cos(a)
    dEa = hx * math.cos(a) * math.cos(b) + hy * math.cos(a) * math.sin(b) - hz * math.sin(a)
    dEb = -hx * math.sin(a) * math.sin(b) + hy * math.sin(a) * math.cos(b)
    assert abs(e.real - E) < TOL and abs(e.imag) < TOL
    assert abs(g[0] - dEa) < TOL and abs(g[1] - dEb) < TOL


@pytest.mark.parametrize("theta", [0.0, 0.3, 1.0, math.pi / 2, 2.5, math.pi, 4.0, 5.9])
def test_ry_under_z_and_x(orc, theta):
    """<Z> = cos(theta), gradient -sin(theta) fixes |alpha| = 1/2; <X> = sin(theta), gradient
    cos(theta) fixes its sign (alpha = -1/2, Appendix A)."""
    gates = W.circuit_table([W.gate_row(W.RY, 0, -1, 0)])
    for code, E, G in ((W.PAULI_Z, math.cos(theta), -math.sin(theta)),
                       (W.PAULI_X, math.sin(theta), math.cos(theta))):
        e, g = orc.adjoint_gradient(1, gates, [theta], np.array([[code]]), [1.0])
        assert abs(e.real - E) < TOL and abs(g[0] - G) < TOL


@pytest.mark.parametrize("a", [0.1, 0.9, 2.2, 3.7, 5.5])
def test_closed_form_two_qubits(orc, a):
    """RY(a) on q0, CNOT(0 -> 1) prepares cos(a/2)|00> + sin(a/2)|11>:
    <Z0Z1> = 1, <Z1> = cos a, <X0X1> = sin a, <Y0Y1> = -sin a."""
    gates = W.circuit_table([W.gate_row(W.RY, 0, -1, 0), W.gate_row(W.CNOT, 0, 1)])
    cases = [([3, 3], 1.0, 0.0), ([0, 3], math.cos(a), -math.sin(a)),
             ([1, 1], math.sin(a), math.cos(a)), ([2, 2], -math.sin(a), -math.cos(a))]
    for codes, E, G in cases:
        e, g = orc.adjoint_gradient(2, gates, [a], np.array([codes], dtype=np.uint8), [1.0])
        assert abs(e.real - E) < TOL and abs(g[0] - G) < TOL


def test_little_endian_and_bell_amplitudes(orc):
    """Qubit q is bit q: X on qubit 0 of |000> gives index 1; RY(a) q0 + CNOT(0->1) puts the
    amplitudes cos(a/2), sin(a/2) at indices 0 and 3."""
    psi = orc.statevector(3, W.circuit_table([W.gate_row(W.X, 0)]), [])
    assert np.argmax(abs(psi)) == 1 and abs(psi[1] - 1) < TOL
    psi = orc.statevector(3, W.circuit_table([W.gate_row(W.X, 2)]), [])
    assert abs(psi[4] - 1) < TOL
    a = 1.234
    psi = orc.statevector(2, W.circuit_table([W.gate_row(W.RY, 0, -1, 0),
                                              W.gate_row(W.CNOT, 0, 1)]), [a])
    assert np.allclose(psi, [math.cos(a / 2), 0, 0, math.sin(a / 2)], atol=TOL)
    # CNOT with control 1 and target 0 acting on |10> (index 2) gives |11> (index 3)
    psi = orc.statevector(2, W.circuit_table([W.gate_row(W.X, 1), W.gate_row(W.CNOT, 1, 0)]), [])
    assert abs(psi[3] - 1) < TOL


def tfim_product_layer(n, rng):
    """One layer RY(a_q), RZ(b_q), no entangler; H = sum J_i Z_i Z_{i+1} + sum h_i X_i.
    Product state with Bloch vectors (sin a cos b, sin a sin b, cos a) per qubit."""
    a = rng.uniform(0, 2 * math.pi, n)
    b = rng.uniform(0, 2 * math.pi, n)
    J = rng.standard_normal(n - 1)
    h = rng.standard_normal(n)
    rows = [W.gate_row(W.RY, q, -1, q) for q in range(n)]
    rows += [W.gate_row(W.RZ, q, -1, n + q) for q in range(n)]
    codes, coeffs = W.ising_chain(n, J, h)
    E = np.sum(J * np.cos(a[:-1]) * np.cos(a[1:])) + np.sum(h * np.sin(a) * np.cos(b))
    ga = h * np.cos(a) * np.cos(b)
    ga[:-1] += -J * np.sin(a[:-1]) * np.cos(a[1:])
    ga[1:] += -J * np.cos(a[:-1]) * np.sin(a[1:])
    gb = -h * np.sin(a) * np.sin(b)
    return W.circuit_table(rows), np.concatenate([a, b]), codes, coeffs, E, np.concatenate([ga, gb])


@pytest.mark.parametrize("n", [2, 5, 9])
def test_scalable_closed_form(orc, n):
    gates, theta, codes, coeffs, E, G = tfim_product_layer(n, np.random.default_rng(n))
    e, g = orc.adjoint_gradient(n, gates, theta, codes, coeffs)
    assert abs(e.real - E) < 1e-12 * n
    assert np.max(abs(g - G)) < 1e-12 * n


def test_theta_zero_hea(orc):
    """At theta = 0 the HEA leaves |0...0> unchanged (CNOTs act trivially), so E is the sum of
    the coefficients of the I/Z-only strings, and every RZ entry of the gradient is 0."""
    n, L = 6, 3
    gates = W.hea_circuit(n, L)
    rng = np.random.default_rng(7)
    codes = W.random_pauli_strings(rng, n, 30)
    coeffs = rng.standard_normal(30)
    theta = np.zeros(2 * n * L)
    e, g = orc.adjoint_gradient(n, gates, theta, codes, coeffs)
    zonly = np.all((codes == 0) | (codes == 3), axis=1)
    assert abs(e.real - coeffs[zonly].sum()) < TOL
    rz = [l * 2 * n + n + q for l in range(L) for q in range(n)]
    assert np.max(abs(g[rz])) < TOL


def test_diagonal_h_last_rz_layer_zero(orc):
    """With an I/Z-only H, the RZ gates of the last layer have zero gradient: the CNOT ladder is
    a permutation, so it keeps U^dag H U diagonal, which commutes with RZ."""
    n, L = 5, 3
    rng = np.random.default_rng(11)
    gates = W.hea_circuit(n, L)
    theta = W.uniform_angles(rng, 2 * n * L)
    codes = rng.choice([0, 3], size=(12, n)).astype(np.uint8)
    coeffs = rng.standard_normal(12)
    e, g = orc.adjoint_gradient(n, gates, theta, codes, coeffs)
    last_rz = [(L - 1) * 2 * n + n + q for q in range(n)]
    assert np.max(abs(g[last_rz])) < TOL
    assert np.max(abs(g)) > 1e-3   # the others are generically nonzero


# --------------------------------------------------------------------------- dense brute force
ALL_KINDS = [W.RX, W.RY, W.RZ, W.H, W.X, W.Y, W.Z, W.S, W.CNOT, W.CZ, W.PHASE, W.CRX, W.CRY,
             W.CRZ, W.RXX, W.RYY, W.RZZ, W.U3, W.T, W.SDG]


@pytest.mark.parametrize("kind", ALL_KINDS)
def test_gate_matrix_vs_expm(orc, kind):
    """Each gate applied by the oracle to a random state equals the dense expm-built operator,
    and U^dag undoes U."""
    n = 3
    rng = np.random.default_rng(100 + kind)
    psi = rng.standard_normal(8) + 1j * rng.standard_normal(8)
    psi /= np.linalg.norm(psi)
    theta = rng.uniform(0, 2 * math.pi, 3)
    nq, npar = W.N_QUBITS[kind], W.N_PARAMS[kind]
    for q0, q1 in ([(0, -1), (1, -1), (2, -1)] if nq == 1 else [(0, 1), (1, 0), (2, 0), (0, 2)]):
        row = W.gate_row(kind, q0, q1, *[j if j < npar else -1 for j in range(3)])
        got = orc.statevector(n, W.circuit_table([row]), theta, psi_in=psi)
        want = D.gate_operator(row, theta, n) @ psi
        assert np.max(abs(got - want)) < TOL
        back = orc.statevector(n, W.circuit_table([row]), theta, psi_in=got, inverse=True)
        assert np.max(abs(back - psi)) < TOL


@pytest.mark.parametrize("kind", [k for k in ALL_KINDS if W.N_PARAMS[k] > 0])
def test_derivative_matrix_vs_difference_quotient(orc, kind):
    """dU/dtheta_j applied by the oracle equals the 5-point difference quotient of the dense
    expm operator."""
    n = 2
    rng = np.random.default_rng(200 + kind)
    psi = rng.standard_normal(4) + 1j * rng.standard_normal(4)
    theta = rng.uniform(0, 2 * math.pi, 3)
    nq, npar = W.N_QUBITS[kind], W.N_PARAMS[kind]
    row = W.gate_row(kind, 1, 0 if nq == 2 else -1, *[j if j < npar else -1 for j in range(3)])
    h = 1e-3
    for j in range(npar):
        got = orc.apply_derivative(n, row, theta, psi, j)
        ops = []
        for k in (-2, -1, 1, 2):
            t = theta.copy()
            t[j] += k * h
            ops.append(D.gate_operator(row, t, n))
        dU = (ops[0] - 8 * ops[1] + 8 * ops[2] - ops[3]) / (12 * h)
        assert np.max(abs(got - dU @ psi)) < 1e-10


@pytest.mark.parametrize("seed", range(5))
def test_pauli_sum_apply_vs_kron(orc, seed):
    n = 5
    rng = np.random.default_rng(300 + seed)
    codes = W.random_pauli_strings(rng, n, 9)
    coeffs = rng.standard_normal(9)
    psi = rng.standard_normal(32) + 1j * rng.standard_normal(32)
    got = orc.apply_pauli_sum(n, codes, coeffs, psi)
    want = D.hamiltonian(codes, coeffs, n) @ psi
    assert np.max(abs(got - want)) < TOL


@pytest.mark.parametrize("seed", range(8))
def test_algorithms_vs_dense(orc, seed):
    """Algorithm 1 (reverse mode) and Algorithm 2 (reference) agree with each other to rounding
    and with a dense-matrix difference quotient of E, on random circuits over every gate kind,
    including repeated parameters and a random input state."""
    rng = np.random.default_rng(400 + seed)
    n = int(rng.integers(1, 6)) if seed else 1
    kinds = ALL_KINDS if n >= 2 else [k for k in ALL_KINDS if W.N_QUBITS[k] == 1]
    gates, P = W.random_circuit(rng, n, int(rng.integers(5, 25)), kinds,
                                n_params=None if seed % 2 else 6)
    theta = W.uniform_angles(rng, P)
    codes = W.random_pauli_strings(rng, n, 7)
    coeffs = rng.standard_normal(7)
    psi_in = None
    if seed % 3 == 2:
        psi_in = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
        psi_in /= np.linalg.norm(psi_in)
    e1, g1 = orc.adjoint_gradient(n, gates, theta, codes, coeffs, psi_in=psi_in)
    g2 = orc.reference_gradient(n, gates, theta, codes, coeffs, psi_in=psi_in)
    e_d = D.energy(gates, theta, codes, coeffs, n, psi_in)
    g_d = D.gradient_fd5(gates, theta, codes, coeffs, n, psi_in=psi_in)
    scale = max(1.0, np.abs(coeffs).sum())
    assert abs(e1 - e_d) < 1e-12 * scale
    assert np.max(abs(g1 - g2)) < 1e-12 * scale
    assert np.max(abs(g1 - g_d)) < 1e-8 * scale


@pytest.mark.parametrize("n", [3, 6])
def test_parameter_shift_exact(orc, n):
    """For rotations exp(-i theta G/2) the two-term shift rule is exact: HEA with RX too."""
    rng = np.random.default_rng(n)
    rows = list(map(tuple, W.hea_circuit(n, 2)))
    rows += [W.gate_row(W.RX, q, -1, 4 * n + q) for q in range(n)]
    gates = W.circuit_table(rows)
    theta = W.uniform_angles(rng, 5 * n)
    codes = W.random_pauli_strings(rng, n, 10)
    coeffs = rng.standard_normal(10)
    _, g = orc.adjoint_gradient(n, gates, theta, codes, coeffs)
    gps = orc.parameter_shift(n, gates, theta, codes, coeffs)
    assert np.max(abs(g - gps)) < 1e-12 * np.abs(coeffs).sum()


def test_central_difference(orc):
    """Central finite differences (h = 1e-5) agree to ~1e-8 relative (Sec. 1, central form)."""
    n = 6
    rng = np.random.default_rng(5)
    gates = W.hea_circuit(n, 3)
    theta = W.uniform_angles(rng, 6 * n)
    codes, coeffs = W.ising_chain(n, rng.standard_normal(n - 1), rng.standard_normal(n))
    _, g = orc.adjoint_gradient(n, gates, theta, codes, coeffs)
    gfd = orc.central_difference(n, gates, theta, codes, coeffs, h=1e-5)
    assert np.max(abs(g - gfd)) < 1e-8 * max(1.0, np.max(abs(g)))


# --------------------------------------------------------------------------- invariants
def test_unitarity_and_norm(orc):
    """Unitaries are reversible: U^dag U |in> = |in>; ||U|in>|| = 1."""
    n = 8
    rng = np.random.default_rng(9)
    gates = W.hea_circuit(n, 4, cz_brickwork=True)
    theta = W.uniform_angles(rng, 8 * n)
    psi = orc.statevector(n, gates, theta)
    assert abs(np.linalg.norm(psi) - 1) < 1e-13
    back = orc.statevector(n, gates, theta, psi_in=psi, inverse=True)
    assert np.max(abs(back - orc.zero_state(n))) < 1e-13


def test_hermitian_energy_is_real(orc):
    p = W.config1()
    e, _ = orc.adjoint_gradient(p.n_qubits, p.gates, p.theta, p.codes, p.coeffs)
    assert abs(e.imag) < 1e-13 * np.abs(p.coeffs).sum()
    e2 = orc.energy(p.n_qubits, p.gates, p.theta, p.codes, p.coeffs)
    assert abs(e - e2) < 1e-13 * np.abs(p.coeffs).sum()


def test_linearity_in_h(orc):
    """g(c1 H1 + c2 H2) = c1 g(H1) + c2 g(H2): lambda = H psi enters the products linearly."""
    n = 6
    rng = np.random.default_rng(3)
    gates = W.hea_circuit(n, 2)
    theta = W.uniform_angles(rng, 4 * n)
    c1, c2 = 0.7, -1.3
    cod1, cf1 = W.random_pauli_strings(rng, n, 5), rng.standard_normal(5)
    cod2, cf2 = W.random_pauli_strings(rng, n, 4), rng.standard_normal(4)
    e1, g1 = orc.adjoint_gradient(n, gates, theta, cod1, cf1)
    e2, g2 = orc.adjoint_gradient(n, gates, theta, cod2, cf2)
    e12, g12 = orc.adjoint_gradient(n, gates, theta, np.vstack([cod1, cod2]),
                                     np.concatenate([c1 * cf1, c2 * cf2]))
    assert abs(e12 - (c1 * e1 + c2 * e2)) < 1e-12
    assert np.max(abs(g12 - (c1 * g1 + c2 * g2))) < 1e-12


def test_repeated_parameters_sum(orc):
    """App. B.2: a parameter shared by several gates gets the sum of the entries it would get if
    each occurrence had its own parameter."""
    n = 4
    rng = np.random.default_rng(21)
    gates = W.hea_circuit(n, 3)
    P = 6 * n
    tie = rng.integers(0, 5, size=P)        # unique parameter p -> shared parameter tie[p]
    theta_t = W.uniform_angles(rng, 5)
    theta_u = theta_t[tie]                  # the untied circuit evaluated at the same point
    tied = gates.copy()
    tied[:, 3] = np.where(gates[:, 3] >= 0, tie[np.maximum(gates[:, 3], 0)], -1)
    codes = W.random_pauli_strings(rng, n, 6)
    coeffs = rng.standard_normal(6)
    _, gu = orc.adjoint_gradient(n, gates, theta_u, codes, coeffs)
    _, gt = orc.adjoint_gradient(n, tied, theta_t, codes, coeffs)
    want = np.zeros(5)
    np.add.at(want, tie, gu)
    assert np.max(abs(gt - want)) < 1e-12


def test_adjoint_products_are_the_gradient(orc):
    """2 Re of the per-occurrence products sums to the gradient; their order is the sweep order
    (last gate first)."""
    p = W.config1()
    e, g, prods = orc.adjoint_gradient(p.n_qubits, p.gates, p.theta, p.codes, p.coeffs,
                                       return_prods=True)
    params = [int(r[3]) for r in p.gates[::-1] if r[3] >= 0]
    acc = np.zeros(p.n_params)
    np.add.at(acc, params, 2 * prods.real)
    assert np.max(abs(acc - g)) < 1e-15
