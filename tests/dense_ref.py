"""Dense brute-force reference for tiny circuits (N <= 7), used to pin the CPU oracle.

Every operator is built as a full 2^N x 2^N matrix, independently of the oracle's construction:

* parameterised gates are matrix exponentials of their generators (``scipy.linalg.expm``):
  R_G(theta) = expm(-i theta G / 2); the phase gate expm(i theta |1><1|); controlled rotations
  expm(-i theta |1><1| (x) G / 2); U3 as the product of exponentials
  e^{i(f+l)/2} RZ(f) RY(t) RZ(l); the non-unitary imaginary-time rotations expm(-theta G / 2);
* each gate is embedded into the full space by index arithmetic;
* a Pauli string is a Kronecker product of 2x2 Paulis (qubit n-1 leftmost);
* E(theta) = psi^dag H psi with psi = (U_G ... U_1) |in>;
* gradients come from a 5-point central-difference stencil on the dense E, or the exact
  parameter-shift rule where it applies.
"""
from __future__ import annotations

import numpy as np
from scipy.linalg import expm

from paper_2009_02823_amd import workloads as W

I2 = np.eye(2, dtype=complex)
PX = np.array([[0, 1], [1, 0]], dtype=complex)
PY = np.array([[0, -1j], [1j, 0]], dtype=complex)
PZ = np.array([[1, 0], [0, -1]], dtype=complex)
PAULIS = [I2, PX, PY, PZ]
P1 = np.array([[0, 0], [0, 1]], dtype=complex)  # |1><1|


def _rot(G, t):
    return expm(-0.5j * t * G)


def local_matrix(kind: int, th) -> np.ndarray:
    """2x2 or 4x4 matrix of a gate; for two-qubit gates the local index is 2 bit(q0) + bit(q1)."""
    if kind in (W.RX, W.RY, W.RZ):
        return _rot(PAULIS[kind - W.RX + 1], th[0])
    if kind == W.H:
        return np.array([[1, 1], [1, -1]], dtype=complex) / np.sqrt(2)
    if kind in (W.X, W.Y, W.Z):
        return PAULIS[kind - W.X + 1].copy()
    if kind == W.S:
        return np.diag([1, 1j])
    if kind == W.SDG:
        return np.diag([1, -1j])
    if kind == W.T:
        return expm(1j * np.pi / 4 * P1)
    if kind == W.PHASE:
        return expm(1j * th[0] * P1)
    if kind == W.U3:
        t, f, l = th
        return np.exp(0.5j * (f + l)) * (_rot(PZ, f) @ _rot(PY, t) @ _rot(PZ, l))
    if kind == W.CNOT:
        return np.kron(np.diag([1, 0]), I2) + np.kron(P1, PX)
    if kind == W.CZ:
        return np.diag([1, 1, 1, -1]).astype(complex)
    if kind in (W.CRX, W.CRY, W.CRZ):
        return expm(-0.5j * th[0] * np.kron(P1, PAULIS[kind - W.CRX + 1]))
    if kind in (W.RXX, W.RYY, W.RZZ):
        s = PAULIS[kind - W.RXX + 1]
        return expm(-0.5j * th[0] * np.kron(s, s))
    if kind in (W.NRX, W.NRY, W.NRZ):  # imaginary-time rotation, not unitary
        return expm(-0.5 * th[0] * PAULIS[kind - W.NRX + 1])
    raise ValueError(kind)


def embed(U: np.ndarray, qubits, n: int) -> np.ndarray:
    """Full-space operator of U acting on ``qubits`` (first = most significant local bit)."""
    dim = 1 << n
    idx = np.arange(dim)
    loc = np.zeros(dim, dtype=np.int64)
    rest = idx.copy()
    for q in qubits:
        loc = (loc << 1) | ((idx >> q) & 1)
        rest &= ~(1 << q)
    same = rest[:, None] == rest[None, :]
    return np.where(same, U[loc[:, None], loc[None, :]], 0.0)


def gate_operator(row, theta, n) -> np.ndarray:
    kind, q0, q1 = int(row[0]), int(row[1]), int(row[2])
    th = [theta[p] if p >= 0 else 0.0 for p in row[3:6]]
    qubits = [q0] if W.N_QUBITS[kind] == 1 else [q0, q1]
    return embed(local_matrix(kind, th), qubits, n)


def circuit_operator(gates, theta, n) -> np.ndarray:
    U = np.eye(1 << n, dtype=complex)
    for row in gates:
        U = gate_operator(row, theta, n) @ U
    return U


def pauli_string(codes_row, n) -> np.ndarray:
    M = np.ones((1, 1), dtype=complex)
    for q in reversed(range(n)):
        M = np.kron(M, PAULIS[int(codes_row[q])])
    return M


def hamiltonian(codes, coeffs, n) -> np.ndarray:
    Hm = np.zeros((1 << n, 1 << n), dtype=complex)
    for row, c in zip(codes, coeffs):
        Hm += c * pauli_string(row, n)
    return Hm


def zero_state(n):
    v = np.zeros(1 << n, dtype=complex)
    v[0] = 1
    return v


def statevector(gates, theta, n, psi_in=None):
    psi = zero_state(n) if psi_in is None else np.asarray(psi_in, dtype=complex)
    return circuit_operator(gates, theta, n) @ psi


def energy(gates, theta, codes, coeffs, n, psi_in=None) -> complex:
    psi = statevector(gates, theta, n, psi_in)
    return complex(np.vdot(psi, hamiltonian(codes, coeffs, n) @ psi))


def gradient_fd5(gates, theta, codes, coeffs, n, h=1e-3, psi_in=None) -> np.ndarray:
    """Five-point central stencil (error O(h^4)) on the dense energy."""
    theta = np.asarray(theta, dtype=float)
    Hm = hamiltonian(codes, coeffs, n)
    psi0 = zero_state(n) if psi_in is None else np.asarray(psi_in, dtype=complex)

    def E(t):
        psi = circuit_operator(gates, t, n) @ psi0
        return np.vdot(psi, Hm @ psi).real

    g = np.zeros(theta.shape[0])
    for p in range(theta.shape[0]):
        vals = []
        for k in (-2, -1, 1, 2):
            t = theta.copy()
            t[p] += k * h
            vals.append(E(t))
        g[p] = (vals[0] - 8 * vals[1] + 8 * vals[2] - vals[3]) / (12 * h)
    return g
