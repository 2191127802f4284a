"""Seeded synthetic inputs: circuits, parameter vectors and Pauli-sum Hamiltonians.

This module only *describes* workloads. It holds none of the gradient method's arithmetic (no
gate matrices, no state-vectors, no sums) so that both the HIP library and the CPU oracle can be
fed the very same inputs without sharing any code that computes a result.

Encodings (these are the C-ABI's plain-data formats, see ``include/qsv.h``):

* A circuit is an ``int32`` table of shape ``(G, 6)``; row ``k`` is gate ``U_{k+1}`` in
  application order: ``(kind, q0, q1, p0, p1, p2)``. ``kind`` is a ``qsv_gate_kind`` code,
  ``q0``/``q1`` are qubits (``q1 = -1`` for one-qubit gates; for controlled gates ``q0`` is the
  control and ``q1`` the target), ``p0..p2`` index into the parameter vector (``-1`` = unused).
  Several gates may share one parameter (the repeated-parameter case of App. B.2).
* A Hamiltonian is ``codes`` (``uint8`` of shape ``(h, n)``, 0=I 1=X 2=Y 3=Z, ``codes[t, q]`` acts
  on qubit ``q``) and real ``coeffs`` (``float64`` of shape ``(h,)``): H = sum_t coeffs[t] P_t.
* Qubit ``q`` is bit ``q`` of an amplitude index (little-endian).

The workloads are the hardware-efficient ansatz (rotation layers plus a linear CNOT entangler, the
family of the paper's "Circuit C", Sec. 3) at the sizes of the five measured configurations, and
the Hamiltonians that go with them.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# qsv_gate_kind codes (one source of truth for Python; the C header repeats them).
RX, RY, RZ, H, X, Y, Z, S, CNOT, CZ = range(10)
PHASE, CRX, CRY, CRZ, RXX, RYY, RZZ, U3, T, SDG = range(10, 20)

GATE_NAMES = {
    RX: "RX", RY: "RY", RZ: "RZ", H: "H", X: "X", Y: "Y", Z: "Z", S: "S", CNOT: "CNOT", CZ: "CZ",
    PHASE: "PHASE", CRX: "CRX", CRY: "CRY", CRZ: "CRZ", RXX: "RXX", RYY: "RYY", RZZ: "RZZ",
    U3: "U3", T: "T", SDG: "SDG",
}
#: non-unitary, invertible gates (App. B.3): imaginary-time rotations exp(-theta G / 2)
NRX, NRY, NRZ = range(20, 23)
NONUNITARY_NAMES = {NRX: "NRX", NRY: "NRY", NRZ: "NRZ"}
#: every kind, unitary or not
KIND_NAMES = {**GATE_NAMES, **NONUNITARY_NAMES}
#: number of parameters each kind takes
N_PARAMS = {k: 0 for k in KIND_NAMES}
N_PARAMS.update({RX: 1, RY: 1, RZ: 1, PHASE: 1, CRX: 1, CRY: 1, CRZ: 1, RXX: 1, RYY: 1, RZZ: 1,
                 U3: 3, NRX: 1, NRY: 1, NRZ: 1})
#: number of qubits each kind acts on
N_QUBITS = {k: 1 for k in KIND_NAMES}
N_QUBITS.update({CNOT: 2, CZ: 2, CRX: 2, CRY: 2, CRZ: 2, RXX: 2, RYY: 2, RZZ: 2})

PAULI_I, PAULI_X, PAULI_Y, PAULI_Z = 0, 1, 2, 3

SEED_ROOT = 2009_02823


def rng_for(config_id: int) -> np.random.Generator:
    """The generator every workload of configuration ``config_id`` draws from."""
    return np.random.default_rng([SEED_ROOT, config_id])


def gate_row(kind: int, q0: int, q1: int = -1, p0: int = -1, p1: int = -1, p2: int = -1):
    return (kind, q0, q1, p0, p1, p2)


def circuit_table(rows) -> np.ndarray:
    t = np.asarray(list(rows), dtype=np.int32).reshape(-1, 6)
    return np.ascontiguousarray(t)


def hea_circuit(n: int, layers: int, cz_brickwork: bool = False) -> np.ndarray:
    """Hardware-efficient ansatz: per layer l, RY(theta[2nl+q]) on every qubit, then
    RZ(theta[2nl+n+q]) on every qubit, then CNOT(q -> q+1) for q = 0..n-2, optionally followed by
    a CZ brickwork (even pairs, then odd pairs). P = 2 n layers parameters, each used once."""
    rows = []
    for l in range(layers):
        base = 2 * n * l
        rows += [gate_row(RY, q, -1, base + q) for q in range(n)]
        rows += [gate_row(RZ, q, -1, base + n + q) for q in range(n)]
        rows += [gate_row(CNOT, q, q + 1) for q in range(n - 1)]
        if cz_brickwork:
            rows += [gate_row(CZ, q, q + 1) for q in range(0, n - 1, 2)]
            rows += [gate_row(CZ, q, q + 1) for q in range(1, n - 1, 2)]
    return circuit_table(rows)


def n_params_of(gates: np.ndarray) -> int:
    p = gates[:, 3:6]
    return int(p.max()) + 1 if p.size and p.max() >= 0 else 0


def uniform_angles(rng: np.random.Generator, count: int) -> np.ndarray:
    return rng.uniform(0.0, 2.0 * math.pi, count).astype(np.float64)


def random_pauli_strings(rng: np.random.Generator, n: int, h: int) -> np.ndarray:
    """``h`` strings with every qubit's letter iid uniform over {I, X, Y, Z}."""
    return rng.integers(0, 4, size=(h, n)).astype(np.uint8)


def random_weight_pauli_strings(rng: np.random.Generator, n: int, h: int,
                                wmin: int = 2, wmax: int = 6) -> np.ndarray:
    """``h`` strings of weight w ~ U{wmin..wmax} on w distinct uniform qubits, letters iid
    uniform over {X, Y, Z}."""
    codes = np.zeros((h, n), dtype=np.uint8)
    for t in range(h):
        w = int(rng.integers(wmin, wmax + 1))
        support = rng.choice(n, size=w, replace=False)
        letters = rng.integers(1, 4, size=w)
        codes[t, support] = letters
    return codes


def ising_chain(n: int, J, hx) -> tuple[np.ndarray, np.ndarray]:
    """Open chain sum_i J_i Z_i Z_{i+1} + sum_i hx_i X_i (scalars broadcast)."""
    J = np.broadcast_to(np.asarray(J, dtype=np.float64), (n - 1,))
    hx = np.broadcast_to(np.asarray(hx, dtype=np.float64), (n,))
    codes = np.zeros((2 * n - 1, n), dtype=np.uint8)
    for i in range(n - 1):
        codes[i, i] = codes[i, i + 1] = PAULI_Z
    for i in range(n):
        codes[n - 1 + i, i] = PAULI_X
    coeffs = np.concatenate([J, hx]).astype(np.float64)
    return codes, coeffs


def heisenberg_chain(n: int) -> tuple[np.ndarray, np.ndarray]:
    """Open chain sum_i (X_i X_{i+1} + Y_i Y_{i+1} + Z_i Z_{i+1}), unit coefficients."""
    codes = np.zeros((3 * (n - 1), n), dtype=np.uint8)
    for i in range(n - 1):
        for k, letter in enumerate((PAULI_X, PAULI_Y, PAULI_Z)):
            codes[3 * i + k, i] = codes[3 * i + k, i + 1] = letter
    return codes, np.ones(3 * (n - 1), dtype=np.float64)


def hadamard_product_observable(n: int) -> tuple[np.ndarray, np.ndarray]:
    """The operator Hadamard^(x)n of the paper's benchmarks (Sec. 3) as an exact Pauli sum:
    Hadamard = (X + Z)/sqrt(2) on every qubit, so the product is the sum of all 2^n strings over
    {X, Z} with coefficient 2^(-n/2)."""
    h = 1 << n
    codes = np.empty((h, n), dtype=np.uint8)
    for t in range(h):
        for q in range(n):
            codes[t, q] = PAULI_X if (t >> q) & 1 else PAULI_Z
    return codes, np.full(h, 2.0 ** (-0.5 * n), dtype=np.float64)


@dataclass
class Problem:
    """One energy-plus-gradient instance."""
    name: str
    n_qubits: int
    gates: np.ndarray          # int32 (G, 6)
    theta: np.ndarray          # float64 (P,)
    codes: np.ndarray          # uint8 (h, n)
    coeffs: np.ndarray         # float64 (h,)
    dtypes: tuple = ("c128",)
    meta: dict = field(default_factory=dict)

    @property
    def n_params(self) -> int:
        return int(self.theta.shape[0])

    @property
    def n_gates(self) -> int:
        return int(self.gates.shape[0])


def config1() -> Problem:
    """10 qubits, 4 HEA layers (P = 80), 20 random Pauli strings, N(0,1) coefficients."""
    n, L = 10, 4
    rng = rng_for(1)
    theta = uniform_angles(rng, 2 * n * L)
    codes = random_pauli_strings(rng, n, 20)
    coeffs = rng.standard_normal(20)
    return Problem("hea10_L4_rand20", n, hea_circuit(n, L), theta, codes, coeffs, ("c128",))


def config2(n: int = 20, layers: int = 20) -> Problem:
    """20 qubits, 20 HEA layers (P = 800), open TFIM sum Z_iZ_{i+1} + 0.7 sum X_i."""
    rng = rng_for(2)
    theta = uniform_angles(rng, 2 * n * layers)
    codes, coeffs = ising_chain(n, 1.0, 0.7)
    return Problem(f"hea{n}_L{layers}_tfim", n, hea_circuit(n, layers), theta, codes, coeffs,
                   ("c128", "c64"))


def config3(n: int = 26, layers: int = 30, h: int = 200) -> Problem:
    """26 qubits, 30 layers RY/RZ + CNOT ladder + CZ brickwork (P = 1560), 200 random strings of
    weight 2..6 with N(0,1) coefficients; complex64 storage."""
    rng = rng_for(3)
    theta = uniform_angles(rng, 2 * n * layers)
    codes = random_weight_pauli_strings(rng, n, h)
    coeffs = rng.standard_normal(h)
    return Problem(f"hea{n}_L{layers}_cz_rand{h}", n, hea_circuit(n, layers, cz_brickwork=True),
                   theta, codes, coeffs, ("c64",))


def config4(batch: int = 512, nmin: int = 12, nmax: int = 18, lmin: int = 5, lmax: int = 15):
    """A batch of independent HEA circuits with uneven sizes, Heisenberg chain per circuit."""
    rng = rng_for(4)
    ns = rng.integers(nmin, nmax + 1, size=batch)
    ls = rng.integers(lmin, lmax + 1, size=batch)
    probs = []
    for b in range(batch):
        n, L = int(ns[b]), int(ls[b])
        theta = uniform_angles(rng, 2 * n * L)
        codes, coeffs = heisenberg_chain(n)
        probs.append(Problem(f"hea{n}_L{L}_heis#{b}", n, hea_circuit(n, L), theta, codes, coeffs,
                             ("c128",)))
    return probs


def config5(n: int = 30, layers: int = 10) -> Problem:
    """30 qubits, 10 layers (P = 600), open Ising chain with N(0,1) couplings and fields."""
    rng = rng_for(5)
    theta = uniform_angles(rng, 2 * n * layers)
    J = rng.standard_normal(n - 1)
    hx = rng.standard_normal(n)
    codes, coeffs = ising_chain(n, J, hx)
    return Problem(f"hea{n}_L{layers}_ising", n, hea_circuit(n, layers), theta, codes, coeffs,
                   ("c128",))


def random_circuit(rng: np.random.Generator, n: int, n_gates: int, kinds=None,
                   n_params: int | None = None) -> tuple[np.ndarray, int]:
    """A random gate sequence over ``kinds`` for tests; parameters are unique unless
    ``n_params`` is given (then they are drawn with repetition from range(n_params))."""
    if kinds is None:
        kinds = [RX, RY, RZ, H, X, Y, Z, S, CNOT, CZ]
    rows = []
    next_p = 0
    for _ in range(n_gates):
        k = int(kinds[int(rng.integers(0, len(kinds)))])
        if N_QUBITS[k] == 2:
            if n < 2:
                continue
            a, b = rng.choice(n, size=2, replace=False)
            q0, q1 = int(a), int(b)
        else:
            q0, q1 = int(rng.integers(0, n)), -1
        ps = []
        for _j in range(N_PARAMS[k]):
            if n_params is None:
                ps.append(next_p)
                next_p += 1
            else:
                ps.append(int(rng.integers(0, n_params)))
        ps += [-1] * (3 - len(ps))
        rows.append((k, q0, q1, *ps))
    P = next_p if n_params is None else n_params
    return circuit_table(rows), P


def paper_benchmark(n: int = 5, layers: int = 129) -> Problem:
    """The paper's benchmark regime (Sec. 3): a few qubits, many parameters, under
    Hadamard^(x)n; the HEA (RY, RZ on every qubit, CNOT ladder) stands in for its ansatz circuits.
    P = 2 n layers (n = 5, 129 layers: P = 1290, the largest count benchmarked there)."""
    rng = rng_for(6)
    theta = uniform_angles(rng, 2 * n * layers)
    codes, coeffs = hadamard_product_observable(n)
    return Problem(f"hea{n}_L{layers}_hadamard", n, hea_circuit(n, layers), theta, codes, coeffs,
                   ("c128",))


CONFIGS = {1: config1, 2: config2, 3: config3, 4: config4, 5: config5}
