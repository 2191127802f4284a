"""ctypes front end of the complex128 CPU oracle (``qsv_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the tests, ``__graft_entry__.smoke()`` and the benchmark's
CPU-baseline leg, never by the GPU library. Every function takes plain numpy inputs in the
interface formats of the library (gate table ``int32 (G, 6)``, Pauli ``codes uint8 (h, n)`` and
``coeffs float64 (h,)``) and returns numpy results.

What each call computes (paper: Jones & Gacon, arXiv:2009.02823):

* ``statevector``       psi = U_G ... U_1 |in>                                    (Sec. 2.2)
* ``energy``            <psi|H|psi> as a complex number (imaginary part ~ 0 for real coeffs)
* ``adjoint_gradient``  Algorithm 1, with three working states (Sec. 2.3)
* ``reference_gradient``  Algorithm 2 / Eq. (reference_gradient), O(P^2) gates (Sec. 3)
* ``parameter_shift`` / ``central_difference``  gradients from energies alone
"""
from __future__ import annotations

import contextlib
import ctypes
import math

import numpy as np

from . import build as _build

_lib = None


def load(path: str):
    """Open a compiled oracle library and declare its signatures."""
    L = ctypes.CDLL(path)
    P = ctypes.c_void_p
    i = ctypes.c_int
    L.orc_num_threads.restype = i
    L.orc_apply_circuit.argtypes = [i, P, P, i, P, i, i]
    L.orc_apply_derivative.argtypes = [i, P, P, P, i, i]
    L.orc_apply_pauli_sum.argtypes = [i, P, P, i, P, P]
    L.orc_inner.argtypes = [i, P, P, P]
    L.orc_energy.argtypes = [i, P, P, i, P, i, i, P, P, P]
    L.orc_adjoint_gradient.argtypes = [i, P, P, i, P, i, i, P, P, P, P, P]
    L.orc_reference_gradient.argtypes = [i, P, P, i, P, i, i, P, P, P]
    L.orc_adjoint_gradient_nonhermitian.argtypes = [i, P, P, i, P, i, i, P, P, P, P, P]
    for f in (L.orc_apply_circuit, L.orc_apply_derivative, L.orc_apply_pauli_sum,
              L.orc_inner, L.orc_energy, L.orc_adjoint_gradient, L.orc_reference_gradient,
              L.orc_adjoint_gradient_nonhermitian):
        f.restype = i
    return L


@contextlib.contextmanager
def using(path: str):
    """Temporarily route every call of this module to another build of the oracle (the
    mutation tests use it to run the pins against deliberately broken copies)."""
    global _lib
    saved = _lib
    _lib = load(path)
    try:
        yield
    finally:
        _lib = saved


def lib():
    global _lib
    if _lib is None:
        _lib = load(_build.build())
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _prep(n, gates, theta, codes=None, coeffs=None, psi_in=None):
    gates = np.ascontiguousarray(np.asarray(gates, dtype=np.int32).reshape(-1, 6))
    theta = np.ascontiguousarray(np.asarray(theta, dtype=np.float64).reshape(-1))
    if codes is not None:
        codes = np.ascontiguousarray(np.asarray(codes, dtype=np.uint8).reshape(-1, n))
        coeffs = np.ascontiguousarray(np.asarray(coeffs, dtype=np.float64).reshape(-1))
        assert codes.shape[0] == coeffs.shape[0]
    if psi_in is not None:
        psi_in = np.ascontiguousarray(np.asarray(psi_in, dtype=np.complex128))
        assert psi_in.shape == (1 << n,)
    return gates, theta, codes, coeffs, psi_in


def _check(rc, what):
    if rc != 0:
        raise ValueError(f"oracle {what} rejected its input (code {rc})")


def num_threads() -> int:
    return int(lib().orc_num_threads())


def zero_state(n: int) -> np.ndarray:
    psi = np.zeros(1 << n, dtype=np.complex128)
    psi[0] = 1.0
    return psi


def statevector(n, gates, theta, psi_in=None, inverse=False) -> np.ndarray:
    """U |in> (or U^dag |in> when ``inverse``)."""
    gates, theta, _, _, psi_in = _prep(n, gates, theta, psi_in=psi_in)
    psi = zero_state(n) if psi_in is None else psi_in.copy()
    _check(lib().orc_apply_circuit(n, _ptr(psi), _ptr(gates), gates.shape[0], _ptr(theta),
                                   theta.shape[0], 1 if inverse else 0), "statevector")
    return psi


def apply_derivative(n, gate_row, theta, psi, j=0) -> np.ndarray:
    """(dU/d theta_j) psi for a single gate row."""
    gates, theta, _, _, psi = _prep(n, [gate_row], theta, psi_in=psi)
    out = psi.copy()
    _check(lib().orc_apply_derivative(n, _ptr(out), _ptr(gates), _ptr(theta), theta.shape[0], j),
           "apply_derivative")
    return out


def apply_pauli_sum(n, codes, coeffs, psi) -> np.ndarray:
    """H psi (unnormalised)."""
    _, _, codes, coeffs, psi = _prep(n, np.zeros((0, 6)), [], codes, coeffs, psi)
    out = np.empty_like(psi)
    _check(lib().orc_apply_pauli_sum(n, _ptr(psi), _ptr(out), codes.shape[0], _ptr(codes),
                                     _ptr(coeffs)), "apply_pauli_sum")
    return out


def inner(a, b) -> complex:
    a = np.ascontiguousarray(a, dtype=np.complex128)
    b = np.ascontiguousarray(b, dtype=np.complex128)
    n = int(round(math.log2(a.shape[0])))
    out = np.zeros(2)
    lib().orc_inner(n, _ptr(a), _ptr(b), _ptr(out))
    return complex(out[0], out[1])


def energy(n, gates, theta, codes, coeffs, psi_in=None) -> complex:
    gates, theta, codes, coeffs, psi_in = _prep(n, gates, theta, codes, coeffs, psi_in)
    out = np.zeros(2)
    _check(lib().orc_energy(n, _ptr(psi_in), _ptr(gates), gates.shape[0], _ptr(theta),
                            theta.shape[0], codes.shape[0], _ptr(codes), _ptr(coeffs), _ptr(out)),
           "energy")
    return complex(out[0], out[1])


def adjoint_gradient(n, gates, theta, codes, coeffs, psi_in=None, return_prods=False):
    """Algorithm 1. Returns (energy (complex), grad (P,)) [, prods (complex, sweep order)]."""
    gates, theta, codes, coeffs, psi_in = _prep(n, gates, theta, codes, coeffs, psi_in)
    out = np.zeros(2)
    grad = np.zeros(theta.shape[0])
    n_occ = int((gates[:, 3:6] >= 0).sum())
    prods = np.zeros(2 * max(n_occ, 1)) if return_prods else None
    _check(lib().orc_adjoint_gradient(n, _ptr(psi_in), _ptr(gates), gates.shape[0], _ptr(theta),
                                      theta.shape[0], codes.shape[0], _ptr(codes), _ptr(coeffs),
                                      _ptr(out), _ptr(grad), _ptr(prods)), "adjoint_gradient")
    e = complex(out[0], out[1])
    if return_prods:
        return e, grad, prods[: 2 * n_occ].view(np.complex128)
    return e, grad


def adjoint_gradient_nonhermitian(n, gates, theta, codes, coeffs, psi_in=None):
    """<A> and its complex gradient for A = sum c_t P_t with complex c (App. B.4): Algorithm 1
    with complex entries run with A and with A^dag, combined as conj(g_A) + g_{A^dag}.
    Returns (energy (complex), grad (P,) complex)."""
    c = np.asarray(coeffs, dtype=np.complex128).reshape(-1)
    cre = np.ascontiguousarray(c.real)
    cim = np.ascontiguousarray(c.imag)
    gates, theta, codes, cre, psi_in = _prep(n, gates, theta, codes, cre, psi_in)
    out = np.zeros(2)
    grad = np.zeros(2 * theta.shape[0])
    _check(lib().orc_adjoint_gradient_nonhermitian(
        n, _ptr(psi_in), _ptr(gates), gates.shape[0], _ptr(theta), theta.shape[0],
        codes.shape[0], _ptr(codes), _ptr(cre), _ptr(cim), _ptr(out), _ptr(grad)),
        "adjoint_gradient_nonhermitian")
    return complex(out[0], out[1]), grad.view(np.complex128)


def reference_gradient(n, gates, theta, codes, coeffs, psi_in=None) -> np.ndarray:
    """Algorithm 2 (one re-simulation per parameter occurrence)."""
    gates, theta, codes, coeffs, psi_in = _prep(n, gates, theta, codes, coeffs, psi_in)
    grad = np.zeros(theta.shape[0])
    _check(lib().orc_reference_gradient(n, _ptr(psi_in), _ptr(gates), gates.shape[0],
                                        _ptr(theta), theta.shape[0], codes.shape[0], _ptr(codes),
                                        _ptr(coeffs), _ptr(grad)), "reference_gradient")
    return grad


def parameter_shift(n, gates, theta, codes, coeffs, psi_in=None, entries=None) -> np.ndarray:
    """g_p = [E(theta + (pi/2) e_p) - E(theta - (pi/2) e_p)] / 2, exact when every occurrence of
    p is a rotation exp(-i theta G / 2) about an involutory G (two-eigenvalue generator +-1/2)."""
    theta = np.asarray(theta, dtype=np.float64)
    P = theta.shape[0]
    entries = range(P) if entries is None else entries
    g = np.zeros(P)
    for p in entries:
        tp, tm = theta.copy(), theta.copy()
        tp[p] += math.pi / 2
        tm[p] -= math.pi / 2
        g[p] = 0.5 * (energy(n, gates, tp, codes, coeffs, psi_in).real
                      - energy(n, gates, tm, codes, coeffs, psi_in).real)
    return g


def central_difference(n, gates, theta, codes, coeffs, h=1e-5, psi_in=None,
                       entries=None) -> np.ndarray:
    """[E(theta + h e_p) - E(theta - h e_p)] / (2h): the finite-difference estimate of Sec. 1
    in its central form."""
    theta = np.asarray(theta, dtype=np.float64)
    P = theta.shape[0]
    entries = range(P) if entries is None else entries
    g = np.zeros(P)
    for p in entries:
        tp, tm = theta.copy(), theta.copy()
        tp[p] += h
        tm[p] -= h
        g[p] = (energy(n, gates, tp, codes, coeffs, psi_in).real
                - energy(n, gates, tm, codes, coeffs, psi_in).real) / (2 * h)
    return g
