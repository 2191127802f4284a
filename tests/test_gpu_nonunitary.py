"""GPU gradients through non-unitary gates (App. B.3) against the CPU oracle.

Mixed circuits of unitary gates and imaginary-time rotations NRX/NRY/NRZ: the fused passes in
several geometries (phi un-done by the stored inverse, lambda by the adjoint), the gate-granular
kernels, the reference gradient (Algorithm 2), a non-Hermitian operator, and the rejection by the
parameter-shift entry point.
"""
import math

import numpy as np
import pytest

from paper_2009_02823_amd import workloads as W

pytestmark = pytest.mark.gpu
MIXED = list(W.GATE_NAMES) + list(W.NONUNITARY_NAMES)


@pytest.fixture(scope="module")
def Q():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2009_02823_amd import qsv
    qsv.lib()
    return qsv


def problem(seed, n, n_gates=100, h=6):
    rng = np.random.default_rng(seed)
    gates, P = W.random_circuit(rng, n, n_gates, MIXED)
    theta = rng.uniform(-0.6, 0.6, P)  # the non-unitary factors stay moderate
    codes = W.random_pauli_strings(rng, n, h)
    coeffs = rng.standard_normal(h)
    return gates, theta, codes, coeffs


def check(dtype, e, g, e_ref, g_ref):
    scale = max(1.0, abs(e_ref), float(np.max(np.abs(g_ref))))
    tol = 1e-10 if dtype == "c128" else 2e-4
    assert abs(e - e_ref) <= tol * scale
    assert np.max(np.abs(g - g_ref)) <= tol * scale


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("n,geom", [(4, None), (10, (3, 8)), (13, (3, 8)), (11, (2, 6)),
                                    (12, (0, 0))])
def test_adjoint_mixed_circuits(Q, orc, dtype, n, geom):
    gates, theta, codes, coeffs = problem(1000 + n, n)
    e_ref, g_ref = orc.adjoint_gradient(n, gates, theta, codes, coeffs)
    with Q.StateVector(n, dtype) as sv:
        if geom == (0, 0):
            sv.set_fusion(0)                 # gate-granular kernels
        elif geom is not None:
            sv.set_fusion(1, *geom)
        e, g = sv.adjoint_gradient(gates, theta, codes, coeffs)
        sv.sync()
        check(dtype, float(e.cpu()[0]), g.cpu().numpy(), e_ref.real, g_ref)


def test_closed_form_norm(Q):
    """exp(-t Y/2)|0> has norm^2 cosh t: <1> = cosh t, derivative sinh t."""
    gates = W.circuit_table([W.gate_row(W.NRY, 0, p0=0)])
    codes = np.zeros((1, 1), dtype=np.uint8)
    for t in (0.4, -1.2):
        with Q.StateVector(1) as sv:
            e, g = sv.adjoint_gradient(gates, np.array([t]), codes, np.array([1.0]))
            sv.sync()
            assert abs(float(e.cpu()[0]) - math.cosh(t)) < 1e-14
            assert abs(float(g.cpu()[0]) - math.sinh(t)) < 1e-14


@pytest.mark.parametrize("n", [5, 9])
def test_reference_gradient(Q, orc, n):
    gates, theta, codes, coeffs = problem(1100 + n, n, 70)
    g_ref = orc.reference_gradient(n, gates, theta, codes, coeffs)
    with Q.StateVector(n) as sv:
        e, g = sv.reference_gradient(gates, theta, codes, coeffs)
        sv.sync()
        assert np.max(np.abs(g.cpu().numpy() - g_ref)) <= 1e-10 * max(1.0, np.max(np.abs(g_ref)))


def test_nonhermitian_through_nonunitary(Q, orc):
    n = 9
    gates, theta, codes, coeffs = problem(1200, n, 80)
    c = coeffs + 1j * np.random.default_rng(1201).standard_normal(coeffs.shape[0])
    e_ref, g_ref = orc.adjoint_gradient_nonhermitian(n, gates, theta, codes, c)
    with Q.StateVector(n) as sv:
        e, g = sv.adjoint_gradient_nonhermitian(gates, theta, codes, c)
        sv.sync()
        e, g = complex(e.cpu()[0]), g.cpu().numpy()
    scale = max(1.0, abs(e_ref), float(np.max(np.abs(g_ref))))
    assert abs(e - e_ref) <= 1e-10 * scale
    assert np.max(np.abs(g - g_ref)) <= 1e-10 * scale


def test_parameter_shift_rejects_nonunitary(Q):
    gates = W.circuit_table([W.gate_row(W.NRX, 0, p0=0)])
    codes = np.array([[W.PAULI_Z]], dtype=np.uint8)
    with Q.StateVector(1) as sv:
        with pytest.raises(Q.QsvError):
            sv.param_shift_gradient(gates, np.array([0.3]), codes, np.array([1.0]))
