"""GPU gradients of non-Hermitian operators (App. B.4) against the CPU oracle.

Complex entries <lambda|mu> from both the lean rotation products and the general derivative
matrices, two sweeps (A and A^dag), single-tile and multi-tile states, both storage types.
"""
import math

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


def run(Q, n, gates, theta, codes, coeffs, dtype="c128", geom=None):
    with Q.StateVector(n, dtype) as sv:
        if geom is not None:
            sv.set_fusion(1, *geom)
        e, g = sv.adjoint_gradient_nonhermitian(gates, theta, codes, coeffs)
        sv.sync()
        return complex(e.cpu()[0]), g.cpu().numpy()


def test_worked_example(Q):
    """RX(t)|0> under |0><1| = (X + iY)/2: <A> = -(i/2) sin t, d<A>/dt = -(i/2) cos t."""
    codes = np.array([[W.PAULI_X], [W.PAULI_Y]], dtype=np.uint8)
    gates = W.circuit_table([W.gate_row(W.RX, 0, p0=0)])
    for t in (0.2, 1.1, 2.9):
        e, g = run(Q, 1, gates, np.array([t]), codes, np.array([0.5, 0.5j]))
        assert abs(e - (-0.5j * math.sin(t))) < 1e-14
        assert abs(g[0] - (-0.5j * math.cos(t))) < 1e-14


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("n,geom", [(3, None), (9, (3, 8)), (13, (3, 8)), (12, (2, 6))])
def test_random_circuits(Q, orc, dtype, n, geom):
    rng = np.random.default_rng(900 + n)
    gates, P = W.random_circuit(rng, n, 120, ALL_KINDS, n_params=None if n != 9 else 30)
    theta = W.uniform_angles(rng, P)
    codes = W.random_pauli_strings(rng, n, 7)
    c = rng.standard_normal(7) + 1j * rng.standard_normal(7)
    e_ref, g_ref = orc.adjoint_gradient_nonhermitian(n, gates, theta, codes, c)
    e, g = run(Q, n, gates, theta, codes, c, dtype, geom)
    if dtype == "c128":
        assert abs(e - e_ref) <= 1e-10
        assert np.max(np.abs(g - g_ref)) <= 1e-10
    else:
        assert abs(e - e_ref) <= 2e-4 * max(abs(e_ref), 1.0)
        scale = max(np.max(np.abs(g_ref)), 1e-5 * np.abs(c).sum())
        assert np.max(np.abs(g - g_ref)) <= 2e-4 * scale


def test_hermitian_weights_match_adjoint(Q):
    p = W.config2(n=14, layers=4)
    with Q.StateVector(p.n_qubits) as sv:
        e1, g1 = sv.adjoint_gradient(p.gates, p.theta, p.codes, p.coeffs)
        e2, g2 = sv.adjoint_gradient_nonhermitian(p.gates, p.theta, p.codes,
                                                  p.coeffs.astype(np.complex128))
        sv.sync()
        g1, g2 = g1.cpu().numpy(), g2.cpu().numpy()
        assert abs(complex(e2.cpu()[0]) - float(e1.cpu()[0])) < 1e-13
    assert np.max(np.abs(g2.real - g1)) < 1e-13
    assert np.max(np.abs(g2.imag)) < 1e-13
