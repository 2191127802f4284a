"""GPU parity on circuits built to exercise rotation macros: layers of RX, RY and RZ on every
qubit (runs of same-axis rotations that cover all register positions of a phase), runs with
leftover rotations, RZ on thread bits inside a run, and repeated parameters. Checked against the
CPU oracle for the Algorithm 1 sweeps in geometries with 2 and 3 register qubits, the
non-Hermitian (complex-entry) sweep, the reference gradient (Algorithm 2) and the batched path.
"""
import numpy as np
import pytest

from paper_2009_02823_amd import workloads as W
from test_schedule_cpu import diagonal_layers

pytestmark = pytest.mark.gpu

GEOMS = {"c128": [(2, 6), (3, 6), (2, 8), (3, 8), (3, 9)],
         "c64": [(2, 6), (3, 6), (2, 8), (3, 8), (3, 9), (4, 9)]}


@pytest.fixture(scope="module")
def Q():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2009_02823_amd import qsv
    qsv.lib()
    return qsv


def rotation_layers(rng, n, layers, n_params=None):
    """Per layer: RX, RY and RZ on every qubit (each axis in a shuffled qubit order), a few
    extra rotations on random qubits (leftovers of a run), then a CNOT ladder."""
    rows = []
    nxt = 0

    def param():
        nonlocal nxt
        if n_params is not None:
            return int(rng.integers(0, n_params))
        nxt += 1
        return nxt - 1

    for _ in range(layers):
        for kind in (W.RX, W.RY, W.RZ):
            for q in rng.permutation(n):
                rows.append(W.gate_row(kind, int(q), p0=param()))
            for q in rng.integers(0, n, size=2):
                rows.append(W.gate_row(kind, int(q), p0=param()))
        rows += [W.gate_row(W.CNOT, q, q + 1) for q in range(n - 1)]
    P = nxt if n_params is None else n_params
    return W.circuit_table(rows), P


def problem(seed, n, layers=3, n_params=None, h=8):
    rng = np.random.default_rng(seed)
    gates, P = rotation_layers(rng, n, layers, n_params)
    theta = W.uniform_angles(rng, P)
    codes = W.random_pauli_strings(rng, n, h)
    coeffs = rng.standard_normal(h)
    return gates, theta, codes, coeffs


def check(dtype, e, g, e_ref, g_ref, coeffs):
    if dtype == "c128":
        assert abs(e - e_ref) <= 1e-10
        assert np.max(np.abs(g - g_ref)) <= 1e-10
    else:
        assert abs(e - e_ref) <= 2e-4 * max(abs(e_ref), 1.0)
        scale = max(np.max(np.abs(g_ref)), 1e-5 * np.abs(coeffs).sum())
        assert np.max(np.abs(g - g_ref)) <= 2e-4 * scale


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("n", [9, 13])
def test_adjoint_every_geometry(Q, orc, dtype, n):
    gates, theta, codes, coeffs = problem(3000 + n, n)
    e_ref, g_ref = orc.adjoint_gradient(n, gates, theta, codes, coeffs)
    for r, w in GEOMS[dtype]:
        with Q.StateVector(n, dtype) as sv:
            sv.set_fusion(1, r, w)
            e, g = sv.adjoint_gradient(gates, theta, codes, coeffs)
            sv.sync()
            check(dtype, float(e.cpu()[0]), g.cpu().numpy(), e_ref.real, g_ref, coeffs)


def test_repeated_parameters(Q, orc):
    n = 12
    gates, theta, codes, coeffs = problem(3100, n, layers=2, n_params=17)
    e_ref, g_ref = orc.adjoint_gradient(n, gates, theta, codes, coeffs)
    for r, w in GEOMS["c128"]:
        with Q.StateVector(n) as sv:
            sv.set_fusion(1, r, w)
            e, g = sv.adjoint_gradient(gates, theta, codes, coeffs)
            sv.sync()
            check("c128", float(e.cpu()[0]), g.cpu().numpy(), e_ref.real, g_ref, coeffs)


@pytest.mark.parametrize("geom", [(2, 8), (3, 8), (3, 9)])
def test_nonhermitian(Q, orc, geom):
    n = 11
    gates, theta, codes, coeffs = problem(3200, n, layers=2)
    c = coeffs + 1j * np.random.default_rng(3201).standard_normal(coeffs.shape[0])
    e_ref, g_ref = orc.adjoint_gradient_nonhermitian(n, gates, theta, codes, c)
    with Q.StateVector(n) as sv:
        sv.set_fusion(1, *geom)
        e, g = sv.adjoint_gradient_nonhermitian(gates, theta, codes, c)
        sv.sync()
        e, g = complex(e.cpu()[0]), g.cpu().numpy()
    assert abs(e - e_ref) <= 1e-10
    assert np.max(np.abs(g - g_ref)) <= 1e-10


@pytest.mark.parametrize("n,geom", [(7, (3, 6)), (12, (3, 8))])
def test_reference_gradient(Q, orc, n, geom):
    gates, theta, codes, coeffs = problem(3300 + n, n, layers=1)
    g_ref = orc.reference_gradient(n, gates, theta, codes, coeffs)
    with Q.StateVector(n) as sv:
        sv.set_fusion(1, *geom)
        e, g = sv.reference_gradient(gates, theta, codes, coeffs)
        sv.sync()
        assert np.max(np.abs(g.cpu().numpy() - g_ref)) <= 1e-10


def test_batched(Q, orc):
    probs = []
    for b, n in enumerate((9, 12, 14)):
        gates, theta, codes, coeffs = problem(3400 + b, n, layers=2)
        probs.append(W.Problem(f"m{b}", n, gates, theta, codes, coeffs))
    batch = Q.Batch(probs, "c128")
    e, g = batch.adjoint_gradient(batch.theta_flat())
    batch.sync()
    e, g = e.cpu().numpy(), g.cpu().numpy()
    for b, p in enumerate(probs):
        e_ref, g_ref = orc.adjoint_gradient(p.n_qubits, p.gates, p.theta, p.codes, p.coeffs)
        gb = g[batch.theta_off[b]: batch.theta_off[b] + p.n_params]
        check("c128", float(e[b]), gb, e_ref.real, g_ref, p.coeffs)


def diag_problem(seed, n, layers=2, cz_repeat=1, h=8):
    rng = np.random.default_rng(seed)
    gates, P = diagonal_layers(rng, n, layers, cz_repeat)
    theta = W.uniform_angles(rng, P)
    codes = W.random_pauli_strings(rng, n, h)
    coeffs = rng.standard_normal(h)
    return gates, theta, codes, coeffs


DIAG_GEOMS = {"c128": [(2, 6), (3, 6), (2, 8), (3, 8), (4, 8), (3, 9)],
              "c64": [(2, 6), (3, 6), (2, 8), (3, 8), (4, 8), (3, 9), (4, 9)]}


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("n,cz_repeat", [(10, 1), (13, 1), (13, 13)])
def test_diagonal_blocks(Q, orc, dtype, n, cz_repeat):
    """RZ and CZ runs on register bits run as diagonal blocks (several RZ per block, blocks of
    CZ alone): both sweeps against the oracle in every geometry."""
    gates, theta, codes, coeffs = diag_problem(3400 + n + cz_repeat, n, cz_repeat=cz_repeat)
    e_ref, g_ref = orc.adjoint_gradient(n, gates, theta, codes, coeffs)
    for r, w in DIAG_GEOMS[dtype]:
        assert Q.schedule_describe(n, gates, True, r, w, dtype)["n_diag_blocks"] > 0
        with Q.StateVector(n, dtype) as sv:
            sv.set_fusion(1, r, w)
            e, g = sv.adjoint_gradient(gates, theta, codes, coeffs)
            sv.sync()
            check(dtype, float(e.cpu()[0]), g.cpu().numpy(), e_ref.real, g_ref, coeffs)


@pytest.mark.parametrize("geom", [(2, 8), (3, 8), (4, 8)])
def test_diagonal_blocks_nonhermitian(Q, orc, geom):
    """Complex gradient entries run a block's members one by one."""
    n = 11
    gates, theta, codes, coeffs = diag_problem(3500, n)
    c = coeffs + 1j * np.random.default_rng(3501).standard_normal(coeffs.shape[0])
    e_ref, g_ref = orc.adjoint_gradient_nonhermitian(n, gates, theta, codes, c)
    with Q.StateVector(n) as sv:
        sv.set_fusion(1, *geom)
        e, g = sv.adjoint_gradient_nonhermitian(gates, theta, codes, c)
        sv.sync()
        e, g = complex(e.cpu()[0]), g.cpu().numpy()
    assert abs(e - e_ref) <= 1e-10
    assert np.max(np.abs(g - g_ref)) <= 1e-10
