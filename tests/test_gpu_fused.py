"""GPU parity of the fused pass kernels in every tile geometry, against the CPU oracle.

Covers: every gate kind in random order (so passes mix dense, diagonal, controlled and two-qubit
ops on register and thread bits), a single tile (no outer qubits), more tiles than workgroups
(grid-stride over tiles), register phases that change layout, and agreement between the fused
and the gate-granular paths.
"""
import numpy as np
import pytest

from paper_2009_02823_amd import workloads as W

pytestmark = pytest.mark.gpu

GEOMS = {"c128": [(2, 8), (3, 8), (4, 8), (2, 9), (3, 9), (2, 6), (3, 6)],
         "c64": [(2, 8), (3, 8), (4, 8), (2, 9), (3, 9), (4, 9), (2, 6), (3, 6)]}
ALL_KINDS = list(W.GATE_NAMES)


@pytest.fixture(scope="module")
def Q():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2009_02823_amd import qsv
    qsv.lib()
    return qsv


def run(Q, n, gates, theta, codes, coeffs, dtype, geom):
    with Q.StateVector(n, dtype) as sv:
        if geom is None:
            sv.set_fusion(0)
        else:
            sv.set_fusion(1, *geom)
        e, g = sv.adjoint_gradient(gates, theta, codes, coeffs)
        sv.reset()
        sv.apply_circuit(gates, theta)
        sv.sync()
        return float(e.cpu()[0]), g.cpu().numpy(), sv.state.cpu().numpy().astype(np.complex128)


def tol_check(dtype, e, g, psi, e_ref, g_ref, psi_ref, coeffs):
    if dtype == "c128":
        assert abs(e - e_ref.real) <= 1e-10
        assert np.max(np.abs(g - g_ref)) <= 1e-10
        assert np.max(np.abs(psi - psi_ref)) <= 1e-12
    else:
        assert abs(e - e_ref.real) <= 2e-4 * max(abs(e_ref), 1.0)
        scale = max(np.max(np.abs(g_ref)), 1e-5 * np.abs(coeffs).sum())
        assert np.max(np.abs(g - g_ref)) <= 2e-4 * scale
        assert np.max(np.abs(psi - psi_ref)) <= 2e-5


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("seed", range(3))
def test_random_circuits_every_geometry(Q, orc, dtype, seed):
    rng = np.random.default_rng(2000 + seed)
    for r, w in GEOMS[dtype]:
        n = r + w + int(rng.integers(0, 3))      # single tile up to 4 tiles
        gates, P = W.random_circuit(rng, n, 160, ALL_KINDS, n_params=None if seed != 1 else 40)
        theta = W.uniform_angles(rng, P)
        codes = W.random_pauli_strings(rng, n, 9)
        coeffs = rng.standard_normal(9)
        e_ref, g_ref = orc.adjoint_gradient(n, gates, theta, codes, coeffs)
        psi_ref = orc.statevector(n, gates, theta)
        e, g, psi = run(Q, n, gates, theta, codes, coeffs, dtype, (r, w))
        tol_check(dtype, e, g, psi, e_ref, g_ref, psi_ref, coeffs)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_hea_many_tiles(Q, orc, dtype):
    """16 qubits with 10/11-qubit tiles: 32..64 tiles, CZ brickwork, random Pauli strings."""
    n = 16
    rng = np.random.default_rng(9)
    gates = W.hea_circuit(n, 6, cz_brickwork=True)
    theta = W.uniform_angles(rng, 12 * n)
    codes = W.random_weight_pauli_strings(rng, n, 30)
    coeffs = rng.standard_normal(30)
    e_ref, g_ref = orc.adjoint_gradient(n, gates, theta, codes, coeffs)
    psi_ref = orc.statevector(n, gates, theta)
    for geom in GEOMS[dtype]:
        e, g, psi = run(Q, n, gates, theta, codes, coeffs, dtype, geom)
        tol_check(dtype, e, g, psi, e_ref, g_ref, psi_ref, coeffs)


def test_fused_matches_gate_granular(Q):
    p = W.config2(n=18, layers=8)
    e0, g0, s0 = run(Q, p.n_qubits, p.gates, p.theta, p.codes, p.coeffs, "c128", None)
    e1, g1, s1 = run(Q, p.n_qubits, p.gates, p.theta, p.codes, p.coeffs, "c128", (3, 8))
    assert abs(e0 - e1) < 1e-13 and np.max(np.abs(g0 - g1)) < 1e-13
    assert np.max(np.abs(s0 - s1)) < 1e-13


def test_more_tiles_than_workgroups(Q):
    """22 qubits, 11-qubit tiles: 2048 tiles over at most 1024 workgroups; closed form."""
    import test_oracle_pins as pins
    n = 22
    gates, theta, codes, coeffs, E, G = pins.tfim_product_layer(n, np.random.default_rng(1))
    with Q.StateVector(n) as sv:
        sv.set_fusion(1, 3, 8)
        e, g = sv.adjoint_gradient(gates, theta, codes, coeffs)
        sv.sync()
    assert abs(float(e.cpu()[0]) - E) < 1e-11
    assert np.max(np.abs(g.cpu().numpy() - G)) < 1e-11


def test_fused_deterministic(Q):
    p = W.config2(n=16, layers=6)
    outs = [run(Q, p.n_qubits, p.gates, p.theta, p.codes, p.coeffs, "c128", (3, 8))[:2]
            for _ in range(3)]
    for e, g in outs[1:]:
        assert e == outs[0][0] and np.array_equal(g, outs[0][1])


def test_set_fusion_validation(Q):
    with Q.StateVector(9) as sv:
        sv.set_fusion(1, 3, 8)          # an 11-qubit tile over 9 qubits: 2 phantom tile bits
        assert sv.get_fusion() == (1, 3, 8)
        with pytest.raises(Q.QsvError):
            sv.set_fusion(1, 7, 8)      # no kernel for 7 register qubits
        sv.set_fusion(1, 3, 6)
        assert sv.get_fusion() == (1, 3, 6)
        sv.set_fusion(0)
        assert sv.get_fusion()[0] == 0


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("n", [1, 2, 3, 5, 7, 9])
def test_states_smaller_than_the_tile(Q, orc, dtype, n):
    """Phantom tile bits: every gate kind on states of 1..9 qubits inside one 8- to 12-bit tile;
    all passes of a sweep run in one launch."""
    rng = np.random.default_rng(300 + n)
    kinds = [k for k in ALL_KINDS if n >= 2 or W.N_QUBITS[k] == 1]
    gates, P = W.random_circuit(rng, n, 120, kinds)
    theta = W.uniform_angles(rng, P)
    codes = W.random_pauli_strings(rng, n, 5)
    coeffs = rng.standard_normal(5)
    e_ref, g_ref = orc.adjoint_gradient(n, gates, theta, codes, coeffs)
    psi_ref = orc.statevector(n, gates, theta)
    geoms = [(2, 6), (3, 8)] + ([(4, 9)] if dtype == "c64" else [(3, 9)])
    for geom in geoms:
        e, g, psi = run(Q, n, gates, theta, codes, coeffs, dtype, geom)
        tol_check(dtype, e, g, psi, e_ref, g_ref, psi_ref, coeffs)
    with Q.StateVector(n, dtype) as sv:       # the automatic mode: one wave up to 6 qubits
        assert sv.get_fusion()[0] == (2 if n <= 6 else 1)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("n", [1, 2, 4, 5, 6])
def test_one_wave_sweep(Q, orc, dtype, n):
    """Algorithm 1 in one wave (states of up to 6 qubits): every gate kind, repeated parameters,
    a prepared input state, against the oracle; the automatic mode takes this path."""
    rng = np.random.default_rng(500 + n)
    kinds = [k for k in ALL_KINDS if n >= 2 or W.N_QUBITS[k] == 1]
    gates, P = W.random_circuit(rng, n, 150, kinds, n_params=40)
    theta = W.uniform_angles(rng, P)
    prep, Pp = W.random_circuit(rng, n, 20, [W.RY, W.RX, W.CNOT] if n >= 2 else [W.RY, W.RX])
    theta_p = W.uniform_angles(rng, Pp)
    codes = W.random_pauli_strings(rng, n, 6)
    coeffs = rng.standard_normal(6)
    psi_in = orc.statevector(n, prep, theta_p)
    e_ref, g_ref = orc.adjoint_gradient(n, gates, theta, codes, coeffs, psi_in=psi_in)
    for mode in (2, -1):
        with Q.StateVector(n, dtype) as sv:
            sv.set_fusion(mode)
            sv.apply_circuit(prep, theta_p)
            e, g = sv.adjoint_gradient(gates, theta, codes, coeffs)
            sv.sync()
            assert sv.get_fusion() == (2, 0, 0)
            e, g = float(e.cpu()[0]), g.cpu().numpy()
        if dtype == "c128":
            assert abs(e - e_ref.real) <= 1e-10 and np.max(np.abs(g - g_ref)) <= 1e-10
        else:
            assert abs(e - e_ref.real) <= 2e-4 * max(abs(e_ref), 1.0)
            assert np.max(np.abs(g - g_ref)) <= 2e-4 * max(np.max(np.abs(g_ref)),
                                                         1e-5 * np.abs(coeffs).sum())


def test_one_wave_mode_needs_a_small_state(Q):
    with Q.StateVector(7) as sv:
        with pytest.raises(Q.QsvError):
            sv.set_fusion(2)


UNITARY_KINDS = [k for k in ALL_KINDS if k not in (W.NRX, W.NRY, W.NRZ)]
assert set(UNITARY_KINDS) == set(ALL_KINDS)  # the named kinds are the unitary ones


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("n", [1, 2, 3, 4, 5])
def test_chunked_sweep(Q, orc, dtype, n):
    """The chunked one-wave sweep (mode 3): chunk operators, boundary states carried by them, and
    the per-chunk steps; every unitary kind, repeated parameters, a prepared input state, gate
    counts of one partial chunk up to many chunks; the automatic mode takes it for long circuits
    and gives the same result; repeated calls and graph replays re-arm the finish counter."""
    import torch
    rng = np.random.default_rng(700 + n)
    kinds = [k for k in UNITARY_KINDS if n >= 2 or W.N_QUBITS[k] == 1]
    prep, Pp = W.random_circuit(rng, n, 20, [W.RY, W.RX, W.CNOT] if n >= 2 else [W.RY, W.RX])
    theta_p = W.uniform_angles(rng, Pp)
    psi_in = orc.statevector(n, prep, theta_p)
    for G in (1, 64, 65, 300):
        gates, P = W.random_circuit(rng, n, G, kinds, n_params=max(3, G // 3))
        theta = W.uniform_angles(rng, P)
        codes = W.random_pauli_strings(rng, n, 6)
        coeffs = rng.standard_normal(6)
        e_ref, g_ref = orc.adjoint_gradient(n, gates, theta, codes, coeffs, psi_in=psi_in)
        results = []
        for mode, graphs in ((3, False), (3, True), (-1, False)):
            with Q.StateVector(n, dtype) as sv:
                sv.set_fusion(mode)
                sv.set_graphs(graphs)
                sv.apply_circuit(prep, theta_p)
                th = torch.as_tensor(theta, device="cuda:0")
                for rep in range(3):
                    e, g = sv.adjoint_gradient(gates, th, codes, coeffs)
                    sv.sync()
                    e, g = float(e.cpu()[0]), g.cpu().numpy()
                    if dtype == "c128":
                        assert abs(e - e_ref.real) <= 1e-10, (G, mode, rep)
                        assert np.max(np.abs(g - g_ref)) <= 1e-10, (G, mode, rep)
                    else:
                        assert abs(e - e_ref.real) <= 2e-4 * max(abs(e_ref), 1.0)
                        assert np.max(np.abs(g - g_ref)) <= 2e-4 * max(
                            np.max(np.abs(g_ref)), 1e-5 * np.abs(coeffs).sum())
                    results.append((e, g))
        if G >= 96:  # the automatic mode ran the chunked kernels too
            assert results[-1][0] == results[0][0] and np.array_equal(results[-1][1], results[0][1])


def test_chunked_mode_limits(Q, orc):
    """Mode 3 needs at most 5 qubits; a circuit with a non-unitary gate runs the plain one-wave
    sweep under mode 3 (phi cannot be carried back by W_c^dag)."""
    with Q.StateVector(6) as sv:
        with pytest.raises(Q.QsvError):
            sv.set_fusion(3)
    rng = np.random.default_rng(9)
    n = 4
    gates, P = W.random_circuit(rng, n, 250, ALL_KINDS)
    rot = [i for i in range(len(gates)) if int(gates[i, 0]) in (W.RX, W.RY, W.RZ)]
    for i in rot[::len(rot) // 4][:4]:  # four rotations become their non-unitary variants
        gates[i, 0] = {W.RX: W.NRX, W.RY: W.NRY, W.RZ: W.NRZ}[int(gates[i, 0])]
    theta = W.uniform_angles(rng, P)
    codes = W.random_pauli_strings(rng, n, 5)
    coeffs = rng.standard_normal(5)
    e_ref, g_ref = orc.adjoint_gradient(n, gates, theta, codes, coeffs)
    with Q.StateVector(n) as sv:
        sv.set_fusion(3)
        assert sv.get_fusion() == (3, 0, 0)
        e, g = sv.adjoint_gradient(gates, theta, codes, coeffs)
        sv.sync()
        scale = max(1.0, abs(e_ref), float(np.max(np.abs(g_ref))))  # the norm is not kept
        assert abs(float(e.cpu()[0]) - e_ref.real) <= 1e-10 * scale
        assert np.max(np.abs(g.cpu().numpy() - g_ref)) <= 1e-10 * scale
