"""Fusion scheduler (host logic, no GPU): the fused schedule is a valid execution of the circuit.

For every schedule: each gate runs exactly once; the gates on every qubit keep their order
(forward) or reversed order (reverse sweep), up to the order inside runs of consecutive diagonal
gates (they commute; the scheduler merges them into diagonal blocks); each gate's qubits lie in its pass's tile; each
gate's non-diagonal targets are register qubits of its phase; passes and phases appear in
increasing order. Executing the gates in the scheduled order on the CPU oracle gives the same
state as the original order.
"""
import numpy as np
import pytest

from paper_2009_02823_amd import qsv
from paper_2009_02823_amd import workloads as W

DIAG = {W.RZ, W.Z, W.S, W.T, W.SDG, W.PHASE, W.CZ, W.RZZ, W.CRZ}


def reg_need(row):
    k, q0, q1 = int(row[0]), int(row[1]), int(row[2])
    if k in DIAG:
        return 0
    if k in (W.CNOT, W.CRX, W.CRY):
        return 1 << q1
    if k in (W.RXX, W.RYY):
        return (1 << q0) | (1 << q1)
    return 1 << q0


def qubits(row):
    return [int(row[1])] + ([int(row[2])] if W.N_QUBITS[int(row[0])] == 2 else [])


def diagonal_runs_sorted(seq, gates):
    """A qubit's gate sequence with every run of consecutive diagonal gates in sorted order."""
    out, run = [], []
    for k in seq:
        if int(gates[k][0]) in DIAG:
            run.append(k)
            continue
        out += sorted(run) + [k]
        run = []
    return out + sorted(run)


def check_schedule(n, gates, backward, r, w):
    info = qsv.schedule_describe(n, gates, backward, r, w)
    G = gates.shape[0]
    order = info["order"]
    assert sorted(order.tolist()) == list(range(G))
    assert np.all(np.diff(info["pass_of"]) >= 0) and np.all(np.diff(info["phase_of"]) >= 0)
    # per-qubit order
    seq = list(range(G))[::-1] if backward else list(range(G))
    for q in range(n):
        want = [k for k in seq if q in qubits(gates[k])]
        got = [int(k) for k in order if q in qubits(gates[k])]
        assert diagonal_runs_sorted(got, gates) == diagonal_runs_sorted(want, gates), \
            f"qubit {q} order changed"
    t = r + w
    for i, k in enumerate(order):
        tile = int(info["tile_mask"][info["pass_of"][i]])
        # a state smaller than the tile fills it; the other tile bits are phantom
        assert bin(tile).count("1") == min(t, n)
        for q in qubits(gates[k]):
            assert (tile >> q) & 1, "gate outside its pass's tile"
        regm = int(info["reg_mask"][info["phase_of"][i]])
        assert (regm & ~tile) == 0
        assert bin(regm).count("1") == r if t <= n else bin(regm).count("1") <= r
        assert (reg_need(gates[k]) & ~regm) == 0, "non-diagonal target not in registers"
    return info


@pytest.mark.parametrize("n,L,cz", [(10, 4, False), (12, 3, True), (16, 5, False),
                                    (20, 20, False), (26, 30, True), (30, 10, False)])
@pytest.mark.parametrize("backward", [False, True])
@pytest.mark.parametrize("r,w", [(3, 8), (4, 8), (2, 6)])
def test_hea_schedules_valid(n, L, cz, backward, r, w):
    if r + w > n:
        pytest.skip("tile larger than the state")
    gates = W.hea_circuit(n, L, cz_brickwork=cz)
    info = check_schedule(n, gates, backward, r, w)
    # fusion must cut the number of HBM passes well below one per gate
    assert info["n_passes"] < gates.shape[0] / 4


@pytest.mark.parametrize("seed", range(12))
def test_random_schedules_valid_and_equivalent(seed, orc):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(2, 13))
    gates, P = W.random_circuit(rng, n, 150, list(W.GATE_NAMES))
    theta = W.uniform_angles(rng, P)
    r, w = (2, 6) if seed % 2 else (3, 6)
    for backward in (False, True):
        info = check_schedule(n, gates, backward, r, w)
        order = info["order"]
        if backward:
            # the reverse sweep applies U^dag in the scheduled order: compare U^dag... products
            psi0 = orc.statevector(n, gates, theta)
            a = orc.statevector(n, gates, theta, psi_in=psi0, inverse=True)
            b = psi0.copy()
            for k in order:
                b = orc.statevector(n, gates[k:k + 1], theta, psi_in=b, inverse=True)
            assert np.max(np.abs(a - b)) < 1e-12
        else:
            a = orc.statevector(n, gates, theta)
            b = orc.statevector(n, gates[order], theta)
            assert np.max(np.abs(a - b)) < 1e-12


def test_schedule_rejects_bad_geometry():
    gates = W.hea_circuit(8, 1)
    with pytest.raises(qsv.QsvError):
        qsv.schedule_describe(8, gates, False, 0, 6)
    with pytest.raises(qsv.QsvError):
        qsv.schedule_describe(8, gates, False, 6, 8)      # more register bits than supported
    with pytest.raises(qsv.QsvError):
        qsv.schedule_describe(8, gates, False, 5, 10)     # tile of 15 > 14 bits


@pytest.mark.parametrize("n", [1, 2, 3, 5, 8])
def test_tile_larger_than_state(n):
    """A 12-bit tile over a smaller state: one tile, every pass over all qubits."""
    gates = W.hea_circuit(n, 6)
    for backward in (False, True):
        info = check_schedule(n, gates, backward, 4, 8)
        assert np.all(info["tile_mask"][:info["n_passes"]] == (1 << n) - 1)


def test_pass_counts_reported():
    """Pass counts for the measured workloads (printed with -s)."""
    for n, L, cz, r in [(20, 20, False, 3), (26, 30, True, 4), (30, 10, False, 3)]:
        gates = W.hea_circuit(n, L, cz_brickwork=cz)
        f = qsv.schedule_describe(n, gates, False, r, 8)
        b = qsv.schedule_describe(n, gates, True, r, 8)
        print(f"n={n} L={L} G={gates.shape[0]} t={r + 8}: forward {f['n_passes']} passes "
              f"{f['n_phases']} phases, backward {b['n_passes']} passes {b['n_phases']} phases")


def rotation_layer_circuit(rng, n, layers):
    """Per layer: RX, RY and RZ on every qubit in shuffled order with two extra rotations per
    axis, then a CNOT ladder (runs of same-axis rotations that rotation macros regroup)."""
    rows, p = [], 0
    for _ in range(layers):
        for kind in (W.RX, W.RY, W.RZ):
            for q in list(rng.permutation(n)) + list(rng.integers(0, n, size=2)):
                rows.append(W.gate_row(kind, int(q), p0=p))
                p += 1
        rows += [W.gate_row(W.CNOT, q, q + 1) for q in range(n - 1)]
    return W.circuit_table(rows), p


@pytest.mark.parametrize("r,w", [(2, 6), (3, 6), (3, 8), (4, 8)])
def test_rotation_macros_regroup_validly(orc, r, w):
    """Rotation macros move same-axis rotations within a run (they commute): the schedule stays
    valid and equivalent, macros form for every r up to 4."""
    rng = np.random.default_rng(77 + r + w)
    n = 13
    gates, P = rotation_layer_circuit(rng, n, 3)
    theta = W.uniform_angles(rng, P)
    for backward in (False, True):
        info = check_schedule(n, gates, backward, r, w)
        assert info["n_macros"] > 0
        order = info["order"]
        if backward:
            psi0 = orc.statevector(n, gates, theta)
            a = orc.statevector(n, gates, theta, psi_in=psi0, inverse=True)
            b = psi0.copy()
            for k in order:
                b = orc.statevector(n, gates[k:k + 1], theta, psi_in=b, inverse=True)
        else:
            a = orc.statevector(n, gates, theta)
            b = orc.statevector(n, gates[order], theta)
        assert np.max(np.abs(a - b)) < 1e-12


def test_headline_schedule_forms_macros():
    gates = W.hea_circuit(20, 20)
    for backward in (False, True):
        assert qsv.schedule_describe(20, gates, backward, 3, 9)["n_macros"] > 0


def diagonal_layers(rng, n, layers, cz_repeat=1):
    """Per layer: RY on every qubit, RZ on every qubit plus extra RZ on random qubits (runs of
    more than four RZ, some on one qubit twice), then CZ on neighbours (each cz_repeat times:
    runs of CZ alone) and a CZ brickwork, so that diagonal blocks of every size form."""
    rows, p = [], 0
    for _ in range(layers):
        for q in range(n):
            rows.append(W.gate_row(W.RY, q, p0=p))
            p += 1
        for q in list(rng.permutation(n)) + list(rng.integers(0, n, size=3)):
            rows.append(W.gate_row(W.RZ, int(q), p0=p))
            p += 1
        for q in range(n - 1):
            rows += [W.gate_row(W.CZ, q, q + 1)] * cz_repeat
        rows += [W.gate_row(W.CZ, q, q + 2) for q in range(0, n - 2, 2)]
    return W.circuit_table(rows), p



@pytest.mark.parametrize("r,w", [(2, 6), (3, 8), (4, 8), (3, 9)])
@pytest.mark.parametrize("cz_repeat", [1, 13])
def test_diagonal_blocks_form_validly(orc, r, w, cz_repeat):
    """Diagonal blocks reorder commuting diagonal gates only: the schedule stays valid and
    executes to the same state, and blocks form in both sweeps."""
    rng = np.random.default_rng(91 + r + w + cz_repeat)
    n = 13
    gates, P = diagonal_layers(rng, n, 2, cz_repeat)
    theta = W.uniform_angles(rng, P)
    for backward in (False, True):
        info = check_schedule(n, gates, backward, r, w)
        assert info["n_diag_blocks"] > 0
        order = info["order"]
        if backward:
            psi0 = orc.statevector(n, gates, theta)
            a = orc.statevector(n, gates, theta, psi_in=psi0, inverse=True)
            b = psi0.copy()
            for k in order:
                b = orc.statevector(n, gates[k:k + 1], theta, psi_in=b, inverse=True)
        else:
            a = orc.statevector(n, gates, theta)
            b = orc.statevector(n, gates[order], theta)
        assert np.max(np.abs(a - b)) < 1e-12


def test_headline_schedule_forms_diagonal_blocks():
    gates = W.hea_circuit(30, 10)
    for backward in (False, True):
        assert qsv.schedule_describe(30, gates, backward, 4, 8)["n_diag_blocks"] > 0


def test_headline_schedule_folds_register_cnots():
    """The reverse sweep's CNOT ladders open phases entered by a relayout: most of the CNOTs
    with both bits in registers become register permutations of that relayout."""
    gates = W.hea_circuit(30, 10)
    assert qsv.schedule_describe(30, gates, True, 4, 8)["n_folded_cnots"] > 100
