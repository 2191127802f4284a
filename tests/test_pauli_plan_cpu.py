"""Host-only checks of how H is applied (qsv_pauli_describe): the X-mask groups, the tiled passes
that apply every group whose X bits lie in their tile, and the groups left to the gather."""
import numpy as np
import pytest

from paper_2009_02823_amd import qsv
from paper_2009_02823_amd import workloads as W


def xmasks(codes):
    return [sum(1 << q for q, c in enumerate(row) if c in (1, 2)) for row in np.asarray(codes)]


CASES = [(2, "c128"), (2, "c64"), (3, "c128"), (3, "c64"), (5, "c128"), (5, "c64")]


@pytest.mark.parametrize("cfg,dtype", CASES)
def test_every_group_once_and_tiles_hold_the_runs(cfg, dtype):
    p = W.CONFIGS[cfg]()
    d = qsv.pauli_describe(p.n_qubits, p.codes, p.coeffs, dtype)
    groups = sorted(set(xmasks(p.codes)))
    assert d["n_groups"] == len(groups)
    assert int(d["pass_groups"].sum()) + d["n_gather_groups"] == d["n_groups"]
    tb = 12 if dtype == "c128" else 13
    runs = 3 if dtype == "c128" or p.n_qubits <= 24 else 4
    for mask, k in zip(d["tile_masks"], d["pass_groups"]):
        mask = int(mask)
        assert bin(mask).count("1") == tb
        assert mask & ((1 << runs) - 1) == (1 << runs) - 1
        assert 3 <= k <= sum(1 for x in groups if x & ~mask == 0)


def test_chain_hamiltonians_need_no_gather():
    """Single-qubit and neighbouring-pair X masks (Ising, transverse-field Ising) fit tiles: at
    30 qubits three passes take all 31 groups, at 20 qubits two take 21."""
    p5, p2 = W.config5(), W.config2()
    d5 = qsv.pauli_describe(30, p5.codes, p5.coeffs, "c128")
    assert (d5["n_tiled_passes"], d5["n_gather_groups"], d5["n_groups"]) == (3, 0, 31)
    d2 = qsv.pauli_describe(20, p2.codes, p2.coeffs, "c128")
    assert (d2["n_tiled_passes"], d2["n_gather_groups"], d2["n_groups"]) == (2, 0, 21)


def test_small_states_gather_only():
    p = W.config1()
    d = qsv.pauli_describe(p.n_qubits, p.codes, p.coeffs, "c128")
    assert d["n_tiled_passes"] == 0 and d["n_gather_groups"] == d["n_groups"]


def test_invalid_sum_rejected():
    with pytest.raises(qsv.QsvError):
        qsv.pauli_describe(4, np.full((1, 4), 7, np.uint8), [1.0])
