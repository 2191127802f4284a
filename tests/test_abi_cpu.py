"""The C-ABI library loads, exports every function ``include/qsv.h`` declares, and validates its
arguments on the host (no GPU, no compute calls)."""
import ctypes
import re
import subprocess

import numpy as np
import pytest

from paper_2009_02823_amd import qsv
from paper_2009_02823_amd import workloads as W


def declared_functions():
    text = open(qsv.HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(qsv_\w+)\s*\(", text)))


def test_header_declares_the_four_calls_of_the_method():
    names = declared_functions()
    for f in ("qsv_create", "qsv_apply_circuit", "qsv_expectation_pauli_sum",
              "qsv_adjoint_gradient"):
        assert f in names


def test_library_exports_every_declared_symbol():
    L = qsv.lib()
    out = subprocess.run(["nm", "-D", "--defined-only", qsv.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (qsv_\w+)", out))
    missing = [f for f in declared_functions() if f not in exported]
    assert not missing, f"declared but not exported: {missing}"
    for f in declared_functions():
        getattr(L, f)   # resolvable through the dynamic loader


def test_sizes():
    assert qsv.state_bytes(10, "c128") == 16 << 10
    assert qsv.state_bytes(10, "c64") == 8 << 10
    assert qsv.workspace_bytes(20, "c128") == 2 * (16 << 20)
    assert qsv.state_bytes(0, "c128") == 0
    assert qsv.state_bytes(35, "c128") == 0
    assert qsv.lib().qsv_state_bytes(10, 7) == 0


def test_valid_inputs_pass():
    p = W.config1()
    qsv.validate_circuit(p.n_qubits, p.gates, p.n_params)
    qsv.validate_pauli_sum(p.n_qubits, p.codes, p.coeffs)
    rng = np.random.default_rng(0)
    g, P = W.random_circuit(rng, 5, 60, kinds=list(W.GATE_NAMES))
    qsv.validate_circuit(5, g, P)
    qsv.validate_circuit(5, np.zeros((0, 6), np.int32), 0)
    qsv.validate_pauli_sum(5, np.zeros((0, 5), np.uint8), np.zeros(0))


BAD_GATES = [
    ("unknown kind", (99, 0, -1, -1, -1, -1)),
    ("negative kind", (-1, 0, -1, -1, -1, -1)),
    ("qubit out of range", (W.RX, 4, -1, 0, -1, -1)),
    ("negative qubit", (W.H, -1, -1, -1, -1, -1)),
    ("q1 on a one-qubit gate", (W.RY, 0, 1, 0, -1, -1)),
    ("two-qubit gate on one qubit", (W.CNOT, 2, 2, -1, -1, -1)),
    ("second qubit out of range", (W.CZ, 0, 4, -1, -1, -1)),
    ("param out of range", (W.RZ, 0, -1, 3, -1, -1)),
    ("missing param", (W.RZ, 0, -1, -1, -1, -1)),
    ("param on a fixed gate", (W.X, 0, -1, 0, -1, -1)),
    ("extra param slot", (W.RX, 0, -1, 0, 1, -1)),
    ("U3 missing third param", (W.U3, 0, -1, 0, 1, -1)),
]


@pytest.mark.parametrize("name,row", BAD_GATES, ids=[b[0] for b in BAD_GATES])
def test_invalid_gate_rejected(name, row):
    good = [(W.H, 0, -1, -1, -1, -1), (W.RY, 1, -1, 0, -1, -1)]
    with pytest.raises(qsv.QsvError) as e:
        qsv.validate_circuit(4, good + [row], 3)
    assert e.value.status == qsv.QSV_ERR_INVALID_ARG
    assert "gate 2" in str(e.value)


def test_invalid_sizes_rejected():
    L = qsv.lib()
    assert L.qsv_validate_circuit(0, None, 0, 0) == qsv.QSV_ERR_INVALID_ARG
    assert L.qsv_validate_circuit(35, None, 0, 0) == qsv.QSV_ERR_INVALID_ARG
    assert L.qsv_validate_circuit(3, None, 2, 0) == qsv.QSV_ERR_INVALID_ARG
    assert L.qsv_validate_circuit(3, None, -1, 0) == qsv.QSV_ERR_INVALID_ARG
    assert L.qsv_validate_pauli_sum(3, None) == qsv.QSV_ERR_INVALID_ARG


def test_invalid_pauli_rejected():
    codes = np.zeros((2, 3), np.uint8)
    codes[1, 2] = 4
    with pytest.raises(qsv.QsvError, match="Pauli code 4 at term 1 qubit 2"):
        qsv.validate_pauli_sum(3, codes, [1.0, 2.0])
    with pytest.raises(qsv.QsvError, match="not finite"):
        qsv.validate_pauli_sum(3, np.zeros((2, 3), np.uint8), [1.0, np.nan])
    with pytest.raises(qsv.QsvError, match="not finite"):
        qsv.validate_pauli_sum(3, np.zeros((1, 3), np.uint8), [np.inf])


def test_create_rejects_bad_arguments_before_touching_the_device():
    L = qsv.lib()
    h = ctypes.c_void_p()
    ws = qsv.workspace_bytes(4, "c128")
    fake = ctypes.c_void_p(1 << 20)  # never dereferenced: validation fails first
    assert L.qsv_create(4, 1, None, fake, ws, None, ctypes.byref(h)) == qsv.QSV_ERR_INVALID_ARG
    assert L.qsv_create(0, 1, fake, fake, ws, None, ctypes.byref(h)) == qsv.QSV_ERR_INVALID_ARG
    assert L.qsv_create(4, 9, fake, fake, ws, None, ctypes.byref(h)) == qsv.QSV_ERR_INVALID_ARG
    assert L.qsv_create(4, 1, fake, fake, ws - 1, None, ctypes.byref(h)) == \
        qsv.QSV_ERR_INVALID_ARG
    assert "workspace" in qsv.last_error()
    assert L.qsv_create(4, 1, ctypes.c_void_p((1 << 20) + 8), fake, ws, None,
                        ctypes.byref(h)) == qsv.QSV_ERR_INVALID_ARG
    assert "aligned" in qsv.last_error()
    assert L.qsv_create(4, 1, fake, fake, ws, None, None) == qsv.QSV_ERR_INVALID_ARG
    assert not h.value
    # calls on a NULL handle are rejected, destroy(NULL) is a no-op
    assert L.qsv_reset(None) == qsv.QSV_ERR_INVALID_ARG
    assert L.qsv_sync(None) == qsv.QSV_ERR_INVALID_ARG
    assert L.qsv_destroy(None) == qsv.QSV_OK


def test_build_id_matches_sources():
    from paper_2009_02823_amd import build as libbuild
    assert qsv.build_id() == libbuild.source_id()


def test_tune_cache_round_trip(tmp_path):
    """Persisted tuning choices: lines tagged with this build's source id are taken, lines of
    other builds, malformed lines and geometries this build lacks are skipped; a save writes
    back what was loaded."""
    sid = qsv.build_id()
    line = ('{{"source": "{s}", "key": "{k}", "n": {n}, "dtype": 1, "mode": {m}, "r": {r}, '
            '"w": {w}, "ms": 12.5}}\n')
    path = tmp_path / "tune.jsonl"
    path.write_text(line.format(s=sid, k="00000000000000aa", n=20, m=1, r=3, w=9)
                    + line.format(s="0123456789abcdef", k="00000000000000bb", n=20, m=1, r=3, w=9)
                    + "not json\n"
                    + line.format(s=sid, k="00000000000000cc", n=20, m=1, r=7, w=9)
                    + line.format(s=sid, k="00000000000000dd", n=12, m=0, r=0, w=0))
    assert qsv.tune_cache_load(str(path)) == 2
    out = tmp_path / "saved.jsonl"
    qsv.tune_cache_save(str(out))
    text = out.read_text()
    assert '"key": "00000000000000aa"' in text and '"key": "00000000000000dd"' in text
    assert "00000000000000bb" not in text and "00000000000000cc" not in text
    assert all(f'"source": "{sid}"' in ln for ln in text.splitlines())
    assert qsv.tune_cache_load(str(tmp_path / "absent.jsonl")) == 0


def test_debug_fail_launch_rejects_negative():
    with pytest.raises(qsv.QsvError):
        qsv.debug_fail_launch(-1)
    qsv.debug_fail_launch(0)


@pytest.mark.parametrize("name", ["qsv_adjoint_gradient_batched", "qsv_reference_gradient_batched"])
def test_batched_entry_points_reject_bad_batches(name):
    """Both batched entry points check the batch size and their host arrays before touching any
    handle or device memory."""
    fn = getattr(qsv.lib(), name)
    z = ctypes.c_void_p(0)
    one = (ctypes.c_int32 * 1)(1)
    off = (ctypes.c_int64 * 1)(0)
    for n_batch in (0, -3):
        assert fn(n_batch, z, z, z, z, z, z, z, z, z) == qsv.QSV_ERR_INVALID_ARG
    # NULL states / gates / counts
    assert fn(1, z, z, one, z, off, one, z, z, z) == qsv.QSV_ERR_INVALID_ARG
    assert "NULL" in qsv.lib().qsv_last_error().decode()
