"""The allocation-free expectation (qsv_expectation_pauli_sum_noalloc) against the cached entry
point (qsv_expectation_pauli_sum) through the C-ABI: two calls in a row on one GPU, the second
with a smaller input (fewer qubits and terms), in both storage types; and its size limit."""
import numpy as np
import pytest

from paper_2009_02823_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def Q():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2009_02823_amd import qsv
    qsv.lib()
    return qsv


def prepared(Q, n, dtype, seed):
    rng = np.random.default_rng(seed)
    gates, P = W.random_circuit(rng, n, 8 * n, list(W.GATE_NAMES))
    sv = Q.StateVector(n, dtype)
    sv.apply_circuit(gates, W.uniform_angles(rng, P))
    return sv, rng


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_two_calls_second_smaller(Q, dtype):
    import torch
    for n, terms, seed in ((16, 48, 1), (9, 7, 2)):
        sv, rng = prepared(Q, n, dtype, seed)
        codes = W.random_pauli_strings(rng, n, terms)
        coeffs = rng.standard_normal(terms)
        ref = sv.expectation(codes, coeffs)
        out = torch.full((1,), 7.0, dtype=torch.float64, device=sv.device)
        sv.expectation_noalloc(codes, coeffs, out)
        sv.sync()
        e_ref, e = float(ref.cpu()[0]), float(out.cpu()[0])
        sv.close()
        if dtype == "c128":
            assert abs(e - e_ref) <= 1e-10, (n, e, e_ref)
        else:
            assert abs(e - e_ref) <= 2e-4 * max(abs(e_ref), 1.0), (n, e, e_ref)


def test_no_terms_and_limits(Q):
    import torch
    sv, rng = prepared(Q, 6, "c128", 3)
    out = torch.full((1,), 7.0, dtype=torch.float64, device=sv.device)
    sv.expectation_noalloc(np.zeros((0, 6), np.uint8), np.zeros(0), out)
    sv.sync()
    assert float(out.cpu()[0]) == 0.0
    out.fill_(7.0)
    codes = np.ones((16385, 6), np.uint8)
    with pytest.raises(Q.QsvError) as e:
        sv.expectation_noalloc(codes, np.ones(16385), out)
    assert e.value.status == Q.QSV_ERR_INVALID_ARG and "16384" in str(e.value)
    sv.sync()
    assert float(out.cpu()[0]) == 7.0
    sv.close()
