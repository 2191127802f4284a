"""hipGraph capture/replay and the autotuner.

Every replay of a captured graph is checked against an eager run, with the program's own eager
work and synchronisations between replays, and with theta changed in place (the graph reads it
from device memory)."""
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


@pytest.mark.parametrize("dtype,geom", [("c128", (3, 8)), ("c64", (3, 8)), ("c128", None)])
def test_graph_replays_match_eager(Q, dtype, geom):
    import torch
    p = W.config2(n=14, layers=5)
    rng = np.random.default_rng(4)
    thetas = [W.uniform_angles(rng, p.n_params) for _ in range(4)]
    # eager references
    with Q.StateVector(p.n_qubits, dtype) as ref:
        if geom is None:
            ref.set_fusion(0)
        else:
            ref.set_fusion(1, *geom)
        want = []
        for th in thetas:
            e, g = ref.adjoint_gradient(p.gates, th, p.codes, p.coeffs)
            ref.sync()
            want.append((e.cpu().clone(), g.cpu().clone()))
    with Q.StateVector(p.n_qubits, dtype) as sv:
        if geom is None:
            sv.set_fusion(0)
        else:
            sv.set_fusion(1, *geom)
        sv.set_graphs(True)
        theta = torch.empty(p.n_params, dtype=torch.float64, device=sv.device)
        e = torch.empty(1, dtype=torch.float64, device=sv.device)
        g = torch.empty(p.n_params, dtype=torch.float64, device=sv.device)
        for rep in range(3):          # eager, capture, replay, replay ...
            for k, th in enumerate(thetas):
                theta.copy_(torch.as_tensor(th, device=sv.device))
                sv.adjoint_gradient(p.gates, theta, p.codes, p.coeffs, e, g)
                sv.sync()
                junk = torch.randn(1 << 16, device=sv.device).sum()   # unrelated eager work
                torch.cuda.synchronize()
                del junk
                assert torch.equal(e.cpu(), want[k][0]) and torch.equal(g.cpu(), want[k][1]), \
                    (rep, k)
        sv.set_graphs(False)


def test_graph_batched(Q):
    import torch
    probs = W.config4(batch=24)
    batch = Q.Batch(probs)
    th = batch.theta_flat()
    e0, g0 = batch.adjoint_gradient(th)
    batch.sync()
    e0, g0 = e0.cpu().clone(), g0.cpu().clone()
    batch.set_graphs(True)
    e = torch.empty(len(probs), dtype=torch.float64, device=batch.device)
    g = torch.empty(batch.n_params, dtype=torch.float64, device=batch.device)
    for _ in range(4):
        e.zero_()
        g.zero_()
        batch.adjoint_gradient(th, e, g)
        batch.sync()
        assert torch.equal(e.cpu(), e0) and torch.equal(g.cpu(), g0)
    batch.set_graphs(False)
    batch.close()


def test_autotune_picks_a_valid_mode_and_caches(Q, orc):
    p = W.config2(n=16, layers=4)
    with Q.StateVector(p.n_qubits) as sv:
        mode, r, w, ms = sv.autotune(p.gates, p.theta, p.codes, p.coeffs, repeats=2)
        assert mode in (0, 1) and ms > 0
        assert sv.get_fusion() == ((mode, r, w) if mode else (0, 0, 0))
        e, g = sv.adjoint_gradient(p.gates, p.theta, p.codes, p.coeffs)
        sv.sync()
    e_ref, g_ref = orc.adjoint_gradient(p.n_qubits, p.gates, p.theta, p.codes, p.coeffs)
    assert np.max(np.abs(g.cpu().numpy() - g_ref)) < 1e-10
    with Q.StateVector(p.n_qubits) as sv2:   # same structure: cached choice, no timing
        m2, r2, w2, ms2 = sv2.autotune(p.gates, p.theta * 0.5, p.codes, p.coeffs)
        assert (m2, r2, w2) == (mode, r, w) and ms2 == ms   # the time the choice was made with
