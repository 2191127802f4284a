"""Batched reverse-mode gradients (one launch per pass level over all circuits) and the autograd
layer, against the CPU oracle."""
import os
import sys

import numpy as np
import pytest

from paper_2009_02823_amd import workloads as W

pytestmark = pytest.mark.gpu

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))


@pytest.fixture(scope="module")
def Q():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2009_02823_amd import qsv
    qsv.lib()
    return qsv


def small_batch(seed, B=7):
    rng = np.random.default_rng(seed)
    probs = []
    for b in range(B):
        n = int(rng.integers(11, 15))
        if b % 2:
            L = int(rng.integers(2, 5))
            gates = W.hea_circuit(n, L, cz_brickwork=bool(b % 3 == 0))
            P = 2 * n * L
            codes, coeffs = W.heisenberg_chain(n)
        else:
            gates, P = W.random_circuit(rng, n, 60, list(W.GATE_NAMES))
            codes = W.random_pauli_strings(rng, n, 6)
            coeffs = rng.standard_normal(6)
        theta = W.uniform_angles(rng, P)
        probs.append(W.Problem(f"b{b}", n, gates, theta, codes, coeffs))
    return probs


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_batch_vs_oracle(Q, orc, dtype):
    probs = small_batch(3)
    batch = Q.Batch(probs, dtype)
    e, g = batch.adjoint_gradient(batch.theta_flat())
    batch.sync()
    e = e.cpu().numpy()
    g = g.cpu().numpy()
    for b, p in enumerate(probs):
        e_ref, g_ref = orc.adjoint_gradient(p.n_qubits, p.gates, p.theta, p.codes, p.coeffs)
        gb = g[batch.theta_off[b]: batch.theta_off[b] + p.n_params]
        if dtype == "c128":
            assert abs(e[b] - e_ref.real) <= 1e-10
            assert np.max(np.abs(gb - g_ref)) <= 1e-10
        else:
            assert abs(e[b] - e_ref.real) < 2e-4 * max(abs(e_ref), 1)
            scale = max(np.max(np.abs(g_ref)), 1e-5 * np.abs(p.coeffs).sum())
            assert np.max(np.abs(gb - g_ref)) < 2e-4 * scale
    batch.close()


def test_batch_equals_single_calls_and_repeats(Q):
    import torch
    probs = small_batch(5, B=5)
    batch = Q.Batch(probs)
    th = batch.theta_flat()
    e1, g1 = batch.adjoint_gradient(th)
    e2, g2 = batch.adjoint_gradient(th)
    batch.sync()
    assert torch.equal(e1, e2) and torch.equal(g1, g2)
    for b, p in enumerate(probs):
        with Q.StateVector(p.n_qubits) as sv:
            e, g = sv.adjoint_gradient(p.gates, p.theta, p.codes, p.coeffs)
            sv.sync()
        o = batch.theta_off[b]
        assert abs(float(e.cpu()[0]) - float(e1[b].cpu())) < 1e-13
        assert float((g - g1[o:o + p.n_params]).abs().max()) < 1e-13
    batch.close()


def test_config4_batch_every_circuit_vs_oracle(Q):
    """The 512-circuit batch (12..18 qubits, 5..15 layers, Heisenberg chains): every circuit's
    energy and every gradient entry against the oracle's stored values, 1e-10 absolute."""
    import make_golden
    ref = make_golden.read_batch()
    if ref is None:
        pytest.skip("batch golden not written (tests/golden/make_golden.py 4)")
    e_ref, g_ref = ref
    probs = W.config4()
    assert len(probs) == len(e_ref)
    batch = Q.Batch(probs)
    e, g = batch.adjoint_gradient(batch.theta_flat())
    batch.sync()
    e = e.cpu().numpy()
    g = g.cpu().numpy()
    batch.close()
    de = np.abs(e - e_ref)
    dg = np.array([np.max(np.abs(g[batch.theta_off[b]: batch.theta_off[b] + p.n_params]
                                 - g_ref[b])) for b, p in enumerate(probs)])
    print(f"512 circuits: max|dE| {de.max():.2e}, max|dg| {dg.max():.2e}", flush=True)
    assert de.max() <= 1e-10, int(np.argmax(de))
    assert dg.max() <= 1e-10, int(np.argmax(dg))


def test_autograd_energy_and_gradcheck(Q, orc):
    import torch
    from paper_2009_02823_amd.autograd import AdjointEnergy
    n = 6
    rng = np.random.default_rng(2)
    gates = W.hea_circuit(n, 2)
    theta0 = W.uniform_angles(rng, 4 * n)
    codes = W.random_pauli_strings(rng, n, 8)
    coeffs = rng.standard_normal(8)
    f = AdjointEnergy(n, gates, codes, coeffs, device="cuda:0")
    theta = torch.tensor(theta0, dtype=torch.float64, device="cuda:0", requires_grad=True)
    e = f(theta)
    e.backward()
    e_ref, g_ref = orc.adjoint_gradient(n, gates, theta0, codes, coeffs)
    assert abs(float(e.detach()) - e_ref.real) < 1e-12
    assert float((theta.grad.cpu() - torch.tensor(g_ref)).abs().max()) < 1e-12
    # no-grad path computes E alone
    with torch.no_grad():
        assert abs(float(f(theta.detach())) - e_ref.real) < 1e-12
    # finite differences of the forward against backward
    th = torch.tensor(theta0[: 4 * n], dtype=torch.float64, device="cuda:0", requires_grad=True)
    assert torch.autograd.gradcheck(lambda t: f(t), (th,), eps=1e-6, atol=1e-7, rtol=1e-5)
    # chain rule through a scalar function of E
    theta.grad = None
    (3.0 * f(theta) ** 2).backward()
    assert float((theta.grad.cpu() - torch.tensor(6.0 * e_ref.real * g_ref)).abs().max()) < 1e-11
    f.sim.close()


def test_autograd_batched(Q, orc):
    import torch
    from paper_2009_02823_amd.autograd import QsvEnergyBatch
    probs = small_batch(8, B=4)
    batch = Q.Batch(probs)
    th = batch.theta_flat().requires_grad_(True)
    e = QsvEnergyBatch.apply(th, batch)
    w = torch.arange(1, len(probs) + 1, dtype=torch.float64, device=th.device)
    (w * e).sum().backward()
    grad = th.grad.cpu().numpy()
    for b, p in enumerate(probs):
        _, g_ref = orc.adjoint_gradient(p.n_qubits, p.gates, p.theta, p.codes, p.coeffs)
        o = batch.theta_off[b]
        assert np.max(np.abs(grad[o:o + p.n_params] - (b + 1) * g_ref)) <= 1e-10 * (b + 1)
    batch.close()


def wave_batch(seed):
    """Circuits of 1 to 6 qubits (one wave each): every gate kind, repeated and unique
    parameters, gate counts around the 64-gate chunks of gate data, slot counts at the 32-slot
    flushes of the product rows, and an empty circuit."""
    rng = np.random.default_rng(seed)
    probs = []
    shapes = [(1, 0, None), (1, 1, None), (2, 63, None), (3, 64, None), (4, 65, None),
              (5, 200, None), (6, 200, 30), (6, 129, 7), (5, 333, None), (2, 40, 3)]
    for b, (n, G, npar) in enumerate(shapes):
        kinds = [k for k in list(W.GATE_NAMES) if n >= 2 or W.N_QUBITS[k] == 1]
        gates, P = W.random_circuit(rng, n, G, kinds, n_params=npar)
        codes = W.random_pauli_strings(rng, n, 5)
        coeffs = rng.standard_normal(5)
        probs.append(W.Problem(f"w{b}", n, gates, W.uniform_angles(rng, P), codes, coeffs))
    # rotations only: exactly 32 and 64 products (the flush boundaries)
    for n, G in ((3, 32), (5, 64)):
        rows = [(int(rng.choice([W.RX, W.RY, W.RZ])), int(rng.integers(0, n)), -1, j, -1, -1)
                for j in range(G)]
        codes = W.random_pauli_strings(rng, n, 4)
        probs.append(W.Problem(f"r{n}", n, W.circuit_table(rows), W.uniform_angles(rng, G),
                               codes, rng.standard_normal(4)))
    return probs


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_wave_batch_vs_oracle(Q, orc, dtype):
    """A batch of circuits of at most 6 qubits runs one wave per circuit in one launch; every
    energy and gradient entry against the oracle, with graphs on, over replays into two pairs of
    output buffers."""
    import torch
    probs = wave_batch(21)
    batch = Q.Batch(probs, dtype)
    batch.set_graphs(True)
    th = batch.theta_flat()
    refs = [orc.adjoint_gradient(p.n_qubits, p.gates, p.theta, p.codes, p.coeffs) for p in probs]
    outs = [(torch.full((len(probs),), np.nan, dtype=torch.float64, device=th.device),
             torch.full((batch.n_params,), np.nan, dtype=torch.float64, device=th.device))
            for _ in range(2)]
    for rep in range(3):
        for e, g in outs:
            batch.adjoint_gradient(th, e, g)
            batch.sync()
            ec, gc = e.cpu().numpy(), g.cpu().numpy()
            for b, (p, (e_ref, g_ref)) in enumerate(zip(probs, refs)):
                gb = gc[batch.theta_off[b]: batch.theta_off[b] + p.n_params]
                if dtype == "c128":
                    assert abs(ec[b] - e_ref.real) <= 1e-10, (rep, b)
                    assert p.n_params == 0 or np.max(np.abs(gb - g_ref)) <= 1e-10, (rep, b)
                else:
                    assert abs(ec[b] - e_ref.real) <= 2e-4 * max(abs(e_ref), 1.0), (rep, b)
                    scale = max(np.max(np.abs(g_ref), initial=0), 1e-5 * np.abs(p.coeffs).sum())
                    assert p.n_params == 0 or np.max(np.abs(gb - g_ref)) <= 2e-4 * scale, (rep, b)
    batch.close()


def test_wave_batch_paper_circuits(Q, orc):
    """The paper's regime at batch scale: 5-qubit circuits with P up to 1290 (Hadamard^(x)5), a
    sample of the batch against the oracle and every circuit against its single call."""
    import torch
    probs = []
    for L in (1, 8, 129):
        base = W.paper_benchmark(5, L)
        rng = np.random.default_rng(L)
        for c in range(3):
            probs.append(W.Problem(f"{base.name}_{c}", 5, base.gates,
                                   W.uniform_angles(rng, base.n_params), base.codes, base.coeffs))
    batch = Q.Batch(probs)
    e, g = batch.adjoint_gradient(batch.theta_flat())
    batch.sync()
    ec, gc = e.cpu().numpy(), g.cpu().numpy()
    for b, p in enumerate(probs):
        gb = gc[batch.theta_off[b]: batch.theta_off[b] + p.n_params]
        if b % 3 == 0:
            e_ref, g_ref = orc.adjoint_gradient(5, p.gates, p.theta, p.codes, p.coeffs)
            assert abs(ec[b] - e_ref.real) <= 1e-10
            assert np.max(np.abs(gb - g_ref)) <= 1e-10
        for mode in (2, -1):  # the plain one-wave sweep is the batch's, bit for bit; the
            with Q.StateVector(5) as sv:  # automatic mode runs long circuits chunked
                sv.set_fusion(mode)
                e1, g1 = sv.adjoint_gradient(p.gates, torch.as_tensor(p.theta, device="cuda:0"),
                                             p.codes, p.coeffs)
                sv.sync()
                e1, g1 = float(e1.cpu()[0]), g1.cpu().numpy()
            if mode == 2:
                assert e1 == ec[b] and np.array_equal(g1, gb)
            else:
                assert abs(e1 - ec[b]) <= 1e-12 and np.max(np.abs(g1 - gb)) <= 1e-12
    batch.close()


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_wave_batch_reference(Q, orc, dtype):
    """Algorithm 2 for a batch of circuits of at most 6 qubits (one wave per circuit for lambda,
    one per (circuit, occurrence)), and for a batch of larger circuits (one after the other),
    against the oracle."""
    for probs in (wave_batch(31), small_batch(4, B=3)):
        batch = Q.Batch(probs, dtype)
        e, g = batch.reference_gradient(batch.theta_flat())
        batch.sync()
        ec, gc = e.cpu().numpy(), g.cpu().numpy()
        for b, p in enumerate(probs):
            e_ref, g_ref = orc.adjoint_gradient(p.n_qubits, p.gates, p.theta, p.codes, p.coeffs)
            gb = gc[batch.theta_off[b]: batch.theta_off[b] + p.n_params]
            if dtype == "c128":
                assert abs(ec[b] - e_ref.real) <= 1e-10, b
                assert p.n_params == 0 or np.max(np.abs(gb - g_ref)) <= 1e-10, b
            else:
                assert abs(ec[b] - e_ref.real) <= 2e-4 * max(abs(e_ref), 1.0), b
                scale = max(np.max(np.abs(g_ref), initial=0), 1e-5 * np.abs(p.coeffs).sum())
                assert p.n_params == 0 or np.max(np.abs(gb - g_ref)) <= 2e-4 * scale, b
        batch.close()


def test_batch_autotune(Q, orc):
    """The batch geometry autotuner times every geometry that fits every circuit, keeps the
    fastest on all handles, and the gradients in that geometry still match the oracle."""
    probs = small_batch(6, B=4)
    batch = Q.Batch(probs)
    mode, r, w, ms = batch.autotune(repeats=1)
    assert ms > 0 and mode in (-1, 1)
    if mode == 1:
        assert (r, w) in Q.Batch.GEOMETRIES["c128"] and r + w <= min(p.n_qubits for p in probs)
        assert all(h.get_fusion() == (1, r, w) for h in batch.handles)
    e, g = batch.adjoint_gradient(batch.theta_flat())
    batch.sync()
    e, g = e.cpu().numpy(), g.cpu().numpy()
    for b, p in enumerate(probs):
        e_ref, g_ref = orc.adjoint_gradient(p.n_qubits, p.gates, p.theta, p.codes, p.coeffs)
        assert abs(e[b] - e_ref.real) <= 1e-10
        assert np.max(np.abs(g[batch.theta_off[b]: batch.theta_off[b] + p.n_params] - g_ref)) <= 1e-10
    batch.close()
