"""Benchmark: full reverse-mode gradients per second on one MI355X, against GPU parameter shift
and the CPU oracle.

Default workload (one "step" = one energy + one full gradient, Algorithm 1): the
hardware-efficient ansatz on 30 qubits with 10 layers of RY and RZ on every qubit plus a CNOT
ladder (P = 600 angles, seeded uniform in [0, 2pi)), under the open Ising chain
sum J_i Z_i Z_{i+1} + sum h_i X_i with N(0,1) couplings and fields, complex128 storage (three
16 GiB states in HBM). Inputs are synthetic and resident on the GPU before the timed region
starts. --config 1 / 2 / 3 / 4 select the 10-qubit, 20-qubit, 26-qubit complex64 workloads and
the 512-circuit batch instead.

Prints one JSON line. Besides the headline value it carries:
  grad_error    energy and gradient against the oracle's stored values (tests/golden/);
  roofline      the dominant kernel family's algorithmic bytes per launch over its average
                launch duration (HIP events around each of its launches, in a second timed region
                of the same steps run without graph replay), against the 8 TB/s HBM peak, with
                the FP64 VALU fraction of the same launches beside it;
  per_step      mean, standard deviation, median and minimum of event-timed steps;
  eager         the step time without graph replay (the second timed region);
  param_shift   the faithful O(P^2) gradient on the same GPU, timed on a sample of entries;
  cpu_baseline  the CPU oracle (Algorithm 1, complex128) on the host cores, on a bounded sample;
  extra         shorter runs of the 20-qubit (complex128, complex64) and 26-qubit (complex64,
                complex128) workloads.
--sweep-p prints the adjoint / parameter-shift times over the number of layers instead.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.join(ROOT, "tests", "golden"))

HBM_PEAK_GBPS = 8000.0
METRIC = "full gradients/sec and HBM GB/s, adjoint vs parameter-shift, at stated grad error"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# The sources that decide what the fused passes read and write: their kernels and headers, the
# scheduler and the host code that builds their launches. Counter runs taken on other versions
# of these files are not used.
FUSED_SOURCES = ("fused_kernels.hip", "fused.h", "schedule.hip", "qsv_api.hip", "qsv_device.h",
                 "qsv_internal.h")


def kernel_source_sha() -> str:
    h = hashlib.sha256()
    for name in FUSED_SOURCES:
        h.update(open(os.path.join(ROOT, "paper_2009_02823_amd", "csrc", name), "rb").read())
    return h.hexdigest()[:16]


def traffic_for(family: str, workload: str, dtype: str, geometry):
    """HBM bytes per launch from committed rocprofv3 counter runs, if they were taken on the
    current kernel sources and the same tile geometry (else None)."""
    if geometry is None:
        return None
    path = os.path.join(ROOT, "profiles",
                        f"traffic_{family}_{workload}_{dtype}_r{geometry[0]}w{geometry[1]}.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("kernel_source_sha") != kernel_source_sha():
        return None
    if list(rec.get("geometry", [])) != list(geometry):
        return None
    return rec.get("bytes_per_launch")


class Single:
    """One circuit on one handle."""

    def __init__(self, qsv, torch, prob, dtype):
        self.torch = torch
        self.prob = prob
        self.sv = qsv.StateVector(prob.n_qubits, dtype, device="cuda:0")
        self.theta = torch.as_tensor(prob.theta, device="cuda:0")
        self.e = torch.empty(1, dtype=torch.float64, device="cuda:0")
        self.g = torch.empty(prob.n_params, dtype=torch.float64, device="cuda:0")
        self.units = 1

    def autotune(self, geometry=None):
        if geometry:
            self.sv.set_fusion(1, *geometry)
            return (1, geometry[0], geometry[1], -1.0)
        return self.sv.autotune(self.prob.gates, self.theta, self.prob.codes, self.prob.coeffs)

    def step(self):
        self.sv.adjoint_gradient(self.prob.gates, self.theta, self.prob.codes, self.prob.coeffs,
                                 self.e, self.g)

    def handle(self):
        return self.sv

    def result(self):
        return float(self.e.cpu()[0]), self.g.cpu().numpy()

    def close(self):
        self.sv.close()


class Batched:
    """The batch of independent circuits (one step = every circuit's energy and gradient)."""

    def __init__(self, qsv, torch, probs, dtype):
        self.torch = torch
        self.batch = qsv.Batch(probs, dtype)
        self.theta = self.batch.theta_flat()
        self.e = torch.empty(len(probs), dtype=torch.float64, device=self.batch.device)
        self.g = torch.empty(self.batch.n_params, dtype=torch.float64, device=self.batch.device)
        self.units = len(probs)

    def autotune(self, geometry=None):
        if geometry:
            for h in self.batch.handles:
                h.set_fusion(1, *geometry)
            return (1, geometry[0], geometry[1], -1.0)
        t = self.batch.autotune()
        log(f"batch autotune: mode {t[0]} r={t[1]} w={t[2]}: {t[3]:.3f} ms")
        return t

    def step(self):
        self.batch.adjoint_gradient(self.theta, self.e, self.g)

    def handle(self):
        return self.batch.handles[0]

    def result(self):
        return self.e.cpu().numpy(), self.g.cpu().numpy()

    def close(self):
        self.batch.close()


def timed_steps(torch, runner, steps):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        runner.step()
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def step_distribution(torch, runner, stream, reps):
    """Each of `reps` steps bracketed by HIP events on the handle's stream, after the timed
    region: mean, standard deviation, median and minimum in ms."""
    import numpy as np
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
    torch.cuda.synchronize()
    ev[0].record(stream)
    for i in range(reps):
        runner.step()
        ev[i + 1].record(stream)
    torch.cuda.synchronize()
    ms = np.array([ev[i].elapsed_time(ev[i + 1]) for i in range(reps)])
    return {"runs": reps, "mean_ms": float(ms.mean()), "std_ms": float(ms.std()),
            "median_ms": float(np.median(ms)), "min_ms": float(ms.min())}


def gate_granular_bytes(prob, state_bytes):
    """Bytes one energy + gradient would move with one HBM pass per gate (mu never in HBM):
    forward rotation 2S, CNOT S, CZ S/2; reverse rotation 4S, CNOT 2S, CZ S; H 2S plus 3S per
    further x-mask group; clones and the energy 6S. Every other gate counts as a rotation."""
    from paper_2009_02823_amd import workloads as W
    S = float(state_bytes)
    fwd = bwd = 0.0
    for row in prob.gates:
        k = int(row[0])
        if k == W.CNOT:
            fwd, bwd = fwd + S, bwd + 2 * S
        elif k == W.CZ:
            fwd, bwd = fwd + S / 2, bwd + S
        else:
            fwd, bwd = fwd + 2 * S, bwd + 4 * S
    xmask = {tuple(int(c) in (1, 2) for c in term) for term in prob.codes}
    return fwd + bwd + 2 * S + 3 * S * (len(xmask) - 1) + 6 * S


def run(qsv, torch, runner, steps, warmup, graphs=True, geometry=None):
    tuned = runner.autotune(geometry)
    h = runner.handle()
    runner.step()   # plans, schedules and code objects load outside the recorded steps
    # warm-up with every kernel timed, to find the dominant kernel family
    h.timing_enable("")
    for _ in range(max(warmup, 1)):
        runner.step()
    stats = h.timing_read()
    h.timing_enable(None)
    dominant = stats[0]["name"]
    # timed region 1: the headline (graph replay of the whole step)
    if graphs:
        h.set_graphs(True)
        for _ in range(2):
            runner.step()      # eager run, then capture
    dt = timed_steps(torch, runner, steps)
    per_step = step_distribution(torch, runner, h.stream, max(3, min(24, steps)))
    if graphs:
        h.set_graphs(False)
    # timed region 2: the same steps launched eagerly, the dominant family timed per launch
    h.timing_enable(dominant)
    dt_eager = timed_steps(torch, runner, steps)
    dom = h.timing_read()
    h.timing_enable(None)
    return {"seconds": dt, "ms_per_step": 1e3 * dt / steps, "value": runner.units * steps / dt,
            "ms_per_step_eager": 1e3 * dt_eager / steps, "per_step": per_step,
            "dominant": dom[0] if dom else None,
            "warmup_stats": stats, "tuned": tuned}


def grad_error(prob, energy, grad, dtype):
    """Energy and gradient against the oracle's stored values, with the per-entry error
    distribution (quantiles of |dg_p| and of |dg_p| / |g_p|)."""
    import numpy as np
    import make_golden
    ref = make_golden.read(prob.name)
    if ref is None:
        return None
    e_ref, g_ref = ref
    scale = max(float(np.max(np.abs(g_ref))), 1e-5 * float(np.abs(prob.coeffs).sum()))
    dg = np.abs(grad - g_ref)
    d = {"max_abs_grad_err": float(dg.max()),
         "abs_energy_err": abs(energy - e_ref.real),
         "max_abs_grad_ref": float(np.max(np.abs(g_ref)))}
    d["rel_grad_err"] = d["max_abs_grad_err"] / scale
    d["tolerance"] = ("1e-10 abs (energy and every entry)" if dtype == "c128" else
                      "2e-4 * max(max|g_oracle|, 1e-5 sum|c|); energy 2e-4 * max(|E|, 1)")
    if dtype == "c128":
        d["ok"] = d["max_abs_grad_err"] <= 1e-10 and d["abs_energy_err"] <= 1e-10
    else:
        d["ok"] = (d["rel_grad_err"] <= 2e-4
                   and d["abs_energy_err"] <= 2e-4 * max(abs(e_ref.real), 1.0))
    q = [0.5, 0.9, 0.99, 1.0]
    rel = dg / np.maximum(np.abs(g_ref), 1e-300)
    d["per_entry"] = {"entries": int(dg.size), "quantiles": q,
                      "abs": [float(x) for x in np.quantile(dg, q)],
                      "rel": [float(x) for x in np.quantile(rel, q)],
                      "note": "relative errors of near-vanishing entries are large by construction; "
                              "reported, not gated"}
    return d


def run_param_shift(qsv, torch, prob, dtype, entries, adj_grad=None, tune=None):
    import numpy as np
    sv = qsv.StateVector(prob.n_qubits, dtype, device="cuda:0")
    if tune:
        sv.set_fusion(*tune)
    theta = torch.as_tensor(prob.theta, device="cuda:0")
    g = torch.zeros(prob.n_params, dtype=torch.float64, device="cuda:0")
    sv.param_shift_gradient(prob.gates, theta, prob.codes, prob.coeffs, 0, 1, g)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sv.param_shift_gradient(prob.gates, theta, prob.codes, prob.coeffs, 0, entries, g)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    gs = g.cpu().numpy()[:entries]
    sv.close()
    per_grad = dt * prob.n_params / entries
    out = {"seconds_per_gradient": per_grad, "value": 1.0 / per_grad,
           "sampled_entries": entries, "sample_seconds": dt,
           "method": "2 energy evaluations per entry (reset + forward + expectation), same "
                     "kernels; sampled entries scaled by P (every entry costs the same)"}
    if adj_grad is not None:
        out["max_abs_diff_vs_adjoint"] = float(np.max(np.abs(gs - adj_grad[:entries])))
    return out


def run_cpu_baseline(prob, W):
    """The oracle's Algorithm 1 (complex128, OpenMP over the host cores) timed on a bounded
    sample (about 10-30 s): the whole energy + gradient of the same workload when its state has
    at most 22 qubits, otherwise of the same ansatz and Hamiltonian recipe at fewer qubits (24
    for the 30-qubit workload, 20 for the 26-qubit one), scaled to one full-size gradient by the
    ratio of the two circuits' one-pass-per-gate bytes (the oracle makes one pass over its
    states per gate primitive, so its time is proportional to them)."""
    from oracle import oracle as O
    O.lib()
    n = prob.n_qubits
    sample = prob
    if n > 22:
        cfg = {30: (W.config5, 24), 26: (W.config3, 20)}.get(n)
        if cfg is None:
            return None
        sample = cfg[0](n=cfg[1])
    t0 = time.perf_counter()
    O.adjoint_gradient(sample.n_qubits, sample.gates, sample.theta, sample.codes, sample.coeffs)
    dt = time.perf_counter() - t0
    factor = gate_granular_bytes(prob, 16 << n) / gate_granular_bytes(sample, 16 << sample.n_qubits)
    sec = dt * factor
    out = {"value": 1.0 / sec, "unit": "gradients/s", "cores": O.num_threads(), "kind": "oracle",
           "seconds_per_gradient": sec, "sample_seconds": dt}
    if sample is prob:
        out["sample"] = (f"one full energy + gradient of {prob.name} (Algorithm 1, complex128, "
                         f"{dt:.1f} s)")
    else:
        out["sample"] = (f"one full energy + gradient of {sample.name} (the same ansatz and "
                         f"Hamiltonian recipe at {sample.n_qubits} qubits, {sample.n_gates} gates; "
                         f"{dt:.1f} s), scaled by {factor:.1f} (ratio of one-pass-per-gate bytes) "
                         f"to {prob.name}")
    return out


def cached_oracle_run(prob):
    """Time of the oracle run that wrote the stored values of this workload (from the golden
    file's header), if present."""
    import re
    import make_golden
    path = make_golden.golden_path(prob.name)
    if not os.path.exists(path):
        return None
    for line in open(path):
        m = re.search(r"oracle threads=(\d+), ([0-9.]+) s", line)
        if m:
            return {"seconds": float(m.group(2)), "threads": int(m.group(1)),
                    "source": os.path.relpath(path, ROOT),
                    "host": "the build container (not the GPU box's host)"}
    return None


def sweep_flops(prob, n_qubits):
    """Algorithmic FP64 flops (an FMA counts 2) of the forward and reverse sweeps, counted per
    gate as the minimal arithmetic of one pass over the state (mu never materialised):
    a rotation costs 6 flops per amplitude on one state (a real 2x2 mix or a complex phase),
    so 6 forward and 6 + 6 + 4 reverse (both states, and the 4-flop product Im<lam|G|phi>);
    CNOT, CZ and the other permutation or sign gates cost none; any other gate counts as a
    dense 2x2 (or 4x4) complex matrix, 14 (or 30) flops per amplitude and state, plus 8 per
    derivative product."""
    from paper_2009_02823_amd import workloads as W
    A = float(1 << n_qubits)
    fwd = bwd = 0.0
    free = {W.CNOT, W.CZ, W.X, W.Y, W.Z, W.S}
    for row in prob.gates:
        k = int(row[0])
        if k in free:
            continue
        if k in (W.RX, W.RY, W.RZ):
            fwd += 6 * A
            bwd += 16 * A
        else:
            m = 30 if W.N_QUBITS.get(k, 1) == 2 else 14
            npar = W.N_PARAMS.get(k, 0)
            fwd += m * A
            bwd += (2 * m + 8 * npar) * A
    return fwd, bwd


FP64_PEAK_TFLOPS = 78.6


def sweep_p(qsv, torch, W, n, layers_list, ps_entries):
    """Adjoint and parameter-shift times over the number of layers (P = 2 n L), with the
    least-squares slopes of log t against log P."""
    import numpy as np
    rows = []
    for L in layers_list:
        prob = W.config2(n=n, layers=L)
        runner = Single(qsv, torch, prob, "c128")
        runner.autotune()
        for _ in range(2):
            runner.step()
        steps = 5
        t_adj = timed_steps(torch, runner, steps) / steps
        runner.close()
        ps = run_param_shift(qsv, torch, prob, "c128", min(ps_entries, prob.n_params))
        rows.append({"layers": L, "P": prob.n_params, "adjoint_s": t_adj,
                     "param_shift_s": ps["seconds_per_gradient"],
                     "speedup": ps["seconds_per_gradient"] / t_adj})
        log(f"L={L} P={prob.n_params}: adjoint {1e3 * t_adj:.3f} ms, parameter shift "
            f"{ps['seconds_per_gradient']:.3f} s, speedup {rows[-1]['speedup']:.0f}")
    lp = np.log([r["P"] for r in rows])
    fit = {k: float(np.polyfit(lp, np.log([r[c] for r in rows]), 1)[0])
           for k, c in (("adjoint", "adjoint_s"), ("param_shift", "param_shift_s"),
                        ("speedup", "speedup"))}
    return {"n_qubits": n, "rows": rows, "loglog_slopes": fit}


def paper_sweep(qsv, torch, W, n, layers_list, runs, cpu):
    """The paper's benchmark (Sec. 3): Algorithm 1 (adjoint) and Algorithm 2 (reference) on the
    GPU at a few qubits under Hadamard^(x)n, P = 2 n L; mean and standard deviation over `runs`
    timed runs each (every run synchronised), and the log-log slopes of time against P. With
    `cpu`, the CPU oracle's Algorithm 1 and 2 times beside them (one run each)."""
    import numpy as np
    rows = []
    for L in layers_list:
        prob = W.paper_benchmark(n, L)
        sv = qsv.StateVector(n, "c128", device="cuda:0")
        theta = torch.as_tensor(prob.theta, device="cuda:0")
        e = torch.empty(1, dtype=torch.float64, device="cuda:0")
        g = torch.empty(prob.n_params, dtype=torch.float64, device="cuda:0")
        row = {"layers": L, "P": prob.n_params, "gates": prob.n_gates}
        for name, fn in (("adjoint", sv.adjoint_gradient), ("reference", sv.reference_gradient)):
            for _ in range(2):
                fn(prob.gates, theta, prob.codes, prob.coeffs, e, g)
            torch.cuda.synchronize()
            ts = []
            for _ in range(runs):
                t0 = time.perf_counter()
                fn(prob.gates, theta, prob.codes, prob.coeffs, e, g)
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t0)
            row[name + "_s"] = float(np.mean(ts))
            row[name + "_std_s"] = float(np.std(ts))
            row[name + "_grad"] = g.cpu().numpy()
        row["max_abs_diff"] = float(np.max(np.abs(row.pop("adjoint_grad") - row.pop("reference_grad"))))
        row["speedup"] = row["reference_s"] / row["adjoint_s"]
        sv.close()
        if cpu:
            from oracle import oracle as O
            t0 = time.perf_counter()
            O.adjoint_gradient(n, prob.gates, prob.theta, prob.codes, prob.coeffs)
            row["cpu_adjoint_s"] = time.perf_counter() - t0
            t0 = time.perf_counter()
            O.reference_gradient(n, prob.gates, prob.theta, prob.codes, prob.coeffs)
            row["cpu_reference_s"] = time.perf_counter() - t0
        rows.append(row)
        log(f"N={n} L={L} P={prob.n_params}: adjoint {1e3 * row['adjoint_s']:.3f} ms, reference "
            f"{1e3 * row['reference_s']:.3f} ms, speedup {row['speedup']:.1f}, "
            f"|dg| {row['max_abs_diff']:.1e}")
    keys = ["adjoint_s", "reference_s", "speedup"] + (["cpu_adjoint_s", "cpu_reference_s"] if cpu else [])
    return {"n_qubits": n, "observable": "Hadamard^(x)n", "runs": runs, "rows": rows,
            "loglog_slopes": loglog_slopes(rows, keys, 0),
            "loglog_slopes_p_ge_160": loglog_slopes(rows, keys, 160)}


def loglog_slopes(rows, keys, p_min):
    """Slopes of log(value) against log(P) over the rows with P >= p_min (least squares)."""
    import numpy as np
    sel = [r for r in rows if r["P"] >= p_min]
    lp = np.log([r["P"] for r in sel])
    return {k: float(np.polyfit(lp, np.log([r[k] for r in sel]), 1)[0]) for k in keys}


def paper_batch(qsv, torch, W, n, layers_list, B, runs):
    """The paper's comparison at batch scale: B circuits of the paper's regime per L (the same
    ansatz, independent uniform angles per circuit) through Algorithm 1
    (qsv_adjoint_gradient_batched, one wave per circuit) and Algorithm 2
    (qsv_reference_gradient_batched, one wave per circuit and parameter occurrence). Device time
    is the sum of the library's event-timed launches per call (mean over `runs` calls); wall time
    also holds the host's per-call work (plan lookups of B handles). A sample of circuits is
    checked between the two algorithms."""
    import numpy as np
    rows = []
    for L in layers_list:
        base = W.paper_benchmark(n, L)
        rng = np.random.default_rng(1000 + L)
        probs = [W.Problem(f"{base.name}_{b}", n, base.gates,
                           W.uniform_angles(rng, base.n_params), base.codes, base.coeffs)
                 for b in range(B)]
        batch = qsv.Batch(probs)
        th = batch.theta_flat()
        e = torch.empty(B, dtype=torch.float64, device="cuda:0")
        g1 = torch.empty(batch.n_params, dtype=torch.float64, device="cuda:0")
        g2 = torch.empty_like(g1)
        row = {"layers": L, "P": base.n_params, "gates": base.n_gates, "circuits": B}
        h0 = batch.handles[0]
        for name, fn, g in (("adjoint", batch.adjoint_gradient, g1),
                            ("reference", batch.reference_gradient, g2)):
            fn(th, e, g)
            torch.cuda.synchronize()
            h0.timing_enable("")
            t0 = time.perf_counter()
            for _ in range(runs):
                fn(th, e, g)
            torch.cuda.synchronize()
            wall = (time.perf_counter() - t0) / runs
            st = h0.timing_read()
            h0.timing_enable(None)
            dev = sum(x["total_ms"] for x in st) * 1e-3 / runs
            row[name + "_device_s"] = dev
            row[name + "_wall_s"] = wall
            row[name + "_gradients_per_s"] = B / dev
            row[name + "_kernels"] = {x["name"]: x["total_ms"] / runs for x in st}
        d = (g1 - g2).abs().max().item()
        row["max_abs_diff"] = d
        row["speedup_device"] = row["reference_device_s"] / row["adjoint_device_s"]
        batch.close()
        del batch, th, e, g1, g2
        rows.append(row)
        log(f"batch N={n} L={L} P={base.n_params} B={B}: Alg. 1 {1e3 * row['adjoint_device_s']:.3f} "
            f"ms ({row['adjoint_gradients_per_s']:.3g} gradients/s), Alg. 2 "
            f"{1e3 * row['reference_device_s']:.3f} ms, speedup {row['speedup_device']:.1f}, "
            f"|dg| {d:.1e}")
    keys = ["adjoint_device_s", "reference_device_s", "speedup_device"]
    return {"n_qubits": n, "observable": "Hadamard^(x)n", "circuits": B, "runs": runs,
            "rows": rows, "loglog_slopes": loglog_slopes(rows, keys, 0),
            "loglog_slopes_p_ge_160": loglog_slopes(rows, keys, 160)}


def roofline_of(res, S, flops_bwd, flops_fwd, steps, workload, dtype):
    """The dominant family's HBM fraction (algorithmic bytes per launch over the event-timed
    average launch) and its FP64 VALU fraction (algorithmic flops of the family's sweep per step
    over the family's event-timed time per step)."""
    dom = res["dominant"]
    if not dom:
        return None
    avg_s = dom["total_ms"] * 1e-3 / dom["launches"]
    achieved = dom["bytes_per_launch"] / avg_s / 1e9
    tuned = res["tuned"]
    roof = {"bound": "hbm", "kernel": dom["name"], "achieved": achieved,
            "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBPS,
            "traffic": traffic_for(dom["name"], workload, dtype,
                                   tuned[1:3] if tuned and tuned[0] else None),
            "bytes_per_launch": dom["bytes_per_launch"], "avg_launch_us": 1e6 * avg_s,
            "launches_per_step": dom["launches"] / steps,
            "share_of_eager_step": dom["total_ms"] / (res["ms_per_step_eager"] * steps),
            "state_bytes": S}
    fl = {"k_pass_bwd": flops_bwd, "k_pass_fwd": flops_fwd}.get(dom["name"])
    if fl:
        t_step = dom["total_ms"] * 1e-3 / steps
        tf = fl / t_step / 1e12
        roof["fp64_valu"] = {"flops_per_step": fl, "achieved": tf, "peak": FP64_PEAK_TFLOPS,
                             "unit": "TFLOP/s", "frac": tf / FP64_PEAK_TFLOPS,
                             "model": "rotation: 6 flops per amplitude and state, 4 per product; "
                                      "CNOT/CZ 0 (see sweep_flops)"}
    return roof


def single_summary(qsv, torch, W, prob, dtype, steps, warmup, graphs, geometry=None):
    """A shorter run of one workload for the `extra` key."""
    r = Single(qsv, torch, prob, dtype)
    res = run(qsv, torch, r, steps, warmup, graphs=graphs, geometry=geometry)
    e, g = r.result()
    r.close()
    S = (16.0 if dtype == "c128" else 8.0) * (1 << prob.n_qubits)
    fl_f, fl_b = sweep_flops(prob, prob.n_qubits)
    return {"workload": prob.name, "storage": "complex128" if dtype == "c128" else "complex64",
            "value": res["value"], "unit": "gradients/s", "ms_per_step": res["ms_per_step"],
            "steps": steps, "per_step": res["per_step"],
            "tuned_mode_r_w": res["tuned"][:3] if res["tuned"] else None,
            "grad_error": grad_error(prob, e, g, dtype),
            "roofline": roofline_of(res, S, fl_b, fl_f, steps, prob.name, dtype),
            "breakdown": [{"kernel": x["name"],
                           "ms_per_step": x["total_ms"] / max(warmup, 1),
                           "launches_per_step": x["launches"] / max(warmup, 1)}
                          for x in res["warmup_stats"]]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--ps-entries", type=int, default=8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-param-shift", action="store_true")
    ap.add_argument("--no-c64", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the shorter 20- and 26-qubit runs of the `extra` key")
    ap.add_argument("--no-graphs", action="store_true")
    ap.add_argument("--geometry", type=str, default="", metavar="R,W",
                    help="run the fused passes with this tile geometry instead of autotuning "
                         "(for profiling a fixed kernel instance)")
    ap.add_argument("--tune-cache", type=str, default="",
                    help="load tuning choices from this file first and save them back at the end")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="first copy MIB MiB device to device twice (a plain copy kernel of known "
                         "size, against which hardware byte counters are scaled)")
    ap.add_argument("--config", type=int, default=5,
                    help="5: 30 qubits complex128 (default); 1: 10 qubits; 2: 20 qubits; "
                         "3: 26 qubits complex64; 4: 512-circuit batch")
    ap.add_argument("--sweep-p", action="store_true",
                    help="adjoint vs parameter shift over the number of layers at 20 qubits")
    ap.add_argument("--paper", type=int, default=0, metavar="N",
                    help="the paper's benchmark at N qubits (4 or 5): Algorithm 1 vs Algorithm 2 "
                         "on the GPU, P up to 1290, 24 runs per point")
    ap.add_argument("--paper-cpu", action="store_true",
                    help="with --paper: also time the CPU oracle's Algorithms 1 and 2")
    ap.add_argument("--paper-batch", type=int, default=0, metavar="B",
                    help="with --paper: also B circuits per point through the batched Algorithms "
                         "1 and 2 (device throughput)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "sharding of the state is a design, not a build, here.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2009_02823_amd import qsv
    from paper_2009_02823_amd import workloads as W

    if args.tune_cache:
        log(f"tuning choices loaded: {qsv.tune_cache_load(args.tune_cache)}")

    if args.copy_calibration:
        src = torch.ones(args.copy_calibration << 18, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(2):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log(f"copy calibration: 2 x {args.copy_calibration} MiB")

    if args.paper:
        n = args.paper
        layers = [1, 2, 4, 8, 16, 32, 64, 1290 // (2 * n)]
        res = paper_sweep(qsv, torch, W, n, layers, 24, args.paper_cpu)
        if args.paper_batch:
            res["batch"] = paper_batch(qsv, torch, W, n, layers, args.paper_batch, 3)
        print(json.dumps({"metric": "Algorithm 1 vs Algorithm 2 gradient time over P", **res}))
        return

    if args.sweep_p:
        res = sweep_p(qsv, torch, W, 20, [1, 2, 4, 8, 16, 20], args.ps_entries)
        print(json.dumps({"metric": "adjoint vs parameter-shift scaling in P", **res}))
        return

    if args.config == 4:
        probs = W.config4()
        main_dt = "c128"
        runner = Batched(qsv, torch, probs, main_dt)
        name = f"batch{len(probs)}_hea12-18_L5-15_heisenberg"
        S = float(sum((16 << p.n_qubits) for p in probs))
        log(f"workload {name}: {len(probs)} circuits, P total {runner.batch.n_params}")
    else:
        prob = W.CONFIGS[args.config]()
        main_dt = "c64" if args.config == 3 else "c128"
        runner = Single(qsv, torch, prob, main_dt)
        name = prob.name
        S = (16.0 if main_dt == "c128" else 8.0) * (1 << prob.n_qubits)
        log(f"workload {name}: n={prob.n_qubits} gates={prob.n_gates} P={prob.n_params}")
    geometry = tuple(int(x) for x in args.geometry.split(",")) if args.geometry else None
    res = run(qsv, torch, runner, args.steps, args.warmup, graphs=not args.no_graphs,
              geometry=geometry)
    log(f"{main_dt} adjoint: {res['ms_per_step']:.3f} ms/step (eager "
        f"{res['ms_per_step_eager']:.3f}), tuned {res['tuned']}")
    e_res, g_res = runner.result()
    err = None if args.config == 4 else grad_error(prob, e_res, g_res, main_dt)
    runner.close()
    probs_ = probs if args.config == 4 else [prob]
    fl_f = fl_b = 0.0
    for p in probs_:
        a, b = sweep_flops(p, p.n_qubits)
        fl_f, fl_b = fl_f + a, fl_b + b
    roof = roofline_of(res, S, fl_b, fl_f, args.steps, name, main_dt)
    out = {
        "metric": METRIC, "value": res["value"],
        "unit": "gradients/s" if args.config != 4 else "circuit gradients/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": res["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if main_dt == "c128" else "f32 (FP64 reductions)",
        "data": "synthetic",
        "config": {"workload": name, "storage": "complex128" if main_dt == "c128" else "complex64",
                   "graph_replay": not args.no_graphs, "parallelism": "single GPU"},
        "grad_error": err,
        "roofline": roof,
        "eager": {"ms_per_step": res["ms_per_step_eager"]},
        "per_step": res["per_step"],
        # per kernel family over the eager warm-up steps (HIP events around every launch)
        "breakdown": [{"kernel": x["name"], "ms_per_step": x["total_ms"] / max(args.warmup, 1),
                       "launches_per_step": x["launches"] / max(args.warmup, 1)}
                      for x in res["warmup_stats"]],
        "execution": {"tuned_mode_r_w": res["tuned"][:3] if res["tuned"] else None},
    }
    if args.config != 4:
        out["config"].update({"n_qubits": prob.n_qubits, "n_params": prob.n_params,
                              "n_gates": prob.n_gates, "pauli_terms": int(len(prob.coeffs))})
    # what fusion saves: the bytes of a one-HBM-pass-per-gate schedule over the measured time
    # (may exceed the peak; it is not a roofline)
    b_adj = sum(gate_granular_bytes(p, (16 if main_dt == "c128" else 8) << p.n_qubits)
                for p in probs_)
    ge = b_adj / (res["ms_per_step"] * 1e-3) / 1e9
    out["gate_equivalent"] = {"bytes_per_step": b_adj, "GBps": ge, "vs_hbm_peak": ge / HBM_PEAK_GBPS,
                              "ms_at_60pct_peak": b_adj / (0.6 * HBM_PEAK_GBPS * 1e9) * 1e3}
    tune = None
    if res["tuned"]:
        m, r, w, _ = res["tuned"]
        tune = (m, r, w) if m else (0, 0, 0)
    if not args.no_c64 and main_dt == "c128" and args.config != 4 and prob.n_qubits <= 26:
        out["c64"] = single_summary(qsv, torch, W, prob, "c64", args.steps, args.warmup,
                                    not args.no_graphs)
        log(f"c64 adjoint: {out['c64']['ms_per_step']:.3f} ms/gradient")
    if not args.no_param_shift and args.config != 4:
        ps = run_param_shift(qsv, torch, prob, main_dt, args.ps_entries, g_res, tune)
        ps["speedup_of_adjoint"] = ps["seconds_per_gradient"] / (res["ms_per_step"] * 1e-3)
        log(f"param shift: {ps['seconds_per_gradient']:.3f} s/gradient (sampled)")
        out["param_shift"] = ps
    if not args.no_cpu_baseline and args.config != 4:
        cb = run_cpu_baseline(prob, W)
        if cb is not None:
            cached = cached_oracle_run(prob)
            if cached:
                cb["cached_full_run"] = cached
            out["cpu_baseline"] = cb
            log(f"cpu oracle: {cb['seconds_per_gradient']:.2f} s/gradient ({cb['sample']})")
    if not args.no_extra and args.config == 5:
        steps_x = max(3, min(args.steps, 10))
        extra = {}
        for key, cfg, dt in (("hea20_L20_tfim_c128", 2, "c128"), ("hea20_L20_tfim_c64", 2, "c64"),
                             ("hea26_L30_cz_rand200_c64", 3, "c64"),
                             ("hea26_L30_cz_rand200_c128", 3, "c128")):
            p = W.CONFIGS[cfg]()
            extra[key] = single_summary(qsv, torch, W, p, dt, steps_x, args.warmup,
                                        not args.no_graphs)
            log(f"extra {key}: {extra[key]['ms_per_step']:.3f} ms/gradient")
        out["extra"] = extra
    if args.tune_cache:
        qsv.tune_cache_save(args.tune_cache)
    out["kernel_source_sha"] = kernel_source_sha()
    print(json.dumps(out, default=float))


if __name__ == "__main__":
    main()
