"""Python binding of the qsv C-ABI (``include/qsv.h``): argument marshalling only.

Device memory and streams come from PyTorch; every step of the computation runs in the HIP
kernels of ``libqsv.so``. There is no CPU fallback: if the library is not built, or no GPU is
present, the calls raise.

Gate tables are ``int32`` arrays of shape ``(G, 6)`` with rows ``(kind, q0, q1, p0, p1, p2)`` (see
``workloads``); Hamiltonians are ``codes`` ``uint8 (h, n)`` plus real ``coeffs`` ``float64 (h,)``.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libqsv.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "qsv.h")

QSV_OK, QSV_ERR_INVALID_ARG, QSV_ERR_UNSUPPORTED, QSV_ERR_OUT_OF_MEMORY, QSV_ERR_HIP, \
    QSV_ERR_INTERNAL = range(6)
QSV_C64, QSV_C128 = 0, 1
DTYPES = {"c64": QSV_C64, "c128": QSV_C128}
STATUS_NAMES = {0: "QSV_OK", 1: "QSV_ERR_INVALID_ARG", 2: "QSV_ERR_UNSUPPORTED",
                3: "QSV_ERR_OUT_OF_MEMORY", 4: "QSV_ERR_HIP", 5: "QSV_ERR_INTERNAL"}


class QsvError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class KernelStat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 48), ("launches", ctypes.c_int64),
                ("total_ms", ctypes.c_double), ("bytes", ctypes.c_double)]


class ScheduleInfo(ctypes.Structure):
    _fields_ = [("n_passes", ctypes.c_int32), ("n_phases", ctypes.c_int32),
                ("order", ctypes.c_void_p), ("pass_of", ctypes.c_void_p),
                ("phase_of", ctypes.c_void_p), ("tile_mask", ctypes.c_void_p),
                ("reg_mask", ctypes.c_void_p), ("n_macros", ctypes.c_int32),
                ("n_direct_loads", ctypes.c_int32), ("n_direct_stores", ctypes.c_int32),
                ("n_diag_blocks", ctypes.c_int32), ("n_folded_cnots", ctypes.c_int32)]


class PauliSum(ctypes.Structure):
    _fields_ = [("n_terms", ctypes.c_int32), ("codes", ctypes.c_void_p),
                ("coeffs", ctypes.c_void_p)]


_lib = None


def lib() -> ctypes.CDLL:
    """The loaded ``libqsv.so``; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_2009_02823_amd.build` (hipcc, gfx950)")
    L = ctypes.CDLL(LIB_PATH)
    P, i32, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_size_t
    PP = ctypes.POINTER(ctypes.c_void_p)
    sigs = {
        "qsv_validate_circuit": ([i32, P, i32, i32], i32),
        "qsv_validate_pauli_sum": ([i32, P], i32),
        "qsv_workspace_bytes": ([i32, i32], sz),
        "qsv_state_bytes": ([i32, i32], sz),
        "qsv_last_error": ([], ctypes.c_char_p),
        "qsv_create": ([i32, i32, P, P, sz, P, PP], i32),
        "qsv_destroy": ([P], i32),
        "qsv_set_stream": ([P, P], i32),
        "qsv_reset": ([P], i32),
        "qsv_sync": ([P], i32),
        "qsv_apply_circuit": ([P, P, i32, P, i32], i32),
        "qsv_expectation_pauli_sum": ([P, P, P], i32),
        "qsv_expectation_pauli_sum_noalloc": ([P, P, P], i32),
        "qsv_adjoint_gradient": ([P, P, i32, P, i32, P, P, P], i32),
        "qsv_energy": ([P, P, i32, P, i32, P, P], i32),
        "qsv_adjoint_gradient_batched": ([i32, P, P, P, P, P, P, P, P, P], i32),
        "qsv_reference_gradient_batched": ([i32, P, P, P, P, P, P, P, P, P], i32),
        "qsv_param_shift_gradient": ([P, P, i32, P, i32, P, i32, i32, P], i32),
        "qsv_reference_gradient": ([P, P, i32, P, i32, P, P, P], i32),
        "qsv_adjoint_gradient_nonhermitian": ([P, P, i32, P, i32, P, P, P, P], i32),
        "qsv_timing_enable": ([P, ctypes.c_char_p], i32),
        "qsv_timing_read": ([P, P, i32, ctypes.POINTER(i32)], i32),
        "qsv_set_fusion": ([P, i32, i32, i32], i32),
        "qsv_get_fusion": ([P, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i32)],
                           i32),
        "qsv_schedule_describe": ([i32, P, i32, i32, i32, i32, i32, P], i32),
        "qsv_set_graphs": ([P, i32], i32),
        "qsv_autotune": ([P, P, i32, P, i32, P, i32, ctypes.POINTER(i32), ctypes.POINTER(i32),
                          ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_double)], i32),
        "qsv_tune_cache_save": ([ctypes.c_char_p], i32),
        "qsv_tune_cache_load": ([ctypes.c_char_p, ctypes.POINTER(i32)], i32),
        "qsv_build_id": ([], ctypes.c_char_p),
        "qsv_pauli_describe": ([i32, i32, P, ctypes.POINTER(i32), ctypes.POINTER(i32),
                                ctypes.POINTER(i32), P, P, i32], i32),
        "qsv_debug_fail_launch": ([i32], i32),
    }
    for name, (args, res) in sigs.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


def last_error() -> str:
    return lib().qsv_last_error().decode()


def check(status: int):
    if status != QSV_OK:
        raise QsvError(status, last_error())


def as_gate_table(gates) -> np.ndarray:
    g = np.ascontiguousarray(np.asarray(gates, dtype=np.int32).reshape(-1, 6))
    return g


def pauli_struct(codes, coeffs, n_qubits):
    codes = np.ascontiguousarray(np.asarray(codes, dtype=np.uint8).reshape(-1, n_qubits))
    coeffs = np.ascontiguousarray(np.asarray(coeffs, dtype=np.float64).reshape(-1))
    if codes.shape[0] != coeffs.shape[0]:
        raise ValueError("codes and coeffs disagree on the number of terms")
    s = PauliSum(codes.shape[0], codes.ctypes.data, coeffs.ctypes.data)
    return s, (codes, coeffs)   # keep the arrays alive with the struct


def build_id() -> str:
    """Source id of the loaded library build (tags persisted tuning choices)."""
    return lib().qsv_build_id().decode()


def debug_fail_launch(k: int):
    """Test hook: the k-th computation launch from now fails with QSV_ERR_HIP (0 disarms)."""
    check(lib().qsv_debug_fail_launch(int(k)))


def tune_cache_save(path: str):
    """Write the process's tuning choices to `path` (see qsv_tune_cache_save)."""
    check(lib().qsv_tune_cache_save(os.fsencode(path)))


def tune_cache_load(path: str) -> int:
    """Merge the tuning choices of `path` made by this library build; returns how many."""
    n = ctypes.c_int32()
    check(lib().qsv_tune_cache_load(os.fsencode(path), ctypes.byref(n)))
    return n.value


def validate_circuit(n_qubits: int, gates, n_theta: int):
    g = as_gate_table(gates)
    check(lib().qsv_validate_circuit(n_qubits, g.ctypes.data, g.shape[0], n_theta))


def validate_pauli_sum(n_qubits: int, codes, coeffs):
    s, keep = pauli_struct(codes, coeffs, n_qubits)
    check(lib().qsv_validate_pauli_sum(n_qubits, ctypes.byref(s)))
    del keep


def pauli_describe(n_qubits: int, codes, coeffs, dtype: str = "c128", max_passes: int = 64):
    """Host-only: how H is applied (see qsv_pauli_describe): groups, tiled passes with their
    qubit masks and group counts, and the groups left to the gather."""
    s, keep = pauli_struct(codes, coeffs, n_qubits)
    ng, npass, nr = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    masks = np.zeros(max_passes, np.uint64)
    pg = np.zeros(max_passes, np.int32)
    check(lib().qsv_pauli_describe(n_qubits, DTYPES[dtype], ctypes.byref(s), ctypes.byref(ng),
                                   ctypes.byref(npass), ctypes.byref(nr), masks.ctypes.data,
                                   pg.ctypes.data, max_passes))
    del keep
    k = min(npass.value, max_passes)
    return {"n_groups": ng.value, "n_tiled_passes": npass.value, "n_gather_groups": nr.value,
            "tile_masks": masks[:k], "pass_groups": pg[:k]}


def schedule_describe(n_qubits: int, gates, backward: bool, reg_qubits: int, threads_log2: int,
                      dtype: str = "c128"):
    """Host-only: the fused schedule of a circuit as numpy arrays (see qsv_schedule_describe)."""
    g = as_gate_table(gates)
    G = g.shape[0]
    order = np.zeros(max(G, 1), np.int32)
    pass_of = np.zeros(max(G, 1), np.int32)
    phase_of = np.zeros(max(G, 1), np.int32)
    tile = np.zeros(max(G, 1), np.uint64)
    reg = np.zeros(max(G, 1), np.uint64)
    info = ScheduleInfo(0, 0, order.ctypes.data, pass_of.ctypes.data, phase_of.ctypes.data,
                        tile.ctypes.data, reg.ctypes.data, 0)
    check(lib().qsv_schedule_describe(n_qubits, g.ctypes.data, G, 1 if backward else 0,
                                      reg_qubits, threads_log2, DTYPES[dtype],
                                      ctypes.byref(info)))
    return {"n_passes": info.n_passes, "n_phases": info.n_phases, "order": order[:G],
            "pass_of": pass_of[:G], "phase_of": phase_of[:G],
            "tile_mask": tile[:info.n_passes], "reg_mask": reg[:info.n_phases],
            "n_macros": info.n_macros, "n_direct_loads": info.n_direct_loads,
            "n_direct_stores": info.n_direct_stores, "n_diag_blocks": info.n_diag_blocks,
            "n_folded_cnots": info.n_folded_cnots}


def state_bytes(n_qubits: int, dtype: str = "c128") -> int:
    return int(lib().qsv_state_bytes(n_qubits, DTYPES[dtype]))


def workspace_bytes(n_qubits: int, dtype: str = "c128") -> int:
    return int(lib().qsv_workspace_bytes(n_qubits, DTYPES[dtype]))


def _torch():
    import torch
    return torch


class StateVector:
    """A handle: the input state |in> (a torch tensor of 2^n complex amplitudes on the GPU) and a
    two-state workspace, with all work ordered on one HIP stream."""

    def __init__(self, n_qubits: int, dtype: str = "c128", device=None, stream=None):
        torch = _torch()
        L = lib()
        if not torch.cuda.is_available():
            raise RuntimeError("qsv needs a ROCm GPU (torch.cuda.is_available() is False)")
        self.n = int(n_qubits)
        self.dtype = dtype
        self.device = torch.device(device if device is not None else "cuda")
        if self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        cdt = torch.complex128 if dtype == "c128" else torch.complex64
        with torch.cuda.device(self.device):
            self.state = torch.empty(1 << self.n, dtype=cdt, device=self.device)
            nbytes = workspace_bytes(self.n, dtype)
            self.work = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
            self._h = ctypes.c_void_p()
            check(L.qsv_create(self.n, DTYPES[dtype], self.state.data_ptr(), self.work.data_ptr(),
                               nbytes, ctypes.c_void_p(self.stream.cuda_stream),
                               ctypes.byref(self._h)))

    # -- lifecycle
    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().qsv_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- views of the workspace (phi and lambda of Algorithm 1)
    def workspace_states(self):
        torch = _torch()
        cdt = self.state.dtype
        half = self.work.numel() // 2
        return (self.work[:half].view(cdt), self.work[half:2 * half].view(cdt))

    def _theta(self, theta):
        torch = _torch()
        t = torch.as_tensor(theta, dtype=torch.float64)
        if t.device != self.device:
            t = t.to(self.device)
        t = t.contiguous()
        self._keep = t   # the enqueued kernels read it after the call returns
        return t

    # -- calls
    def sync(self):
        check(lib().qsv_sync(self._h))

    def set_stream(self, stream):
        check(lib().qsv_set_stream(self._h, ctypes.c_void_p(stream.cuda_stream)))
        self.stream = stream

    def reset(self):
        check(lib().qsv_reset(self._h))

    def apply_circuit(self, gates, theta=()):
        g = as_gate_table(gates)
        t = self._theta(theta)
        check(lib().qsv_apply_circuit(self._h, g.ctypes.data, g.shape[0],
                                      t.data_ptr() if t.numel() else None, t.numel()))
        return self

    def expectation(self, codes, coeffs, out=None):
        torch = _torch()
        s, keep = pauli_struct(codes, coeffs, self.n)
        e = out if out is not None else torch.empty(1, dtype=torch.float64, device=self.device)
        check(lib().qsv_expectation_pauli_sum(self._h, ctypes.byref(s), e.data_ptr()))
        del keep
        return e

    def expectation_noalloc(self, codes, coeffs, out):
        """<state|H|state> into the float64 device tensor `out` without any allocation (see
        qsv_expectation_pauli_sum_noalloc); `out` must be given."""
        s, keep = pauli_struct(codes, coeffs, self.n)
        check(lib().qsv_expectation_pauli_sum_noalloc(self._h, ctypes.byref(s), out.data_ptr()))
        del keep
        return out

    def energy(self, gates, theta, codes, coeffs, out=None):
        """<psi|H|psi> with psi = U(theta)|in> as a float64 device tensor of shape (1,)."""
        torch = _torch()
        g = as_gate_table(gates)
        t = self._theta(theta)
        s, keep = pauli_struct(codes, coeffs, self.n)
        e = out if out is not None else torch.empty(1, dtype=torch.float64, device=self.device)
        check(lib().qsv_energy(self._h, g.ctypes.data, g.shape[0],
                               t.data_ptr() if t.numel() else None, t.numel(), ctypes.byref(s),
                               e.data_ptr()))
        del keep
        return e

    def adjoint_gradient(self, gates, theta, codes, coeffs, energy=None, grad=None):
        """(E, grad) of Algorithm 1 as float64 device tensors (E has shape (1,))."""
        torch = _torch()
        g = as_gate_table(gates)
        t = self._theta(theta)
        s, keep = pauli_struct(codes, coeffs, self.n)
        e = energy if energy is not None else torch.empty(1, dtype=torch.float64,
                                                         device=self.device)
        gr = grad if grad is not None else torch.empty(t.numel(), dtype=torch.float64,
                                                      device=self.device)
        check(lib().qsv_adjoint_gradient(self._h, g.ctypes.data, g.shape[0],
                                         t.data_ptr() if t.numel() else None, t.numel(),
                                         ctypes.byref(s), e.data_ptr(),
                                         gr.data_ptr() if gr.numel() else None))
        del keep
        return e, gr

    def reference_gradient(self, gates, theta, codes, coeffs, energy=None, grad=None):
        """(E, grad) by the reference scheme of Algorithm 2: one simulation per parameter
        occurrence with that gate replaced by its derivative (O(P^2) gates)."""
        torch = _torch()
        g = as_gate_table(gates)
        t = self._theta(theta)
        s, keep = pauli_struct(codes, coeffs, self.n)
        e = energy if energy is not None else torch.empty(1, dtype=torch.float64,
                                                         device=self.device)
        gr = grad if grad is not None else torch.empty(t.numel(), dtype=torch.float64,
                                                      device=self.device)
        check(lib().qsv_reference_gradient(self._h, g.ctypes.data, g.shape[0],
                                           t.data_ptr() if t.numel() else None, t.numel(),
                                           ctypes.byref(s), e.data_ptr(),
                                           gr.data_ptr() if gr.numel() else None))
        del keep
        return e, gr

    def adjoint_gradient_nonhermitian(self, gates, theta, codes, coeffs):
        """(<A>, grad) for A = sum c_t P_t with complex coefficients (App. B.4) as complex128
        device tensors (<A> has shape (1,), grad shape (P,))."""
        torch = _torch()
        g = as_gate_table(gates)
        t = self._theta(theta)
        c = np.asarray(coeffs, dtype=np.complex128).reshape(-1)
        s, keep = pauli_struct(codes, np.ascontiguousarray(c.real), self.n)
        cim = np.ascontiguousarray(c.imag)
        e = torch.empty(2, dtype=torch.float64, device=self.device)
        gr = torch.empty(2 * t.numel(), dtype=torch.float64, device=self.device)
        check(lib().qsv_adjoint_gradient_nonhermitian(
            self._h, g.ctypes.data, g.shape[0], t.data_ptr() if t.numel() else None, t.numel(),
            ctypes.byref(s), cim.ctypes.data, e.data_ptr(), gr.data_ptr() if gr.numel() else None))
        del keep
        return torch.view_as_complex(e.view(1, 2)), torch.view_as_complex(gr.view(-1, 2))

    def param_shift_gradient(self, gates, theta, codes, coeffs, first=0, count=None, grad=None):
        """GPU parameter-shift entries [first, first + count) (the faithful O(P^2) baseline)."""
        torch = _torch()
        g = as_gate_table(gates)
        t = self._theta(theta)
        count = t.numel() - first if count is None else count
        s, keep = pauli_struct(codes, coeffs, self.n)
        gr = grad if grad is not None else torch.zeros(t.numel(), dtype=torch.float64,
                                                      device=self.device)
        check(lib().qsv_param_shift_gradient(self._h, g.ctypes.data, g.shape[0],
                                             t.data_ptr() if t.numel() else None, t.numel(),
                                             ctypes.byref(s), first, count,
                                             gr.data_ptr() if gr.numel() else None))
        del keep
        return gr

    def set_fusion(self, mode: int, reg_qubits: int = 0, threads_log2: int = 0):
        """mode 0: gate-granular; 1: fused with the given geometry; 2: one wave (at most 6
        qubits); 3: the chunked one-wave sweep (at most 5 qubits); -1: automatic."""
        check(lib().qsv_set_fusion(self._h, mode, reg_qubits, threads_log2))

    def get_fusion(self):
        m, r, w = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        check(lib().qsv_get_fusion(self._h, ctypes.byref(m), ctypes.byref(r), ctypes.byref(w)))
        return m.value, r.value, w.value

    def set_graphs(self, on: bool = True):
        """Capture repeated adjoint calls into hipGraphs and replay them (see qsv_set_graphs)."""
        check(lib().qsv_set_graphs(self._h, 1 if on else 0))

    def autotune(self, gates, theta, codes, coeffs, repeats: int = 2):
        """Time every execution mode on this circuit and keep the fastest; returns
        (mode, reg_qubits, threads_log2, ms per gradient; for a cached choice the time it was
        measured with, -1 if unknown)."""
        g = as_gate_table(gates)
        t = self._theta(theta)
        s, keep = pauli_struct(codes, coeffs, self.n)
        m, r, w = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        ms = ctypes.c_double()
        check(lib().qsv_autotune(self._h, g.ctypes.data, g.shape[0],
                                 t.data_ptr() if t.numel() else None, t.numel(), ctypes.byref(s),
                                 repeats, ctypes.byref(m), ctypes.byref(r), ctypes.byref(w),
                                 ctypes.byref(ms)))
        del keep
        return m.value, r.value, w.value, ms.value

    def timing_enable(self, name_filter: str | None = ""):
        check(lib().qsv_timing_enable(self._h, None if name_filter is None
                                      else name_filter.encode()))

    def timing_read(self, max_out: int = 64):
        """[{name, launches, total_ms, bytes, avg_us, gbps}] sorted by total time."""
        arr = (KernelStat * max_out)()
        n = ctypes.c_int32(0)
        check(lib().qsv_timing_read(self._h, arr, max_out, ctypes.byref(n)))
        out = []
        for k in range(n.value):
            st = arr[k]
            avg_ms = st.total_ms / max(st.launches, 1)
            out.append({"name": st.name.decode(), "launches": int(st.launches),
                        "total_ms": float(st.total_ms), "bytes": float(st.bytes),
                        "avg_us": 1e3 * avg_ms,
                        "bytes_per_launch": float(st.bytes) / max(st.launches, 1),
                        "gbps": (float(st.bytes) / (st.total_ms * 1e-3) / 1e9)
                        if st.total_ms > 0 else 0.0})
        return out


class Batch:
    """Independent circuits (one handle each) whose energies and gradients are computed by one
    qsv_adjoint_gradient_batched call from a flat parameter vector.

    problems: objects with n_qubits, gates, codes, coeffs and n_params (workloads.Problem)."""

    def __init__(self, problems, dtype: str = "c128", device=None):
        torch = _torch()
        self.problems = list(problems)
        B = len(self.problems)
        self.handles = [StateVector(p.n_qubits, dtype, device=device) for p in self.problems]
        self.device = self.handles[0].device
        self.gates = [as_gate_table(p.gates) for p in self.problems]
        self._paulis = [pauli_struct(p.codes, p.coeffs, p.n_qubits) for p in self.problems]
        self.n_theta = [int(p.n_params) for p in self.problems]
        off = np.zeros(B + 1, dtype=np.int64)
        off[1:] = np.cumsum(self.n_theta)
        self.theta_off = off[:-1]
        self.n_params = int(off[-1])
        self._states = (ctypes.c_void_p * B)(*[h._h.value for h in self.handles])
        self._gates = (ctypes.c_void_p * B)(*[g.ctypes.data for g in self.gates])
        self._n_gates = (ctypes.c_int32 * B)(*[g.shape[0] for g in self.gates])
        self._theta_off = (ctypes.c_int64 * B)(*self.theta_off.tolist())
        self._n_theta = (ctypes.c_int32 * B)(*self.n_theta)
        self._H = (PauliSum * B)(*[ps for ps, _ in self._paulis])
        self._seg = None
        del torch

    def theta_flat(self):
        """The problems' parameter vectors concatenated (float64, on the device)."""
        torch = _torch()
        return torch.as_tensor(np.concatenate([p.theta for p in self.problems]),
                               dtype=torch.float64, device=self.device)

    def segment_ids(self, device=None):
        torch = _torch()
        if self._seg is None:
            self._seg = torch.as_tensor(np.repeat(np.arange(len(self.n_theta)), self.n_theta),
                                        device=self.device)
        return self._seg

    def adjoint_gradient(self, theta_flat, energy=None, grad=None):
        """(E[b], flat gradient) of every circuit by Algorithm 1 (qsv_adjoint_gradient_batched)."""
        return self._call(lib().qsv_adjoint_gradient_batched, theta_flat, energy, grad)

    def reference_gradient(self, theta_flat, energy=None, grad=None):
        """The same by Algorithm 2 (qsv_reference_gradient_batched)."""
        return self._call(lib().qsv_reference_gradient_batched, theta_flat, energy, grad)

    def _call(self, fn, theta_flat, energy, grad):
        torch = _torch()
        t = torch.as_tensor(theta_flat, dtype=torch.float64)
        if t.device != self.device:
            t = t.to(self.device)
        t = t.contiguous()
        self._keep = t
        B = len(self.handles)
        e = energy if energy is not None else torch.empty(B, dtype=torch.float64,
                                                         device=self.device)
        g = grad if grad is not None else torch.empty(self.n_params, dtype=torch.float64,
                                                     device=self.device)
        check(fn(B, self._states, self._gates, self._n_gates, t.data_ptr(), self._theta_off,
                 self._n_theta, self._H, e.data_ptr(), g.data_ptr()))
        return e, g

    def sync(self):
        self.handles[0].sync()

    # tile geometries (reg_qubits, threads_log2) of the fused kernels, as qsv_set_fusion accepts
    GEOMETRIES = {"c128": [(2, 8), (3, 8), (4, 8), (2, 9), (3, 9), (2, 6), (3, 6)],
                  "c64": [(2, 8), (3, 8), (4, 8), (2, 9), (3, 9), (4, 9), (2, 6), (3, 6)]}

    def autotune(self, repeats: int = 3):
        """Time the batched gradient in every tile geometry that fits every circuit (and the
        one-wave or automatic mode) and keep the fastest for all handles; returns
        (mode, reg_qubits, threads_log2, ms per batch). The batch runs one common geometry (its
        passes of all circuits launch together)."""
        torch = _torch()
        th = self.theta_flat()
        e = torch.empty(len(self.handles), dtype=torch.float64, device=self.device)
        g = torch.empty(max(self.n_params, 1), dtype=torch.float64, device=self.device)
        n_min = min(h.n for h in self.handles)
        dt = self.handles[0].dtype
        cands = [(-1, 0, 0)] + [(1, r, w) for r, w in self.GEOMETRIES[dt] if r + w <= n_min]
        best = None
        stream = self.handles[0].stream  # the batched call runs on the first handle's stream
        for c in cands:
            for h in self.handles:
                h.set_fusion(*c)
            self.adjoint_gradient(th, e, g)   # builds the schedules
            torch.cuda.synchronize(self.device)
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(stream)
            for _ in range(repeats):
                self.adjoint_gradient(th, e, g)
            b.record(stream)
            b.synchronize()
            ms = a.elapsed_time(b) / repeats
            if best is None or ms < best[3]:
                best = (*c, ms)
        for h in self.handles:
            h.set_fusion(*best[:3])
        return best

    def set_graphs(self, on: bool = True):
        self.handles[0].set_graphs(on)

    def close(self):
        for h in self.handles:
            h.close()
