"""torch.autograd integration: the energy E(theta) of a circuit under a Pauli-sum Hamiltonian as a
differentiable function whose backward is the reverse-mode gradient of Algorithm 1.

The forward call runs the adjoint sweep once when theta requires a gradient (one forward pass,
one H application and one reverse sweep give both E and dE/dtheta) and keeps the gradient for
backward; otherwise it computes E alone. backward scales the stored gradient by the incoming
gradient of E. Every step runs in the HIP library; theta must be a float64 tensor on the GPU of
the handle.
"""
from __future__ import annotations

import numpy as np
import torch

from . import qsv


class QsvEnergy(torch.autograd.Function):
    """E = QsvEnergy.apply(theta, sim, gates, codes, coeffs) with sim a qsv.StateVector whose
    state is the input |in> of the circuit (left unchanged)."""

    @staticmethod
    def forward(ctx, theta, sim, gates, codes, coeffs):
        if theta.requires_grad:
            e, g = sim.adjoint_gradient(gates, theta.detach(), codes, coeffs)
            ctx.save_for_backward(g)
        else:
            e = sim.energy(gates, theta, codes, coeffs)
        return e.reshape(())

    @staticmethod
    def backward(ctx, grad_out):
        (g,) = ctx.saved_tensors
        return grad_out * g, None, None, None, None


class AdjointEnergy(torch.nn.Module):
    """A circuit and Hamiltonian bound to a device handle; calling it with theta returns E.

    >>> f = AdjointEnergy(n, gates, codes, coeffs)          # doctest: +SKIP
    >>> e = f(theta); e.backward()                           # theta.grad = dE/dtheta
    """

    def __init__(self, n_qubits, gates, codes, coeffs, dtype="c128", device=None):
        super().__init__()
        self.sim = qsv.StateVector(n_qubits, dtype, device=device)
        self.gates = qsv.as_gate_table(gates)
        self.codes = np.ascontiguousarray(np.asarray(codes, dtype=np.uint8))
        self.coeffs = np.ascontiguousarray(np.asarray(coeffs, dtype=np.float64))

    def forward(self, theta):
        return QsvEnergy.apply(theta, self.sim, self.gates, self.codes, self.coeffs)


class QsvEnergyBatch(torch.autograd.Function):
    """Energies of several independent circuits from one flat parameter vector.

    E = QsvEnergyBatch.apply(theta_flat, batch) with batch a qsv.Batch; returns the (B,) energies;
    backward maps the (B,) incoming gradient onto theta_flat segment by segment."""

    @staticmethod
    def forward(ctx, theta_flat, batch):
        e, g = batch.adjoint_gradient(theta_flat.detach())
        ctx.save_for_backward(g)
        ctx.seg = batch.segment_ids(theta_flat.device)
        return e

    @staticmethod
    def backward(ctx, grad_out):
        (g,) = ctx.saved_tensors
        return grad_out[ctx.seg] * g, None
