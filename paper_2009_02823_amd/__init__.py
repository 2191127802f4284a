"""MI355X-native reverse-mode energy gradients for state-vector circuit simulation.

Implements, as hand-written HIP for gfx950 behind the C-ABI of ``include/qsv.h``, the O(P)
gradient of Jones & Gacon (arXiv:2009.02823, Algorithm 1): one forward pass to |psi>,
lambda = H|psi>, then a backward sweep that un-applies every gate from phi and lambda and
accumulates 2 Re <lambda| dU/dtheta |phi> per parameter.

Importing the package loads nothing; ``qsv.lib()`` loads ``libqsv.so`` on first use and raises if
it is missing.
"""
from . import workloads  # noqa: F401

__all__ = ["workloads", "qsv"]
