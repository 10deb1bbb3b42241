"""MI355X (gfx950) SPH particle update: cell-linked-list neighbour search,
WCSPH sweeps with surface tension and a predictor-corrector step, in HIP,
behind the C-ABI of include/sph.h.

``Simulation`` is a thin ctypes handle on that library; PyTorch only provides
device memory and the stream. ``closure`` holds the learned curvature closure's
trainer handle, training data and shipped weights; ``train_closure`` trains and
evaluates it.
"""
from . import native  # noqa: F401
from .sim import Simulation, autotune  # noqa: F401

__all__ = ["Simulation", "autotune", "native"]
