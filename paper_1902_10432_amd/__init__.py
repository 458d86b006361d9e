"""MI355X-native coupled multi-phase-field / lattice-Boltzmann step (arXiv:1902.10432).

The step runs as hand-written HIP kernels for gfx950 behind the C-ABI of ``include/pf_lbm.h``
(``libpflbm.so``); :mod:`.binding` mirrors it one to one and :class:`.simulation.Simulation`
owns a handle with a PyTorch-allocated workspace.
"""
from .binding import EXPORTED, LIB_PATH, load_library  # noqa: F401


def Simulation(*args, **kwargs):  # noqa: N802 - class factory, imports torch lazily
    from .simulation import Simulation as _S
    return _S(*args, **kwargs)
