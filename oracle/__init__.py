"""FP64 CPU oracle of the coupled multi-phase-field / lattice-Boltzmann step (arXiv:1902.10432).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the CPU-baseline
leg of the benchmark; never by the GPU library or its Python binding.
"""
from .oracle import Oracle, build, library_path, lattice_of  # noqa: F401
