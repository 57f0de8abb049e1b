"""FP64 CPU oracle for the incident-wave hot path (HOS step, modal evaluation
on the intermediate grid, interpolation to cell centres, divergence).

TEST INFRASTRUCTURE ONLY.  Nothing in the product library imports or calls
this package; only the tests, the smoke check and the benchmark's CPU
baseline do.  It shares no code with the HIP path; the only common inputs
are the seeded generators of the `synth` module.

Each function states the passage of the paper (section / equation) it
follows.  The method is a truncated perturbation series iterated by RK4, so
the oracle takes the algorithm's steps in order (no fusion, no blocking),
using numpy's FFT as a library step.  The readings adopted where the paper
is silent are listed in the design notes and in the docstrings.
"""
from .spectral import Grid  # noqa: F401
from . import sea, hos, reconstruct  # noqa: F401
