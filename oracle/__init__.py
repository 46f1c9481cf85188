"""Plain CPU FP64 oracle for the GLR prior step and its data-fidelity loop.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only the tests, the smoke check and the CPU-baseline leg
of the benchmark use it.  It shares no code with the HIP library; the only
common dependency is the seeded input generator module ``synth``.

Every function follows a passage of the paper (arXiv 2301.03047), cited in its
docstring; where the paper is silent the reading taken is stated there too.
Arithmetic is NumPy FP64 unless a step fixes another precision (the detector
quantiser works in IEEE FP32, emulated exactly with ``np.float32``).
"""
from . import operators, detector, matching, lowrank, aggregate, prior, reconstruct, metrics, edges

__all__ = ["operators", "detector", "matching", "lowrank", "aggregate", "prior",
           "reconstruct", "metrics", "edges"]
