"""Seeded synthetic wideband inputs (sky cubes, uv coverages, noise draws).

This package only draws random numbers and lays them out with the shapes of
the paper's simulations (Section 4.1).  It contains none of the imaging
method's arithmetic: the measurement operator is passed in by the caller
(the oracle in tests, the HIP library in the benchmark), so both sides of a
parity check are fed from the same draws.
"""
from .synth import CONFIGS, WorkloadConfig, make_problem_inputs, make_measurements, make_state  # noqa: F401
