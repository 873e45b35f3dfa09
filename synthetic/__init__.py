"""Seeded synthetic inputs for the full-space Gauss-Newton KKT solver.

This package only *produces inputs*: velocity models (squared slowness on the
grid), acquisition geometry (source and receiver node indices), weights, and
seeded random complex vectors.  It contains none of the method's arithmetic
(no Helmholtz operator, no PML, no KKT algebra), so both the oracle and the
GPU path may use it without sharing any of the computation they are compared
on.

The paper's experiments use part of the Marmousi model (Section 6), which is
not available here; the seeded layered / faulted / lens models below stand in
for it, with the same kind of structure (layered sediments, dipping faults, a
high-velocity body) and velocities in the paper's range.
"""

from .models import (layered_model, faulted_lens_model, gaussian_smooth,
                     model_pair)
from .configs import CONFIGS, get_config, make_problem_inputs, geometry
from .rand import complex_normal

__all__ = [
    "layered_model", "faulted_lens_model", "gaussian_smooth", "model_pair",
    "CONFIGS", "get_config", "make_problem_inputs", "geometry",
    "complex_normal",
]
