"""Seeded synthetic workloads shared by the tests, the benchmark and the oracle.

This package holds the *problem definitions* only: the detector error models
(H, p, l) of the codes and noise models decoded here, their canonical
detector/mechanism numbering, and the seeded Bernoulli samplers that draw error
patterns and turn them into syndromes.  It contains none of the decoder's
arithmetic (no tensor network, no contraction, no truncation), so both the
oracle and the GPU path may consume what it produces without sharing code.
"""

from .codes import (  # noqa: F401
    Dem,
    surface3d_point,
    surface3d_faces,
    surface3d_depolarizing,
    surface3d_loop,
    rotated_phenom,
    repetition_line,
    surface2d_bitflip,
    five_qubit_stabilizers,
)
from .sample import sample_syndromes, sample_pauli, config_workload, CONFIG_SEED_BASE  # noqa: F401
