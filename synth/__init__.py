"""Seeded synthetic inputs for the NNP workloads (gas-phase clusters, molecule
batches and periodic boxes).

This module draws inputs only: atom positions, species, masses, initial
velocities, molecule boundaries and network weights.  It holds none of the
method's arithmetic (no descriptors, no network evaluation, no forces, no
integration) so that the CPU oracle and the HIP path can both consume the
same inputs without sharing any code that computes results.
"""

from .generate import (  # noqa: F401
    ELEMENTS,
    MASSES_AMU,
    WEIGHT_SHAPES,
    N_WEIGHTS_PER_ELEMENT,
    N_WEIGHTS,
    System,
    composition_counts,
    rsa_cube,
    rsa_ball,
    rsa_periodic,
    box_edge,
    ball_radius,
    maxwell_boltzmann,
    xavier_weights,
    molecule_sizes,
    make_config,
    CONFIGS,
)
