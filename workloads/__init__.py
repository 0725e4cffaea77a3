"""Seeded synthetic inputs for the density-matrix solver.

This package only draws inputs (Hamiltonians, perturbations, weights and
the synthetic charge model, the inputs of the canonical integrator).  It holds none of the solver's arithmetic, so
both the FP64 oracle and the GPU path can take their inputs from here
without sharing any code with each other.
"""

from .hamiltonians import (  # noqa: F401
    random_orthogonal_hamiltonian,
    water_box_positions,
    water_box_hamiltonian,
    water_box_length,
    symmetric_normal,
    trajectory_perturbation,
    trajectory_hamiltonian,
    pad_matrix,
    WATER_ONSITE,
)
from .charges import (  # noqa: F401
    water_charge_model,
    random_charges,
    charge_shifted_hamiltonian,
    WATER_VALENCE,
)
from .canonical import (  # noqa: F401
    AMU,
    KB_EV,
    morse_energy,
    morse_force,
    laplace_unit,
    canonical_noise,
    water_atom_masses,
)
