"""Seeded synthetic inputs (Hamiltonian, trial, walkers, fields) shared by the
CPU oracle and the GPU path.  Holds no part of the method's arithmetic."""
from .generator import (SystemSpec, RunSpec, make_hamiltonian, make_trial, make_system,
                        initial_walkers, FieldStream, batching_walker_counts, batching_specs,
                        SMALL, MEDIUM, HEADLINE, BENZENE_SCALE)
