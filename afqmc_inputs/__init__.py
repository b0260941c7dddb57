"""Seeded synthetic inputs (Hamiltonian, trial, walkers, fields) shared by the
CPU oracle and the GPU path.  Holds no part of the method's arithmetic."""
from .generator import (SystemSpec, RunSpec, make_hamiltonian, make_trial, make_system,
                        make_system_without_chol, make_chol_counter, chol_factors, splitmix64_outputs,
                        make_trial_from_h, initial_walkers, FieldStream, batching_walker_counts,
                        batching_specs, SMALL, MEDIUM, HEADLINE, BENZENE_SCALE)
