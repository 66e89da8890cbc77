"""Seeded synthetic tight-binding workloads.

This package only builds input matrices (Hamiltonians, perturbations and the
per-system parameters of a batch).  It holds none of the method's arithmetic,
so both the FP64 CPU oracle and the GPU library can be fed from it without
sharing any computation.
"""
from .tb import (chain_1d, dimer_chain, cubic_lattice, banded, lattice_dipoles, grid_dipoles,
                 batched_systems, config, CONFIGS, overlap, inverse_factor)

__all__ = ["chain_1d", "dimer_chain", "cubic_lattice", "banded", "lattice_dipoles", "grid_dipoles",
           "batched_systems", "config", "CONFIGS", "overlap", "inverse_factor"]
