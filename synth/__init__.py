"""Seeded synthetic inputs shared by the oracle and the HIP path.

This package draws random numbers and slices them into the arrays a
closed-shell polarization-propagator calculation consumes (orbital energies,
density-fitted three-index tensors, dipole integrals).  It performs none of
the method's arithmetic: no integrals are contracted, no amplitudes are
formed, nothing is solved.
"""
from .gen import System, gen, gen_request, CONFIGS, WINDOWS, REQUEST_SEED_BASE

__all__ = ["System", "gen", "gen_request", "CONFIGS", "WINDOWS", "REQUEST_SEED_BASE"]
