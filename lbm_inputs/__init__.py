"""Seeded synthetic inputs for the two-phase D2Q9 lattice-Boltzmann step.

This package is shared by the GPU library's callers and the CPU oracle's
tests.  It builds geometry (solid masks, cut links with their wall fraction
q of Eq. 6, wall velocities), initial density fields and parameter sets.  It
contains none of the method's arithmetic: no equilibrium, no collision, no
equation of state, no boundary rule.  Randomness comes from a counter-based
splitmix64 generator (``rng.py``).
"""
from .problem import Problem, LINK_DTYPE  # noqa: F401
