"""Seeded synthetic inputs for the G1-G2 propagator.

This package only draws random numbers and builds model inputs (one-particle
Hamiltonians, pair interactions, initial density matrices and drive
parameters).  It contains none of the method's arithmetic, so both the CPU
oracle (tests) and the GPU library's callers (tests, benchmark) can use it.
"""
from .systems import *  # noqa: F401,F403
