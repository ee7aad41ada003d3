"""Seeded synthetic workloads: kernel factors in CP form and initial concentrations.

This module only builds inputs (factor columns such as i**a, initial vectors,
random seeds).  It holds none of the method's arithmetic and is the one piece
shared by the HIP path's tests/bench and the oracle.
"""
from .workloads import *  # noqa: F401,F403
