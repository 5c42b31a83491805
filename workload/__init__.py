"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package only draws parameters and defines the user-supplied potential
V(r) (and, optionally, a non-local kernel W(r, r')) of the coupled-channel equation (Sec. 2, Eq. cc_schrodinger): the
physics input that an R-matrix solver takes as given.  It holds none of the
solver's arithmetic (no mesh, no kinetic/Bloch matrix, no linear algebra, no
matching).
"""
from .generator import (  # noqa: F401
    CONFIGS, HBAR2_2MU, E2, SystemParams, make_system, energies, batch_systems,
    served_requests, perey_buck_factors, with_perey_buck,
)
