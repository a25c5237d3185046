"""Seeded synthetic particle loads shared by the tests, the bench and the oracle checks.

This package draws random numbers and shapes them into initial conditions; it holds
none of the particle-mesh step's arithmetic (no deposit, no Poisson kernel, no
interpolation, no integrator, no codec), so the HIP path and the oracle can both be
fed from it without sharing any of the method.
"""

from .ic import (  # noqa: F401
    CONFIGS,
    PMWorkload,
    SpeciesLoad,
    cdm_zeldovich,
    fd_speed_table,
    make_workload,
    neutrinos_fermi_dirac,
)
