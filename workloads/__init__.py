"""Seeded synthetic inputs shared by the oracle-side tests and the HIP-side
tests/bench.

This package holds only problem DATA: domain descriptors, manufactured exact
solutions and seeded random fields.  It contains none of the KFBI method's
arithmetic (no geometry processing, jumps, corrections, grid solves or
Krylov iterations); each side computes its own collocation points, and a
boundary field is evaluated by calling the functions here at whichever points
that side produced.
"""

from .domains import (  # noqa: F401
    domain_c1_heat,
    domain_c2_wave,
    domain_c3_schrodinger,
    domain_c4_instance,
    domain_neumann_wave,
    domain_nls_example,
    grid_coords,
)
from . import manufactured  # noqa: F401
from . import fields  # noqa: F401
