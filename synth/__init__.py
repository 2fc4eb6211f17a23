"""Seeded synthetic inputs shared by the oracle-side tests and the GPU path.

This package generates *inputs only*: column layouts, the hydrostatic
background, the vortex initial state and its seeded noise, evaluated at
whatever node coordinates the caller supplies.  It contains none of the
discretisation (no basis, derivative, assembly, projection or time-stepping
arithmetic), so the oracle and the HIP library stay independent.
"""

from . import atmosphere, cases, columns, noise  # noqa: F401
