"""Seeded synthetic inputs shared by the oracle and the GPU library's tests.

Holds the counter-based input streams and the upwind discretisations that
produce the linear systems A x = b.  It holds none of the solver's arithmetic.
"""
from . import rng, fv, dg, fd, workloads  # noqa: F401
from .fv import FVProblem, fv_advection, inflow_values  # noqa: F401
from .dg import DGProblem, dg_advection  # noqa: F401
from .fd import FDProblem, fd_advection  # noqa: F401
