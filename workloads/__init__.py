"""Seeded synthetic workloads and physics input tables for the DLRA proton
transport solver.  Data generation only; no part of the transport method."""
from .problem import Beam, Grid, Materials, Options, Problem  # noqa: F401
from . import configs, materials  # noqa: F401
