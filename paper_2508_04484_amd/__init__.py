"""MI355X-native dynamical low-rank (DLRA) proton transport.

The compute path is the HIP library libdlra.so (C ABI in include/dlra.h);
`binding` marshals arguments to it, with PyTorch supplying device memory and
the stream.  Build the library with `python -m paper_2508_04484_amd.build`.
"""
from .binding import (BeamSolver, DlraError, Solver, batch_solvers, load, run_batch,  # noqa: F401
                      solve, workspace_size)
