"""MI355X (gfx950) imaginary-time Schroedinger eigensolver (arXiv:2006.16935 method).

The hot path (transforms, kinetic multiply, update, reductions, projections,
Gram-Schmidt) runs in the HIP library ``libitse.so`` behind the C ABI of
``include/itse.h``; this package is its Python binding.  Importing it does not
touch the GPU; constructing a Lattice requires the built library and a GPU.
"""
from ._lib import (CENTER_CELL, CENTER_ORIGIN, FP32, FP64, KIN_FDTD, KIN_NR_CONT, KIN_NR_LAT,
                   KIN_REL_CONT, KIN_REL_LAT, MAX_STATES, ItseError, load)
from .lattice import (Batch, Lattice, Server, autotune, autotune_batch, make_opts, schedule, schedule_variants,
                      set_schedule)
from .solver import SnapshotResult, SolveResult, run_snapshot_overlap, run_to_convergence, solve

__all__ = ["Lattice", "Batch", "Server", "solve", "run_to_convergence", "SolveResult", "run_snapshot_overlap",
           "SnapshotResult", "autotune", "autotune_batch",
           "schedule", "schedule_variants", "set_schedule", "make_opts", "load", "ItseError", "KIN_FDTD", "KIN_NR_CONT", "KIN_NR_LAT",
           "KIN_REL_LAT", "KIN_REL_CONT", "FP32", "FP64", "CENTER_CELL", "CENTER_ORIGIN",
           "MAX_STATES"]
