"""MI355X-native MGCNN solver (arXiv 2312.11093): HIP kernels for gfx950 behind a C-ABI
library (include/mgcnn.h), with a thin ctypes binding.

    from paper_2312_11093_amd import Solver
"""
from .mgcnn import GroupSolver, Solver, MGCNNError, lib  # noqa: F401
