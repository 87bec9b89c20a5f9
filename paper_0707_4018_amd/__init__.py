"""MI355X (gfx950) adaptive multigrid solver for the Wilson-Dirac equation D(U) psi = chi.

Python binding of libamg (ctypes).  PyTorch provides device memory and
streams; every step of the solve runs in the library's HIP kernels.  The
binding only marshals arguments: it raises if the library is missing or a
call fails, and never computes anything itself.

Method: Brannick, Brower, Clark, Osborn, Rebbi, "Adaptive Multigrid Algorithm
for Lattice QCD", arXiv:0707.4018.
"""
from .binding import (  # noqa: F401
    AMGError, Batch, Cnn, Gauge, MGParams, NormalInfo, NormalMG, NormalParams, Solver, SolveInfo, F32, F64,
    lib_path, load_library,
    use_torch_allocator,
)
