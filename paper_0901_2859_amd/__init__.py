"""tdsolve for MI355X: series of symmetric tridiagonal systems A X_n = F_n by
the parallel sweep method (Terekhov, arXiv:0901.2859), hand-written HIP
kernels for gfx950 behind a C ABI (include/tdsolve.h).

Importing the package loads nothing; ``paper_0901_2859_amd.tdsolve`` loads
the shared library on first use.
"""
__all__ = ["tdsolve", "workloads"]
