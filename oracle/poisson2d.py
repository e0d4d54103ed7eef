"""CPU ORACLE -- test infrastructure only: the 2-D Poisson problem of the
paper's section on the variable separation method, solved directly.

-Delta u = f on an N1 x N2 mesh (steps h1, h2) with zero boundary values,
the standard 5-point difference operators (eq. operator2); unknowns u[i-1,
j-1] for i = 1..N1-1, j = 1..N2-1.  The discrete operator is assembled as a
sparse matrix (Kronecker sums of the 1-D second differences) and solved by
scipy's sparse LU -- the plain definition of the discrete solution, with no
transform and no tridiagonal series.
"""
from __future__ import annotations

import numpy as np


def laplacian(N1: int, N2: int, h1: float, h2: float):
    """Sparse matrix of -Delta_h on the interior points, row-major (i, j)."""
    import scipy.sparse as sp
    M, L = N1 - 1, N2 - 1
    T1 = sp.diags([-np.ones(M - 1), 2 * np.ones(M), -np.ones(M - 1)], [-1, 0, 1])
    T2 = sp.diags([-np.ones(L - 1), 2 * np.ones(L), -np.ones(L - 1)], [-1, 0, 1])
    return (sp.kron(T1, sp.identity(L)) / h1 ** 2 + sp.kron(sp.identity(M), T2) / h2 ** 2).tocsc()


def solve_direct(f, h1: float, h2: float):
    """u with -Delta_h u = f for one (N1-1, N2-1) array or a stack (S, N1-1, N2-1)."""
    from scipy.sparse.linalg import splu
    f = np.asarray(f, dtype=np.float64)
    single = f.ndim == 2
    fs = f[None] if single else f
    S, M, L = fs.shape
    lu = splu(laplacian(M + 1, L + 1, h1, h2))
    u = np.stack([lu.solve(fs[s].reshape(-1)).reshape(M, L) for s in range(S)])
    return u[0] if single else u
