"""Application driver: a series of 2-D Poisson problems by the alternating
direction (Peaceman-Rachford) method on top of the series solver.

The paper's section "Alternating Direction Method": -Delta u = f on an
N1 x N2 mesh with zero boundary values is the steady state of
u_t = Delta u + f; with Lambda = Lambda_1 + Lambda_2 (eq. operator2) each
iteration takes two half steps (eq. adi_iter, adi_iter2) with a parameter
omega_k = 1 / tau_k,

    (omega_k - Lambda_1) v = (omega_k + Lambda_2) u + f      (lines along x)
    (omega_k - Lambda_2) u = (omega_k + Lambda_1) v + f      (lines along y)

and the parameters repeat with a period n0 (eq. ocenka1:
n0 = 0.2 ln(4N/pi) ln(4/eps) for a square mesh).  For a fixed k every line
of a half step solves the same tridiagonal matrix
h_a^2 omega_k + 2 on the diagonal, -1 off it (the matrices C^(1), C^(2)
of the paper, negated), so a half step is one series solve of the library
and the preliminary step prepares only 2 n0 matrices.

Reading taken here: the paper leaves the parameter set to the literature;
this driver uses geometrically spaced parameters between the extreme
eigenvalues delta, Delta of -Lambda_a (omega_k = delta (Delta/delta)^((2k-1)
/ (2 n0)), the Wachspress-type set) with the paper's n0, and the sign
convention -Delta u = f throughout.

Layout: u and f are (S, N1-1, N2-1) device tensors for S problems on the
same mesh; the half steps solve the lines of all S problems together (S (N2-1)
right-hand sides along x, S (N1-1) along y), the y half step on a transposed
copy.  Right-hand sides and transposes are torch operations; the line solves
run in the library's kernels.
"""
from __future__ import annotations

import math
from typing import Optional

import numpy as np

from . import tdsolve as t


def n0_iterations(N: int, eps: float) -> int:
    """The paper's iteration count per parameter cycle (eq. ocenka1)."""
    return max(1, int(math.ceil(0.2 * math.log(4 * N / math.pi) * math.log(4 / eps))))


class ADIPoisson2D:
    def __init__(self, N1: int, N2: int, S: int, h1: float = None, h2: float = None,
                 eps: float = 1e-6, mode: str = "f64", P: Optional[int] = None):
        if N1 < 3 or N2 < 3 or S < 1:
            raise ValueError("need N1, N2 >= 3 and S >= 1")
        self.N1, self.N2, self.S = N1, N2, S
        self.h1 = h1 if h1 is not None else 1.0 / N1
        self.h2 = h2 if h2 is not None else 1.0 / N2
        self.mode = mode
        # spectrum of -Lambda_a: 4/h^2 sin^2(pi l / 2N), l = 1..N-1
        lo = min(4 / self.h1 ** 2 * math.sin(math.pi / (2 * N1)) ** 2,
                 4 / self.h2 ** 2 * math.sin(math.pi / (2 * N2)) ** 2)
        hi = max(4 / self.h1 ** 2 * math.cos(math.pi / (2 * N1)) ** 2,
                 4 / self.h2 ** 2 * math.cos(math.pi / (2 * N2)) ** 2)
        self.n0 = n0_iterations(max(N1, N2), eps)
        k = np.arange(1, self.n0 + 1)
        self.omega = lo * (hi / lo) ** ((2 * k - 1) / (2 * self.n0))
        M1, M2 = N1 - 1, N2 - 1
        self.plans_x = [t.Plan(np.full(M1 - 1, -1.0), np.full(M1, 2.0 + self.h1 ** 2 * w), P)
                        for w in self.omega]
        self.plans_y = [t.Plan(np.full(M2 - 1, -1.0), np.full(M2, 2.0 + self.h2 ** 2 * w), P)
                        for w in self.omega]

    @staticmethod
    def _lap(u, axis: int, h: float):
        """Second difference along `axis` with zero boundary values, / h^2."""
        import torch
        d = -2.0 * u
        n = u.shape[axis]
        d.narrow(axis, 1, n - 1).add_(u.narrow(axis, 0, n - 1))
        d.narrow(axis, 0, n - 1).add_(u.narrow(axis, 1, n - 1))
        return d / (h * h)

    def _solve_lines(self, plan, rhs_lines):
        """rhs_lines: (M, R) lines of one direction; the library's series solve."""
        import torch
        F = rhs_lines if self.mode == "f64" else rhs_lines.float()
        X = plan.solve(F.contiguous(), mode=self.mode)
        return X if X.dtype == torch.float64 else X.double()

    def step(self, u, f, k: int):
        """One Peaceman-Rachford iteration with parameter omega_k."""
        S, M1, M2 = u.shape
        w = float(self.omega[k])
        # half step along x: (omega - Lambda_1) v = (omega + Lambda_2) u + f
        r = w * u + self._lap(u, 2, self.h2) + f
        lines = (self.h1 ** 2 * r).permute(1, 0, 2).reshape(M1, S * M2)
        v = self._solve_lines(self.plans_x[k], lines).reshape(M1, S, M2).permute(1, 0, 2)
        # half step along y: (omega - Lambda_2) u = (omega + Lambda_1) v + f
        r = w * v + self._lap(v, 1, self.h1) + f
        lines = (self.h2 ** 2 * r).permute(2, 0, 1).reshape(M2, S * M1)
        return self._solve_lines(self.plans_y[k], lines).reshape(M2, S, M1).permute(1, 2, 0)

    def solve(self, f, cycles: int = 1, u0=None):
        """u after `cycles` full parameter cycles (n0 iterations each) from u0
        (default zero); f, u: (S, N1-1, N2-1) FP64 device tensors."""
        import torch
        u = torch.zeros_like(f) if u0 is None else u0.clone()
        for _ in range(cycles):
            for k in range(self.n0):
                u = self.step(u, f, k).contiguous()
        return u
