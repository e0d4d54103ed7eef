"""Application driver: a series of 2-D Poisson problems by the variable
separation (Fourier) method on top of the uneven-batch solver.

The paper's section "Variable separation method": on an N1 x N2 mesh with
steps h1, h2 and zero boundary values, -Delta u = f_n (n = 1..S problems on
the same mesh) is expanded in the eigenfunctions sin(pi l j / N2) of the
difference operator in y; harmonic l then obeys, for every problem n, the
tridiagonal system (eq. SLAU_FFT, here multiplied by -1)

    (2 + d_l) u_i(l) - u_{i-1}(l) - u_{i+1}(l) = h1^2 f_i(l),  i = 1..N1-1,
    d_l = 4 (h1 / h2)^2 sin^2(pi l / (2 N2)),               (eq. series_fft)

one fixed matrix per harmonic with S right-hand sides (eq. poisson_end):
N2-1 series of the kind the library solves, handed to it as one batch.  The
sine transforms along y are FFTs of the odd extension (torch.fft); the
transposes that bring the S problems next to each other (RHS-interleaved
layout per harmonic) and back are the library's tiled strided copies
(tdsolve_strided_copy), the tridiagonal series its batch solve.

Layout: f and u are (S, N1-1, N2-1) device tensors, u[n, i-1, j-1] = u_n at
mesh point (i, j).
"""
from __future__ import annotations

import math
from typing import Optional

import numpy as np

from . import tdsolve as t


def _dst1_view(x):
    """-y of the type-I sine transform along the last axis, as a strided view:
    y_l = sum_j x_j sin(pi l j / (m + 1)) = -Im sum_j x_j exp(-i pi l j /
    (m + 1)), the real FFT of length 2 (m + 1) of x placed at positions
    1..m (one padded copy; x may be any strided view)."""
    import torch
    m = x.shape[-1]
    return torch.fft.rfft(torch.nn.functional.pad(x, (1, m + 1)), dim=-1).imag[..., 1:m + 1]


def dst1(x):
    """Type-I sine transform along the last axis: y_l = sum_j x_j
    sin(pi l j / (m + 1)), l, j = 1..m."""
    return -_dst1_view(x)


class FourierPoisson2D:
    """Series of S Poisson problems -Delta u = f on an N1 x N2 mesh of the
    rectangle [0, N1 h1] x [0, N2 h2], zero Dirichlet boundary values.

    mode: the library's solve mode for the per-harmonic series ("f64",
    "f32_refined", "f32_wide", "f32"); the transforms run in FP64 for "f64"
    and FP32 otherwise.  P: blocks per harmonic matrix (None: the batch
    autotuner's choice for S right-hand sides)."""

    def __init__(self, N1: int, N2: int, S: int, h1: float = None, h2: float = None,
                 mode: str = "f64", P: Optional[int] = None, autotune_cache: bool = True):
        if N1 < 2 or N2 < 2 or S < 1:
            raise ValueError("need N1, N2 >= 2 and S >= 1")
        self.N1, self.N2, self.S = N1, N2, S
        self.h1 = h1 if h1 is not None else 1.0 / N1
        self.h2 = h2 if h2 is not None else 1.0 / N2
        self.mode = mode
        M = N1 - 1
        L = N2 - 1
        ratio = (self.h1 / self.h2) ** 2
        l = np.arange(1, L + 1)
        self.d = 4.0 * ratio * np.sin(np.pi * l / (2 * N2)) ** 2          # eq. series_fft
        a = np.full(M - 1, -1.0)
        self._a = [a] * L
        self._b = [np.full(M, 2.0 + dl) for dl in self.d]
        if P is None:
            Ps, _ = t.batch_autotune(self._a, self._b, [S] * L, mode, cache=autotune_cache)
        else:
            Ps = [P] * L
        self.P = Ps
        self.plan = t.BatchPlan(self._a, self._b, Ps)

    def solve(self, f, stream=None):
        """u for the S right-hand sides f, shape (S, N1-1, N2-1).  With
        `stream` (a torch.cuda.Stream), every step (the transforms, the
        copies and the batch solve) runs on it, in order."""
        import contextlib

        import torch
        S, M, L = self.S, self.N1 - 1, self.N2 - 1
        if tuple(f.shape) != (S, M, L):
            raise ValueError(f"f must have shape {(S, M, L)}")
        ctx = torch.cuda.stream(stream) if stream is not None else contextlib.nullcontext()
        with ctx:
            return self._solve(f, None)

    def _solve(self, f, stream):
        import torch
        S, M, L = self.S, self.N1 - 1, self.N2 - 1
        wdt = torch.float64 if self.mode == "f64" else torch.float32
        # harmonics of f along y, scaled to the right-hand side h1^2 f~(l) and
        # written straight into the RHS-interleaved layout (l, i, S) by one
        # strided multiply (scale and transpose in one pass)
        scale = self.h1 ** 2 * 2.0 / self.N2
        rhs = torch.empty((L, M, S), dtype=wdt, device=f.device)
        t.strided_copy(rhs.permute(2, 1, 0), _dst1_view(f.to(wdt)), -scale, stream=stream)
        X = self.plan.solve_stacked(rhs, mode=self.mode, stream=stream)
        # back to mesh values in y: X (l, i, S) into the padded odd-extension
        # rows of the inverse transform, again by one tiled transposing copy
        Y = torch.zeros((S, M, 2 * (L + 1)), dtype=X.dtype, device=X.device)
        t.strided_copy(Y[..., 1:L + 1], X.permute(2, 1, 0), 1.0, stream=stream)
        return -torch.fft.rfft(Y, dim=-1).imag[..., 1:L + 1]

    @staticmethod
    def eigen_rhs(N1, N2, k, l, h1=None, h2=None):
        """(f, u) of one discrete eigenfunction sin(pi k i/N1) sin(pi l j/N2):
        the exact discrete solution is f divided by its eigenvalue."""
        h1 = h1 if h1 is not None else 1.0 / N1
        h2 = h2 if h2 is not None else 1.0 / N2
        i = np.arange(1, N1)[:, None]
        j = np.arange(1, N2)[None, :]
        phi = np.sin(math.pi * k * i / N1) * np.sin(math.pi * l * j / N2)
        lam = 4 / h1 ** 2 * math.sin(math.pi * k / (2 * N1)) ** 2 + \
            4 / h2 ** 2 * math.sin(math.pi * l / (2 * N2)) ** 2
        return phi, phi / lam
