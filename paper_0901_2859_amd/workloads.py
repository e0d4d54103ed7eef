"""Seeded synthetic inputs for series of symmetric tridiagonal systems.

This module only draws numbers: matrix coefficients (a, b), right-hand sides F
and loss weights W.  It holds none of the solver's arithmetic, so both the
CPU oracle (through the tests) and the GPU path can be fed from it.

Matrix convention (statement of the problem, section 2 of the paper): A is
M x M, symmetric tridiagonal, diagonal b[0..M-1], off-diagonal a[0..M-2] with
A[i, i+1] = A[i+1, i] = a[i].  A series of N right-hand sides is stored
RHS-interleaved: F has shape (M, N) and F[i, n] is row i of right-hand side n.

The five workloads follow the shapes of the paper's experiments: a small
diagonally dominant system, 1-D Poisson series (the Fourier-method shape: one
matrix, many right-hand sides), an uneven batch of shifted Poisson matrices
(one matrix per Fourier harmonic), ADI line solves on a smooth random field,
and a random dominant matrix for gradients.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "small", "poisson_series", "uneven_batch", "adi_lines", "gradient_case",
    "random_dominant", "poisson_coeffs",
]


def _rng(seed):
    return np.random.default_rng(np.random.SeedSequence(seed))


def poisson_coeffs(M: int, shift: float = 0.0):
    """Coefficients of the 3-point Dirichlet Laplacian (+ shift on the diagonal)."""
    a = np.full(max(M - 1, 0), -1.0)
    b = np.full(M, 2.0 + shift)
    return a, b


def small(seed: int = 1, M: int = 64, N: int = 16, P: int = 4):
    """Plain method, small: b_i = 4, a_i = 1, F ~ U[-1, 1] in FP64."""
    r = _rng(seed)
    a = np.full(M - 1, 1.0)
    b = np.full(M, 4.0)
    F = r.uniform(-1.0, 1.0, size=(M, N))
    return dict(name="small", a=a, b=b, F=F, P=P, M=M, N=N, dtype="f64")


def _sine_table(M: int):
    # sin(pi * j / (M + 1)) for j = 0 .. 2M+1: one full period of the modes
    j = np.arange(2 * (M + 1), dtype=np.float64)
    return np.sin(np.pi * j / (M + 1))


def poisson_series(seed: int = 2, M: int = 4096, N: int = 4096, P: int = 64,
                   modes: int = 8, noise: float = 1e-3, as_f32: bool = True):
    """1-D Poisson series: b_i = 2, a_i = -1; each RHS is a sum of `modes`
    sine modes sin(pi m i / (M+1)) (m uniform in 1..M, amplitude U[-1, 1])
    plus U[-noise, noise] noise.  Built in FP64, stored as FP32 when `as_f32`
    (the FP32 values are then the definitive input)."""
    r = _rng(seed)
    a, b = poisson_coeffs(M)
    m = r.integers(1, M + 1, size=(N, modes))
    c = r.uniform(-1.0, 1.0, size=(N, modes))
    tab = _sine_table(M)
    period = 2 * (M + 1)
    rows = np.arange(1, M + 1, dtype=np.int64)[:, None]
    F = np.zeros((M, N))
    for k in range(modes):
        idx = (rows * m[None, :, k]) % period
        F += tab[idx] * c[None, :, k]
    F += r.uniform(-noise, noise, size=(M, N))
    if as_f32:
        F = F.astype(np.float32)
    return dict(name="poisson_series", a=a, b=b, F=F, P=P, M=M, N=N,
                dtype="f32" if as_f32 else "f64", modes=m, amps=c)


def uneven_batch(seed: int = 3, K: int = 256, M_lo: int = 128, M_hi: int = 16384,
                 N_hi: int = 2048, c_lo: float = 0.01, c_hi: float = 1.0):
    """Uneven batch: K independent matrices, M_k log-uniform in [M_lo, M_hi],
    b_i = 2 + c_i with c_i ~ U[c_lo, c_hi] per row, a_i = -1; N_k ~ U{1..N_hi};
    F ~ U[-1, 1] stored as FP32.  Each matrix gets its own spawned stream."""
    root = np.random.SeedSequence(seed)
    top = np.random.default_rng(root)
    Ms = np.rint(np.exp(top.uniform(np.log(M_lo), np.log(M_hi), size=K))).astype(np.int64)
    Ns = top.integers(1, N_hi + 1, size=K).astype(np.int64)
    items = []
    for k, ss in enumerate(root.spawn(K)):
        r = np.random.default_rng(ss)
        M, N = int(Ms[k]), int(Ns[k])
        a = np.full(M - 1, -1.0)
        b = 2.0 + r.uniform(c_lo, c_hi, size=M)
        F = r.uniform(-1.0, 1.0, size=(M, N)).astype(np.float32)
        items.append(dict(a=a, b=b, F=F, M=M, N=N))
    return dict(name="uneven_batch", items=items, K=K)


def gaussian_field(seed: int, rows: int, cols: int, corr: float = 64.0):
    """Periodic Gaussian random field with correlation exp(-r^2 / (2 corr^2)),
    made by filtering white noise in Fourier space; unit variance, FP32."""
    import scipy.fft as sfft
    r = _rng(seed)
    w = r.standard_normal((rows, cols), dtype=np.float32)
    W = sfft.rfft2(w, workers=-1)
    ky = np.fft.fftfreq(rows).astype(np.float32)[:, None]
    kx = np.fft.rfftfreq(cols).astype(np.float32)[None, :]
    # the filter's square is the Fourier transform of the correlation function
    filt = np.exp(-(np.pi ** 2) * (corr ** 2) * (kx ** 2 + ky ** 2)).astype(np.float32)
    W *= filt
    f = sfft.irfft2(W, s=(rows, cols), workers=-1).astype(np.float32)
    f /= np.float32(f.std())
    return f


def adi_lines(seed: int = 4, M: int = 8192, N: int = 8192, sigma: float = 0.05,
              corr: float = 64.0, P: int = 128):
    """ADI-shaped line solves: b_i = 2 + sigma, a_i = -1; the N right-hand
    sides are the N grid lines of an M x N smooth Gaussian random field."""
    a, b = poisson_coeffs(M, sigma)
    F = gaussian_field(seed, M, N, corr)
    return dict(name="adi_lines", a=a, b=b, F=F, P=P, M=M, N=N, dtype="f32")


def gradient_case(seed: int = 5, M: int = 2048, N: int = 1024, P: int = 32):
    """Differentiation: b_i = 3 + U[0, 1], a_i ~ U[-1, -0.5], F ~ U[-1, 1]
    (FP32), loss weights W ~ U[-1, 1] (FP64)."""
    r = _rng(seed)
    b = 3.0 + r.uniform(0.0, 1.0, size=M)
    a = r.uniform(-1.0, -0.5, size=M - 1)
    F = r.uniform(-1.0, 1.0, size=(M, N)).astype(np.float32)
    W = r.uniform(-1.0, 1.0, size=(M, N))
    return dict(name="gradient_case", a=a, b=b, F=F, W=W, P=P, M=M, N=N, dtype="f32")


def random_dominant(seed: int, M: int, N: int, strict: float = 0.1,
                    dtype=np.float64, sign_mix: bool = True):
    """Random symmetric tridiagonal with |b_i| >= |a_{i-1}| + |a_i| + strict,
    off-diagonals of mixed sign; F ~ U[-1, 1]."""
    r = _rng(seed)
    a = r.uniform(0.2, 1.0, size=max(M - 1, 0))
    if sign_mix:
        a *= r.choice([-1.0, 1.0], size=a.shape)
    left = np.concatenate([[0.0], np.abs(a)])
    right = np.concatenate([np.abs(a), [0.0]])
    b = (left + right + strict + r.uniform(0.0, 0.5, size=M))
    b *= r.choice([-1.0, 1.0], size=M) if sign_mix else 1.0
    F = r.uniform(-1.0, 1.0, size=(M, N)).astype(dtype)
    return dict(name="random_dominant", a=a, b=b, F=F, M=M, N=N)
