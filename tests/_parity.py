"""Parity gates shared by the GPU tests: the HIP path against the CPU oracle.

Every step of the method is exact in exact arithmetic (Lemma 1, Lemma 2,
Theorem 2), so a GPU solution and the oracle's differ by rounding only.  A
first-order error model of the two gives, per right-hand side n (column of
the [M][N] arrays), with u = 2^-53:

* the method's interface values are dot products of F with rows G_k of
  A^{-1} (eq. beta_symn) chained through the transfer factors (eq. theor_2):
  their error is a multiple of u * max_k sum_i |G_k(i)| |F_i|, the
  interface condition number cs_n (times |X_n|_inf);
* a block sweep (Lemma 1) and the oracle's sweep of the whole matrix are
  backward stable on these diagonally dominant matrices, (T + dT) x = f with
  |dT| a small multiple of u |T|; their forward error is then a multiple of
  u * (|T^{-1}| |T| |x|)_i <= u * (<A>^{-1} |A| |x|)_i, where <A> (|b| on the
  diagonal, -|a| off it) bounds |A^{-1}| and every |T_j^{-1}| entrywise for
  these H-matrices: the componentwise condition number co_n (times |X_n|_inf);
* each block sweep accumulates over its t rows.

Hence the gate  e_n = |X_n - X_or,n|_inf / |X_or,n|_inf
                    <= C u (cs_n + co_n + t),   C = 2.
The worst-case first-order constants are larger (t + 2P + 3 for the
interface values, about twice the LU backward-error constant for the two
sweeps); rounding errors of long sums behave like random walks, and the
largest ratio e_n / (u (cs_n + co_n)) measured over the parity workloads is
0.29 (the 4096 x 4096 Poisson series), so C = 2 keeps the bound within about
an order of magnitude of what the method shows.

The residual gates read the accuracy target, "within 1e-10 relative
residual of the FP64 oracle", with r2 = |F - A X|_2 / |F|_2 computed on the
host by the oracle's pinned residual routine (oracle.method.residual_columns)
for both solutions: per column r2_n <= r2_or,n + 1e-10, and over the series
max_n r2_n <= R_GATE max_n r2_or,n, R_GATE = 2 (equal residual: the worst
column of the GPU solution within a small factor of the oracle's worst;
1.28 is the largest factor measured over the parity workloads).

Each gate records its largest ratio (e / tol, r2 / r2_or and the series
maxima) on stdout and, when TDS_PARITY_LOG names a file, as one JSON line.
"""
import json
import os

import numpy as np

import oracle
from oracle import method

U = 2.0 ** -53
C_GATE = 2.0
R_GATE = 2.0


def col_err(X, ref):
    X = np.asarray(X, dtype=np.float64)
    return np.max(np.abs(X - ref), axis=0) / np.maximum(np.max(np.abs(ref), axis=0), 1e-300)


def _abs_times(lower, diag, upper, X):
    """|A| |X| for the tridiagonal A (lower[i] = A[i+1][i], upper[i] = A[i][i+1])."""
    Y = np.abs(diag)[:, None] * np.abs(X)
    if len(diag) > 1:
        Y[:-1] += np.abs(upper)[:, None] * np.abs(X[1:])
        Y[1:] += np.abs(lower)[:, None] * np.abs(X[:-1])
    return Y


def conditions(a, b, F, ref, P, lower=None):
    """(cs_n, co_n) of the module docstring.  a: the super-diagonal
    (A[i][i+1]); lower: the sub-diagonal when A is not symmetric."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    F = np.asarray(F, dtype=np.float64)
    M = len(b)
    lo = a if lower is None else np.asarray(lower, dtype=np.float64)
    xin = np.maximum(np.max(np.abs(ref), axis=0), 1e-300)
    if P >= 2:
        _, s = method.partition(M, P)
        if lower is None:
            G = method.green_rows(a, b, s[1:P])              # columns = rows of A^{-1}
        else:
            A = np.diag(b) + np.diag(a, 1) + np.diag(lo, -1)
            G = np.linalg.inv(A)[s[1:P], :].T
        cs = (np.abs(G).T @ np.abs(F)).max(axis=0) / xin
    else:
        cs = np.zeros(F.shape[1])
    Y = _abs_times(lo, b, a, ref)
    if lower is None:
        Z = oracle.thomas(-np.abs(a), np.abs(b), Y)
    else:
        low = np.concatenate([[0.0], -np.abs(lo)])
        upp = np.concatenate([-np.abs(a), [0.0]])
        Z = np.stack([oracle.tridiag_general(low, np.abs(b), upp, Y[:, n])
                      for n in range(Y.shape[1])], 1)
    co = np.max(Z, axis=0) / xin
    assert np.all(np.isfinite(co)) and np.all(co >= 1.0 - 1e-12), "comparison matrix not an M-matrix"
    return cs, co


def tol64(a, b, F, ref, P, lower=None):
    """Per-column forward-error bound C u (cs_n + co_n + t)."""
    M = len(b)
    t = int(np.ceil(M / max(P, 1)))
    cs, co = conditions(a, b, F, ref, P, lower)
    return C_GATE * U * (cs + co + t)


def record(what, **kv):
    line = {"what": what, **{k: (float(v) if v is not None else None) for k, v in kv.items()}}
    print("parity " + json.dumps(line), flush=True)
    path = os.environ.get("TDS_PARITY_LOG")
    if path:
        with open(path, "a") as f:
            f.write(json.dumps(line) + "\n")


def check(X, ref, tol, what):
    """Forward-error gate e_n <= tol_n on every column."""
    e = col_err(X, ref)
    record(what, max_e_over_tol=float(np.max(e / tol)), e_max=float(e.max()))
    bad = np.nonzero(e > tol)[0]
    assert bad.size == 0, f"{what}: columns {bad[:5]} e={e[bad[:5]]} tol={tol[bad[:5]]}"
    return e


def check_residual(a, b, F, X, ref, what, lower=None):
    """Residual gate r2_n <= r2_or,n + 1e-10 on every column, both residuals
    from the oracle's pinned routine on the host."""
    if lower is not None:
        raise NotImplementedError("residual gate of symmetric plans only")
    r2 = method.residual_columns(a, b, F, X)["r2"]
    r2_or = method.residual_columns(a, b, F, ref)["r2"]
    record(what, max_r2_over_r2or=float(np.max(r2 / np.maximum(r2_or, 1e-300))),
           r2_max=float(r2.max()), r2_or_max=float(r2_or.max()),
           series_r2_over_r2or=float(r2.max() / max(r2_or.max(), 1e-300)))
    bad = np.nonzero(r2 > r2_or + 1e-10)[0]
    assert bad.size == 0, f"{what}: columns {bad[:5]} r2={r2[bad[:5]]} r2_or={r2_or[bad[:5]]}"
    assert r2.max() <= R_GATE * r2_or.max(), f"{what}: series r2 {r2.max()} vs oracle {r2_or.max()}"
    return r2, r2_or
