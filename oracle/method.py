"""CPU ORACLE (test infrastructure only): the paper's method, step by step.

FP64 NumPy, written from the paper's text in its order and notation, with
0-based row indices.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may use it; the GPU library shares no code with it.

Readings of the paper taken here (the paper is garbled or silent on them):

* Data decomposition (section 2): P contiguous blocks of sizes t_j >= 2 that
  tile rows 0..M-1; when P does not divide M the first M mod P blocks get one
  extra row.  Block j starts at row s_j (s_0 = 0, s_P = M).
* Lemma 1 needs the first and last element of each block system; we take one
  interface row per block boundary: the separators are s_1 .. s_{P-1}, the
  first rows of blocks 1..P-1 (the set Omega of Theorem 2 excludes rows 1
  and n).  Block j's identity-bordered system of Lemma 1 spans rows
  s_j .. s_{j+1} (both separators known), block 0 keeps row 0 of A and block
  P-1 keeps row M-1 of A.
* Segment j (eq. define_vectorF) is rows s_j .. s_{j+1}-1, i.e. block j.
  beta^R_j uses the row of A^{-1} at its right separator s_{j+1} (j <= P-2),
  beta^L_j the row at its left separator s_j (j >= 1)   (eq. beta_symn).
* Theorem 2 (eq. theor_2), separator k = 1..P-1:
      x(s_k) = sum_{j<k}  beta^R_j Z^R_{s_{j+1}}(s_k)
             + sum_{j>=k} beta^L_j Z^L_{s_j}(s_k)
  (the second sum uses Z^L at the segment's left separator, as the proof
  defines it; the case split of eq. AL is read with this orientation).
* Theorem 3 (dichotomy): between known separators k1 < i < k2 we carry the
  left and right partial sums SR, SL (not x alone):
      SR_i = SR_{k1} Z^R_{s_k1}(s_i) + sum_{j=k1}^{i-1} beta^R_j Z^R_{s_{j+1}}(s_i)
      SL_i = SL_{k2} Z^L_{s_k2}(s_i) + sum_{j=i}^{k2-1} beta^L_j Z^L_{s_j}(s_i)
      x(s_i) = SR_i + SL_i,
  with SR = 0 at the left end of the domain and SL = 0 at the right end.
"""
from __future__ import annotations

import math

import numpy as np

from . import core


# ---------------------------------------------------------------- decomposition
def partition(M: int, P: int):
    """Block sizes t_j and starts s_j (data decomposition, section 2)."""
    if P < 1 or M < 2 * P and P > 1:
        raise ValueError("need 1 <= P and blocks of at least 2 rows")
    base, extra = divmod(M, P)
    t = np.array([base + (1 if j < extra else 0) for j in range(P)], dtype=np.int64)
    s = np.concatenate([[0], np.cumsum(t)])
    return t, s


def separators(M: int, P: int):
    """Interface rows s_1..s_{P-1}."""
    _, s = partition(M, P)
    return s[1:P].copy()


def dense(a, b):
    """The matrix of section 2 as a dense array (for tiny pins only)."""
    M = len(b)
    A = np.diag(np.asarray(b, dtype=np.float64))
    if M > 1:
        A += np.diag(a, 1) + np.diag(a, -1)
    return A


# ------------------------------------------------------ preliminary step (Alg. 3, step 1)
def green_rows(a, b, ks):
    """Lemma 2 / eq. green_v: G_k solves A G_k = e_k; for symmetric A it is
    both row and column k of A^{-1}.  Returns an (M, len(ks)) array."""
    M = len(b)
    E = np.zeros((M, len(ks)))
    for m, k in enumerate(ks):
        E[k, m] = 1.0
    return core.thomas(a, b, E)


def z_right(a, b, k):
    """Z^R_k of eq. z_vector: B^R_k Z = e^R over rows k..M-1, where B^R_k has
    an identity first row and rows k+1..M-1 of A.  Returned on all M rows
    (NaN above k)."""
    M = len(b)
    n = M - k
    lower = np.zeros(n)
    diag = np.zeros(n)
    upper = np.zeros(n)
    diag[0] = 1.0
    for r in range(1, n):
        i = k + r
        lower[r] = a[i - 1]
        diag[r] = b[i]
        upper[r] = a[i] if i < M - 1 else 0.0
    rhs = np.zeros(n)
    rhs[0] = 1.0
    z = np.full(M, np.nan)
    z[k:] = core.tridiag_general(lower, diag, upper, rhs)
    return z


def z_left(a, b, k):
    """Z^L_k of eq. z_vector: B^L_k Z = e^L over rows 0..k, where B^L_k has
    rows 0..k-1 of A and an identity last row.  NaN below k."""
    M = len(b)
    n = k + 1
    lower = np.zeros(n)
    diag = np.zeros(n)
    upper = np.zeros(n)
    for i in range(k):
        lower[i] = a[i - 1] if i > 0 else 0.0
        diag[i] = b[i]
        upper[i] = a[i]
    diag[k] = 1.0
    rhs = np.zeros(n)
    rhs[k] = 1.0
    z = np.full(M, np.nan)
    z[: k + 1] = core.tridiag_general(lower, diag, upper, rhs)
    return z


def prepare(a, b, P):
    """Preliminary step of Algorithm 3 (once per matrix): G at every
    separator and Z^R, Z^L at every separator."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    M = len(b)
    t, s = partition(M, P)
    seps = s[1:P]
    G = green_rows(a, b, seps) if P > 1 else np.zeros((M, 0))
    ZR = {int(k): z_right(a, b, int(k)) for k in seps}
    ZL = {int(k): z_left(a, b, int(k)) for k in seps}
    return dict(a=a, b=b, M=M, P=P, t=t, s=s, seps=seps, G=G, ZR=ZR, ZL=ZL)


# ------------------------------------------------------ per right-hand side (Alg. 3, step 2)
def betas(prep, F):
    """eq. beta_symn: beta^R_j = F_seg . G_{s_{j+1}}, beta^L_j = F_seg . G_{s_j}
    over segment j = rows s_j..s_{j+1}-1.  Returns (bR, bL), each (P, N);
    bR[P-1] and bL[0] are unused (zero)."""
    F = np.asarray(F, dtype=np.float64)
    if F.ndim == 1:
        F = F[:, None]
    P, s, G = prep["P"], prep["s"], prep["G"]
    N = F.shape[1]
    bR = np.zeros((P, N))
    bL = np.zeros((P, N))
    for j in range(P):
        lo, hi = s[j], s[j + 1]
        if j <= P - 2:
            bR[j] = G[lo:hi, j].T @ F[lo:hi]          # row of A^{-1} at s_{j+1}
        if j >= 1:
            bL[j] = G[lo:hi, j - 1].T @ F[lo:hi]      # row of A^{-1} at s_j
    return bR, bL


def interface_theor2(prep, bR, bL):
    """Theorem 2 (eq. theor_2), the O(P^2) double sum: x at s_1..s_{P-1}.
    Returns (P-1, N)."""
    P, s, ZR, ZL = prep["P"], prep["s"], prep["ZR"], prep["ZL"]
    N = bR.shape[1]
    X = np.zeros((P - 1, N))
    for k in range(1, P):
        sk = s[k]
        acc = np.zeros(N)
        for j in range(0, k):
            acc += bR[j] * ZR[int(s[j + 1])][sk]
        for j in range(k, P):
            acc += bL[j] * ZL[int(s[j])][sk]
        X[k - 1] = acc
    return X


def block_solves(prep, F, xsep):
    """Lemma 1 / Algorithm 1 step 3: each block's identity-bordered system
    solved independently once the separator values are known."""
    a, b, M, P, s = prep["a"], prep["b"], prep["M"], prep["P"], prep["s"]
    F = np.asarray(F, dtype=np.float64)
    N = F.shape[1]
    X = np.zeros((M, N))
    for j in range(P):
        lo = s[j]
        hi = s[j + 1] if j < P - 1 else M - 1          # window rows lo..hi
        n = hi - lo + 1
        lower = np.zeros(n)
        diag = np.zeros(n)
        upper = np.zeros(n)
        for r in range(n):
            i = lo + r
            known_left = (r == 0 and j > 0)
            known_right = (r == n - 1 and j < P - 1)
            if known_left or known_right:
                diag[r] = 1.0
            else:
                lower[r] = a[i - 1] if i > 0 else 0.0
                diag[r] = b[i]
                upper[r] = a[i] if i < M - 1 else 0.0
        for col in range(N):
            rhs = F[lo:hi + 1, col].copy()
            if j > 0:
                rhs[0] = xsep[j - 1, col]
            if j < P - 1:
                rhs[-1] = xsep[j, col]
            X[lo:hi + 1, col] = core.tridiag_general(lower, diag, upper, rhs)
    return X


def solve_by_method(a, b, F, P):
    """Algorithm 1 with Algorithm 3 for the boundary elements, end to end."""
    F = np.asarray(F, dtype=np.float64)
    if F.ndim == 1:
        F = F[:, None]
    prep = prepare(a, b, P)
    if P == 1:
        return core.thomas(a, b, F)
    bR, bL = betas(prep, F)
    xsep = interface_theor2(prep, bR, bL)
    return block_solves(prep, F, xsep)


# ------------------------------------------------------ dichotomy (Alg. 4)
def omega_levels(p: int):
    """eq. omega_i: level sets of the separator indices 1..p, level
    i = 1..floor(log2 p)+1 takes j = 2^(floor(log2 p)+1-i) * k,
    k = 1..2^i - 1, minus the earlier levels (and indices beyond p)."""
    L = int(math.floor(math.log2(p))) + 1
    seen = set()
    levels = []
    for i in range(1, L + 1):
        step = 2 ** (L - i)
        cur = []
        for k in range(1, 2 ** i):
            j = step * k
            if j <= p and j not in seen:
                cur.append(j)
        seen.update(cur)
        levels.append(cur)
    return levels


def interface_dichotomy(prep, bR, bL):
    """Algorithm 4, step 2.2: separators computed level by level from the
    nearest already-known separators (Theorem 3, with the partial sums SR,
    SL carried per known separator).  Returns (P-1, N)."""
    P, s, ZR, ZL = prep["P"], prep["s"], prep["ZR"], prep["ZL"]
    N = bR.shape[1]
    p = P - 1
    SR = {0: np.zeros(N)}        # left domain end
    SL = {P: np.zeros(N)}        # right domain end
    known = [0, P]
    for level in omega_levels(p):
        new = {}
        for i in level:
            k1 = max(k for k in known if k < i)
            k2 = min(k for k in known if k > i)
            si = s[i]
            sr = np.zeros(N) if k1 == 0 else SR[k1] * ZR[int(s[k1])][si]
            for j in range(k1, i):
                sr = sr + bR[j] * ZR[int(s[j + 1])][si]
            sl = np.zeros(N) if k2 == P else SL[k2] * ZL[int(s[k2])][si]
            for j in range(i, k2):
                sl = sl + bL[j] * ZL[int(s[j])][si]
            new[i] = (sr, sl)
        for i, (sr, sl) in new.items():
            SR[i], SL[i] = sr, sl
        known = sorted(set(known) | set(new))
    X = np.zeros((P - 1, N))
    for k in range(1, P):
        X[k - 1] = SR[k] + SL[k]
    return X


# ------------------------------------------------------ metrics
def residual_columns(a, b, F, X, X_ref=None):
    """Per right-hand side n (column of the [M][N] arrays), with
    R = F - A X computed row by row from the matrix of section 2:
        eta_n = |R_n|_inf / (|A|_inf |X_n|_inf + |F_n|_inf)   (normwise backward error),
        r2_n  = |R_n|_2 / |F_n|_2                               (relative residual),
        e_n   = |X_n - X_ref,n|_inf / |X_ref,n|_inf             (forward error, if X_ref).
    Returns a dict of length-N arrays."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    F = np.asarray(F, dtype=np.float64)
    X = np.asarray(X, dtype=np.float64)
    if F.ndim == 1:
        F, X = F[:, None], X[:, None]
    R = F - b[:, None] * X
    if len(b) > 1:
        R[:-1] -= a[:, None] * X[1:]
        R[1:] -= a[:, None] * X[:-1]
    normA = np.max(np.abs(b) + np.concatenate([[0.0], np.abs(a)]) + np.concatenate([np.abs(a), [0.0]]))
    xinf = np.max(np.abs(X), axis=0)
    finf = np.max(np.abs(F), axis=0)
    rinf = np.max(np.abs(R), axis=0)
    out = dict(eta=rinf / np.maximum(normA * xinf + finf, 1e-300),
               r2=np.linalg.norm(R, axis=0) / np.maximum(np.linalg.norm(F, axis=0), 1e-300))
    if X_ref is not None:
        X_ref = np.asarray(X_ref, dtype=np.float64)
        if X_ref.ndim == 1:
            X_ref = X_ref[:, None]
        out["e"] = np.max(np.abs(X - X_ref), axis=0) / np.maximum(np.max(np.abs(X_ref), axis=0), 1e-300)
    return out


def residual_metrics(a, b, F, X, X_ref=None):
    """The maxima over the series of residual_columns' eta, r2 (and e)."""
    cols = residual_columns(a, b, F, X, X_ref)
    return {k: float(v.max()) for k, v in cols.items()}
