"""CPU-only checks of the library's host side: the shared library loads and
exports every symbol the header declares, the FP64 preliminary step matches
the oracle's rows of A^{-1} and Z vectors, argument errors are reported
without touching a GPU, and a NumPy replay of the per-RHS recurrences built
from the library's own tables reproduces the oracle's interface values
(this validates the index conventions before any kernel runs)."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
from oracle import method
from paper_0901_2859_amd import tdsolve as t
from paper_0901_2859_amd import workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_symbols():
    src = open(os.path.join(ROOT, "include", "tdsolve.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(tdsolve_\w+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = t.lib()
    names = _header_symbols()
    assert len(names) >= 10
    for name in names:
        assert hasattr(L, name), name
    assert set(names) == set(t.SYMBOLS)


def test_strerror_and_default_blocks():
    L = t.lib()
    assert L.tdsolve_strerror(0) == b"ok"
    assert b"singular" in L.tdsolve_strerror(-2) or b"pivot" in L.tdsolve_strerror(-2)
    assert t.default_blocks(4096) == 64
    assert t.default_blocks(3) == 1


def _rand(rng, M):
    a = rng.uniform(-1, 1, size=M - 1)
    b = np.sign(rng.uniform(-1, 1, size=M) + 1e-9) * (
        np.concatenate([[0], np.abs(a)]) + np.concatenate([np.abs(a), [0]]) + 0.3)
    return a, b


@pytest.mark.parametrize("M,P", [(64, 4), (67, 5), (200, 16), (9, 4), (130, 3)])
def test_prepare_host_matches_oracle_rows(M, P):
    rng = np.random.default_rng(M * 7 + P)
    a, b = _rand(rng, M)
    h = t.prepare_host(a, b, P)
    prep = method.prepare(a, b, P)
    s = prep["s"]
    assert np.array_equal(h["starts"], s)
    G = prep["G"]                                   # columns: rows of A^{-1} at s_1..s_{P-1}
    for j in range(P):
        lo, hi = s[j], s[j + 1]
        if j <= P - 2:
            assert np.allclose(h["wR"][lo:hi], G[lo:hi, j], rtol=1e-13, atol=1e-15)
        if j >= 1:
            assert np.allclose(h["wL"][lo:hi], G[lo:hi, j - 1], rtol=1e-13, atol=1e-15)
    for k in range(1, P - 1):
        assert np.isclose(h["rho"][k], prep["ZR"][int(s[k])][s[k + 1]], rtol=1e-13, atol=1e-300)
        assert np.isclose(h["lam"][k], prep["ZL"][int(s[k + 1])][s[k]], rtol=1e-13, atol=1e-300)
    Ginv = method.green_rows(a, b, list(range(M)))
    assert np.allclose(h["diag_inv"], np.diag(Ginv), rtol=1e-13)


def test_prepare_host_poisson_closed_form():
    M, P = 64, 4
    a, b = wl.poisson_coeffs(M)
    h = t.prepare_host(a, b, P)
    i = np.arange(1, M + 1)
    assert np.allclose(h["diag_inv"], i * (M + 1 - i) / (M + 1), rtol=1e-13)
    s = h["starts"]
    # Z^R of the Poisson matrix is linear: rho_k = (M+1-s_{k+1}-1)/(M+1-s_k-1) in 1-based rows
    for k in range(1, P - 1):
        sk, sk1 = s[k] + 1, s[k + 1] + 1
        assert np.isclose(h["rho"][k], (M + 1 - sk1) / (M + 1 - sk), rtol=1e-13)
        assert np.isclose(h["lam"][k], sk / sk1, rtol=1e-13)


def _replay(h, a, b, F):
    """NumPy replay of beta -> recurrences -> block sweeps with the library tables."""
    s, P = h["starts"], h["P"]
    M, N = F.shape
    bR = np.zeros((P, N)); bL = np.zeros((P, N))
    for j in range(P):
        lo, hi = s[j], s[j + 1]
        bR[j] = h["wR"][lo:hi] @ F[lo:hi]
        bL[j] = h["wL"][lo:hi] @ F[lo:hi]
    xs = np.zeros((P - 1, N))
    SR = bR[0].copy(); xs[0] = SR
    for k in range(1, P - 1):
        SR = h["rho"][k] * SR + bR[k]; xs[k] = SR
    SL = bL[P - 1].copy(); xs[P - 2] += SL
    for k in range(P - 2, 0, -1):
        SL = bL[k] + h["lam"][k] * SL; xs[k - 1] += SL
    return xs


@pytest.mark.parametrize("M,P", [(64, 4), (101, 7), (256, 32), (50, 25)])
def test_replay_with_library_tables_matches_oracle(M, P):
    rng = np.random.default_rng(M + 3 * P)
    a, b = _rand(rng, M)
    F = rng.uniform(-1, 1, size=(M, 5))
    h = t.prepare_host(a, b, P)
    xs = _replay(h, a, b, F)
    X = oracle.thomas(a, b, F)
    assert np.max(np.abs(xs - X[h["starts"][1:P]])) <= 1e-13


def test_prepare_errors_without_gpu():
    L = t.lib()
    h = ctypes.c_void_p()
    a = np.ones(9); b = np.full(10, 4.0)
    pa, pb = a.ctypes.data_as(ctypes.c_void_p), b.ctypes.data_as(ctypes.c_void_p)
    assert L.tdsolve_prepare(pa, pb, 0, 1, ctypes.byref(h)) == -1          # M = 0
    assert L.tdsolve_prepare(pa, pb, 10, 6, ctypes.byref(h)) == -1         # blocks < 2 rows
    assert L.tdsolve_prepare(pa, pb, 10, -1, ctypes.byref(h)) == -1
    assert L.tdsolve_prepare(None, pb, 10, 1, ctypes.byref(h)) == -1
    bn = b.copy(); bn[3] = np.nan
    assert L.tdsolve_prepare(pa, bn.ctypes.data_as(ctypes.c_void_p), 10, 2, ctypes.byref(h)) == -1
    ai = a.copy(); ai[0] = np.inf
    assert L.tdsolve_prepare(ai.ctypes.data_as(ctypes.c_void_p), pb, 10, 2, ctypes.byref(h)) == -1
    # nondegenerate [[0,1],[1,0]] has no elimination without pivoting
    with pytest.raises(t.TdsError) as ei:
        t.prepare_host(np.array([1.0]), np.array([0.0, 0.0]), 1)
    assert ei.value.code == -2
    assert L.tdsolve_series(None, None, None, 0, 0, None) == -1
    assert L.tdsolve_destroy(None) == -1


def test_prepare_host_default_and_ragged_blocks():
    M = 1000
    a, b = wl.poisson_coeffs(M, 0.1)
    h = t.prepare_host(a, b, 0)
    assert h["P"] == t.default_blocks(M)
    sizes = np.diff(h["starts"])
    assert sizes.sum() == M and sizes.max() - sizes.min() <= 1 and sizes.min() >= 2
    t13 = np.diff(t.prepare_host(a, b, 13)["starts"])
    assert list(t13[: M % 13]) == [M // 13 + 1] * (M % 13)


def test_dominance_ratios_bounded():
    rng = np.random.default_rng(5)
    a, b = _rand(rng, 300)
    # ratios are the Z transfer factors; |rho|, |lam| <= 1 under dominance (Theorem 4)
    h = t.prepare_host(a, b, 10)
    assert np.all(np.abs(h["rho"]) <= 1.0) and np.all(np.abs(h["lam"]) <= 1.0)
