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


def _rand_general(rng, M):
    """Non-symmetric, diagonally dominant, lower[i] * upper[i] > 0."""
    up = rng.uniform(0.2, 1.0, size=M - 1) * rng.choice([-1.0, 1.0], size=M - 1)
    lo = np.sign(up) * rng.uniform(0.2, 1.0, size=M - 1)
    d = (np.concatenate([[0], np.abs(lo)]) + np.concatenate([np.abs(up), [0]]) + 0.3
         + rng.uniform(0, 0.5, size=M)) * rng.choice([-1.0, 1.0], size=M)
    return lo, d, up


def _dense(lo, d, up):
    return np.diag(d) + np.diag(lo, -1) + np.diag(up, 1)


@pytest.mark.parametrize("M,P", [(64, 4), (67, 5), (200, 16), (9, 4)])
def test_prepare_host_general_rows_of_inverse(M, P):
    # weights = rows of A^{-1} at the interface rows (the non-symmetric A,
    # not its symmetrisation), diagonal of A^{-1}
    rng = np.random.default_rng(M * 11 + P)
    lo, d, up = _rand_general(rng, M)
    h = t.prepare_host_general(lo, d, up, P)
    Ainv = np.linalg.inv(_dense(lo, d, up))
    s = h["starts"]
    for j in range(P):
        a_, b_ = s[j], s[j + 1]
        if j <= P - 2:
            assert np.allclose(h["wR"][a_:b_], Ainv[s[j + 1], a_:b_], rtol=1e-12, atol=1e-15)
        if j >= 1:
            assert np.allclose(h["wL"][a_:b_], Ainv[s[j], a_:b_], rtol=1e-12, atol=1e-15)
    assert np.allclose(h["diag_inv"], np.diag(Ainv), rtol=1e-12)


@pytest.mark.parametrize("M,P", [(64, 4), (101, 7), (256, 32)])
def test_replay_with_general_tables_matches_oracle(M, P):
    # the per-RHS recurrences with the general tables give A^{-1} F at the
    # interface rows, against the oracle's general elimination per column
    rng = np.random.default_rng(M + 5 * P)
    lo, d, up = _rand_general(rng, M)
    F = rng.uniform(-1, 1, size=(M, 4))
    h = t.prepare_host_general(lo, d, up, P)
    xs = _replay(h, None, None, F)
    low = np.concatenate([[0.0], lo])
    upp = np.concatenate([up, [0.0]])
    X = np.stack([oracle.tridiag_general(low, d, upp, F[:, n]) for n in range(F.shape[1])], 1)
    assert np.max(np.abs(xs - X[h["starts"][1:P]])) <= 1e-12 * np.max(np.abs(X))


def test_prepare_general_symmetric_input_matches_symmetric_tables():
    rng = np.random.default_rng(3)
    a, b = _rand(rng, 120)
    hg = t.prepare_host_general(a, b, a, 8)
    hs = t.prepare_host(a, b, 8)
    for key in ("wR", "wL", "rho", "lam", "diag_inv"):
        assert np.allclose(hg[key], hs[key], rtol=1e-14, atol=1e-300), key


def test_prepare_general_errors_without_gpu():
    L = t.lib()
    h = ctypes.c_void_p()
    lo, d, up = np.ones(9), np.full(10, 4.0), np.ones(9)
    P_ = lambda x: x.ctypes.data_as(ctypes.c_void_p)
    bad = up.copy(); bad[4] = -1.0                   # lower * upper < 0: no similarity
    assert L.tdsolve_prepare_general(P_(lo), P_(d), P_(bad), 10, 2, ctypes.byref(h)) == -6
    zero = lo.copy(); zero[2] = 0.0
    assert L.tdsolve_prepare_general(P_(zero), P_(d), P_(up), 10, 2, ctypes.byref(h)) == -6
    nan = lo.copy(); nan[0] = np.nan
    assert L.tdsolve_prepare_general(P_(nan), P_(d), P_(up), 10, 2, ctypes.byref(h)) == -1
    assert L.tdsolve_prepare_general(None, P_(d), P_(up), 10, 2, ctypes.byref(h)) == -1


def test_adi_iteration_count_formula():
    # eq. ocenka1: n0 = 0.2 ln(4N/pi) ln(4/eps); N = 64, eps = 1e-6 gives 13.4
    from paper_0901_2859_amd.adi import n0_iterations
    assert n0_iterations(64, 1e-6) == 14
    assert n0_iterations(1024, 1e-5) == int(np.ceil(0.2 * np.log(4096 / np.pi) * np.log(4e5)))


def test_new_entry_points_reject_bad_arguments_without_gpu():
    # argument checks come before any HIP call
    L = t.lib()
    a, b = -np.ones(9), 3 * np.ones(10)
    P_ = lambda x: x.ctypes.data_as(ctypes.c_void_p)
    Pout = ctypes.c_int32()
    ms = ctypes.c_double()
    assert L.tdsolve_autotune(P_(a), P_(b), 10, 0, 0, 3, ctypes.byref(Pout), ctypes.byref(ms),
                              None) == -1                              # N = 0
    assert L.tdsolve_autotune(P_(a), P_(b), 10, 5, 9, 3, ctypes.byref(Pout), ctypes.byref(ms),
                              None) == -1                              # bad mode
    assert L.tdsolve_autotune(P_(a), P_(b), 10, 5, 0, 3, None, None, None) == -1
    assert L.tdsolve_batch_autotune(0, None, None, None, None, 0, 3, None, None, None,
                                    None, None) == -1
    tun = t.Tuning()
    assert L.tdsolve_autotune_plan(P_(a), P_(b), 10, 0, 0, 0, None, 3, ctypes.byref(tun),
                                   None) == -1                         # N = 0
    assert L.tdsolve_autotune_plan(P_(a), P_(b), 10, 5, 9, 0, None, 3, ctypes.byref(tun),
                                   None) == -1                         # bad mode
    assert L.tdsolve_autotune_plan(P_(a), P_(b), 10, 5, 0, -1, None, 3, ctypes.byref(tun),
                                   None) == -1                         # P < 0
    assert L.tdsolve_autotune_plan(P_(a), P_(b), 10, 5, 0, 0, None, 3, None, None) == -1
    assert L.tdsolve_set_interface(None, 1) == -1
    assert L.tdsolve_prepare_host_general(P_(a), P_(b), None, 10, 2, None, None, None, None,
                                          None, None) == -1


@pytest.mark.parametrize("M,P", [(64, 8), (300, 10), (1000, 37), (4096, 64), (2000, 130)])
def test_dense_table_host_is_theorem2_ratio_products(M, P):
    # the coefficient matrix of the dense interface order, entry by entry
    # against the oracle's Z vectors at the interface rows, and its product
    # with the oracle's betas against the oracle's literal double sum
    w = wl.random_dominant(seed=M + P, M=M, N=5)
    a, b, F = w["a"], w["b"], w["F"]
    prep = method.prepare(a, b, P)
    s, ZR, ZL = prep["s"], prep["ZR"], prep["ZL"]
    K = t.dense_table_host(a, b, P)
    assert K.shape == (P - 1, 2 * P)
    Kor = np.zeros((P - 1, 2 * P))
    for k in range(1, P):
        sk = int(s[k])
        for j in range(k):
            Kor[k - 1, j] = ZR[int(s[j + 1])][sk]
        for j in range(k, P):
            Kor[k - 1, P + j] = ZL[int(s[j])][sk]
    np.testing.assert_allclose(K, Kor, rtol=1e-11, atol=1e-300)
    bR, bL = method.betas(prep, F)
    xs = method.interface_theor2(prep, bR, bL)
    X = K[:, :P] @ bR + K[:, P:] @ bL
    assert np.max(np.abs(X - xs)) <= 1e-12 * np.max(np.abs(xs))


def test_dense_table_host_limits():
    a, b = -np.ones(2099), 3 * np.ones(2100)
    with pytest.raises(t.TdsError) as err:
        t.dense_table_host(a, b, 1)
    assert err.value.code == -1                 # TDS_EINVAL: no interface rows
    with pytest.raises(t.TdsError) as err:
        t.dense_table_host(a, b, 1025)
    assert err.value.code == -6                 # TDS_EUNSUPPORTED: P > 1024
    K = t.dense_table_host(a[:3], b[:4], 2)     # one interface row: both parts 1 at j = 0, 1
    assert np.array_equal(K, np.array([[1.0, 0.0, 0.0, 1.0]]))


def test_status_and_overlap_checks_without_gpu():
    # tdsolve_status needs a handle that has solved something; a NULL
    # handle is rejected before any HIP call
    L = t.lib()
    err = ctypes.c_double()
    passes = ctypes.c_int32()
    assert L.tdsolve_status(None, None, ctypes.byref(err), ctypes.byref(passes)) == -1
