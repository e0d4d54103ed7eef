"""Pins for the CPU oracle, independent of the oracle itself.

Each test fixes the oracle to something the paper or mathematics determines:
a dense LU solve (library), closed forms of the 1-D Poisson matrix (its sine
eigenvectors, used by the paper's Fourier method, and its explicit inverse,
the discrete analog of the linear Green's function of Theorem 1), exact
integer manufactured solutions, Theorem 4's bound, brute-force Algorithm 2,
the worked dichotomy example, and finite differences for the gradient.
The last group plants plausible mistakes in copies of the oracle and checks
that the pins catch them.
"""
import json
import os

import numpy as np
import pytest

import oracle
from oracle import method
from paper_0901_2859_amd import workloads as wl

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rand_tridiag(rng, M, dominant=True):
    a = rng.uniform(-1, 1, size=M - 1)
    b = rng.uniform(-1, 1, size=M)
    if dominant:
        b = np.sign(b + 1e-3) * (np.concatenate([[0], np.abs(a)]) + np.concatenate([np.abs(a), [0]]) + 0.2 + np.abs(b))
    return a, b


# ------------------------------------------------------------------ whole solve
@pytest.mark.parametrize("M", [1, 2, 3, 5, 17, 64])
def test_thomas_matches_dense_lu(M):
    rng = np.random.default_rng(100 + M)
    a, b = _rand_tridiag(rng, M) if M > 1 else (np.zeros(0), np.array([2.5]))
    F = rng.uniform(-1, 1, size=(M, 7))
    X = oracle.thomas(a, b, F)
    Xd = np.linalg.solve(method.dense(a, b), F)
    assert np.max(np.abs(X - Xd)) <= 1e-13 * max(1.0, np.max(np.abs(Xd)))


def test_thomas_small_config_matches_dense():
    w = wl.small()
    X = oracle.thomas(w["a"], w["b"], w["F"])
    Xd = np.linalg.solve(method.dense(w["a"], w["b"]), w["F"])
    assert np.max(np.abs(X - Xd)) <= 1e-14


@pytest.mark.parametrize("M,l", [(64, 1), (64, 7), (64, 64), (500, 3), (500, 250)])
def test_thomas_poisson_sine_modes(M, l):
    # sin(pi l i/(M+1)) is an eigenvector of the Poisson matrix with
    # eigenvalue 2 - 2 cos(pi l/(M+1)) (the basis of the Fourier method)
    a, b = wl.poisson_coeffs(M)
    i = np.arange(1, M + 1)
    v = np.sin(np.pi * l * i / (M + 1))
    lam = 2.0 - 2.0 * np.cos(np.pi * l / (M + 1))
    X = oracle.thomas(a, b, v)
    kappa = 4.0 / (2.0 - 2.0 * np.cos(np.pi / (M + 1)))
    assert np.max(np.abs(X - v / lam)) <= 50 * kappa * 2.2e-16 * np.max(np.abs(v / lam)) + 1e-15


def test_thomas_manufactured_integer_solution():
    rng = np.random.default_rng(7)
    M, N = 200, 9
    a = np.full(M - 1, 1.0)
    b = np.full(M, 4.0)
    Xs = rng.integers(-5, 6, size=(M, N)).astype(np.float64)
    F = method.dense(a, b) @ Xs          # exact in FP64 (small integers)
    X = oracle.thomas(a, b, F)
    assert np.max(np.abs(X - Xs)) <= 1e-13


def test_thomas_detects_zero_pivot():
    # [[0, 1], [1, 0]] is nondegenerate but has no elimination without pivoting
    with pytest.raises(oracle.OracleError):
        oracle.thomas(np.array([1.0]), np.array([0.0, 0.0]), np.ones((2, 1)))


# ------------------------------------------------------------------ preliminary step
def _poisson_inv(M):
    i = np.arange(1, M + 1)
    I, J = np.meshgrid(i, i, indexing="ij")
    return np.minimum(I, J) * (M + 1 - np.maximum(I, J)) / (M + 1)


def test_green_rows_poisson_closed_form():
    M = 64
    a, b = wl.poisson_coeffs(M)
    ks = [0, 5, 31, 63]
    G = method.green_rows(a, b, ks)
    Ainv = _poisson_inv(M)
    assert np.max(np.abs(G - Ainv[:, ks])) <= 1e-12


def test_z_vectors_poisson_linear():
    # for the Poisson matrix the homogeneous solutions are linear:
    # Z^R_k(i) = (M+1-i)/(M+1-k), Z^L_k(i) = i/k (1-based rows)
    M = 64
    a, b = wl.poisson_coeffs(M)
    for k0 in [3, 16, 40]:
        k = k0 + 1
        zr = method.z_right(a, b, k0)
        zl = method.z_left(a, b, k0)
        i = np.arange(1, M + 1)
        assert np.allclose(zr[k0:], ((M + 1 - i) / (M + 1 - k))[k0:], atol=1e-13)
        assert np.allclose(zl[: k0 + 1], (i / k)[: k0 + 1], atol=1e-13)


def test_z_vectors_bounded_under_dominance():
    # Theorem 4: diagonal dominance (one strict) => |Z^{R,L}| <= 1
    rng = np.random.default_rng(11)
    for _ in range(5):
        M = 80
        a, b = _rand_tridiag(rng, M)
        for k in [0, 10, 41, 79]:
            zr = method.z_right(a, b, k)
            zl = method.z_left(a, b, k)
            assert np.nanmax(np.abs(zr)) <= 1.0 + 1e-15
            assert np.nanmax(np.abs(zl)) <= 1.0 + 1e-15


def test_inverse_symmetry_lemma2():
    rng = np.random.default_rng(12)
    M = 40
    a, b = _rand_tridiag(rng, M)
    G = method.green_rows(a, b, list(range(M)))
    assert np.max(np.abs(G - G.T)) <= 1e-14


# ------------------------------------------------------------------ interface step
@pytest.mark.parametrize("M,P", [(64, 4), (64, 8), (67, 5), (128, 16), (9, 4)])
def test_theor2_matches_brute_force_algorithm2(M, P):
    rng = np.random.default_rng(M * 31 + P)
    a, b = _rand_tridiag(rng, M)
    F = rng.uniform(-1, 1, size=(M, 6))
    prep = method.prepare(a, b, P)
    bR, bL = method.betas(prep, F)
    xs = method.interface_theor2(prep, bR, bL)
    Ainv = np.linalg.inv(method.dense(a, b))        # Algorithm 2: x_k = G_k^T F
    brute = Ainv[prep["seps"]] @ F
    assert np.max(np.abs(xs - brute)) <= 1e-13


def test_theor2_poisson_small_config():
    w = wl.small()
    prep = method.prepare(w["a"], w["b"], w["P"])
    bR, bL = method.betas(prep, w["F"])
    xs = method.interface_theor2(prep, bR, bL)
    X = np.linalg.solve(method.dense(w["a"], w["b"]), w["F"])
    assert np.max(np.abs(xs - X[prep["seps"]])) <= 1e-14


@pytest.mark.parametrize("M,P", [(64, 4), (66, 7), (200, 16), (10, 5), (5, 1)])
def test_method_end_to_end_matches_dense(M, P):
    rng = np.random.default_rng(M + 1000 * P)
    a, b = _rand_tridiag(rng, M)
    F = rng.uniform(-1, 1, size=(M, 5))
    X = method.solve_by_method(a, b, F, P)
    Xd = np.linalg.solve(method.dense(a, b), F)
    assert np.max(np.abs(X - Xd)) <= 1e-13


def test_partition_rule():
    t, s = method.partition(10, 4)
    assert list(t) == [3, 3, 2, 2] and list(s) == [0, 3, 6, 8, 10]
    with pytest.raises(ValueError):
        method.partition(7, 4)


# ------------------------------------------------------------------ dichotomy
def test_omega_levels_worked_example():
    with open(os.path.join(GOLDEN, "dichotomy_levels_p15.json")) as fh:
        g = json.load(fh)
    assert method.omega_levels(g["p"]) == g["levels"]


@pytest.mark.parametrize("p", [1, 2, 3, 6, 15, 20, 31])
def test_omega_levels_partition_all(p):
    levels = method.omega_levels(p)
    flat = [j for L in levels for j in L]
    assert sorted(flat) == list(range(1, p + 1))
    assert len(levels) == int(np.floor(np.log2(p))) + 1


@pytest.mark.parametrize("M,P", [(64, 16), (96, 7), (130, 32)])
def test_dichotomy_matches_brute_force(M, P):
    rng = np.random.default_rng(M + P)
    a, b = _rand_tridiag(rng, M)
    F = rng.uniform(-1, 1, size=(M, 4))
    prep = method.prepare(a, b, P)
    bR, bL = method.betas(prep, F)
    xd = method.interface_dichotomy(prep, bR, bL)
    brute = np.linalg.inv(method.dense(a, b))[prep["seps"]] @ F
    assert np.max(np.abs(xd - brute)) <= 1e-13


# ------------------------------------------------------------------ gradient
def test_grad_matches_central_differences():
    rng = np.random.default_rng(21)
    M, N = 24, 5
    a, b = _rand_tridiag(rng, M)
    F = rng.uniform(-1, 1, size=(M, N))
    W = rng.uniform(-1, 1, size=(M, N))

    def loss(a_, b_, F_):
        return float(np.sum(W * np.linalg.solve(method.dense(a_, b_), F_)))

    X = oracle.thomas(a, b, F)
    gF, ga, gb = oracle.grad(a, b, X, W)
    h = 1e-6
    for i in range(M - 1):
        d = np.zeros(M - 1); d[i] = h
        fd = (loss(a + d, b, F) - loss(a - d, b, F)) / (2 * h)
        assert abs(fd - ga[i]) <= 1e-7 * max(1.0, abs(fd))
    for i in range(M):
        d = np.zeros(M); d[i] = h
        fd = (loss(a, b + d, F) - loss(a, b - d, F)) / (2 * h)
        assert abs(fd - gb[i]) <= 1e-7 * max(1.0, abs(fd))
    for (i, n) in [(0, 0), (5, 2), (M - 1, N - 1)]:
        d = np.zeros((M, N)); d[i, n] = h
        fd = (loss(a, b, F + d) - loss(a, b, F - d)) / (2 * h)
        assert abs(fd - gF[i, n]) <= 1e-7 * max(1.0, abs(fd))


@pytest.mark.slow
def test_grad_matches_central_differences_gradient_case():
    # the differentiation workload at full size (M = 2048, N = 1024; the
    # FP32 right-hand sides widened exactly): central differences with the
    # absolute step h = 1e-6 on every a_i, every b_i and 64 seeded entries
    # of F plus its two corners, each difference taken of the loss
    # sum(W * X) through two full oracle solves of the perturbed series
    w = wl.gradient_case()
    a, b, W = w["a"], w["b"], w["W"]
    F = w["F"].astype(np.float64)
    M, N = F.shape
    X = oracle.thomas(a, b, F)
    gF, ga, gb = oracle.grad(a, b, X, W)
    h = 1e-6

    def fd(ap, bp, am, bm):
        dX = oracle.thomas(ap, bp, F) - oracle.thomas(am, bm, F)
        return float(np.sum(W * dX)) / (2 * h)

    worst = 0.0
    for i in range(M - 1):
        d = np.zeros(M - 1); d[i] = h
        g = fd(a + d, b, a - d, b)
        worst = max(worst, abs(g - ga[i]) / max(1.0, abs(g)))
    for i in range(M):
        d = np.zeros(M); d[i] = h
        g = fd(a, b + d, a, b - d)
        worst = max(worst, abs(g - gb[i]) / max(1.0, abs(g)))
    rng = np.random.default_rng(55)
    cells = list(zip(rng.integers(0, M, 64), rng.integers(0, N, 64))) + [(0, 0), (M - 1, N - 1)]
    for i, n in cells:
        e = np.zeros(M); e[i] = h
        # only column n of X depends on F[i, n]
        dX = oracle.thomas(a, b, F[:, n] + e) - oracle.thomas(a, b, F[:, n] - e)
        g = float(np.dot(W[:, n], dX)) / (2 * h)
        worst = max(worst, abs(g - gF[i, n]) / max(1.0, abs(g)))
    print(f"gradient case: max |fd - grad| / max(1, |fd|) = {worst:.3e}")
    assert worst <= 1e-7


def test_grad_self_adjoint_identity():
    rng = np.random.default_rng(22)
    M, N = 50, 3
    a, b = _rand_tridiag(rng, M)
    F = rng.uniform(-1, 1, size=(M, N))
    W = rng.uniform(-1, 1, size=(M, N))
    X = oracle.thomas(a, b, F)
    gF, _, _ = oracle.grad(a, b, X, W)
    assert abs(np.sum(W * X) - np.sum(gF * F)) <= 1e-12 * np.sum(np.abs(W * X))


# ------------------------------------------------------------------ residual metrics
def _manufactured_residual_case():
    # integer A (mixed-sign, non-constant off-diagonals, dominant diagonal)
    # and integer X*: F0 = A X* is exact in FP64, and F = F0 + delta_n e_{k_n}
    # with delta_n a power of two is exact too, so F - A X* is exactly
    # delta_n e_{k_n} in column n: the residual is known in closed form.
    rng = np.random.default_rng(41)
    M, N = 57, 6
    a = rng.integers(1, 4, size=M - 1) * rng.choice([-1.0, 1.0], size=M - 1)
    b = (np.concatenate([[0], np.abs(a)]) + np.concatenate([np.abs(a), [0]]) + rng.integers(1, 3, size=M)).astype(np.float64)
    Xs = rng.integers(-9, 10, size=(M, N)).astype(np.float64)
    F = method.dense(a, b) @ Xs
    rows = np.array([0, 1, 28, M - 2, M - 1, 13])
    delta = np.array([2.0 ** -3, -(2.0 ** -7), 2.0 ** -20, -(2.0 ** 2), 2.0 ** -1, 2.0 ** -30])
    F[rows, np.arange(N)] += delta
    return a, b, Xs, F, rows, delta


def test_residual_columns_manufactured_closed_form():
    a, b, Xs, F, rows, delta = _manufactured_residual_case()
    D = method.dense(a, b)
    normA = np.abs(D).sum(axis=1).max()              # |A|_inf, max row sum
    want_eta = np.abs(delta) / (normA * np.abs(Xs).max(axis=0) + np.abs(F).max(axis=0))
    want_r2 = np.abs(delta) / np.sqrt((F ** 2).sum(axis=0))
    got = method.residual_columns(a, b, F, Xs)
    assert np.allclose(got["eta"], want_eta, rtol=1e-15, atol=0)
    assert np.allclose(got["r2"], want_r2, rtol=1e-15, atol=0)
    m = method.residual_metrics(a, b, F, Xs)
    assert m["eta"] == want_eta.max() or abs(m["eta"] - want_eta.max()) <= 1e-15 * want_eta.max()
    assert abs(m["r2"] - want_r2.max()) <= 1e-15 * want_r2.max()
    # forward error against a reference with a known difference
    X = Xs.copy()
    X[rows, np.arange(len(rows))] += 0.5
    e = method.residual_columns(a, b, F, X, Xs)["e"]
    assert np.array_equal(e, 0.5 / np.abs(Xs).max(axis=0))


def test_residual_columns_exact_solution_is_zero():
    a, b, Xs, F, rows, delta = _manufactured_residual_case()
    F0 = F.copy()
    F0[rows, np.arange(len(rows))] -= delta
    got = method.residual_columns(a, b, F0, Xs)
    assert np.all(got["eta"] == 0.0) and np.all(got["r2"] == 0.0)


def _residual_wrong_coupling(a, b, F, X):
    # plausible slip: the upper neighbour's coupling applied to the row itself
    R = F - b[:, None] * X
    R[:-1] -= a[:, None] * X[:-1]
    R[1:] -= a[:, None] * X[:-1]
    return np.linalg.norm(R, axis=0) / np.linalg.norm(F, axis=0)


def test_planted_mistake_in_residual_is_caught():
    a, b, Xs, F, rows, delta = _manufactured_residual_case()
    want_r2 = np.abs(delta) / np.sqrt((F ** 2).sum(axis=0))
    assert not np.allclose(_residual_wrong_coupling(a, b, F, Xs), want_r2, rtol=1e-6, atol=0)


# ------------------------------------------------------------------ planted mistakes
def _theor2_wrong_zl(prep, bR, bL):
    # plausible slip: Z^L taken at the right separator s_{j+1}
    P, s, ZR, ZL = prep["P"], prep["s"], prep["ZR"], prep["ZL"]
    X = np.zeros((P - 1, bR.shape[1]))
    for k in range(1, P):
        acc = sum(bR[j] * ZR[int(s[j + 1])][s[k]] for j in range(k))
        for j in range(k, P):
            key = int(s[j + 1]) if j + 1 < P else int(s[j])
            acc = acc + bL[j] * ZL[key][s[k]] if s[k] <= key else acc
        X[k - 1] = acc
    return X


def test_planted_mistake_in_theor2_is_caught():
    rng = np.random.default_rng(31)
    M, P = 64, 4
    a, b = _rand_tridiag(rng, M)
    F = rng.uniform(-1, 1, size=(M, 3))
    prep = method.prepare(a, b, P)
    bR, bL = method.betas(prep, F)
    brute = np.linalg.inv(method.dense(a, b))[prep["seps"]] @ F
    assert np.max(np.abs(_theor2_wrong_zl(prep, bR, bL) - brute)) > 1e-6
    # swapped beta^R / beta^L
    assert np.max(np.abs(method.interface_theor2(prep, bL, bR) - brute)) > 1e-6


def test_planted_mistake_in_sweep_is_caught():
    # a sign slip on the off-diagonal, or a transposed (shifted) off-diagonal
    rng = np.random.default_rng(32)
    M = 30
    a, b = _rand_tridiag(rng, M)
    F = rng.uniform(-1, 1, size=(M, 2))
    Xd = np.linalg.solve(method.dense(a, b), F)
    assert np.max(np.abs(oracle.thomas(-a, b, F) - Xd)) > 1e-6
    assert np.max(np.abs(oracle.thomas(np.roll(a, 1), b, F) - Xd)) > 1e-6


# ---------------------------------------------------- general (non-symmetric)
@pytest.mark.parametrize("M", [1, 2, 7, 60])
def test_tridiag_general_matches_dense_lu(M):
    # the oracle's plain elimination for a non-symmetric tridiagonal system
    # against dense LU (numpy), on a diagonally dominant random matrix
    rng = np.random.default_rng(40 + M)
    lower = np.concatenate([[0.0], rng.uniform(-1, 1, size=M - 1)])
    upper = np.concatenate([rng.uniform(-1, 1, size=M - 1), [0.0]])
    diag = np.abs(lower) + np.abs(upper) + rng.uniform(0.5, 1.5, size=M)
    A = np.diag(diag)
    if M > 1:
        A += np.diag(lower[1:], -1) + np.diag(upper[:-1], 1)
    f = rng.uniform(-1, 1, size=M)
    x = oracle.tridiag_general(lower, diag, upper, f)
    assert np.allclose(x, np.linalg.solve(A, f), rtol=1e-13, atol=1e-14)


def test_tridiag_general_manufactured_integer_solution():
    # exact arithmetic: integer solution, small integer coefficients
    M = 9
    lower = np.array([0, 1, 2, 1, 3, 1, 2, 1, 1], dtype=float)
    upper = np.array([2, 1, 1, 2, 1, 1, 3, 1, 0], dtype=float)
    diag = np.full(M, 8.0)
    x_true = np.arange(1, M + 1, dtype=float) * np.array([1, -1] * 4 + [1])
    f = diag * x_true
    f[1:] += lower[1:] * x_true[:-1]
    f[:-1] += upper[:-1] * x_true[1:]
    assert np.allclose(oracle.tridiag_general(lower, diag, upper, f), x_true, rtol=0, atol=1e-12)


# ---------------------------------------------------- 2-D Poisson (direct)
def test_poisson2d_direct_discrete_eigenfunction():
    # sin(pi k i/N1) sin(pi l j/N2) is an eigenvector of the 5-point operator
    # with eigenvalue 4/h1^2 sin^2(pi k/2N1) + 4/h2^2 sin^2(pi l/2N2)
    from oracle import poisson2d
    N1, N2, h1, h2 = 24, 17, 0.1, 0.07
    i = np.arange(1, N1)[:, None]
    j = np.arange(1, N2)[None, :]
    for k, l in ((1, 1), (5, 3), (23, 16)):
        phi = np.sin(np.pi * k * i / N1) * np.sin(np.pi * l * j / N2)
        lam = 4 / h1 ** 2 * np.sin(np.pi * k / (2 * N1)) ** 2 + \
            4 / h2 ** 2 * np.sin(np.pi * l / (2 * N2)) ** 2
        u = poisson2d.solve_direct(phi, h1, h2)
        assert np.allclose(u, phi / lam, rtol=0, atol=1e-12 * np.max(np.abs(phi / lam)))


def test_poisson2d_direct_manufactured_second_order():
    # u = sin(2 pi x) sin(2 pi y), -Delta u = 8 pi^2 u on the unit square
    # (the paper's test problem): the discrete error falls 4x per halving of h
    from oracle import poisson2d
    errs = []
    for n in (16, 32, 64):
        h = 1.0 / n
        x = np.arange(1, n)[:, None] * h
        y = np.arange(1, n)[None, :] * h
        ue = np.sin(2 * np.pi * x) * np.sin(2 * np.pi * y)
        u = poisson2d.solve_direct(8 * np.pi ** 2 * ue, h, h)
        errs.append(np.max(np.abs(u - ue)))
    assert 3.6 < errs[0] / errs[1] < 4.4 and 3.8 < errs[1] / errs[2] < 4.2, errs
