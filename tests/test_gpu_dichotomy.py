"""GPU: the interface step by the dichotomy (Algorithm 4, Theorem 3,
eq. omega_i; tdsolve_set_interface(TDS_IFACE_DICHOTOMY)) against the CPU
oracle's level-by-level evaluation (oracle.method.interface_dichotomy, which
is pinned to the paper's p = 15 level sets and to brute force), against the
recurrence order, and end to end against the oracle's sweep.

Tolerance: the interface values carry the same rounding bound as in the
parity tests, 1e-11 + 8 (t + 2P) u cond_n per right-hand side (relative to
the largest solution component of that right-hand side)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
from oracle import method  # noqa: E402
from tests import _parity  # noqa: E402
from paper_0901_2859_amd import tdsolve as t  # noqa: E402
from paper_0901_2859_amd import workloads as wl  # noqa: E402

DEV = "cuda:0"


def _tol(a, b, F, ref, P):
    return _parity.tol64(a, b, F, ref, P)


@pytest.mark.parametrize("M,N,P", [(64, 16, 16), (300, 77, 10), (1024, 300, 64), (130, 5, 65),
                                   (40, 9, 2), (90, 33, 3), (4096, 64, 128),
                                   # P > 129: the recurrence order's scan groups hold more
                                   # blocks than it keeps in registers
                                   (1200, 50, 300), (8192, 20, 1024)])
def test_dichotomy_components_match_oracle(M, N, P):
    print(f"dichotomy M={M} N={N} P={P}", flush=True)
    w = wl.random_dominant(seed=M + P, M=M, N=N)
    a, b, F = w["a"], w["b"], w["F"]
    prep = method.prepare(a, b, P)
    bR, bL = method.betas(prep, F)
    xs_or = method.interface_dichotomy(prep, bR, bL)
    ref = oracle.thomas(a, b, F)
    tol = _tol(a, b, F, ref, P)
    scale = np.max(np.abs(ref), axis=0)
    plan = t.Plan(a, b, P)
    Fd = torch.from_numpy(F).to(DEV)
    plan.set_interface("dichotomy")
    xs_d = plan.components(Fd, mode="f64").cpu().numpy()
    plan.set_interface("recurrence")
    xs_r = plan.components(Fd, mode="f64").cpu().numpy()
    for xs, what in ((xs_d, "dichotomy vs oracle"), ):
        e = np.max(np.abs(xs - xs_or), axis=0) / scale
        assert np.all(e <= tol), (what, e.max())
    e = np.max(np.abs(xs_d - xs_r), axis=0) / scale
    assert np.all(e <= tol), ("dichotomy vs recurrence", e.max())


def test_dichotomy_full_solve_poisson_all_modes():
    # the Poisson series at 1024 x 512 with P = 64: the full solve with the
    # dichotomy order, every FP64-result mode, against the oracle's sweep
    w = wl.poisson_series(M=1024, N=512, P=64)
    a, b, F32 = w["a"], w["b"], w["F"]
    Fw = F32.astype(np.float64)
    ref = oracle.thomas(a, b, Fw)
    tol = _tol(a, b, Fw, ref, 64)
    plan = t.Plan(a, b, 64)
    plan.set_interface("dichotomy")
    Fs = torch.from_numpy(F32).to(DEV)
    for mode, Fin in (("f64", Fs.double()), ("f32_refined", Fs), ("f32_wide", Fs)):
        X = plan.solve(Fin, mode=mode).cpu().numpy()
        _parity.check(X, ref, tol, f"dichotomy poisson 1024x512 {mode}")
        _parity.check_residual(a, b, Fw, X, ref, f"dichotomy poisson 1024x512 {mode}")


def test_set_interface_rejects_unknown_order():
    a, b = -np.ones(63), 3 * np.ones(64)
    plan = t.Plan(a, b, 4)
    with pytest.raises(t.TdsError):
        t._check(t.lib().tdsolve_set_interface(plan._h, 7), "tdsolve_set_interface")


def test_dichotomy_general_matrix_matches_oracle():
    # non-symmetric A: the dichotomy's products of transfer factors carry the
    # similarity's ratios as the recurrences do
    rng = np.random.default_rng(8)
    M, N, P = 1200, 40, 20
    up = rng.uniform(0.2, 1.0, size=M - 1) * rng.choice([-1.0, 1.0], size=M - 1)
    lo = np.sign(up) * rng.uniform(0.2, 1.0, size=M - 1)
    d = (np.concatenate([[0], np.abs(lo)]) + np.concatenate([np.abs(up), [0]]) + 0.3) * \
        rng.choice([-1.0, 1.0], size=M)
    F = rng.uniform(-1, 1, size=(M, N))
    low, upp = np.concatenate([[0.0], lo]), np.concatenate([up, [0.0]])
    ref = np.stack([oracle.tridiag_general(low, d, upp, F[:, n]) for n in range(N)], 1)
    plan = t.Plan.general(lo, d, up, P)
    Fd = torch.from_numpy(F).to(DEV)
    plan.set_interface("dichotomy")
    X = plan.solve(Fd, mode="f64").cpu().numpy()
    scale = np.max(np.abs(ref), axis=0)
    assert np.max(np.abs(X - ref).max(axis=0) / scale) <= 1e-11
