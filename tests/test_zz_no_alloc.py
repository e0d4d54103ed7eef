"""The entry point that allocates nothing (tdsolve_series_noalloc) against
tdsolve_series on the same plan, through the C ABI.

Both run the same kernels on the same tables; only the work area of the beta
weights and interface values differs (the library's fixed device scratch
instead of the plan's buffer), so the solutions must be bitwise equal, and
both are held to the oracle's bound as in the parity tests.
"""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
from paper_0901_2859_amd import tdsolve as t  # noqa: E402

DEV = "cuda:0"
SCRATCH = 32 << 20
ESCRATCH = -7


def _rand(rng, M, strict=0.3):
    a = rng.uniform(-1, 1, size=M - 1)
    b = np.sign(rng.uniform(-1, 1, size=M) + 1e-9) * (
        np.concatenate([[0], np.abs(a)]) + np.concatenate([np.abs(a), [0]]) + strict)
    return a, b


def _work_bytes(P, N, dichotomy=False):
    # beta^R, beta^L, interface values, the dichotomy's two partial sums and
    # the fused order's counters (2 + 2 ceil(N / 256) of them, one 256-byte
    # line each), each slice rounded up to 256 bytes
    up = lambda x: (x + 255) // 256 * 256          # noqa: E731
    nb, nx = up(8 * P * N), up(8 * max(P - 1, 1) * N)
    ns = up(8 * (P + 1) * N) if dichotomy else 0
    nc = 256 * (2 + 2 * ((N + 255) // 256))
    return 2 * nb + nx + 2 * ns + nc


def _noalloc(plan, F, X, mode):
    return t.lib().tdsolve_series_noalloc(plan._h, ctypes.c_void_p(F.data_ptr()),
                                          ctypes.c_void_p(X.data_ptr()), F.shape[1],
                                          t.MODES[mode], t._stream_ptr(None))


def _inputs(rng, M, N, mode):
    F = rng.uniform(-1, 1, size=(M, N))
    if mode != "f64":
        F = F.astype(np.float32)
    Fd = torch.from_numpy(F).to(DEV)
    xdt = torch.float32 if mode == "f32" else torch.float64
    return F, Fd, xdt


@pytest.mark.parametrize("M,P,order", [
    (3000, 32, "recurrence"),      # 93-94-row blocks: the register sweep
    (4096, 64, "dense"),           # 64-row blocks: the halves sweep, MFMA interface
    (2000, 40, "dichotomy"),       # the dichotomy's two extra work slices
])
@pytest.mark.parametrize("mode", ["f64", "f32_refined", "f32_wide", "f32"])
def test_noalloc_equals_series_two_calls(M, P, order, mode):
    print(f"case M={M} P={P} order={order} mode={mode}", flush=True)
    rng = np.random.default_rng(M + P + len(mode))
    a, b = _rand(rng, M)
    plan = t.Plan(a, b, P)
    plan.set_interface(order)
    for N in (1000, 301):                      # the second call is smaller
        F, Fd, xdt = _inputs(rng, M, N, mode)
        X0 = plan.solve(Fd, mode=mode)
        X1 = torch.full((M, N), float("nan"), dtype=xdt, device=DEV)
        assert _noalloc(plan, Fd, X1, mode) == 0
        torch.cuda.synchronize()
        assert torch.equal(X0, X1), (N, mode)
        if mode != "f32":
            ref = oracle.thomas(a, b, F.astype(np.float64))
            e = np.max(np.abs(X1.cpu().numpy() - ref)) / np.max(np.abs(ref))
            assert e <= 1e-12, (N, e)


def test_noalloc_rejects_work_beyond_scratch():
    # P = 64: the largest N whose work area fits is 21930 (include/tdsolve.h)
    rng = np.random.default_rng(5)
    M, P = 128, 64
    a, b = _rand(rng, M)
    plan = t.Plan(a, b, P)
    assert _work_bytes(P, 21930) <= SCRATCH < _work_bytes(P, 21931)
    assert _work_bytes(128, 10943) <= SCRATCH < _work_bytes(128, 10944)
    for N, want in ((21931, ESCRATCH), (21930, 0)):
        F = torch.from_numpy(rng.uniform(-1, 1, size=(M, N)).astype(np.float32)).to(DEV)
        X = torch.empty((M, N), dtype=torch.float64, device=DEV)
        assert _noalloc(plan, F, X, "f32_refined") == want, N
        if want == 0:
            torch.cuda.synchronize()
            assert torch.equal(X, plan.solve(F, mode="f32_refined"))
    with pytest.raises(t.TdsError):
        plan.solve_noalloc(torch.zeros((M, 21931), dtype=torch.float32, device=DEV),
                           torch.empty((M, 21931), dtype=torch.float64, device=DEV))


def test_noalloc_stale_scratch_does_not_leak():
    # A call whose inputs are all NaN leaves NaN weights in the shared
    # scratch, over the rows that a later plan with fewer blocks never writes
    # (beta^L of its first block); the dense order must not read them.
    rng = np.random.default_rng(8)
    M, N = 1024, 64
    a, b = _rand(rng, M)
    pa = t.Plan(a, b, 16)
    Fa = torch.full((M, N), float("nan"), dtype=torch.float64, device=DEV)
    Xa = torch.empty((M, N), dtype=torch.float64, device=DEV)
    assert _noalloc(pa, Fa, Xa, "f64") == 0
    pb = t.Plan(a, b, 8)
    pb.set_interface("dense")
    F = rng.uniform(-1, 1, size=(M, N))
    Fd = torch.from_numpy(F).to(DEV)
    X = torch.empty((M, N), dtype=torch.float64, device=DEV)
    assert _noalloc(pb, Fd, X, "f64") == 0
    torch.cuda.synchronize()
    assert torch.isfinite(X).all()
    assert torch.equal(X, pb.solve(Fd, mode="f64"))
