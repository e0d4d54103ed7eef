"""GPU: the fused order of a single-matrix solve (tdsolve_set_fused): one
launch whose workgroups take the beta, interface and sweep items in ticket
order, tile by tile of 256 right-hand sides, the interface items waiting on
their tile's weights and the sweeps (after their zero-boundary solves) on
their tile's interface values.  The work items and their arithmetic are
those of the three-launch order, so X must be bitwise equal to it; the
solution is also held to the oracle's gates (tests/_parity.py).

Shapes: several tiles with a ragged last one, a lag longer than the series,
N not a multiple of the 256-RHS tile, both interface orders, every mode
with FP64 results, a non-symmetric matrix, the entry point that allocates
nothing, and replays of a captured graph.  Shapes outside the fused order
(odd N, unaligned F, the dichotomy order, the FP32-result mode) must fall
back to the three launches with the same result.
"""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
from tests import _parity  # noqa: E402
from paper_0901_2859_amd import tdsolve as t  # noqa: E402
from paper_0901_2859_amd import workloads as wl  # noqa: E402

DEV = "cuda:0"


def _dominant(rng, M):
    a = rng.uniform(-1, -0.3, size=M - 1)
    b = np.concatenate([[0], np.abs(a)]) + np.concatenate([np.abs(a), [0]]) + rng.uniform(0.05, 0.5, size=M)
    return a, b


def _both(plan, F, mode, lag, tile=1024):
    plan.set_fused(0)
    X0 = plan.solve(F, mode=mode)
    plan.set_fused(lag, tile)
    X1 = torch.full_like(X0, float("nan"))
    plan.solve(F, X1, mode=mode)
    torch.cuda.synchronize()
    return X0, X1


@pytest.mark.parametrize("M,N,P,lag,tile,order", [
    (4096, 4096, 64, 4, 256, "dense"),          # 16 tiles
    (4096, 3000, 64, 2, 512, "dense"),          # ragged last tile
    (4096, 1000, 64, 8, 256, "recurrence"),     # lag longer than the series (4 tiles)
    (8192, 2052, 128, 3, 512, "recurrence"),    # P = 128, N % 256 = 4
    (8192, 2048, 128, 1, 1024, "dense"),        # the shortest lag
    (2543, 772, 40, 2, 256, "recurrence"),      # ragged 63/64-row blocks
    (4096, 4, 64, 1, 2048, "dense"),            # one tile of 4 columns
    (4096, 4100, 64, 1, 2048, "recurrence"),    # 3 tiles, the last of 4 columns
])
@pytest.mark.parametrize("mode", ["f32_refined", "f32_wide", "f64"])
def test_fused_bitwise_equals_three_launches(M, N, P, lag, tile, order, mode):
    print(f"fused M={M} N={N} P={P} lag={lag} tile={tile} {order} {mode}", flush=True)
    rng = np.random.default_rng(M + N + P + lag)
    a, b = _dominant(rng, M)
    F32 = rng.uniform(-1, 1, size=(M, N)).astype(np.float32)
    plan = t.Plan(a, b, P)
    assert plan.info().sweep_halves == 1
    plan.set_interface(order)
    Fd = torch.from_numpy(F32).to(DEV)
    if mode == "f64":
        Fd = Fd.double()
    X0, X1 = _both(plan, Fd, mode, lag, tile)
    assert torch.equal(X0, X1)
    if N <= 2052:
        Fw = F32.astype(np.float64)
        ref = oracle.thomas(a, b, Fw)
        Xh = X1.cpu().numpy()
        what = f"fused M={M} N={N} P={P} {order} {mode}"
        _parity.check(Xh, ref, _parity.tol64(a, b, Fw, ref, P), what)
        _parity.check_residual(a, b, Fw, Xh, ref, what)


def test_fused_adi_full_size_against_oracle():
    # the ADI line solves (8192 x 8192, P = 128) in the fused order, every
    # column against the oracle
    w = wl.adi_lines()
    a, b, F32 = w["a"], w["b"], w["F"]
    Fw = F32.astype(np.float64)
    ref = oracle.thomas(a, b, Fw)
    tol = _parity.tol64(a, b, Fw, ref, w["P"])
    plan = t.Plan(a, b, w["P"])
    plan.set_fused(2, 1024)
    Fs = torch.from_numpy(F32).to(DEV)
    for mode in ("f32_refined", "f32_wide"):
        Xh = plan.solve(Fs, mode=mode).cpu().numpy()
        what = f"fused adi 8192x8192 {mode}"
        _parity.check(Xh, ref, tol, what)
        _parity.check_residual(a, b, Fw, Xh, ref, what)
        del Xh


def test_fused_general_matrix():
    rng = np.random.default_rng(3)
    M, N, P = 64 * 40, 1024, 40
    up = rng.uniform(0.2, 1.0, size=M - 1) * rng.choice([-1.0, 1.0], size=M - 1)
    lo = np.sign(up) * rng.uniform(0.2, 1.0, size=M - 1)
    d = (np.concatenate([[0], np.abs(lo)]) + np.concatenate([np.abs(up), [0]]) + 0.3) * \
        rng.choice([-1.0, 1.0], size=M)
    plan = t.Plan.general(lo, d, up, P)
    assert plan.info().sweep_halves == 1
    F = torch.from_numpy(rng.uniform(-1, 1, size=(M, N)).astype(np.float32)).to(DEV)
    for mode in ("f32_refined", "f32_wide"):
        X0, X1 = _both(plan, F, mode, 2)
        assert torch.equal(X0, X1), mode


@pytest.mark.parametrize("case", ["n_odd", "unaligned", "dichotomy", "f32"])
def test_fused_falls_back_outside_its_shapes(case):
    rng = np.random.default_rng(9)
    M, N, P = 4096, 1025 if case == "n_odd" else 1024, 64
    a, b = _dominant(rng, M)
    plan = t.Plan(a, b, P)
    F32 = rng.uniform(-1, 1, size=(M, N)).astype(np.float32)
    if case == "unaligned":
        buf = torch.empty(M * N + 1, dtype=torch.float32, device=DEV)
        F = buf[1:].view(M, N)
        F.copy_(torch.from_numpy(F32))
    else:
        F = torch.from_numpy(F32).to(DEV)
    if case == "dichotomy":
        plan.set_interface("dichotomy")
    mode = "f32" if case == "f32" else "f32_refined"
    X0, X1 = _both(plan, F, mode, 2)
    assert torch.equal(X0, X1)


def test_fused_noalloc_and_graph_replays():
    rng = np.random.default_rng(11)
    M, N, P = 4096, 2048, 64
    a, b = _dominant(rng, M)
    plan = t.Plan(a, b, P)
    plan.set_interface("dense")
    F = torch.from_numpy(rng.uniform(-1, 1, size=(M, N)).astype(np.float32)).to(DEV)
    plan.set_fused(0)
    ref = plan.solve(F, mode="f32_refined")
    plan.set_fused(2)
    X = torch.full_like(ref, float("nan"))
    rc = t.lib().tdsolve_series_noalloc(plan._h, ctypes.c_void_p(F.data_ptr()),
                                        ctypes.c_void_p(X.data_ptr()), N, t.MODES["f32_refined"],
                                        t._stream_ptr(None))
    assert rc == 0
    torch.cuda.synchronize()
    assert torch.equal(X, ref)
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        plan.solve(F, X, mode="f32_refined")
    for rep in range(3):
        X.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(X, ref), rep
        _ = (F * 2).sum().item()


def test_set_fused_rejects_bad_arguments():
    plan = t.Plan(-np.ones(127), 3 * np.ones(128), 2)
    for lag, tile in ((-1, 1024), (65, 1024), (1, 100), (1, 0), (1, 3 << 20)):
        with pytest.raises(t.TdsError):
            plan.set_fused(lag, tile)
    plan.set_fused(0, 0)
    plan.set_fused(64, 256)
