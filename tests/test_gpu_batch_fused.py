"""GPU: the one-launch order of the uneven batch (tdsolve_batch_set_fused):
the beta, interface and sweep items of every matrix in one grid, taken in
ticket order tile by tile of 256 right-hand sides, the interface items
waiting on their tile's weights and the sweeps on their tile's interface
values.  The work items and their arithmetic are those of the separate
launches, so X must be bitwise equal to them; one case is also held to the
oracle's gates (tests/_parity.py).

Shapes: an uneven batch with 32-row blocks, ragged matrices (M = 2 with
P = 1, empty series, one right-hand side, N not a multiple of 256), lags
shorter and longer than the batch's tiles, every mode, replays of a captured graph,
the full benchmark batch; a batch with a 64-row-block matrix must fall
back to the separate launches with the same result.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
from tests import _parity  # noqa: E402
from paper_0901_2859_amd import tdsolve as t  # noqa: E402
from paper_0901_2859_amd import workloads as wl  # noqa: E402

DEV = "cuda:0"


def _rows32(M):
    # blocks of at most 32 rows, within the method's limits (P <= M / 2)
    return max(1, min(-(-M // 32), M // 2))


def _inputs(items, mode):
    Fs = [torch.from_numpy(it["F"]).to(DEV) for it in items]
    return [F.double() for F in Fs] if mode == "f64" else Fs


def _both(bp, Fs, mode, lag):
    bp.set_fused(0)
    X0 = bp.solve(Fs, mode=mode)
    bp.set_fused(lag)
    X1 = [torch.full_like(X, float("nan")) for X in X0]
    bp.solve(Fs, X1, mode=mode)
    torch.cuda.synchronize()
    return X0, X1


@pytest.mark.parametrize("lag", [1, 2, 5, 40])
@pytest.mark.parametrize("mode", ["f32_refined", "f32_wide", "f64", "f32"])
def test_fused_batch_bitwise_equals_separate_launches(mode, lag):
    w = wl.uneven_batch(seed=3, K=24, M_lo=128, M_hi=3000, N_hi=700)
    items = w["items"]
    print(f"fused batch K={len(items)} mode={mode} lag={lag}", flush=True)
    bp = t.BatchPlan([it["a"] for it in items], [it["b"] for it in items],
                     [_rows32(it["M"]) for it in items])
    X0, X1 = _both(bp, _inputs(items, mode), mode, lag)
    for k in range(len(items)):
        assert torch.equal(X0[k], X1[k]), (mode, lag, k)


def test_fused_batch_ragged_shapes_meet_oracle_gates():
    rng = np.random.default_rng(14)
    Ms = [2, 5, 64, 65, 129, 1000, 300, 33]
    Ns = [3, 0, 1, 257, 513, 40, 2, 700]
    a_l, b_l, F_l = [], [], []
    for M, N in zip(Ms, Ns):
        a_l.append(rng.uniform(-1, -0.5, size=M - 1))
        b_l.append(2.2 + rng.uniform(0, 1, size=M))
        F_l.append(rng.uniform(-1, 1, size=(M, N)).astype(np.float32))
    P_l = [_rows32(M) for M in Ms]
    bp = t.BatchPlan(a_l, b_l, P_l)
    Fs = [torch.from_numpy(F).to(DEV) for F in F_l]
    for lag in (1, 3, 12, 64):
        print(f"ragged fused batch lag={lag}", flush=True)
        X0, X1 = _both(bp, Fs, "f32_refined", lag)
        for k in range(len(Ms)):
            assert torch.equal(X0[k], X1[k]), (lag, k)
    for k in range(len(Ms)):
        if Ns[k] == 0:
            continue
        F64 = F_l[k].astype(np.float64)
        ref = oracle.thomas(a_l[k], b_l[k], F64)
        X = X1[k].cpu().numpy()
        what = f"fused batch M={Ms[k]} N={Ns[k]}"
        _parity.check(X, ref, _parity.tol64(a_l[k], b_l[k], F64, ref, P_l[k]), what)
        _parity.check_residual(a_l[k], b_l[k], F64, X, ref, what)


def test_fused_batch_falls_back_with_a_64_row_matrix():
    # one matrix with 64-row blocks: the separate launches run, same X
    w = wl.uneven_batch(seed=8, K=6, M_lo=200, M_hi=2000, N_hi=300)
    items = w["items"]
    P_l = [_rows32(it["M"]) for it in items]
    P_l[2] = -(-items[2]["M"] // 64)
    bp = t.BatchPlan([it["a"] for it in items], [it["b"] for it in items], P_l)
    X0, X1 = _both(bp, _inputs(items, "f32_refined"), "f32_refined", 2)
    for k in range(len(items)):
        assert torch.equal(X0[k], X1[k]), k


def test_fused_batch_graph_replays():
    w = wl.uneven_batch(seed=5, K=16, M_lo=128, M_hi=2500, N_hi=600)
    items = w["items"]
    bp = t.BatchPlan([it["a"] for it in items], [it["b"] for it in items],
                     [_rows32(it["M"]) for it in items])
    Fs = _inputs(items, "f32_refined")
    bp.set_fused(0)
    ref = [X.clone() for X in bp.solve(Fs, mode="f32_refined")]
    bp.set_fused(2)
    Xs = [torch.empty_like(X) for X in ref]
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        bp.solve(Fs, Xs, mode="f32_refined", stream=s)     # uploads the ticket table
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        bp.solve(Fs, Xs, mode="f32_refined", stream=s)
    for rep in range(4):
        for X in Xs:
            X.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for k in range(len(items)):
            assert torch.equal(Xs[k], ref[k]), (rep, k)
        _ = (Fs[0] * 2).sum().item()


def test_fused_batch_full_benchmark_batch():
    # the 256-matrix benchmark batch with 32-row blocks
    w = wl.uneven_batch()
    items = w["items"]
    bp = t.BatchPlan([it["a"] for it in items], [it["b"] for it in items],
                     [_rows32(it["M"]) for it in items])
    Fs = _inputs(items, "f32_refined")
    X0, X1 = _both(bp, Fs, "f32_refined", 2)
    for k in range(len(items)):
        assert torch.equal(X0[k], X1[k]), k


def test_fused_batch_lag_limits():
    w = wl.uneven_batch(seed=2, K=3, M_lo=100, M_hi=200, N_hi=10)
    items = w["items"]
    bp = t.BatchPlan([it["a"] for it in items], [it["b"] for it in items])
    for lag in (-1, 65):
        with pytest.raises(RuntimeError):
            bp.set_fused(lag)
    bp.set_fused(64)
    bp.set_fused(0)


def test_fused_batch_status_and_phase_timing():
    # the last one-launch solve is what tdsolve_status checks, and phase
    # timing reports the one launch as the sweep phase
    w = wl.uneven_batch(seed=6, K=10, M_lo=128, M_hi=2000, N_hi=500)
    items = w["items"]
    bp = t.BatchPlan([it["a"] for it in items], [it["b"] for it in items],
                     [_rows32(it["M"]) for it in items])
    bp.set_refinement(2)
    Fs = _inputs(items, "f32_refined")
    bp.set_fused(0)
    bp.solve(Fs, mode="f32_refined")
    eta0, passes0 = bp.status()
    bp.set_fused(4)
    Xs = bp.solve(Fs, mode="f32_refined")
    eta1, passes1 = bp.status()
    assert eta1 == eta0 and passes1 == passes0 == 2
    assert 0.0 < eta1 < 1e-14
    bp.timing(True)
    bp.timing_read()
    for _ in range(3):
        bp.solve(Fs, Xs, mode="f32_refined")
    mb, mi, ms, calls = bp.timing_read()
    bp.timing(False)
    assert calls == 3 and mb == 0.0 and mi == 0.0 and ms > 0.0
