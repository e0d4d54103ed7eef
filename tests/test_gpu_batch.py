"""GPU parity of the uneven batch (many matrices of different sizes and
series lengths solved by one launch per step) against the CPU oracle, and
of its replays from a captured HIP graph.

Gates as in the single-matrix parity tests (tests/_parity.py): per
right-hand side the forward error within C u (cs_n + co_n + t) of the
oracle's solution and the relative residual, computed on the host by the
oracle's routine, within 1e-10 of the oracle's; the batch matrices are
shifted Poisson matrices with b_i = 2 + c_i, c_i >= 0.01.
"""
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


def _check(a, b, F64, X, P, what="batch item"):
    ref = oracle.thomas(a, b, F64)
    _parity.check(X, ref, _parity.tol64(a, b, F64, ref, P), what)
    _parity.check_residual(a, b, F64, X, ref, what)


@pytest.mark.parametrize("mode", ["f32_refined", "f32_wide", "f64"])
def test_uneven_batch_parity(mode):
    w = wl.uneven_batch(seed=3, K=24, M_lo=128, M_hi=3000, N_hi=700)
    items = w["items"]
    print(f"batch K={len(items)} mode={mode}", flush=True)
    bp = t.BatchPlan([it["a"] for it in items], [it["b"] for it in items])
    Fs = []
    for it in items:
        F = torch.from_numpy(it["F"]).to(DEV)
        Fs.append(F.double() if mode == "f64" else F)
    Xs = bp.solve(Fs, mode=mode)
    torch.cuda.synchronize()
    plans = [t.Plan(it["a"], it["b"], 0) for it in items]
    for k, it in enumerate(items):
        _check(it["a"], it["b"], it["F"].astype(np.float64), Xs[k].cpu().numpy(), plans[k].P)


def test_batch_ragged_shapes_and_empty_series():
    rng = np.random.default_rng(4)
    Ms = [2, 5, 64, 65, 129, 1000, 300]
    Ns = [3, 0, 1, 257, 513, 40, 2]
    a_l, b_l, F_l = [], [], []
    for M, N in zip(Ms, Ns):
        a = rng.uniform(-1, -0.5, size=M - 1)
        b = 2.2 + rng.uniform(0, 1, size=M)
        a_l.append(a); b_l.append(b)
        F_l.append(rng.uniform(-1, 1, size=(M, N)).astype(np.float32))
    P_l = [1, 2, 0, 0, 4, 0, 5]
    bp = t.BatchPlan(a_l, b_l, P_l)
    Xs = bp.solve([torch.from_numpy(F).to(DEV) for F in F_l], mode="f32_refined")
    for k in range(len(Ms)):
        if Ns[k] == 0:
            continue
        P = P_l[k] or t.default_blocks(Ms[k])
        _check(a_l[k], b_l[k], F_l[k].astype(np.float64), Xs[k].cpu().numpy(), P)


@pytest.mark.parametrize("mode", ["f32_refined", "f64", "f32_wide"])
def test_batch_matches_single_plans_bitwise(mode):
    # 64-row blocks that every matrix's halves fit: the batch and the single
    # plans take the same sweep
    w = wl.uneven_batch(seed=11, K=6, M_lo=128, M_hi=1500, N_hi=400)
    items = w["items"]
    bp = t.BatchPlan([it["a"] for it in items], [it["b"] for it in items])
    Fs = [torch.from_numpy(it["F"]).to(DEV) for it in items]
    if mode == "f64":
        Fs = [F.double() for F in Fs]
    Xs = bp.solve(Fs, mode=mode)
    for k, it in enumerate(items):
        X1 = t.Plan(it["a"], it["b"], 0).solve(Fs[k], mode=mode)
        assert torch.equal(X1, Xs[k])


@pytest.mark.parametrize("mode", ["f32_refined", "f64", "f32_wide"])
def test_batch_mixed_row_buckets_bitwise(mode):
    # per-matrix block counts: 32-row blocks for some matrices, 64-row blocks
    # (swept in halves) for the others, one launch of each kernel per bucket;
    # every matrix bitwise its single plan, and the parity gates
    w = wl.uneven_batch(seed=13, K=8, M_lo=300, M_hi=2500, N_hi=600)
    items = w["items"]
    P_l = [-(-it["M"] // (32 if k % 2 else 64)) for k, it in enumerate(items)]
    rows = [-(-it["M"] // p) for it, p in zip(items, P_l)]
    assert any(r <= 32 for r in rows) and any(35 <= r <= 64 for r in rows)
    print(f"mixed buckets rows={rows} mode={mode}", flush=True)
    bp = t.BatchPlan([it["a"] for it in items], [it["b"] for it in items], P_l)
    Fs = [torch.from_numpy(it["F"]).to(DEV) for it in items]
    if mode == "f64":
        Fs = [F.double() for F in Fs]
    Xs = bp.solve(Fs, mode=mode)
    for k, it in enumerate(items):
        X1 = t.Plan(it["a"], it["b"], P_l[k]).solve(Fs[k], mode=mode)
        assert torch.equal(X1, Xs[k]), f"matrix {k} ({rows[k]} rows per block)"
        _check(it["a"], it["b"], it["F"].astype(np.float64), Xs[k].cpu().numpy(), P_l[k])


def test_batch_graph_replays():
    # capture the batch solve once, replay it several times with eager work
    # and synchronizations in between; every replay must equal the eager solve
    w = wl.uneven_batch(seed=12, K=8, M_lo=128, M_hi=2000, N_hi=500)
    items = w["items"]
    bp = t.BatchPlan([it["a"] for it in items], [it["b"] for it in items])
    Fs = [torch.from_numpy(it["F"]).to(DEV) for it in items]
    Xs = [torch.empty((it["M"], it["N"]), dtype=torch.float64, device=DEV) for it in items]
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        bp.solve(Fs, Xs, mode="f32_refined")          # eager: uploads descriptors
    torch.cuda.synchronize()
    ref = [X.clone() for X in Xs]
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        bp.solve(Fs, Xs, mode="f32_refined")
    for rep in range(4):
        for X in Xs:
            X.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for X, R in zip(Xs, ref):
            assert torch.equal(X, R), rep
        _ = (Fs[0] * 2).sum().item()                   # eager work between replays


@pytest.fixture(scope="module")
def full_batch(tmp_path_factory):
    # the full uneven batch (256 matrices, M log-uniform in [128, 16384],
    # N uniform in [1, 2048], FP32 storage with refinement) with the batch
    # autotuner's block counts, in the launch configuration the benchmark
    # times; solved once, checked in four parts below
    import os
    old = os.environ.get("TDSOLVE_AUTOTUNE_CACHE")
    os.environ["TDSOLVE_AUTOTUNE_CACHE"] = str(tmp_path_factory.mktemp("tune") / "autotune.json")
    try:
        items = wl.uneven_batch()["items"]
        a_l, b_l = [it["a"] for it in items], [it["b"] for it in items]
        P_l, ms = t.batch_autotune(a_l, b_l, [it["N"] for it in items], "f32_refined")
    finally:
        if old is None:
            del os.environ["TDSOLVE_AUTOTUNE_CACHE"]
        else:
            os.environ["TDSOLVE_AUTOTUNE_CACHE"] = old
    print(f"full batch: {sum(it['M'] * it['N'] for it in items)} unknowns, {ms:.3f} ms",
          flush=True)
    bp = t.BatchPlan(a_l, b_l, P_l)
    Xs = bp.solve([torch.from_numpy(it["F"]).to(DEV) for it in items], mode="f32_refined")
    torch.cuda.synchronize()
    return items, P_l, Xs


@pytest.mark.timeout(600)
@pytest.mark.parametrize("part", range(4))
def test_uneven_batch_full_size_every_column(full_batch, part):
    # every right-hand side of every matrix against the oracle
    items, P_l, Xs = full_batch
    for k in range(part, len(items), 4):
        it = items[k]
        _check(it["a"], it["b"], it["F"].astype(np.float64), Xs[k].cpu().numpy(), P_l[k],
               f"full batch item {k} M={it['M']} N={it['N']} P={P_l[k]}")


def test_batch_many_small_matrices():
    # 600 matrices of 2..200 rows and 0..40 right-hand sides: most own one to
    # a few work items, so neighbouring items belong to different matrices
    # (the per-item owner table), and some series are empty
    rng = np.random.default_rng(31)
    K = 600
    Ms = rng.integers(2, 201, size=K)
    Ns = rng.integers(0, 41, size=K)
    a_l, b_l, F_l = [], [], []
    for M, N in zip(Ms, Ns):
        a = rng.uniform(-1, -0.5, size=M - 1)
        b = 2.2 + rng.uniform(0, 1, size=M)
        a_l.append(a)
        b_l.append(b)
        F_l.append(rng.uniform(-1, 1, size=(M, N)).astype(np.float32))
    print(f"batch K={K} small matrices", flush=True)
    bp = t.BatchPlan(a_l, b_l)
    Xs = bp.solve([torch.from_numpy(F).to(DEV) for F in F_l], mode="f32_refined")
    for k in range(K):
        if Ns[k] == 0:
            continue
        P = t.default_blocks(int(Ms[k]))
        _check(a_l[k], b_l[k], F_l[k].astype(np.float64), Xs[k].cpu().numpy(), P)
