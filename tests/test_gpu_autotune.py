"""GPU: the measured choices (tdsolve_autotune, tdsolve_autotune_plan,
tdsolve_batch_autotune) and their JSON cache.  The chosen decomposition,
interface order and launch order are free parameters of the method, so the
checks are that each choice is one of the candidates, that a plan built
with it solves to the oracle's tolerance, that the refinement passes meet
the stated accuracy rule, and that the cache returns the stored choice
without measuring again."""
import json

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
from paper_0901_2859_amd import tdsolve as t  # noqa: E402
from paper_0901_2859_amd import workloads as wl  # noqa: E402

DEV = "cuda:0"


def _candidates(M):
    out = set()
    for rows in (16, 32, 64, 128):
        P = 1 if M < 4 else max(1, min(-(-M // rows), M // 2, 65535))
        out.add(P)
    if M <= 128:
        out.add(1)
    return out


@pytest.mark.parametrize("M,N,mode", [(4096, 512, "f32_refined"), (1000, 300, "f64"),
                                      (100, 17, "f32_wide")])
def test_autotune_choice_solves(M, N, mode, tmp_path, monkeypatch):
    monkeypatch.setenv("TDSOLVE_AUTOTUNE_CACHE", str(tmp_path / "cache.json"))
    rng = np.random.default_rng(M + N)
    a = -rng.uniform(0.5, 1.0, size=M - 1)
    b = 2.2 + rng.uniform(0.0, 1.0, size=M)
    P, ms = t.autotune(a, b, N, mode)
    print(f"autotune M={M} N={N} mode={mode}: P={P} {ms:.4f} ms", flush=True)
    assert P in _candidates(M) and ms > 0
    F = rng.uniform(-1, 1, size=(M, N))
    Fin = torch.from_numpy(F if mode == "f64" else F.astype(np.float32)).to(DEV)
    X = t.Plan(a, b, P).solve(Fin, mode=mode).cpu().numpy()
    ref = oracle.thomas(a, b, Fin.cpu().double().numpy())
    assert np.max(np.abs(X - ref)) <= 1e-11 * np.max(np.abs(ref))
    # second call: answered from the cache file
    data = json.loads((tmp_path / "cache.json").read_text())
    assert any(v["P"] == P for v in data.values())
    key = next(iter(data))
    data[key]["P"] = 1            # a value measurement could not give here
    (tmp_path / "cache.json").write_text(json.dumps(data))
    if M > 128:
        assert t.autotune(a, b, N, mode)[0] == 1
        assert t.autotune(a, b, N, mode, cache=False)[0] in _candidates(M)


def test_batch_autotune_choice_solves(tmp_path, monkeypatch):
    monkeypatch.setenv("TDSOLVE_AUTOTUNE_CACHE", str(tmp_path / "cache.json"))
    w = wl.uneven_batch(seed=9, K=12, M_lo=64, M_hi=3000, N_hi=600)
    items = w["items"]
    a_l, b_l = [it["a"] for it in items], [it["b"] for it in items]
    P_l, ms = t.batch_autotune(a_l, b_l, [it["N"] for it in items], "f32_refined")
    assert ms > 0 and len(P_l) == len(items)
    rows = {32, 64}
    ok = [r for r in rows
          if all(P == (1 if it["M"] < 4 else max(1, min(-(-it["M"] // r), it["M"] // 2)))
                 for P, it in zip(P_l, items))]
    assert ok, P_l
    bp = t.BatchPlan(a_l, b_l, P_l)
    Xs = bp.solve([torch.from_numpy(it["F"]).to(DEV) for it in items], mode="f32_refined")
    torch.cuda.synchronize()
    for k, it in enumerate(items):
        ref = oracle.thomas(it["a"], it["b"], it["F"].astype(np.float64))
        X = Xs[k].cpu().numpy()
        assert np.max(np.abs(X - ref)) <= 1e-11 * np.max(np.abs(ref)), k
    assert t.batch_autotune(a_l, b_l, [it["N"] for it in items], "f32_refined")[0] == P_l


def test_autotune_rejects_bad_arguments():
    a, b = -np.ones(9), 3 * np.ones(10)
    with pytest.raises(t.TdsError):
        t.autotune(a, b, 0, "f64", cache=False)
    with pytest.raises(t.TdsError):
        t.autotune(a, b, 4, 7, cache=False)


SLACK = 1.25     # the autotuner's passes rule: residual within this factor of FP64 arithmetic's


@pytest.mark.parametrize("mode", ["f32_refined", "f32_wide", "f64"])
def test_autotune_plan_choice_solves(mode):
    # the Poisson series (ill-conditioned, P fixed at 64) and its own
    # right-hand sides: the plan configured as chosen meets the parity gates,
    # and in the refined mode the chosen passes are the fewest whose residual
    # stays within 1.25 times the FP64-arithmetic solve's
    from tests import _parity
    w = wl.poisson_series(M=4096, N=1024, P=64)
    a, b, F32 = w["a"], w["b"], w["F"]
    Fs = torch.from_numpy(F32).to(DEV)
    Fin = Fs.double() if mode == "f64" else Fs
    tun = t.autotune_plan(a, b, 1024, mode, P=64, F=Fin)
    print(f"autotune_plan {mode}: {tun}", flush=True)
    assert tun["P"] == 64 and tun["order"] in ("recurrence", "dense") and tun["ms"] > 0
    assert (tun["fuse_lag"], tun["fuse_tile"]) in ((0, 0), (8, 512))
    plan = t.Plan(a, b, 64)
    plan.set_interface(tun["order"])
    plan.set_fused(tun["fuse_lag"], tun["fuse_tile"] or 512)
    if mode == "f32_refined":
        assert 1 <= tun["passes"] <= 3
        plan.set_refinement(tun["passes"])
    else:
        assert tun["passes"] == 0
    Xh = plan.solve(Fin, mode=mode).cpu().numpy()
    Fw = F32.astype(np.float64)
    ref = oracle.thomas(a, b, Fw)
    _parity.check(Xh, ref, _parity.tol64(a, b, Fw, ref, 64), f"autotuned poisson {mode}")
    r2 = _parity.method.residual_columns(a, b, Fw, Xh)["r2"].max()
    assert abs(r2 - tun["r2"]) <= 1e-3 * r2
    if mode == "f32_refined":
        # the rule is applied on a fresh plan (recurrence order, three launches)
        p0 = t.Plan(a, b, 64)
        Xw = p0.solve(Fs, mode="f32_wide").cpu().numpy()
        r2w = _parity.method.residual_columns(a, b, Fw, Xw)["r2"].max()
        p0.set_refinement(tun["passes"])
        Xp = p0.solve(Fs, mode=mode).cpu().numpy()
        assert _parity.method.residual_columns(a, b, Fw, Xp)["r2"].max() <= SLACK * r2w * (1 + 1e-3)
        if tun["passes"] > 1:
            p0.set_refinement(tun["passes"] - 1)
            Xp = p0.solve(Fs, mode=mode).cpu().numpy()
            assert _parity.method.residual_columns(a, b, Fw, Xp)["r2"].max() > SLACK * r2w * (1 - 1e-3)


def test_batch_autotune_passes(tmp_path, monkeypatch):
    monkeypatch.setenv("TDSOLVE_AUTOTUNE_CACHE", str(tmp_path / "cache.json"))
    w = wl.uneven_batch(seed=9, K=12, M_lo=64, M_hi=3000, N_hi=600)
    items = w["items"]
    a_l, b_l = [it["a"] for it in items], [it["b"] for it in items]
    Ns = [it["N"] for it in items]
    P_l, passes, ms = t.batch_autotune(a_l, b_l, Ns, "f32_refined", with_passes=True)
    assert 1 <= passes <= 3 and ms > 0
    # per matrix, 32 or 64 rows per block
    for it, P in zip(items, P_l):
        M = it["M"]
        assert P in (max(1, min(-(-M // 32), M // 2)), max(1, min(-(-M // 64), M // 2))), (M, P)
    assert t.batch_autotune(a_l, b_l, Ns, "f32_refined", with_passes=True) == (P_l, passes, ms)
    assert t.batch_autotune(a_l, b_l, Ns, "f64", with_passes=True)[1] == 0
    # the launch order: a lag of the one-launch order only when every
    # matrix has 32-row blocks, and the chosen order solves as the other
    P_l, passes, lag, ms = t.batch_autotune(a_l, b_l, Ns, "f64", with_order=True)
    assert lag in (0, 8, 16, 32) and ms > 0
    if lag:
        assert all(P == max(1, min(-(-it["M"] // 32), it["M"] // 2)) for it, P in zip(items, P_l))
    bp = t.BatchPlan(a_l, b_l, P_l)
    Fs = [torch.from_numpy(it["F"]).to(DEV).double() for it in items]
    X0 = bp.solve(Fs, mode="f64")
    bp.set_fused(lag)
    X1 = bp.solve(Fs, mode="f64")
    for k in range(len(items)):
        assert torch.equal(X0[k], X1[k]), k
