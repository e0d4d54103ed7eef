"""GPU: the library's per-phase timing (tdsolve_timing_enable/read).  Each
timed call launches its three kernels with start and stop events that take
the kernels' own timestamps, so the phases are positive, are counted per
call, and add up to no more than the wall time of the calls; a phase without
a kernel (one block: no beta weights, no interface step) reads zero."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_0901_2859_amd import tdsolve as t  # noqa: E402
from paper_0901_2859_amd import workloads as wl  # noqa: E402

DEV = "cuda:0"


def _wall_ms(fn, reps):
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b)


@pytest.mark.parametrize("order", ["recurrence", "dense"])
def test_single_plan_phases(order):
    w = wl.poisson_series(M=2048, N=2048, P=32)
    plan = t.Plan(w["a"], w["b"], 32)
    plan.set_interface(order)
    F = torch.from_numpy(w["F"]).to(DEV)
    X = torch.empty((2048, 2048), dtype=torch.float64, device=DEV)
    plan.solve(F, X, mode="f32_refined")
    plan.timing(True)
    plan.timing_read()
    wall = _wall_ms(lambda: plan.solve(F, X, mode="f32_refined"), 7)
    b, i, s, calls = plan.timing_read()
    plan.timing(False)
    assert calls == 7
    assert b > 0 and i > 0 and s > 0
    assert b + i + s <= wall * 1.001
    # timing off: nothing recorded
    plan.solve(F, X, mode="f32_refined")
    torch.cuda.synchronize()
    assert plan.timing_read()[3] == 0


def test_single_block_has_empty_phases():
    a, b = -np.ones(99), 3 * np.ones(100)
    plan = t.Plan(a, b, 1)
    F = torch.ones((100, 300), dtype=torch.float64, device=DEV)
    plan.timing(True)
    for _ in range(3):
        plan.solve(F, mode="f64")
    mb, mi, ms, calls = plan.timing_read()
    assert calls == 3 and mb == 0.0 and mi == 0.0 and ms > 0


def test_batch_phases():
    items = wl.uneven_batch(seed=4, K=12, M_lo=200, M_hi=3000, N_hi=700)["items"]
    bp = t.BatchPlan([it["a"] for it in items], [it["b"] for it in items])
    Fs = [torch.from_numpy(it["F"]).to(DEV) for it in items]
    bp.solve(Fs, mode="f32_refined")
    bp.timing(True)
    bp.timing_read()
    wall = _wall_ms(lambda: bp.solve(Fs, mode="f32_refined"), 4)
    b, i, s, calls = bp.timing_read()
    assert calls == 4 and b > 0 and i > 0 and s > 0
    assert b + i + s <= wall * 1.001
