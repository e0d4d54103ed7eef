"""GPU: the sweep of blocks of 34..65 interior rows in the modes with FP64
results, which the library solves in two halves per block (a left half of
32 rows, the middle row from its own equation, a right half of 1..31 rows;
Lemma 1 per half), against the CPU oracle's sweep.

The shapes cover even and ragged partitions, the shortest right half (one
row: blocks of 35 rows), one block (no interface rows), column counts that
leave part of the last workgroup idle, a non-symmetric matrix, and the
partition just below the split (blocks of 34 rows, swept whole).

Gates as in the parity tests (tests/_parity.py): per right-hand side the
forward error within C u (cs_n + co_n + t) of the oracle's solution, and
the relative residual, computed on the host by the oracle's routine, within
1e-10 of the oracle's."""
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


def _r2(a, b, F, X):
    return method.residual_columns(a, b, F, X)["r2"]


@pytest.mark.parametrize("M,N,P,halves", [
    (4096, 300, 64, 1),    # 64-row segments: 32 + middle + 30 rows (block 0: + 31)
    (2543, 129, 40, 1),    # ragged, 63 and 64 rows; one live column in the last workgroup
    (700, 64, 20, 1),      # 35-row segments: right halves of one row
    (720, 200, 20, 1),     # 36-row segments
    (50, 10, 1, 1),        # one block, no interface rows
    (64 * 30 - 7, 257, 30, 1),  # 64 and 63 rows; one live column in the last workgroup
    (2048, 2000, 32, 1),   # 16 tiles of 128: the XCD-matched tile order, last tile partial
    (680, 70, 20, 0),      # 34-row segments: below the split, swept whole
])
@pytest.mark.parametrize("mode", ["f32_refined", "f64", "f32_wide"])
def test_halves_match_oracle(M, N, P, halves, mode):
    print(f"halves M={M} N={N} P={P} mode={mode}", flush=True)
    rng = np.random.default_rng(M + N + P)
    a = rng.uniform(-1, -0.2, size=M - 1)
    b = np.concatenate([[0], np.abs(a)]) + np.concatenate([np.abs(a), [0]]) + rng.uniform(0.05, 0.5, size=M)
    F32 = rng.uniform(-1, 1, size=(M, N)).astype(np.float32)
    F = F32.astype(np.float64)
    ref = oracle.thomas(a, b, F)
    plan = t.Plan(a, b, P)
    assert plan.P == P and plan.info().sweep_halves == halves
    Fd = torch.from_numpy(F32).to(DEV)
    X = plan.solve(Fd.double() if mode == "f64" else Fd, mode=mode).cpu().numpy()
    what = f"halves M={M} N={N} P={P} {mode}"
    _parity.check(X, ref, _tol(a, b, F, ref, P), what)
    _parity.check_residual(a, b, F, X, ref, what)


def test_refined_halves_poisson_passes():
    # the Poisson series on 64-row blocks with 0, 1 and 3 refinement passes:
    # each pass brings the halves' zero-boundary solves closer to FP64
    w = wl.poisson_series(M=4096, N=256, P=64)
    a, b, F32 = w["a"], w["b"], w["F"]
    F = F32.astype(np.float64)
    ref = oracle.thomas(a, b, F)
    r2_or = _r2(a, b, F, ref)
    plan = t.Plan(a, b, 64)
    Fd = torch.from_numpy(F32).to(DEV)
    r2 = {}
    for passes in (0, 1, 3):
        plan.set_refinement(passes)
        X = plan.solve(Fd, mode="f32_refined").cpu().numpy()
        r2[passes] = _r2(a, b, F, X)
    assert np.all(r2[1] <= r2_or + 1e-10) and np.all(r2[3] <= r2_or + 1e-10)
    assert r2[1].max() < r2[0].max()


def test_refined_halves_general_matrix():
    # non-symmetric A (sub- and super-diagonal of one sign per row pair) on
    # ragged 56/57-row segments
    rng = np.random.default_rng(21)
    M, N, P = 57 * 25 - 9, 150, 25
    up = rng.uniform(0.2, 1.0, size=M - 1) * rng.choice([-1.0, 1.0], size=M - 1)
    lo = np.sign(up) * rng.uniform(0.2, 1.0, size=M - 1)
    d = (np.concatenate([[0], np.abs(lo)]) + np.concatenate([np.abs(up), [0]]) + 0.3) * \
        rng.choice([-1.0, 1.0], size=M)
    F32 = rng.uniform(-1, 1, size=(M, N)).astype(np.float32)
    F = F32.astype(np.float64)
    low, upp = np.concatenate([[0.0], lo]), np.concatenate([up, [0.0]])
    ref = np.stack([oracle.tridiag_general(low, d, upp, F[:, n]) for n in range(N)], 1)
    plan = t.Plan.general(lo, d, up, P)
    assert plan.info().sweep_halves == 1
    X = plan.solve(torch.from_numpy(F32).to(DEV), mode="f32_refined").cpu().numpy()
    _parity.check(X, ref, _parity.tol64(up, d, F, ref, P, lower=lo), "halves general refined")


def test_refined_halves_reproducible_and_in_place_of_rows():
    # two solves give the same bits; every row is written (X starts as NaN)
    rng = np.random.default_rng(5)
    M, N, P = 4096, 384, 64
    a = rng.uniform(-1, -0.5, size=M - 1)
    b = 2.2 + rng.uniform(0, 1, size=M)
    F = torch.from_numpy(rng.uniform(-1, 1, size=(M, N)).astype(np.float32)).to(DEV)
    plan = t.Plan(a, b, P)
    X1 = torch.full((M, N), float("nan"), dtype=torch.float64, device=DEV)
    X2 = torch.full((M, N), float("nan"), dtype=torch.float64, device=DEV)
    plan.solve(F, X1, mode="f32_refined")
    plan.solve(F, X2, mode="f32_refined")
    assert not torch.isnan(X1).any()
    assert torch.equal(X1, X2)


@pytest.mark.parametrize("mode", ["f32_refined", "f64", "f32_wide"])
def test_unaligned_series_takes_the_scalar_beta_path_bitwise(mode):
    # F starting one element past a 16-byte boundary cannot be read by the
    # vector-load beta kernel (8-byte loads on FP32 input, 16-byte on
    # FP64); the one-RHS-per-lane kernel forms the same
    # weights in the same order, so X is bitwise that of the aligned solve
    rng = np.random.default_rng(17)
    M, N, P = 4096, 512, 64
    a = rng.uniform(-1, -0.5, size=M - 1)
    b = 2.2 + rng.uniform(0, 1, size=M)
    dt = torch.float64 if mode == "f64" else torch.float32
    F = torch.from_numpy(rng.uniform(-1, 1, size=(M, N))).to(DEV, dt)
    buf = torch.empty(M * N + 1, dtype=dt, device=DEV)
    Fu = buf[1:].view(M, N)
    Fu.copy_(F)
    assert Fu.data_ptr() % 16 != 0 and F.data_ptr() % 16 == 0
    plan = t.Plan(a, b, P)
    X1 = plan.solve(F, mode=mode)
    X2 = plan.solve(Fu, mode=mode)
    assert torch.equal(X1, X2)
