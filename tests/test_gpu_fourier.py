"""GPU: the series of 2-D Poisson problems by the variable separation
method (paper_0901_2859_amd.fourier: sine transforms along y, one
tridiagonal series per harmonic solved as a batch) against the oracle's
direct sparse solve of the 5-point problem, the exact discrete
eigenfunctions, and the paper's manufactured problem sin(2 pi x) sin(2 pi y).

Tolerances: FP64 mode, 1e-11 relative (transforms and solves round at
~1e-15 times the condition of the low harmonics, ~N^2); FP32 storage with
refinement, 2e-6 relative (the transformed right-hand sides are rounded to
FP32 before the solve)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import poisson2d  # noqa: E402
from paper_0901_2859_amd.fourier import FourierPoisson2D  # noqa: E402

DEV = "cuda:0"


@pytest.mark.parametrize("N1,N2,S,h1,h2", [(64, 64, 8, None, None), (50, 33, 5, 0.02, 0.03),
                                            (129, 70, 300, None, None)])
def test_fourier_matches_direct_solve(N1, N2, S, h1, h2, tmp_path, monkeypatch):
    monkeypatch.setenv("TDSOLVE_AUTOTUNE_CACHE", str(tmp_path / "autotune.json"))
    print(f"fourier N1={N1} N2={N2} S={S}", flush=True)
    rng = np.random.default_rng(N1 + N2 + S)
    f = rng.uniform(-1, 1, size=(S, N1 - 1, N2 - 1))
    fp = FourierPoisson2D(N1, N2, S, h1, h2, mode="f64")
    u = fp.solve(torch.from_numpy(f).to(DEV)).cpu().numpy()
    ks = range(S) if S <= 8 else (0, S // 2, S - 1)
    for s in ks:
        ref = poisson2d.solve_direct(f[s], fp.h1, fp.h2)
        assert np.max(np.abs(u[s] - ref)) <= 1e-11 * np.max(np.abs(ref)), s
    fr = FourierPoisson2D(N1, N2, S, h1, h2, mode="f32_refined")
    u32 = fr.solve(torch.from_numpy(f).to(DEV)).cpu().numpy()
    ref = poisson2d.solve_direct(f[0], fp.h1, fp.h2)
    assert np.max(np.abs(u32[0] - ref)) <= 2e-6 * np.max(np.abs(ref))


def test_fourier_eigenfunctions_and_manufactured(tmp_path, monkeypatch):
    monkeypatch.setenv("TDSOLVE_AUTOTUNE_CACHE", str(tmp_path / "autotune.json"))
    N = 128
    fp = FourierPoisson2D(N, N, 3, mode="f64")
    fs, us = [], []
    for k, l in ((1, 1), (7, 100), (127, 2)):
        f, u = FourierPoisson2D.eigen_rhs(N, N, k, l)
        fs.append(f)
        us.append(u)
    u = fp.solve(torch.from_numpy(np.stack(fs)).to(DEV)).cpu().numpy()
    for s in range(3):
        # rounding in the transforms puts ~1e-16 |f| into the other
        # harmonics; the inverse operator (norm <= 1 / (2 pi^2) here) keeps
        # it at that absolute level, whatever the size of this eigenvalue
        err = np.max(np.abs(u[s] - us[s]))
        assert err <= 1e-12 * np.max(np.abs(us[s])) + 1e-14 * np.max(np.abs(fs[s])), s
    # the paper's problem: -Delta u = 8 pi^2 sin(2 pi x) sin(2 pi y)
    errs = []
    for n in (64, 128):
        h = 1.0 / n
        x = np.arange(1, n)[:, None] * h
        ue = np.sin(2 * np.pi * x) * np.sin(2 * np.pi * x.T)
        fq = FourierPoisson2D(n, n, 1, mode="f64")
        u = fq.solve(torch.from_numpy((8 * np.pi ** 2 * ue)[None]).to(DEV)).cpu().numpy()[0]
        errs.append(np.max(np.abs(u - ue)))
    assert 3.8 < errs[0] / errs[1] < 4.2, errs


def test_fourier_on_a_side_stream(tmp_path, monkeypatch):
    # with a stream argument every step (transforms, copies, batch solve)
    # runs on that stream: the result equals the default-stream solve
    monkeypatch.setenv("TDSOLVE_AUTOTUNE_CACHE", str(tmp_path / "autotune.json"))
    rng = np.random.default_rng(77)
    N1, N2, S = 96, 80, 40
    f = torch.from_numpy(rng.uniform(-1, 1, size=(S, N1 - 1, N2 - 1))).to(DEV)
    fp = FourierPoisson2D(N1, N2, S, mode="f64")
    ref = fp.solve(f)
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    for rep in range(3):
        u = fp.solve(f, stream=side)
        side.synchronize()
        assert torch.equal(u, ref), rep
