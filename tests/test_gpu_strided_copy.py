"""GPU: the library's tiled strided copy (tdsolve_strided_copy), used by the
Fourier driver to move S problems between the mesh layout (s, i, l) and the
per-harmonic RHS-interleaved layout (l, i, s), against torch's own strided
copy of the same views.  Exact: a copy times alpha is one rounding per
element on both sides."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_0901_2859_amd import tdsolve as t  # noqa: E402

DEV = "cuda:0"


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
@pytest.mark.parametrize("S,M,L", [(256, 5, 1023), (1, 1, 1), (65, 3, 129), (130, 2, 63)])
def test_transposing_copy_both_ways(dtype, S, M, L):
    print(f"strided copy S={S} M={M} L={L} {dtype}", flush=True)
    g = torch.Generator(device="cpu").manual_seed(S + M + L)
    A = torch.rand((S, M, L), generator=g, dtype=torch.float64).to(DEV, dtype)
    # (s, i, l) -> (l, i, s), scaled
    B = torch.empty((L, M, S), dtype=dtype, device=DEV)
    t.strided_copy(B.permute(2, 1, 0), A, -0.25)
    assert torch.equal(B, (A * -0.25).permute(2, 1, 0).contiguous())
    # and back into the padded rows of a wider array, pads untouched
    W = 2 * (L + 1)
    Y = torch.full((S, M, W), 7.0, dtype=dtype, device=DEV)
    t.strided_copy(Y[..., 1:L + 1], B.permute(2, 1, 0), 1.0)
    assert torch.equal(Y[..., 1:L + 1], A * -0.25)
    assert torch.all(Y[..., 0] == 7.0) and torch.all(Y[..., L + 1:] == 7.0)


def test_copy_from_the_imaginary_part_of_a_spectrum():
    # the driver's forward copy reads the imaginary parts of a complex FFT
    # output: every other float, offset by one element
    x = torch.rand((64, 3, 200), dtype=torch.float32, device=DEV)
    z = torch.fft.rfft(x, dim=-1)                     # (64, 3, 101) complex64
    src = z.imag[..., 1:100]
    out = torch.empty((99, 3, 64), dtype=torch.float32, device=DEV)
    t.strided_copy(out.permute(2, 1, 0), src, 2.0)
    assert torch.equal(out, (src * 2.0).permute(2, 1, 0).contiguous())


def test_rejects_bad_arguments():
    a = torch.zeros((2, 2, 2), device=DEV)
    with pytest.raises(TypeError):
        t.strided_copy(a.double(), a)
    with pytest.raises(ValueError):
        t.strided_copy(torch.zeros((2, 2, 3), device=DEV), a)
    ss = np.array([4, 2, -1], dtype=np.int64)
    rc = t.lib().tdsolve_strided_copy(a.data_ptr(), a.data_ptr(), 0, 2, 2, 2, t._ptr(ss),
                                      t._ptr(ss), 1.0, None)
    assert rc == -1                                   # TDS_EINVAL: negative stride
