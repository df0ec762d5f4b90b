"""The allocation-free product (h2_matvec_noalloc): the same result as
h2_matvec, bitwise, with the intermediate vectors in the library's static
device scratch array; consecutive calls of different sizes reuse the array."""
import numpy as np
import pytest

from paper_1902_01829_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _h2mv():
    from paper_1902_01829_amd import h2mv
    return h2mv


def _build(w, storage=0):
    return _h2mv().H2Matrix(W.points(w), w.dim, w.leaf, w.cheb_p, w.eta, w.corr_len, storage=storage)


def _both(A, seed):
    """y from h2_matvec and from h2_matvec_noalloc on the same x (through the C ABI)."""
    h2mv = _h2mv()
    gen = torch.Generator(device="cuda").manual_seed(seed)
    x = torch.randn(A.n, dtype=torch.float64, device="cuda", generator=gen)
    st = torch.cuda.current_stream().cuda_stream
    y_ref = torch.full_like(x, float("nan"))
    y_na = torch.full_like(x, float("nan"))
    h2mv.h2_matvec(A.handle, x.data_ptr(), y_ref.data_ptr(), st)
    h2mv.h2_matvec_noalloc(A.handle, x.data_ptr(), y_na.data_ptr(), st)
    torch.cuda.synchronize()
    return y_ref, y_na


LARGE = W.C1.with_(name="2d-n20000-m64-p8", n=20000, leaf=64, cheb_p=8, seed=82)
SMALL = W.C1   # 4096 points: fewer block rows than the split threshold, so partial sums are used


@pytest.mark.parametrize("storage", [0, 1, 2], ids=["fp64", "fp32", "bf16"])
def test_noalloc_equals_matvec_two_calls(storage):
    """Two calls in a row, the second on a smaller matrix: both bitwise equal
    to h2_matvec (so nothing left in the array by the first call leaks)."""
    A, B = _build(LARGE, storage), _build(SMALL, storage)
    for M, seed in ((A, 1), (B, 2), (A, 3)):
        y_ref, y_na = _both(M, seed)
        print(f"n={M.n} storage={storage}: max |diff| {(y_ref - y_na).abs().max().item():.3e}", flush=True)
        assert torch.isfinite(y_ref).all()
        assert torch.equal(y_ref, y_na)
    A.close()
    B.close()


def test_noalloc_half_storage_small():
    h2mv = _h2mv()
    A = _build(SMALL, h2mv.H2_HALF_STORAGE)
    y_ref, y_na = _both(A, 4)
    assert torch.equal(y_ref, y_na)
    A.close()


def test_noalloc_headline_matrix_fits():
    """The 2^20-point rank-64 FP64 matrix needs 42 MB of scratch."""
    A = _build(W.C2)
    y_ref, y_na = _both(A, 5)
    assert torch.equal(y_ref, y_na)
    A.close()


def test_noalloc_rejects_what_does_not_fit():
    """A half-stored 2^20-point rank-64 FP64 matrix needs ~150 MB of partial
    slots: refused with UNSUPPORTED before anything is enqueued."""
    h2mv = _h2mv()
    w = W.C2.with_(name="2d-n1048576-m64-k64-s91", seed=91)
    A = _build(w, h2mv.H2_HALF_STORAGE)
    x = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    y = torch.full_like(x, 7.0)
    with pytest.raises(h2mv.H2Error) as e:
        h2mv.h2_matvec_noalloc(A.handle, x.data_ptr(), y.data_ptr(), torch.cuda.current_stream().cuda_stream)
    assert e.value.code == h2mv.H2_ERR_UNSUPPORTED
    assert "scratch" in h2mv.h2_last_error()
    torch.cuda.synchronize()
    assert torch.all(y == 7.0)
    with pytest.raises(h2mv.H2Error) as e:
        h2mv.h2_matvec_noalloc(A.handle, 0, y.data_ptr(), 0)
    assert e.value.code == h2mv.H2_ERR_INVALID_ARG
    A.close()
