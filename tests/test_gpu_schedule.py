"""The streamed schedule of the single-vector product (the near field on the
handle's second stream, concurrent with the low-rank phases: the overlap of
Sec. 4.5) against the merged one, through the C ABI.

Both schedules run the same rows with the same block order and the same
summation order, so their products must be bitwise equal, whatever the cap
on the near-field launch's workgroups per compute unit and the share of its
rows started with the product: eagerly, replayed from a HIP graph (the second
stream joins the capture through events), through the allocation-free entry
point, and on every storage mode.  The merged products themselves are held to
the FP64 oracle by test_gpu_matvec.py.
"""
import numpy as np
import pytest

from paper_1902_01829_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

# (near_wg_per_cu, near_early): no cap, all rows early; no cap, all rows after
# the coupling launch; caps 2 and 3 with the rows split or all early
SETTINGS = [(0, 1.0), (0, 0.0), (3, 0.5), (2, 1.0), (3, 0.0), (2, 0.25)]

CASES = [
    W.C1,                                                                   # split (chunked) stream list
    W.C1.with_(name="2d-n5000-m32-p4-ragged", n=5000, seed=78),
    W.C1.with_(name="3d-n3000-m24-p3", n=3000, dim=3, leaf=24, cheb_p=3, corr_len=0.2, seed=77),
    W.C1.with_(name="2d-n999-m7-p2-eta2", n=999, leaf=7, cheb_p=2, eta=2.0, seed=81),
    W.C1.with_(name="2d-n200000-m64-p8", n=200000, leaf=64, cheb_p=8, seed=87),   # one row per wavefront
    W.C1.with_(name="3d-n150000-m64-p4", n=150000, dim=3, leaf=64, cheb_p=4, corr_len=0.2, seed=88),
    W.C1.with_(name="2d-n3-m2-p1", n=3, leaf=2, cheb_p=1, seed=84),
    W.C1.with_(name="3d-n50-m64-single-leaf", n=50, dim=3, leaf=64, seed=86),   # near field only
]


def _h2mv():
    from paper_1902_01829_amd import h2mv
    return h2mv


def _build(w, storage=0):
    h2mv = _h2mv()
    return h2mv.H2Matrix(W.points(w), w.dim, w.leaf, w.cheb_p, w.eta, w.corr_len, storage=storage)


def _x(A, w):
    return torch.from_numpy(np.ascontiguousarray(W.rhs(w)[A.perm()])).cuda()


@pytest.mark.parametrize("w", CASES, ids=lambda w: w.name)
def test_streamed_equals_merged_fp64(w):
    print(f"case {w.name}", flush=True)
    h2mv = _h2mv()
    A = _build(w)
    x = _x(A, w)
    y0 = A.matvec(x)
    for cap, early in SETTINGS:
        A.set_schedule(h2mv.H2_SCHEDULE_STREAMED, cap, early)
        for _ in range(2):
            y = A.matvec(x)
            torch.cuda.synchronize()
            assert torch.equal(y, y0), (cap, early)
    A.set_schedule(h2mv.H2_SCHEDULE_MERGED)
    assert torch.equal(A.matvec(x), y0)
    A.close()


@pytest.mark.parametrize("storage", [1, 2], ids=["fp32", "bf16"])
@pytest.mark.parametrize("w", [CASES[0], CASES[4]], ids=lambda w: w.name)
def test_streamed_equals_merged_reduced(w, storage):
    print(f"case {w.name} storage {storage}", flush=True)
    h2mv = _h2mv()
    A = _build(w, storage)
    x = _x(A, w)
    y0 = A.matvec(x)
    for cap, early in SETTINGS[:3]:
        A.set_schedule(h2mv.H2_SCHEDULE_STREAMED, cap, early)
        y = A.matvec(x)
        torch.cuda.synchronize()
        assert torch.equal(y, y0), (cap, early)
    A.close()


def test_streamed_headline_matrix():
    """The 2^20-point 2-D FP64 matrix under the schedules the benchmark times."""
    w = W.C2
    print(f"case {w.name}", flush=True)
    h2mv = _h2mv()
    A = _build(w)
    x = _x(A, w)
    y0 = A.matvec(x)
    for cap, early in ((0, 1.0), (3, 1.0), (3, 0.5)):
        A.set_schedule(h2mv.H2_SCHEDULE_STREAMED, cap, early)
        y = A.matvec(x)
        torch.cuda.synchronize()
        assert torch.equal(y, y0), (cap, early)
    A.close()


@pytest.mark.parametrize("w", [CASES[0], CASES[4]], ids=lambda w: w.name)
def test_streamed_graph_replays(w):
    """A streamed product captured into a HIP graph, replayed several times
    with eager work and synchronizations between the replays."""
    print(f"case {w.name}", flush=True)
    h2mv = _h2mv()
    A = _build(w)
    x = _x(A, w)
    y0 = A.matvec(x)
    torch.cuda.synchronize()
    A.set_schedule(h2mv.H2_SCHEDULE_STREAMED, 3, 0.5)
    yg = torch.empty_like(x)
    A.matvec(x, out=yg)             # warm-up outside the capture
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        A.matvec(x, out=yg)
    for _ in range(4):
        yg.fill_(-1.0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(yg, y0)
        assert torch.equal(A.matvec(x), y0)   # eager product between replays
    del g
    A.close()


def test_streamed_noalloc():
    """The allocation-free entry point under the streamed schedule, two calls
    in a row, the second on a smaller matrix."""
    h2mv = _h2mv()
    for w in (CASES[4], CASES[1]):
        print(f"case {w.name}", flush=True)
        A = _build(w)
        x = _x(A, w)
        y0 = A.matvec(x)
        A.set_schedule(h2mv.H2_SCHEDULE_STREAMED, 3, 0.5)
        y = torch.full_like(x, -1.0)
        h2mv.h2_matvec_noalloc(A.handle, x.data_ptr(), y.data_ptr(), torch.cuda.current_stream().cuda_stream)
        torch.cuda.synchronize()
        assert torch.equal(y, y0)
        A.close()


def test_set_schedule_rejects():
    h2mv = _h2mv()
    w = CASES[1]
    A = _build(w)
    for args in ((2, 0, 1.0), (-1, 0, 1.0), (1, -1, 1.0), (1, 0, 1.5), (1, 0, -0.1), (1, 0, float("nan"))):
        with pytest.raises(h2mv.H2Error) as e:
            A.set_schedule(*args)
        assert e.value.code == h2mv.H2_ERR_INVALID_ARG, args
    # a cap the LDS request cannot express (above one workgroup per 1 KiB of
    # the compute unit's LDS)
    with pytest.raises(h2mv.H2Error) as e:
        A.set_schedule(h2mv.H2_SCHEDULE_STREAMED, 1000, 1.0)
    assert e.value.code == h2mv.H2_ERR_UNSUPPORTED
    assert "LDS" in h2mv.h2_last_error()
    A.close()
    H = _h2mv().H2Matrix(W.points(w), w.dim, w.leaf, w.cheb_p, w.eta, w.corr_len,
                         storage=h2mv.H2_FP64 | h2mv.H2_HALF_STORAGE)
    with pytest.raises(h2mv.H2Error) as e:
        H.set_schedule(h2mv.H2_SCHEDULE_STREAMED)
    assert e.value.code == h2mv.H2_ERR_UNSUPPORTED
    H.set_schedule(h2mv.H2_SCHEDULE_MERGED)
    H.close()
