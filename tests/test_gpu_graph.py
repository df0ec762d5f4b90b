"""The products captured into a HIP graph (torch.cuda.CUDAGraph) and replayed:
every replay, with eager work and synchronizations between replays, equals the
eager product bitwise (the replay runs the same kernels on the same data)."""
import pytest

from paper_1902_01829_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _build(w, storage):
    from paper_1902_01829_amd import h2mv
    return h2mv.H2Matrix(W.points(w), w.dim, w.leaf, w.cheb_p, w.eta, w.corr_len, storage=storage)


@pytest.mark.parametrize("storage", [0, 1, 2, 16, 18], ids=["fp64", "fp32", "bf16", "fp64-half", "bf16-half"])
def test_matvec_graph_replays(storage):
    w = W.C1
    A = _build(w, storage)
    x = torch.zeros(w.n, dtype=torch.float64, device="cuda")
    y = torch.zeros_like(x)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        A.matvec(x, out=y)                     # warm-up outside the capture
    torch.cuda.current_stream().wait_stream(s)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        A.matvec(x, out=y)
    gen = torch.Generator(device="cuda").manual_seed(3)
    for _ in range(4):
        x.copy_(torch.randn(w.n, dtype=torch.float64, device="cuda", generator=gen))
        g.replay()
        torch.cuda.synchronize()
        ref = A.matvec(x)                      # eager, between replays
        torch.cuda.synchronize()
        assert torch.equal(y, ref)
    del g
    A.close()


@pytest.mark.parametrize("storage", [1, 2], ids=["fp32", "bf16"])
def test_matmat_graph_replays(storage):
    w = W.C1
    A = _build(w, storage)
    X = torch.zeros(12, w.n, dtype=torch.float64, device="cuda")
    Y = torch.zeros_like(X)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        A.matmat(X, out=Y)                     # first call: tunes (synchronizes), not capturable
    torch.cuda.current_stream().wait_stream(s)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        A.matmat(X, out=Y)
    gen = torch.Generator(device="cuda").manual_seed(4)
    for _ in range(3):
        X.copy_(torch.randn(12, w.n, dtype=torch.float64, device="cuda", generator=gen))
        g.replay()
        torch.cuda.synchronize()
        ref = A.matmat(X)
        torch.cuda.synchronize()
        assert torch.equal(Y, ref)
    del g
    A.close()
