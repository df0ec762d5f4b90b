"""The transposed matrix (h2_transpose) on the GPU, against the oracle's
transpose_arrays (pinned on the CPU against the transpose of the dense
expansion): its arrays are A's stored values moved, compared bitwise; its
products match the oracle's products of the transposed arrays."""
import numpy as np
import pytest

from paper_1902_01829_amd import workloads as W
from test_gpu_arrays import _assert_arrays_equal, _stored, _structure_arrays

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12
REDUCED_TOL = 1e-6   # FP32 arithmetic on the same stored values


def _h2mv():
    from paper_1902_01829_amd import h2mv
    return h2mv


def _rel(y, ref):
    return float(np.linalg.norm(y - ref) / np.linalg.norm(ref))


@pytest.mark.parametrize("storage", [0, 1, 2], ids=["fp64", "fp32", "bf16"])
@pytest.mark.parametrize("n,d,m,seed", [(3000, 2, 32, 81), (2500, 3, 16, 82)])
def test_transpose_of_nonsymmetric_arrays(oracle_mod, n, d, m, seed, storage):
    """Random values with a rank per level (U != V, E != F, S_ji != S_ij^T):
    the transposed handle reads back as the oracle's transpose of A's stored
    arrays, bitwise, and its products (one and many right-hand sides) match
    the oracle's product of those arrays."""
    h2mv = _h2mv()
    print(f"case transpose n={n} d={d} storage={storage}", flush=True)
    arr = _structure_arrays(oracle_mod, n, d, m, 2, seed, 400 + seed, 48)
    assert not np.array_equal(arr["U"], arr["V"])
    A = h2mv.H2Matrix.from_arrays(arr, storage)
    At = A.transpose()
    ref = oracle_mod.transpose_arrays(_stored(oracle_mod, arr, storage))
    got = h2mv.h2_export_arrays(At.handle)
    assert np.array_equal(got["level_rank"], arr["level_rank"])
    _assert_arrays_equal(ref, got, 0.0, f"transpose storage {storage}")
    tol = FP64_TOL if storage == 0 else REDUCED_TOL
    rng = np.random.Generator(np.random.PCG64(83))
    x = rng.standard_normal(n)
    y = At.matvec(torch.from_numpy(x).cuda()).cpu().numpy()
    assert _rel(y, oracle_mod.arrays_matvec(ref, x)) <= tol
    X = rng.standard_normal((8, n))
    Y = At.matmat(torch.from_numpy(X).cuda()).cpu().numpy()
    for j in (0, 7):
        assert _rel(Y[j], oracle_mod.arrays_matvec(ref, X[j])) <= tol
    # A is unchanged and independent of At
    At.close()
    y_a = A.matvec(torch.from_numpy(x).cuda()).cpu().numpy()
    assert _rel(y_a, oracle_mod.arrays_matvec(_stored(oracle_mod, arr, storage), x)) <= tol
    A.close()


def test_transpose_twice_is_the_matrix(oracle_mod):
    h2mv = _h2mv()
    arr = _structure_arrays(oracle_mod, 2000, 2, 32, 2, 84, 484, 40)
    A = h2mv.H2Matrix.from_arrays(arr, 0)
    Att = A.transpose().transpose()
    _assert_arrays_equal(h2mv.h2_export_arrays(A.handle), h2mv.h2_export_arrays(Att.handle), 0.0, "twice")


def test_transpose_of_a_points_build_is_the_matrix(oracle_mod):
    """The covariance matrices built from points are symmetric (the kernel is
    symmetric bit for bit and the two trees are one), so A^T x = A x."""
    h2mv = _h2mv()
    w = W.C1
    A = h2mv.H2Matrix(W.points(w), w.dim, w.leaf, w.cheb_p, w.eta, w.corr_len, storage=0)
    At = A.transpose()
    x = torch.from_numpy(W.rhs(w)[A.perm()]).cuda()
    y, yt = A.matvec(x).cpu().numpy(), At.matvec(x).cpu().numpy()
    print(f"A x vs A^T x: {_rel(yt, y):.2e}", flush=True)
    assert _rel(yt, y) <= 1e-14
    # the transposed handle keeps V = U, F = E: it can be compressed
    ranks = At.compress(1e-6)
    assert int(ranks.max()) <= w.rank


def test_transpose_rejections():
    h2mv = _h2mv()
    with pytest.raises(h2mv.H2Error) as e:
        h2mv.h2_transpose(None)
    assert e.value.code == h2mv.H2_ERR_INVALID_ARG
