"""Blocks stored by halves (H2_HALF_STORAGE) on the GPU: a symmetric H^2
matrix holds only its blocks with column >= row, and the product reads each
stored block once for both S_ij x_j and S_ij^T x_i.  The matrix is the same as
with full storage, so the products are compared with the FP64 oracle (the
bounds of the full-storage tests), with the full-storage GPU product (rounding
order only), and the exported arrays with the full arrays, bitwise."""
import numpy as np
import pytest

from paper_1902_01829_amd import workloads as W
from test_gpu_arrays import _assert_arrays_equal, _stored, _structure_arrays
from test_gpu_matvec import (BF16_VS_FP64_TOL, FP32_VS_FP64_TOL, FP64_TOL, REDUCED_VS_DEQUANT_TOL, SMALL,
                             _check_fp64)

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

HALF = 16
# Same stored values, other summation order: per-block partial sums of the
# transposed products formed across lanes instead of along a row, and the
# segment's transposed contributions added after its row sum.
FP64_VS_FULL_TOL = 1e-13
REDUCED_VS_FULL_TOL = 1e-6


def _h2mv():
    from paper_1902_01829_amd import h2mv
    return h2mv


def _rel(y, ref):
    return float(np.linalg.norm(y - ref) / np.linalg.norm(ref))


def _build(w, storage):
    h2mv = _h2mv()
    return h2mv.H2Matrix(W.points(w), w.dim, w.leaf, w.cheb_p, w.eta, w.corr_len, storage=storage)


def _matvec(A, xt):
    y = A.matvec(torch.from_numpy(np.ascontiguousarray(xt)).cuda())
    torch.cuda.synchronize()
    return y.cpu().numpy()


def _symmetrize(arr):
    """Arrays of a symmetric matrix on the same partition: V = U, F = E, and
    every block below the diagonal replaced by its mirror's transpose."""
    out = dict(arr)
    out["V"] = np.array(arr["U"], copy=True)
    out["F"] = np.array(arr["E"], copy=True)
    q = int(arr["q"])
    S = []
    for l in range(q + 1):
        rp, ci = arr["S_rowptr"][l], arr["S_colidx"][l]
        k = int(arr["level_rank"][l])
        kk = k * k
        Sl = np.array(arr["S"][l], copy=True)
        pos = {(i, int(ci[t])): t for i in range(1 << l) for t in range(rp[i], rp[i + 1])}
        for (i, j), t in pos.items():
            if j < i:
                u = pos[(j, i)]
                Sl[t * kk:(t + 1) * kk] = Sl[u * kk:(u + 1) * kk].reshape(k, k, order="F").T.reshape(-1, order="F")
        S.append(Sl)
    out["S"] = S
    b, e = arr["begin"], arr["end"]
    lf = (1 << q) - 1
    size = lambda i: int(e[lf + i] - b[lf + i])
    D = np.array(arr["D"], copy=True)
    pos, off = {}, 0
    for i in range(1 << q):
        for t in range(arr["D_rowptr"][i], arr["D_rowptr"][i + 1]):
            j = int(arr["D_colidx"][t])
            pos[(i, j)] = off
            off += size(i) * size(j)
    for (i, j), o in pos.items():
        if j < i:
            u = pos[(j, i)]
            blk = D[u:u + size(j) * size(i)].reshape(size(j), size(i), order="F")
            D[o:o + size(i) * size(j)] = blk.T.reshape(-1, order="F")
    out["D"] = D
    return out


@pytest.mark.parametrize("w", SMALL, ids=lambda w: w.name)
def test_half_fp64_matches_oracle_and_full(oracle_mod, w):
    print(f"case half fp64 {w.name}", flush=True)
    H, F = _build(w, HALF), _build(w, 0)
    o = oracle_mod.OracleH2(W.points(w), w.leaf, w.cheb_p, w.eta, w.corr_len, keep_blocks=False)
    perm = H.perm()
    assert np.array_equal(perm, o.perm())
    xt = W.rhs(w)[perm]
    y, yf = _matvec(H, xt), _matvec(F, xt)
    _check_fp64(y, o.matvec(xt))
    assert _rel(y, yf) <= FP64_VS_FULL_TOL
    assert np.array_equal(y, _matvec(H, xt))   # no atomics: the same sums every call
    hi, fi = H.info, F.info
    assert hi.storage == HALF and fi.storage == 0
    assert hi.coupling_blocks == fi.coupling_blocks and hi.dense_blocks == fi.dense_blocks
    if fi.coupling_blocks:
        assert hi.bytes_coupling * 2 == fi.bytes_coupling   # no diagonal coupling blocks
    assert hi.bytes_dense <= fi.bytes_dense   # strictly less when a dense block is off the diagonal
    # partial slots: at most one per stored off-diagonal block (a group of
    # block rows shares one per column segment), none with full storage
    off_diagonal = fi.coupling_blocks // 2 + (fi.dense_blocks - (1 << fi.levels_q)) // 2
    assert fi.partial_slots == 0
    assert (hi.partial_slots > 0) == (off_diagonal > 0) and hi.partial_slots <= off_diagonal
    H.close()
    F.close()


@pytest.mark.parametrize("w", [W.C1, SMALL[2], SMALL[4], SMALL[5]], ids=lambda w: w.name)
@pytest.mark.parametrize("storage", [1, 2], ids=["fp32", "bf16"])
def test_half_reduced_storage(oracle_mod, w, storage):
    print(f"case half {w.name} storage {storage}", flush=True)
    H, F = _build(w, storage | HALF), _build(w, storage)
    perm = H.perm()
    xt = W.rhs(w)[perm]
    y, yf = _matvec(H, xt), _matvec(F, xt)
    oq = oracle_mod.OracleH2(W.points(w), w.leaf, w.cheb_p, w.eta, w.corr_len, storage=storage, keep_blocks=False)
    refq = oq.matvec(xt)
    print(f"  vs dequantized {_rel(y, refq):.3e}  vs full storage {_rel(y, yf):.3e}", flush=True)
    assert _rel(y, refq) <= REDUCED_VS_DEQUANT_TOL
    assert _rel(y, yf) <= REDUCED_VS_FULL_TOL
    H.close()
    F.close()


def _sampled(oracle_mod, w, storage, nleaves, tol):
    print(f"case half full-size {w.name} storage {storage}", flush=True)
    A = _build(w, storage | HALF)
    perm = A.perm()
    xt = W.rhs(w)[perm]
    y = _matvec(A, xt)
    A.close()
    o = oracle_mod.OracleH2(W.points(w), w.leaf, w.cheb_p, w.eta, w.corr_len, keep_blocks=False)
    rng = np.random.Generator(np.random.PCG64(11))
    leaves = np.sort(rng.choice(o.leaf_nodes(), size=nleaves, replace=False))
    rows = o.leaf_rows(leaves)
    ref = o.matvec_leaves(xt, leaves)
    rel = _rel(y[rows], ref)
    print(f"  rel err vs fp64 oracle on {len(rows)} rows: {rel:.3e}", flush=True)
    assert rel <= tol
    if storage == 0:
        assert np.abs(y[rows] - ref).max() <= FP64_TOL * np.abs(ref).max()


@pytest.mark.parametrize("rows", [1, 2, 3, 4])
@pytest.mark.parametrize("w", [SMALL[1], SMALL[2], SMALL[4], SMALL[5]], ids=lambda w: w.name)
def test_half_row_groups(oracle_mod, monkeypatch, w, rows):
    """The stored-by-halves product with the block rows taken in groups of
    1 .. 4 rows per wavefront (forced on small matrices, which the library
    would otherwise run one row per wavefront): the oracle's bound, and the
    full-storage product up to rounding order, in FP64 and BF16."""
    print(f"case half groups of {rows} {w.name}", flush=True)
    monkeypatch.setenv("H2MV_HALF_GROUP_ROWS", str(rows))
    o = oracle_mod.OracleH2(W.points(w), w.leaf, w.cheb_p, w.eta, w.corr_len, keep_blocks=False)
    for storage in (0, 2):
        H, F = _build(w, HALF | storage), _build(w, storage)
        xt = W.rhs(w)[H.perm()]
        y, yf = _matvec(H, xt), _matvec(F, xt)
        if storage == 0:
            _check_fp64(y, o.matvec(xt))
            assert _rel(y, yf) <= FP64_VS_FULL_TOL
        else:
            assert _rel(y, yf) <= REDUCED_VS_FULL_TOL
        assert np.array_equal(y, _matvec(H, xt))
        off_diagonal = F.info.coupling_blocks // 2 + (F.info.dense_blocks - (1 << F.info.levels_q)) // 2
        assert H.info.partial_slots <= off_diagonal
        H.close()
        F.close()


def test_half_fp64_full_2d_1m(oracle_mod):
    _sampled(oracle_mod, W.C2, 0, 48, FP64_TOL)


def test_half_fp64_full_3d_512k(oracle_mod):
    _sampled(oracle_mod, W.C3, 0, 48, FP64_TOL)


@pytest.mark.parametrize("storage", [1, 2], ids=["fp32", "bf16"])
def test_half_reduced_full_3d_512k(oracle_mod, storage):
    _sampled(oracle_mod, W.C3, storage, 16, FP32_VS_FP64_TOL if storage == 1 else BF16_VS_FP64_TOL)


@pytest.mark.parametrize("storage", [0, 1, 2], ids=["fp64", "fp32", "bf16"])
@pytest.mark.parametrize("n,d,m,seed", [(3000, 2, 32, 91), (2500, 3, 16, 92)])
def test_half_from_symmetric_arrays(oracle_mod, n, d, m, seed, storage):
    """Random symmetric arrays with a rank per level (ragged leaves): the
    export gives the full arrays back (mirrors transposed from the stored
    halves, bitwise), and the product matches the oracle's."""
    h2mv = _h2mv()
    print(f"case half arrays n={n} d={d} storage={storage}", flush=True)
    arr = _symmetrize(_structure_arrays(oracle_mod, n, d, m, 2, seed, 500 + seed, 48))
    H = h2mv.H2Matrix.from_arrays(arr, storage | HALF)
    F = h2mv.H2Matrix.from_arrays(arr, storage)
    _assert_arrays_equal(h2mv.h2_export_arrays(F.handle), h2mv.h2_export_arrays(H.handle), 0.0, "half export")
    ref_arr = _stored(oracle_mod, arr, storage)
    rng = np.random.Generator(np.random.PCG64(seed))
    x = rng.standard_normal(n)
    y = _matvec(H, x)
    tol = FP64_TOL if storage == 0 else REDUCED_VS_DEQUANT_TOL
    assert _rel(y, oracle_mod.arrays_matvec(ref_arr, x)) <= tol
    assert _rel(y, _matvec(F, x)) <= (FP64_VS_FULL_TOL if storage == 0 else REDUCED_VS_FULL_TOL)
    H.close()
    F.close()


def test_half_rejects_nonsymmetric_arrays(oracle_mod):
    h2mv = _h2mv()
    arr = _structure_arrays(oracle_mod, 2000, 2, 32, 2, 93, 593, 40)
    with pytest.raises(h2mv.H2Error) as e:      # V != U
        h2mv.H2Matrix.from_arrays(arr, HALF)
    assert e.value.code == h2mv.H2_ERR_INVALID_ARG
    sym = _symmetrize(arr)
    bad = dict(sym)
    l = next(l for l in range(int(arr["q"]) + 1) if len(arr["S_colidx"][l]) > 1)
    bad["S"] = [np.array(s, copy=True) for s in sym["S"]]
    bad["S"][l][0] += 1.0                        # one block no longer its mirror's transpose
    with pytest.raises(h2mv.H2Error) as e:
        h2mv.H2Matrix.from_arrays(bad, HALF)
    assert e.value.code == h2mv.H2_ERR_INVALID_ARG
    bad = dict(sym)
    bad["D"] = np.array(sym["D"], copy=True)
    lf = (1 << int(arr["q"])) - 1
    i = next(i for i in range(1 << int(arr["q"])) if arr["D_rowptr"][i + 1] - arr["D_rowptr"][i] > 1)
    t = next(t for t in range(arr["D_rowptr"][i], arr["D_rowptr"][i + 1]) if arr["D_colidx"][t] != i)
    off = sum(int(arr["end"][lf + a] - arr["begin"][lf + a]) * int(arr["end"][lf + arr["D_colidx"][u]]
                                                                  - arr["begin"][lf + arr["D_colidx"][u]])
              for a in range(1 << int(arr["q"])) for u in range(arr["D_rowptr"][a], arr["D_rowptr"][a + 1]) if u < t)
    bad["D"][off] += 1.0                         # an off-diagonal dense block
    with pytest.raises(h2mv.H2Error) as e:
        h2mv.H2Matrix.from_arrays(bad, HALF)
    assert e.value.code == h2mv.H2_ERR_INVALID_ARG
    H = h2mv.H2Matrix.from_arrays(sym, HALF)     # the symmetric arrays themselves are accepted
    H.close()


def test_half_matmat_columns_and_rejections():
    h2mv = _h2mv()
    w = W.C1
    H = _build(w, 1 | HALF)
    X = torch.randn(3, w.n, dtype=torch.float64, device="cuda")
    Y = H.matmat(X)
    for j in range(3):
        yj = H.matvec(X[j].contiguous())
        assert torch.equal(Y[j], yj)   # one single-vector product per column
    for call in (H.orthogonalize, H.transpose, lambda: H.compress(1e-6)):
        with pytest.raises(h2mv.H2Error) as e:
            call()
        assert e.value.code == h2mv.H2_ERR_UNSUPPORTED
    with pytest.raises(h2mv.H2Error) as e:
        h2mv.H2Batch([H], 4)
    assert e.value.code == h2mv.H2_ERR_UNSUPPORTED
    H.close()
    H64 = _build(w, HALF)
    for call in (H64.orthogonalize, lambda: H64.compress(1e-6)):
        with pytest.raises(h2mv.H2Error) as e:
            call()
        assert e.value.code == h2mv.H2_ERR_UNSUPPORTED
    H64.close()
