"""Algebraic compression (Sec. 5: orthogonalization, basis generation of
Sec. 5.2, truncation of Sec. 5.3, projection) on the GPU, against the
oracle's compress_arrays (pinned on the CPU by brute-force far-field singular
values, a planted rank, the zero threshold and the error bound).

What is unique is compared exactly: the new rank of every level (a count of
singular values above a threshold, decided on both sides in FP64; each case
checks that no singular value lies near its threshold), the product of the
compressed matrix, and the kept subspace of every leaf whose singular values
have a gap at the cut.  The bases themselves are unique only up to the
signs of their columns (and rotations among equal singular values), so they
are checked for orthonormality instead."""
import numpy as np
import pytest

from paper_1902_01829_amd import workloads as W
from test_oracle import _explicit_bases, _explicit_col_bases, _inflate, _nonsymmetric_coupling, _two_trees

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

# Relative product difference, GPU compression vs the oracle's.  Where every
# cut falls between distinct singular values both keep the same subspaces
# and the compressed matrices differ by rounding amplified by 1 / gap (the
# cases here measure 2e-15 .. 8e-15).  The bound allows gaps down to ~1e-4
# relative; a cut inside a cluster of equal singular values could exceed it,
# and none of the seeded cases has one.
PARITY_TOL = 1e-11
ORTHO_TOL = 1e-12     # explicit new bases: Q^T Q = I
LAYOUT_TOL = 1e-13    # GPU product vs the oracle's product of the GPU's exported arrays
# kept leaf subspaces, |P_gpu - P_oracle| <= 1e-14 s_0 / gap + 1e-13 where the
# gap s_(kt-1) - s_kt at the cut exceeds 1e-9 s_0 (perturbation of a subspace)

CASES = [
    (W.C1.with_(name="2d-n4096-m32-p4", n=4096, leaf=32, cheb_p=4, seed=601), (0.0, 1e-4, 1e-8)),
    (W.C1.with_(name="3d-n3000-m64-p3", n=3000, dim=3, leaf=64, cheb_p=3, corr_len=0.2, seed=602), (1e-3, 1e-6)),
    (W.C1.with_(name="2d-n8192-m64-p8", n=8192, leaf=64, cheb_p=8, seed=603), (1e-7,)),
]


def _h2mv():
    from paper_1902_01829_amd import h2mv
    return h2mv


def _lmin(arr):
    q = int(arr["q"])
    return next((l for l in range(q + 1) if len(arr["S_colidx"][l]) > 0), q + 1)


def _rel(y, ref):
    return float(np.linalg.norm(y - ref) / np.linalg.norm(ref))


def _check_margin(info, eps):
    """No singular value within a relative 1e-6 of its node's threshold."""
    if eps == 0.0:
        return
    for v, s in info["sigma"].items():
        if s.size and s[0] > 0.0:
            r = s / s[0]
            assert not np.any(np.abs(r - eps) <= 1e-6 * eps), f"node {v}: singular value at the threshold"


def _leaf_bases(arr):
    q, kq = int(arr["q"]), int(arr["level_rank"][int(arr["q"])])
    b, e = arr["begin"], arr["end"]
    lf = (1 << q) - 1
    out, off = {}, 0
    for j in range(1 << q):
        m = int(e[lf + j] - b[lf + j])
        out[lf + j] = arr["U"][off:off + m * kq].reshape(kq, m).T
        off += m * kq
    return out


@pytest.mark.parametrize("w,epss", CASES, ids=lambda c: c.name if hasattr(c, "name") else str(c))
def test_compress_matches_oracle(oracle_mod, w, epss):
    h2mv = _h2mv()
    o = oracle_mod.OracleH2(W.points(w), w.leaf, w.cheb_p, w.eta, w.corr_len)
    arr0 = o.export_arrays()
    x = W.rhs(w)[o.perm()]
    y0 = o.matvec(x)
    for eps in epss:
        print(f"case {w.name} eps {eps}", flush=True)
        A = h2mv.H2Matrix(W.points(w), w.dim, w.leaf, w.cheb_p, w.eta, w.corr_len, storage=0)
        ranks = A.compress(eps)
        ref, info = oracle_mod.compress_arrays(arr0, eps)
        _check_margin(info, eps)
        assert list(ranks) == [int(r) for r in ref["level_rank"]], (list(ranks), list(ref["level_rank"]))
        assert A.info.rank == max(int(r) for r in ref["level_rank"])
        y = A.matvec(torch.from_numpy(x).cuda()).cpu().numpy()
        y_ref = oracle_mod.arrays_matvec(ref, x)
        par, err = _rel(y, y_ref), _rel(y, y0)
        got = h2mv.h2_export_arrays(A.handle)
        lay = _rel(oracle_mod.arrays_matvec(got, x), y)
        new = _explicit_bases(got)
        lmin = _lmin(got)
        worst_o = max(float(np.abs(new[v].T @ new[v] - np.eye(new[v].shape[1])).max())
                      for v in range((1 << lmin) - 1, o.nnodes))
        # kept leaf subspaces where the cut has a gap
        gu, ru = _leaf_bases(got), _leaf_bases(ref)
        worst_p, gapped = 0.0, 0
        kt = int(ref["level_rank"][o.q])
        for v, Q in gu.items():
            s = info["sigma"][v]
            if kt < len(s) and s[0] > 0.0 and (s[kt - 1] - s[kt]) > 1e-9 * s[0]:
                bound = 1e-14 * s[0] / (s[kt - 1] - s[kt]) + 1e-13
                worst_p = max(worst_p, float(np.abs(Q @ Q.T - ru[v] @ ru[v].T).max()) / bound)
                gapped += 1
        print(f"  ranks {[int(r) for r in ranks]} vs oracle {par:.2e}, vs uncompressed {err:.2e}, layout {lay:.2e}, "
              f"orthonormality {worst_o:.1e}, leaf subspaces ({gapped} gapped) {worst_p:.2f} of bound", flush=True)
        assert par <= PARITY_TOL
        assert err <= max(eps, 1e-12)
        assert lay <= LAYOUT_TOL
        assert worst_o <= ORTHO_TOL
        assert worst_p <= 1.0
        A.close()


@pytest.mark.parametrize("d,eps", [(2, 1e-6), (3, 1e-4)])
def test_compress_nonsymmetric_coupling_matches_oracle(oracle_mod, d, eps):
    """One basis tree for rows and columns (V = U, F = E) with coupling blocks
    that are not symmetric: the basis generation stacks block rows and block
    columns on both sides; ranks, products and orthonormality as above."""
    h2mv = _h2mv()
    n = 4000
    pts = np.random.Generator(np.random.PCG64(670 + d)).random((n, d))
    o = oracle_mod.OracleH2(pts, 64, 5 if d == 2 else 3, 0.9, 0.2)
    arr = _nonsymmetric_coupling(o.export_arrays())
    assert not oracle_mod.coupling_is_symmetric(arr)
    ref, info = oracle_mod.compress_arrays(arr, eps)
    _check_margin(info, eps)
    A = h2mv.H2Matrix.from_arrays(arr, storage=0)
    ranks = A.compress(eps)
    assert list(ranks) == [int(r) for r in ref["level_rank"]], (list(ranks), list(ref["level_rank"]))
    x = np.random.Generator(np.random.PCG64(671)).standard_normal(n)
    y = A.matvec(torch.from_numpy(x).cuda()).cpu().numpy()
    par, err = _rel(y, oracle_mod.arrays_matvec(ref, x)), _rel(y, oracle_mod.arrays_matvec(arr, x))
    got = h2mv.h2_export_arrays(A.handle)
    new = _explicit_bases(got)
    lmin = _lmin(got)
    worst_o = max(float(np.abs(new[v].T @ new[v] - np.eye(new[v].shape[1])).max())
                  for v in range((1 << lmin) - 1, o.nnodes))
    print(f"d={d} eps={eps}: ranks {[int(r) for r in ranks]} vs oracle {par:.2e}, vs uncompressed {err:.2e}, "
          f"orthonormality {worst_o:.1e}", flush=True)
    assert par <= PARITY_TOL
    assert err <= eps
    assert worst_o <= ORTHO_TOL


def _row_projected(arr, r, seed):
    """Coupling blocks S_ij <- P_i P_i^T S_ij, P_i a random rank-r projector
    per row node: block rows need few directions, block columns many."""
    rng = np.random.Generator(np.random.PCG64(seed))
    S = []
    for l in range(int(arr["q"]) + 1):
        k = int(arr["level_rank"][l])
        rp = arr["S_rowptr"][l]
        Sl = np.array(arr["S"][l], dtype=np.float64, copy=True)
        for i in range(1 << l):
            P = np.linalg.qr(rng.standard_normal((k, r)))[0]
            for t in range(int(rp[i]), int(rp[i + 1])):
                Sb = Sl[t * k * k:(t + 1) * k * k].reshape(k, k).T
                Sl[t * k * k:(t + 1) * k * k] = (P @ (P.T @ Sb)).ravel(order="F")
        S.append(Sl)
    return dict(arr, S=S)


@pytest.mark.parametrize("case,eps", [("nonsymmetric", 1e-6), ("nonsymmetric", 1e-4), ("row-projected", 1e-8)])
def test_compress_two_trees_matches_oracle(oracle_mod, case, eps):
    """Different row and column trees (V != U, F != E): each tree's R from its
    own blocks, a level's rank the larger count of the two trees; ranks,
    products and both trees' orthonormality against the oracle's
    compress_two_trees.  The row-projected case has the column tree decide
    the ranks."""
    h2mv = _h2mv()
    n = 4000
    pts = np.random.Generator(np.random.PCG64(680)).random((n, 2))
    o = oracle_mod.OracleH2(pts, 64, 5, 0.9, 0.2)
    base = o.export_arrays()
    base = _nonsymmetric_coupling(base) if case == "nonsymmetric" else _row_projected(base, 4, 681)
    arr = _two_trees(base, 682)
    ref, info = oracle_mod.compress_arrays(arr, eps)
    _check_margin(info, eps)
    _check_margin({"sigma": info["sigma_col"]}, eps)
    A = h2mv.H2Matrix.from_arrays(arr, storage=0)
    ranks = A.compress(eps)
    assert list(ranks) == [int(r) for r in ref["level_rank"]], (list(ranks), list(ref["level_rank"]))
    x = np.random.Generator(np.random.PCG64(683)).standard_normal(n)
    y = A.matvec(torch.from_numpy(x).cuda()).cpu().numpy()
    par, err = _rel(y, oracle_mod.arrays_matvec(ref, x)), _rel(y, oracle_mod.arrays_matvec(arr, x))
    got = h2mv.h2_export_arrays(A.handle)
    lmin = _lmin(got)
    worst_o = 0.0
    for expl in (_explicit_bases(got), _explicit_col_bases(got)):
        worst_o = max(worst_o, max(float(np.abs(expl[v].T @ expl[v] - np.eye(expl[v].shape[1])).max())
                                   for v in range((1 << lmin) - 1, o.nnodes)))
    q = o.q
    leaves = range((1 << q) - 1, (2 << q) - 1)
    rows, cols = max(info["count"][v] for v in leaves), max(info["count_col"][v] for v in leaves)
    print(f"{case} eps={eps}: ranks {[int(r) for r in ranks]} (leaf counts rows {rows}, columns {cols}) vs oracle "
          f"{par:.2e}, vs uncompressed {err:.2e}, orthonormality {worst_o:.1e}", flush=True)
    if case == "row-projected":
        assert rows < cols
    assert par <= PARITY_TOL
    assert err <= eps
    assert worst_o <= ORTHO_TOL


def test_compress_zero_threshold_keeps_ranks_and_product(oracle_mod):
    h2mv = _h2mv()
    w = W.C1
    A = h2mv.H2Matrix(W.points(w), w.dim, w.leaf, w.cheb_p, w.eta, w.corr_len, storage=0)
    x = torch.from_numpy(W.rhs(w)[A.perm()]).cuda()
    y0 = A.matvec(x).cpu().numpy()
    k = A.info.rank
    ranks = A.compress(0.0)
    assert list(ranks) == [k] * (A.info.levels_q + 1)
    y1 = A.matvec(x).cpu().numpy()
    assert _rel(y1, y0) <= 1e-12


@pytest.mark.parametrize("d,extra", [(2, 6), (3, 5)])
def test_compress_recovers_a_planted_rank(oracle_mod, d, extra):
    """A rank-4 (2-D) / rank-8 (3-D) matrix written with redundant basis
    columns compresses back to its own rank, product unchanged."""
    h2mv = _h2mv()
    n = 3000
    pts = np.random.Generator(np.random.PCG64(650 + d)).random((n, d))
    o = oracle_mod.OracleH2(pts, 32, 2, 0.9, 0.2)
    arr = o.export_arrays()
    big = _inflate(arr, extra, 651)
    x = np.random.Generator(np.random.PCG64(652)).standard_normal(n)
    y0 = oracle_mod.arrays_matvec(arr, x)
    A = h2mv.H2Matrix.from_arrays(big, storage=0)
    ranks = A.compress(1e-10)
    lmin = _lmin(arr)
    print(f"d={d}: ranks {[int(r) for r in ranks]}", flush=True)
    assert all(int(ranks[l]) == o.k for l in range(lmin, o.q + 1))
    y = A.matvec(torch.from_numpy(x).cuda()).cpu().numpy()
    assert _rel(y, y0) <= 1e-12


def test_compressed_arrays_in_reduced_storage(oracle_mod):
    """The compressed representation, exported and imported with FP32
    storage (per-level ranks), multiplies many right-hand sides on the
    matrix cores like the oracle's product of the same arrays."""
    h2mv = _h2mv()
    w = W.C1.with_(name="2d-n8192-m64-p6", n=8192, leaf=64, cheb_p=6, seed=660)
    A = h2mv.H2Matrix(W.points(w), w.dim, w.leaf, w.cheb_p, w.eta, w.corr_len, storage=0)
    ranks = A.compress(1e-6)
    assert len(set(int(r) for r in ranks)) > 1   # ranks differ by level
    arr = h2mv.h2_export_arrays(A.handle)
    B = h2mv.H2Matrix.from_arrays(arr, storage=h2mv.H2_FP32)
    X = np.random.Generator(np.random.PCG64(661)).standard_normal((8, w.n))
    Y = B.matmat(torch.from_numpy(X).cuda()).cpu().numpy()
    worst = max(_rel(Y[j], oracle_mod.arrays_matvec(arr, X[j])) for j in range(8))
    print(f"ranks {[int(r) for r in ranks]}, FP32 matmat vs oracle {worst:.2e}", flush=True)
    assert worst <= 1e-5   # FP32 storage and products, FP64 sums (the FP32 matmat bound)


def test_compress_rejections():
    h2mv = _h2mv()
    w = W.C1
    A = h2mv.H2Matrix(W.points(w), w.dim, w.leaf, w.cheb_p, w.eta, w.corr_len, storage=0)
    for bad in (-1e-3, float("nan"), float("inf")):
        with pytest.raises(h2mv.H2Error) as e:
            A.compress(bad)
        assert e.value.code == h2mv.H2_ERR_INVALID_ARG
    F = h2mv.H2Matrix(W.points(w), w.dim, w.leaf, w.cheb_p, w.eta, w.corr_len, storage=h2mv.H2_FP32)
    batch = h2mv.H2Batch([F], 4)
    with pytest.raises(h2mv.H2Error) as e:   # its addresses are held by the batch
        F.compress(1e-6)
    assert e.value.code == h2mv.H2_ERR_INVALID_ARG
    batch.close()
    with pytest.raises(h2mv.H2Error) as e:
        F.compress(1e-6)
    assert e.value.code == h2mv.H2_ERR_UNSUPPORTED
    # the failed calls left A usable
    ranks = A.compress(1e-6)
    assert int(ranks.max()) <= A.info.rank <= 16


def test_compress_full_size_2d(oracle_mod):
    """2^20 points, rank 64, the paper's 2-D threshold 1e-7 (Table 2): the
    product changes by at most eps per truncated level (a property at any size; the
    oracle's compression of this size does not finish in seconds), every
    level's rank drops, and the stored bytes shrink."""
    h2mv = _h2mv()
    w = W.C2
    print(f"case {w.name}", flush=True)
    A = h2mv.H2Matrix(W.points(w), w.dim, w.leaf, w.cheb_p, w.eta, w.corr_len, storage=0)
    x = torch.from_numpy(W.rhs(w)[A.perm()]).cuda()
    y0 = A.matvec(x).cpu().numpy()
    bytes0 = A.info.bytes_coupling + A.info.bytes_leaf_bases + A.info.bytes_transfers
    ranks = A.compress(1e-7)
    y1 = A.matvec(x).cpu().numpy()
    bytes1 = A.info.bytes_coupling + A.info.bytes_leaf_bases + A.info.bytes_transfers
    err = _rel(y1, y0)
    levels = A.info.levels_q - A.info.lmin + 1
    print(f"ranks {[int(r) for r in ranks]}, product change {err:.2e}, low-rank bytes {bytes0 / 1e9:.2f} -> "
          f"{bytes1 / 1e9:.2f} GB", flush=True)
    # each truncated level drops singular values below eps times those of the
    # block rows it represents; the levels' errors add up
    assert err <= levels * 1e-7
    assert int(ranks[A.info.lmin:].max()) < 64
    assert bytes1 < bytes0


def test_compress_without_coupling_blocks():
    """A single leaf (only a dense block): nothing to compress; ranks and
    product unchanged."""
    h2mv = _h2mv()
    rng = np.random.Generator(np.random.PCG64(690))
    n = 40
    D = rng.standard_normal((n, n))
    arr = {"n": n, "q": 0, "level_rank": np.array([8], dtype=np.int32), "begin": np.array([0]),
           "end": np.array([n]), "U": np.zeros(8 * n), "V": np.zeros(8 * n), "E": np.zeros(0), "F": np.zeros(0),
           "S_rowptr": [np.array([0, 0], dtype=np.int32)], "S_colidx": [np.zeros(0, dtype=np.int32)],
           "S": [np.zeros(0)], "D_rowptr": np.array([0, 1], dtype=np.int32),
           "D_colidx": np.array([0], dtype=np.int32), "D": D.ravel(order="F")}
    A = h2mv.H2Matrix.from_arrays(arr, storage=0)
    x = rng.standard_normal(n)
    ranks = A.compress(1e-3)
    assert list(ranks) == [8]
    y = A.matvec(torch.from_numpy(x).cuda()).cpu().numpy()
    assert _rel(y, D @ x) <= 1e-14


def test_compress_twice_does_not_grow():
    """Compressing a compressed matrix again at the same threshold keeps or
    lowers every rank and changes the product by less than eps per level."""
    h2mv = _h2mv()
    w = W.C1.with_(name="2d-n8192-m64-p6", n=8192, leaf=64, cheb_p=6, seed=691)
    A = h2mv.H2Matrix(W.points(w), w.dim, w.leaf, w.cheb_p, w.eta, w.corr_len, storage=0)
    x = torch.from_numpy(W.rhs(w)[A.perm()]).cuda()
    r1 = A.compress(1e-6)
    y1 = A.matvec(x).cpu().numpy()
    r2 = A.compress(1e-6)
    y2 = A.matvec(x).cpu().numpy()
    print(f"ranks {[int(r) for r in r1]} -> {[int(r) for r in r2]}, product change {_rel(y2, y1):.2e}", flush=True)
    assert all(int(b) <= int(a) for a, b in zip(r1, r2))
    assert _rel(y2, y1) <= 1e-6 * (A.info.levels_q - A.info.lmin + 1)


def test_transpose_of_a_compressed_nonsymmetric_matrix(oracle_mod):
    """Per-level ranks after compression, then the transposed handle: its
    product is the oracle's product of the transposed compressed arrays."""
    h2mv = _h2mv()
    n = 3000
    pts = np.random.Generator(np.random.PCG64(692)).random((n, 2))
    o = oracle_mod.OracleH2(pts, 64, 5, 0.9, 0.2)
    arr = _two_trees(_nonsymmetric_coupling(o.export_arrays()), 693)
    A = h2mv.H2Matrix.from_arrays(arr, storage=0)
    A.compress(1e-5)
    At = A.transpose()
    got = h2mv.h2_export_arrays(A.handle)
    ref = oracle_mod.transpose_arrays(got)
    x = np.random.Generator(np.random.PCG64(694)).standard_normal(n)
    y = At.matvec(torch.from_numpy(x).cuda()).cpu().numpy()
    assert _rel(y, oracle_mod.arrays_matvec(ref, x)) <= 1e-12
