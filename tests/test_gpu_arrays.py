"""H^2 matrices given by their arrays (h2_build_from_arrays): the paper's
statement of the problem -- flattened cluster tree, bases, transfers, per-level
coupling blocks and dense blocks in, y = A x out -- with a rank per level.

References: the oracle's product of the same arrays (or_arrays_matvec), which
is pinned on the CPU against the definition written out (tests/test_oracle.py);
in reduced storage, the same arrays rounded as the library stores them (bases
and transfers FP32; blocks FP32, or BF16 with a per-block FP32 scale)."""
import numpy as np
import pytest

from paper_1902_01829_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12
REDUCED_TOL = 1e-6   # FP32 arithmetic on the same stored values (as for points-built matrices)


def _h2mv():
    from paper_1902_01829_amd import h2mv
    return h2mv


def _structure_arrays(oracle_mod, n, d, m, p, ranks_seed, values_seed, kmax):
    """Block structure of an oracle H^2 (a valid partition), a random rank per
    level in [1, kmax] and random values."""
    pts = np.random.Generator(np.random.PCG64(60 + n)).random((n, d))
    o = oracle_mod.OracleH2(pts, m, p, 0.9, 0.2)
    b, e = o.ranges()
    q, lf = o.q, (1 << o.q) - 1
    rng = np.random.Generator(np.random.PCG64(ranks_seed))
    level_rank = rng.integers(1, kmax + 1, size=q + 1).astype(np.int32)
    level_rank[q] = kmax   # the leaf level at the largest rank (above the leaf size)
    S_rowptr, S_colidx = [], []
    for l in range(q + 1):
        rp, ci = o.coupling_bsr(l)
        S_rowptr.append(rp)
        S_colidx.append(ci)
    drp, dci = o.dense_bsr()
    sizes = e - b
    shapes = [(int(sizes[lf + i]), int(sizes[lf + dci[t]])) for i in range(1 << q) for t in range(drp[i], drp[i + 1])]
    vals = W.random_h2_values(values_seed, sizes[lf:], level_rank, [len(c) for c in S_colidx], shapes)
    return {"n": n, "q": q, "level_rank": level_rank, "begin": b, "end": e, "S_rowptr": S_rowptr,
            "S_colidx": S_colidx, "D_rowptr": drp, "D_colidx": dci, **vals}


def _stored(oracle_mod, arr, storage):
    """The arrays as the library stores them in a reduced mode (exact FP64)."""
    if storage == 0:
        return arr
    out = dict(arr)
    for key in ("U", "V", "E", "F"):
        out[key] = oracle_mod.quantize(1, np.array(arr[key], dtype=np.float64))
    S = []
    for l, Sl in enumerate(arr["S"]):
        kk = int(arr["level_rank"][l]) ** 2
        S.append(np.concatenate([oracle_mod.quantize(storage, Sl[i:i + kk].copy()) for i in range(0, len(Sl), kk)])
                 if len(Sl) else Sl)
    out["S"] = S
    b, e, q = arr["begin"], arr["end"], int(arr["q"])
    lf = (1 << q) - 1
    blocks, off = [], 0
    for i in range(1 << q):
        for t in range(arr["D_rowptr"][i], arr["D_rowptr"][i + 1]):
            sz = int(e[lf + i] - b[lf + i]) * int(e[lf + arr["D_colidx"][t]] - b[lf + arr["D_colidx"][t]])
            blocks.append(oracle_mod.quantize(storage, arr["D"][off:off + sz].copy()))
            off += sz
    out["D"] = np.concatenate(blocks)
    return out


def _rel(y, ref):
    return float(np.linalg.norm(y - ref) / np.linalg.norm(ref))


@pytest.mark.parametrize("n,d,m,p", [(5000, 2, 32, 4), (3000, 3, 24, 3), (1, 2, 8, 2)])
def test_arrays_of_oracle_h2_fp64(oracle_mod, n, d, m, p):
    """The oracle's own H^2 handed over as arrays: the product matches the
    oracle's to 1e-12, element by element."""
    h2mv = _h2mv()
    print(f"case oracle arrays n={n} d={d}", flush=True)
    pts = np.random.Generator(np.random.PCG64(70 + n)).random((n, d))
    o = oracle_mod.OracleH2(pts, m, p, 0.9, 0.15)
    A = h2mv.H2Matrix.from_arrays(o.export_arrays(), 0)
    assert np.array_equal(A.perm(), np.arange(n))
    x = np.random.Generator(np.random.PCG64(71)).standard_normal(n)
    y = A.matvec(torch.from_numpy(x).cuda()).cpu().numpy()
    ref = o.matvec(x)
    assert _rel(y, ref) <= FP64_TOL
    assert np.abs(y - ref).max() <= FP64_TOL * np.abs(ref).max()
    A.close()


@pytest.mark.parametrize("n,d,m,seed", [(4000, 2, 32, 1), (2500, 3, 16, 2), (700, 2, 8, 3)])
def test_arrays_level_ranks_fp64(oracle_mod, n, d, m, seed):
    """Random ranks per level up to 64 (above the leaf size at the leaves)."""
    h2mv = _h2mv()
    print(f"case level ranks n={n} d={d} seed={seed}", flush=True)
    arr = _structure_arrays(oracle_mod, n, d, m, 2, seed, 200 + seed, 64)
    A = h2mv.H2Matrix.from_arrays(arr, 0)
    assert A.info.rank == 64 and A.info.dim == 0
    X = np.random.Generator(np.random.PCG64(72)).standard_normal((3, n))
    Y = A.matmat(torch.from_numpy(X).cuda()).cpu().numpy()
    for j in range(3):
        ref = oracle_mod.arrays_matvec(arr, X[j])
        assert _rel(Y[j], ref) <= FP64_TOL
    A.close()


@pytest.mark.parametrize("storage", [1, 2], ids=["fp32", "bf16"])
@pytest.mark.parametrize("n,d,m,seed", [(4000, 2, 32, 4), (2500, 3, 16, 5)])
def test_arrays_level_ranks_reduced(oracle_mod, n, d, m, seed, storage):
    """Reduced storage of the same arrays: single vector and the matrix cores
    (16- and 32-wide tiles) against the stored values in exact arithmetic."""
    h2mv = _h2mv()
    print(f"case level ranks reduced n={n} d={d} storage={storage}", flush=True)
    arr = _structure_arrays(oracle_mod, n, d, m, 2, seed, 300 + seed, 64)
    ref_arr = _stored(oracle_mod, arr, storage)
    A = h2mv.H2Matrix.from_arrays(arr, storage)
    rng = np.random.Generator(np.random.PCG64(73))
    x = rng.standard_normal(n)
    y = A.matvec(torch.from_numpy(x).cuda()).cpu().numpy()
    assert _rel(y, oracle_mod.arrays_matvec(ref_arr, x)) <= REDUCED_TOL
    for nrhs in (5, 40):
        X = rng.standard_normal((nrhs, n))
        Y = A.matmat(torch.from_numpy(X).cuda()).cpu().numpy()
        for j in (0, nrhs - 1):
            assert _rel(Y[j], oracle_mod.arrays_matvec(ref_arr, X[j])) <= REDUCED_TOL, (nrhs, j)
    A.close()


def test_batch_with_array_members(oracle_mod):
    """Members given by arrays (ranks per level) batched with points-built ones."""
    h2mv = _h2mv()
    mats = [h2mv.H2Matrix.from_arrays(_structure_arrays(oracle_mod, 3000, 2, 32, 2, 6, 406, 48), 1),
            h2mv.H2Matrix.from_arrays(_structure_arrays(oracle_mod, 1200, 3, 16, 2, 7, 407, 27), 1)]
    w = W.C1
    mats.append(h2mv.H2Matrix(W.points(w), w.dim, w.leaf, w.cheb_p, w.eta, w.corr_len, storage=1))
    batch = h2mv.H2Batch(mats, 8)
    Xs = [torch.randn(8, m.n, dtype=torch.float64, device="cuda") for m in mats]
    Ys = batch.matmat(Xs)
    for m, X, Y in zip(mats, Xs, Ys):
        R = m.matmat(X)
        assert ((Y - R).norm() / R.norm()).item() <= 1e-12
    batch.close()
    for m in mats:
        m.close()


def _lmin(arr):
    q = int(arr["q"])
    return next((l for l in range(q + 1) if len(arr["S_colidx"][l]) > 0), q + 1)


def _transfer_mask(arr):
    """Entries of E / F of nodes below the first coupling level (the stored ones)."""
    q, kr = int(arr["q"]), [int(k) for k in arr["level_rank"]]
    lmin = _lmin(arr)
    mask = []
    for l in range(1, q + 1):
        mask.append(np.full((kr[l] * kr[l - 1]) << l, l > lmin))
    return np.concatenate(mask) if mask else np.zeros(0, dtype=bool)


def _assert_arrays_equal(a, b, tol, what):
    m = _transfer_mask(a)
    for key in ("U", "V"):
        assert np.abs(a[key] - b[key]).max(initial=0.0) <= tol, (what, key)
    for key in ("E", "F"):
        assert np.abs(a[key][m] - b[key][m]).max(initial=0.0) <= tol, (what, key)
        assert not np.any(b[key][~m]), (what, key, "unstored transfers read back as zero")
    for l in range(int(a["q"]) + 1):
        assert np.array_equal(a["S_rowptr"][l], b["S_rowptr"][l]) and np.array_equal(a["S_colidx"][l], b["S_colidx"][l])
        assert np.abs(np.asarray(a["S"][l]) - b["S"][l]).max(initial=0.0) <= tol, (what, "S", l)
    assert np.array_equal(a["D_rowptr"], b["D_rowptr"]) and np.array_equal(a["D_colidx"], b["D_colidx"])
    assert np.abs(a["D"] - b["D"]).max(initial=0.0) <= tol, (what, "D")


@pytest.mark.parametrize("storage", [0, 1, 2], ids=["fp64", "fp32", "bf16"])
def test_export_round_trip(oracle_mod, storage):
    """Arrays in, arrays out: exactly the stored values (FP64 as given; FP32
    rounded; BF16 code x scale), bitwise."""
    h2mv = _h2mv()
    arr = _structure_arrays(oracle_mod, 3000, 2, 32, 2, 8, 408, 40)
    A = h2mv.H2Matrix.from_arrays(arr, storage)
    got = h2mv.h2_export_arrays(A.handle)
    assert np.array_equal(got["level_rank"], arr["level_rank"])
    assert np.array_equal(got["begin"], arr["begin"]) and np.array_equal(got["end"], arr["end"])
    _assert_arrays_equal(_stored(oracle_mod, arr, storage), got, 0.0, f"storage {storage}")
    A.close()


def test_export_of_points_build_matches_oracle(oracle_mod):
    """A matrix built on the device from points reads back as the oracle's
    arrays of the same H^2, to the rounding of the entries."""
    h2mv = _h2mv()
    w = W.C1
    A = h2mv.H2Matrix(W.points(w), w.dim, w.leaf, w.cheb_p, w.eta, w.corr_len, storage=0)
    got = h2mv.h2_export_arrays(A.handle)
    o = oracle_mod.OracleH2(W.points(w), w.leaf, w.cheb_p, w.eta, w.corr_len)
    ref = o.export_arrays()
    scale = max(np.abs(ref["U"]).max(), np.abs(ref["E"]).max(), 1.0)
    _assert_arrays_equal(ref, got, 1e-13 * scale, "points build")
    A.close()
