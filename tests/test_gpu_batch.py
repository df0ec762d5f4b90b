"""Batches of uneven H^2 matrices in one launch per level slot (HIP graph).

Each member's batched product runs the same block arithmetic as its own
many-right-hand-side product, so the two must agree to rounding (the batch
may choose the non-pipelined block loop, which sums in the same order); the
members are also compared with the oracle on the same dequantized values.
"""
import numpy as np
import pytest

from paper_1902_01829_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

MEMBERS = [
    W.C1.with_(name="b0-2d-n3000-m32-p4", n=3000, leaf=32, cheb_p=4, corr_len=0.1, seed=301),
    W.C1.with_(name="b1-2d-n5000-m64-p8", n=5000, leaf=64, cheb_p=8, corr_len=0.2, seed=302),
    W.C1.with_(name="b2-3d-n4000-m32-p3", n=4000, dim=3, leaf=32, cheb_p=3, corr_len=0.15, seed=303),
    W.C1.with_(name="b3-3d-n2500-m64-p4", n=2500, dim=3, leaf=64, cheb_p=4, corr_len=0.3, seed=304),
    W.C1.with_(name="b4-2d-n777-m32-p4", n=777, leaf=32, cheb_p=4, corr_len=0.05, seed=305),
    W.C1.with_(name="b5-3d-n9000-m32-p4", n=9000, dim=3, leaf=32, cheb_p=4, corr_len=0.2, seed=306),
]


def _h2mv():
    from paper_1902_01829_amd import h2mv
    return h2mv


def _build(w, storage):
    return _h2mv().H2Matrix(W.points(w), w.dim, w.leaf, w.cheb_p, w.eta, w.corr_len, storage=storage)


def _pin_members(mats, nrhs, tile_width):
    """Members' own products with the batch's MFMA tile width (the prefetch
    depth does not change any sum): the same block arithmetic as the batch."""
    for m in mats:
        m.set_matmat_tuning(1 if nrhs <= 16 else 0, 1, tile_width, 0)


@pytest.mark.parametrize("storage", [1, 2], ids=["fp32", "bf16"])
def test_batch_equals_member_products(oracle_mod, storage):
    h2mv = _h2mv()
    nrhs = 8
    mats = [_build(w, storage) for w in MEMBERS]
    batch = h2mv.H2Batch(mats, nrhs)
    gen = torch.Generator(device="cuda").manual_seed(7)
    for call in range(3):   # the first call tunes and captures; the others replay the graph
        Xs = [torch.randn(nrhs, m.n, dtype=torch.float64, device="cuda", generator=gen) for m in mats]
        Ys = batch.matmat(Xs)
        _pin_members(mats, nrhs, batch.tuning()["tile_width"])
        refs = [m.matmat(X) for m, X in zip(mats, Xs)]
        torch.cuda.synchronize()
        for w, Y, R in zip(MEMBERS, Ys, refs):
            rel = ((Y - R).norm() / R.norm()).item()
            assert rel <= 1e-12, (call, w.name, rel)
    print("tuning:", batch.tuning(), flush=True)
    # two members against the oracle on the same dequantized values
    for idx in (0, 2):
        w, m = MEMBERS[idx], mats[idx]
        o = oracle_mod.OracleH2(W.points(w), w.leaf, w.cheb_p, w.eta, w.corr_len, storage=storage)
        X = Xs[idx].cpu().numpy()
        Y = Ys[idx].cpu().numpy()
        for j in (0, nrhs - 1):
            ref = o.matvec(X[j])
            assert np.linalg.norm(Y[j] - ref) / np.linalg.norm(ref) <= 1e-6
    batch.close()
    for m in mats:
        m.close()


def test_batch_rejects_fp64_mixed_and_wide():
    h2mv = _h2mv()
    a32 = _build(MEMBERS[0], 1)
    a64 = _build(MEMBERS[4], 0)
    abf = _build(MEMBERS[4], 2)
    for handles, nrhs, code in (([a32.handle, a64.handle], 8, h2mv.H2_ERR_UNSUPPORTED),
                                ([a32.handle, abf.handle], 8, h2mv.H2_ERR_UNSUPPORTED),
                                ([a32.handle], 33, h2mv.H2_ERR_UNSUPPORTED),
                                ([a32.handle], 0, h2mv.H2_ERR_INVALID_ARG)):
        with pytest.raises(h2mv.H2Error) as e:
            h2mv.h2_batch_create(handles, nrhs)
        assert e.value.code == code
    h2mv.h2_batch_free(0)
    for m in (a32, a64, abf):
        m.close()


DEGENERATE = [
    W.C1.with_(name="d0-2d-n1", n=1, seed=311),
    W.C1.with_(name="d1-2d-n3-m2-p1", n=3, leaf=2, cheb_p=1, seed=312),
    W.C1.with_(name="d2-3d-n50-m64", n=50, dim=3, leaf=64, seed=313),
    W.C1.with_(name="d3-2d-n4096-m32-p4", seed=314),
]


@pytest.mark.parametrize("nrhs", [1, 32])
@pytest.mark.parametrize("storage", [1, 2], ids=["fp32", "bf16"])
def test_batch_degenerate_members(storage, nrhs):
    """Members of one point, of leaves holding one or two points and of a
    single leaf, batched with a regular one; one and 32 right-hand sides."""
    h2mv = _h2mv()
    mats = [_build(w, storage) for w in DEGENERATE]
    batch = h2mv.H2Batch(mats, nrhs)
    gen = torch.Generator(device="cuda").manual_seed(11)
    Xs = [torch.randn(nrhs, m.n, dtype=torch.float64, device="cuda", generator=gen) for m in mats]
    for _ in range(2):
        Ys = batch.matmat(Xs)
        refs = [m.matmat(X) for m, X in zip(mats, Xs)]
        torch.cuda.synchronize()
        for w, Y, R in zip(DEGENERATE, Ys, refs):
            rel = ((Y - R).norm() / R.norm()).item()
            # the members' own products may have chosen another tile width
            assert rel <= (1e-12 if _same_width(batch, mats, nrhs) else 2e-6), (w.name, rel)
    batch.close()
    for m in mats:
        m.close()


def _same_width(batch, mats, nrhs):
    tw = batch.tuning()["tile_width"]
    return all(m.matmat_tuning(1 if nrhs <= 16 else 0)["tile_width"] == tw for m in mats)


def test_batch_tuning_cache_file(tmp_path, monkeypatch):
    """The chosen launch shape is appended to the file named by
    H2MV_AUTOTUNE_CACHE, and a second batch of the same members reuses it."""
    h2mv = _h2mv()
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("H2MV_AUTOTUNE_CACHE", str(cache))
    members = [W.C1.with_(name=f"c{i}", n=1500 + 250 * i, seed=320 + i) for i in range(3)]
    mats = [_build(w, 1) for w in members]
    Xs = [torch.randn(4, m.n, dtype=torch.float64, device="cuda") for m in mats]
    b1 = h2mv.H2Batch(mats, 4)
    assert b1.tuning()["tuned_ms"] < 0          # nothing chosen before the first product
    Y1 = b1.matmat(Xs)
    t1 = b1.tuning()
    assert t1["tuned_ms"] > 0
    lines = cache.read_text().split("\n")
    assert any(line.endswith(f" {t1['pipelined']} {t1['grid']} {t1['tile_width']}") for line in lines if line)
    b2 = h2mv.H2Batch(mats, 4)
    Y2 = b2.matmat(Xs)
    t2 = b2.tuning()
    assert (t2["pipelined"], t2["grid"], t2["tile_width"], t2["tuned_ms"]) == \
        (t1["pipelined"], t1["grid"], t1["tile_width"], 0.0)
    for a, b in zip(Y1, Y2):
        assert torch.equal(a, b)
    b1.close()
    b2.close()
    for m in mats:
        m.close()


@pytest.mark.parametrize("storage", [1, 2], ids=["fp32", "bf16"])
def test_batch_every_launch_shape(oracle_mod, storage):
    """Every configuration the tuner may pick -- prefetch depth 0..3, 4..5
    with tiles shared by a row's halves (32-wide), 6..7 with rings of column
    chunks (16-wide), one workgroup per item group or
    persistent grids, 16- or 32-wide tiles -- gives
    each member's own product with the same tile width (to 1e-12: the same
    block arithmetic in the same order) and matches the oracle on the same
    dequantized values (1e-6), on two consecutive products per shape."""
    h2mv = _h2mv()
    nrhs = 8
    mats = [_build(w, storage) for w in MEMBERS]
    batch = h2mv.H2Batch(mats, nrhs)
    gen = torch.Generator(device="cuda").manual_seed(17)
    Xs = [torch.randn(nrhs, m.n, dtype=torch.float64, device="cuda", generator=gen) for m in mats]
    oracles = {i: oracle_mod.OracleH2(W.points(MEMBERS[i]), MEMBERS[i].leaf, MEMBERS[i].cheb_p, MEMBERS[i].eta,
                                      MEMBERS[i].corr_len, storage=storage) for i in (0, 5)}
    oref = {i: [oracles[i].matvec(Xs[i][j].cpu().numpy()) for j in (0, nrhs - 1)] for i in oracles}
    refs = {}
    for tw in (16, 32):
        _pin_members(mats, nrhs, tw)
        refs[tw] = [m.matmat(X) for m, X in zip(mats, Xs)]
    for tw in (16, 32):
        for depth in ((0, 1, 2, 3, 4, 5) if tw == 32 else (0, 1, 2, 3, 6, 7)):
            for grid in (0, 64, 2048):
                batch.set_tuning(depth, grid, tw)
                for call in range(2):
                    Ys = batch.matmat(Xs)
                    torch.cuda.synchronize()
                    for w, Y, R in zip(MEMBERS, Ys, refs[tw]):
                        rel = ((Y - R).norm() / R.norm()).item()
                        assert rel <= 1e-12, (tw, depth, grid, call, w.name, rel)
                for i in oref:
                    Yi = Ys[i].cpu().numpy()
                    for jj, j in enumerate((0, nrhs - 1)):
                        ref = oref[i][jj]
                        assert np.linalg.norm(Yi[j] - ref) / np.linalg.norm(ref) <= 1e-6, (tw, depth, grid, i, j)
    batch.close()
    for m in mats:
        m.close()


def test_batch_set_tuning_rejects():
    h2mv = _h2mv()
    mats = [_build(MEMBERS[0], 1)]
    b8 = h2mv.H2Batch(mats, 8)
    b20 = h2mv.H2Batch(mats, 20)
    for B, args in ((b8, (8, 0, 16)), (b8, (6, 0, 32)), (b8, (4, 0, 16)), (b8, (-1, 0, 16)), (b8, (1, -5, 16)), (b8, (1, 0, 24)),
                    (b20, (1, 0, 16))):
        with pytest.raises(h2mv.H2Error) as e:
            B.set_tuning(*args)
        assert e.value.code == h2mv.H2_ERR_INVALID_ARG
    b8.close()
    b20.close()
    mats[0].close()


def test_batch_64_uneven_members(oracle_mod):
    """The 64-member batch of the benchmark (n log-uniform in [2^12, 2^17],
    2-D ranks 16 / 64 and 3-D ranks 27 / 64, leaves of 32 or 64, FP32, 8
    right-hand sides), autotuned and replayed from its graph: every member's
    batched product equals its own product with the same tile width (1e-12),
    and members of each kind match the oracle on all rows of sampled leaves."""
    h2mv = _h2mv()
    nrhs = 8
    members = W.batch_members()
    mats = [_build(w, 1) for w in members]
    batch = h2mv.H2Batch(mats, nrhs)
    gen = torch.Generator(device="cuda").manual_seed(23)
    Xs = [torch.randn(nrhs, m.n, dtype=torch.float64, device="cuda", generator=gen) for m in mats]
    Ys = batch.matmat(Xs)       # tunes, captures, runs
    Ys = batch.matmat(Xs)       # graph replay
    tw = batch.tuning()["tile_width"]
    print("tuning:", batch.tuning(), flush=True)
    _pin_members(mats, nrhs, tw)
    worst = 0.0
    for w, m, X, Y in zip(members, mats, Xs, Ys):
        R = m.matmat(X)
        rel = ((Y - R).norm() / R.norm()).item()
        worst = max(worst, rel)
        assert rel <= 1e-12, (w.name, rel)
    print(f"  worst batched vs own product: {worst:.3e}", flush=True)
    # one member of each kind: 2-D and 3-D, low and high rank, smallest and largest n
    kinds = {}
    for i, w in enumerate(members):
        kinds.setdefault((w.dim, w.rank), []).append(i)
    picks = sorted({min(v, key=lambda i: members[i].n) for v in kinds.values()} |
                   {max(v, key=lambda i: members[i].n) for v in kinds.values()})
    rng = np.random.Generator(np.random.PCG64(29))
    for i in picks:
        w = members[i]
        o = oracle_mod.OracleH2(W.points(w), w.leaf, w.cheb_p, w.eta, w.corr_len, storage=1, keep_blocks=False)
        leaves = np.sort(rng.choice(o.leaf_nodes(), size=min(4, len(o.leaf_nodes())), replace=False))
        rows = o.leaf_rows(leaves)
        Yi, Xi = Ys[i].cpu().numpy(), Xs[i].cpu().numpy()
        for j in (0, nrhs - 1):
            ref = o.matvec_leaves(Xi[j], leaves)
            rel = np.linalg.norm(Yi[j][rows] - ref) / np.linalg.norm(ref)
            print(f"  member {i} ({w.name}) column {j}: rel err vs dequantized oracle {rel:.3e}", flush=True)
            assert rel <= 1e-6
    batch.close()
    for m in mats:
        m.close()
