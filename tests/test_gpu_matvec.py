"""GPU parity of the HIP H^2 product against the FP64 oracle, through the C ABI.

Both sides build the H^2 from the same seeded points with the same rules (the
structure is identical, see test_structure.py); their entries differ only by
the rounding of exp and of the interpolation weights, so the FP64 products
must agree to 1e-12 relative (2-norm, the error measure of Sec. 4.6) and
elementwise to 1e-12 of the largest entry.  Reduced storage is compared with
the oracle's exact dequantized values (isolating the FP32 arithmetic) and with
the FP64 oracle (the storage error itself).
"""
import numpy as np
import pytest

from paper_1902_01829_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12
# FP32 arithmetic on the same stored values: per-block partial sums of <= 64
# FP32 products (relative error <= 64 u_32 ~ 4e-6 worst case, ~1e-7 typical),
# FP32 input and vector trees (u_32 = 6e-8 each), FP64 sums over blocks.
REDUCED_VS_DEQUANT_TOL = 1e-6
FP32_VS_FP64_TOL = 1e-6
# BF16 storage against the FP64 oracle.  The workloads state their bound,
# 2e-3 (the 4096-point 2-D matrix, the 2^19-point 3-D matrix, the 2^20-point
# 2-D matrix with 32 right-hand sides).  For any other case the bound is
# derived rather than chosen: the GPU result differs from the FP64 product by
# the storage error of the representation itself, e_store = |y_q - y_64| /
# |y_64| with y_q the oracle's exact product on the dequantized values (a
# property of the BF16 matrix, computed by the oracle alone), plus the
# arithmetic error, at most REDUCED_VS_DEQUANT_TOL relative to |y_q| (triangle
# inequality).  Where leaves hold fewer points than the rank, e_store exceeds
# 2e-3 (rounding reaches y through overcomplete leaf bases).
BF16_VS_FP64_TOL = 2e-3


def bf16_derived_bound(y_q, y_64):
    """Storage error of the BF16 representation plus the arithmetic bound."""
    n64 = np.linalg.norm(y_64)
    return np.linalg.norm(y_q - y_64) / n64 + REDUCED_VS_DEQUANT_TOL * np.linalg.norm(y_q) / n64


def _h2mv():
    from paper_1902_01829_amd import h2mv
    return h2mv


def _build(w, storage=0):
    h2mv = _h2mv()
    return h2mv.H2Matrix(W.points(w), w.dim, w.leaf, w.cheb_p, w.eta, w.corr_len, storage=storage)


def _gpu_matvec(A, x_tree):
    x = torch.from_numpy(np.ascontiguousarray(x_tree)).cuda()
    y = A.matvec(x)
    torch.cuda.synchronize()
    return y.cpu().numpy()


def _check_fp64(y, ref):
    rel = np.linalg.norm(y - ref) / np.linalg.norm(ref)
    assert rel <= FP64_TOL, rel
    assert np.abs(y - ref).max() <= FP64_TOL * np.abs(ref).max()


SMALL = [
    W.C1,
    W.C1.with_(name="2d-n5000-m32-p4-ragged", n=5000, seed=78),
    W.C1.with_(name="3d-n3000-m24-p3", n=3000, dim=3, leaf=24, cheb_p=3, corr_len=0.2, seed=77),
    W.C1.with_(name="2d-n999-m7-p2-eta2", n=999, leaf=7, cheb_p=2, eta=2.0, seed=81),
    W.C1.with_(name="2d-n20000-m64-p8", n=20000, leaf=64, cheb_p=8, seed=82),
    W.C1.with_(name="3d-n20000-m64-p4", n=20000, dim=3, leaf=64, cheb_p=4, corr_len=0.2, seed=83),
    W.C1.with_(name="2d-n3-m2-p1", n=3, leaf=2, cheb_p=1, seed=84),
    W.C1.with_(name="2d-n1", n=1, seed=85),
    W.C1.with_(name="3d-n50-m64-single-leaf", n=50, dim=3, leaf=64, seed=86),
]


@pytest.mark.parametrize("w", SMALL, ids=lambda w: w.name)
def test_fp64_matvec_matches_oracle(oracle_mod, w):
    print(f"case {w.name}", flush=True)
    A = _build(w)
    o = oracle_mod.OracleH2(W.points(w), w.leaf, w.cheb_p, w.eta, w.corr_len, keep_blocks=w.n <= 6000)
    perm = A.perm()
    assert np.array_equal(perm, o.perm())
    xt = W.rhs(w)[perm]
    _check_fp64(_gpu_matvec(A, xt), o.matvec(xt))
    A.close()


def test_fp64_deterministic_linear_zero(oracle_mod):
    w = W.C1
    A = _build(w)
    x = torch.from_numpy(W.rhs(w)[A.perm()]).cuda()
    z = torch.randn(w.n, dtype=torch.float64, device="cuda")
    y1, y2 = A.matvec(x), A.matvec(x)
    assert torch.equal(y1, y2)
    assert torch.count_nonzero(A.matvec(torch.zeros_like(x))) == 0
    lin = A.matvec(2.0 * x - z)
    ref = 2.0 * y1 - A.matvec(z)
    assert (lin - ref).abs().max().item() <= 1e-12 * y1.abs().max().item()
    A.close()


def _sampled_parity(oracle_mod, w, storage, nleaves, tol, quant_ref_tol=None):
    """Full-size workload: every leaf row of a seeded sample of leaves."""
    print(f"case {w.name} storage {storage}", flush=True)
    A = _build(w, storage)
    perm = A.perm()
    xt = W.rhs(w)[perm]
    y = _gpu_matvec(A, xt)
    A.close()
    o = oracle_mod.OracleH2(W.points(w), w.leaf, w.cheb_p, w.eta, w.corr_len, keep_blocks=False)
    assert np.array_equal(perm, o.perm())
    rng = np.random.Generator(np.random.PCG64(7))
    leaves = np.sort(rng.choice(o.leaf_nodes(), size=nleaves, replace=False))
    rows = o.leaf_rows(leaves)
    ref = o.matvec_leaves(xt, leaves)
    rel = np.linalg.norm(y[rows] - ref) / np.linalg.norm(ref)
    print(f"  rel err vs fp64 oracle on {len(rows)} rows: {rel:.3e}", flush=True)
    assert rel <= tol
    if storage == 0:
        assert np.abs(y[rows] - ref).max() <= FP64_TOL * np.abs(ref).max()
    if quant_ref_tol is not None:
        oq = oracle_mod.OracleH2(W.points(w), w.leaf, w.cheb_p, w.eta, w.corr_len, storage=storage,
                                 keep_blocks=False)
        refq = oq.matvec_leaves(xt, leaves)
        relq = np.linalg.norm(y[rows] - refq) / np.linalg.norm(refq)
        print(f"  rel err vs dequantized oracle: {relq:.3e}", flush=True)
        assert relq <= quant_ref_tol
    return rel


def _all_rows_fp64(oracle_mod, w):
    """Full-size workload, FP64: every row against the matrix-free oracle,
    elementwise and in the 2-norm."""
    print(f"case {w.name} fp64 all rows", flush=True)
    A = _build(w, 0)
    perm = A.perm()
    xt = W.rhs(w)[perm]
    y = _gpu_matvec(A, xt)
    A.close()
    o = oracle_mod.OracleH2(W.points(w), w.leaf, w.cheb_p, w.eta, w.corr_len, keep_blocks=False)
    assert np.array_equal(perm, o.perm())
    ref = o.matvec(xt)
    rel = np.linalg.norm(y - ref) / np.linalg.norm(ref)
    print(f"  rel err vs fp64 oracle on all {w.n} rows: {rel:.3e}, "
          f"max abs err / max |y|: {np.abs(y - ref).max() / np.abs(ref).max():.3e}", flush=True)
    _check_fp64(y, ref)


def test_fp64_full_2d_1m_all_rows(oracle_mod):
    _all_rows_fp64(oracle_mod, W.C2)


def test_fp64_full_3d_512k_all_rows(oracle_mod):
    _all_rows_fp64(oracle_mod, W.C3)


@pytest.mark.parametrize("w", [W.C1, SMALL[2], SMALL[4], SMALL[5]], ids=lambda w: w.name)
@pytest.mark.parametrize("storage", [1, 2], ids=["fp32", "bf16"])
def test_reduced_storage_small(oracle_mod, w, storage):
    print(f"case {w.name} storage {storage}", flush=True)
    A = _build(w, storage)
    perm = A.perm()
    xt = W.rhs(w)[perm]
    y = _gpu_matvec(A, xt)
    A.close()
    o64 = oracle_mod.OracleH2(W.points(w), w.leaf, w.cheb_p, w.eta, w.corr_len, keep_blocks=False)
    oq = oracle_mod.OracleH2(W.points(w), w.leaf, w.cheb_p, w.eta, w.corr_len, storage=storage,
                             keep_blocks=False)
    ref, refq = o64.matvec(xt), oq.matvec(xt)
    relq = np.linalg.norm(y - refq) / np.linalg.norm(refq)
    rel = np.linalg.norm(y - ref) / np.linalg.norm(ref)
    print(f"  vs dequantized {relq:.3e}  vs fp64 {rel:.3e}", flush=True)
    assert relq <= REDUCED_VS_DEQUANT_TOL
    if storage == 1:
        assert rel <= FP32_VS_FP64_TOL
    else:
        assert rel <= bf16_derived_bound(refq, ref)
        if w == W.C1:
            assert rel <= BF16_VS_FP64_TOL


@pytest.mark.parametrize("storage", [1, 2], ids=["fp32", "bf16"])
def test_reduced_storage_full_3d_512k(oracle_mod, storage):
    _sampled_parity(oracle_mod, W.C3, storage, 16, FP32_VS_FP64_TOL if storage == 1 else BF16_VS_FP64_TOL,
                    quant_ref_tol=REDUCED_VS_DEQUANT_TOL)


@pytest.mark.parametrize("storage", [0, 1, 2], ids=["fp64", "fp32", "bf16"])
def test_matmat_columns_equal_matvec(storage):
    w = W.C1.with_(name="2d-n20000-m64-p8", n=20000, leaf=64, cheb_p=8, seed=82)
    A = _build(w, storage)
    X = torch.randn(5, w.n, dtype=torch.float64, device="cuda")
    Y = A.matmat(X)
    for j in range(5):
        yj = A.matvec(X[j].contiguous())
        tol = 1e-13 if storage == 0 else 1e-6
        assert (Y[j] - yj).norm().item() <= tol * yj.norm().item()
    A.close()
