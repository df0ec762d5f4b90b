"""ctypes wrapper of the FP64 CPU oracle (h2oracle.c).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg use it; the HIP library never does.  It imports nothing from
the HIP package.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# H2_ORACLE_LIBRARY names another build of h2oracle.c (the sanitizer test's)
LIB_PATH = os.environ.get("H2_ORACLE_LIBRARY") or os.path.join(HERE, "liboracle.so")
SRC = os.path.join(HERE, "h2oracle.c")

KERNEL_EXP, KERNEL_POLY2 = 0, 1
STORE_FP64, STORE_FP32, STORE_BF16 = 0, 1, 2

_i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, no fast-math, no FMA contraction)."""
    if force or not os.path.exists(LIB_PATH):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-shared", "-fPIC",
                               "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            if os.environ.get("H2_ORACLE_LIBRARY"):
                raise RuntimeError(f"H2_ORACLE_LIBRARY={LIB_PATH} does not exist")
            build()
        L = C.CDLL(LIB_PATH)
        L.or_cheb_nodes.argtypes = [C.c_int, _f64p]
        L.or_lagrange_1d.argtypes = [C.c_int, _f64p, C.c_int, C.c_double]
        L.or_lagrange_1d.restype = C.c_double
        L.or_kernel.argtypes = [C.c_int, C.c_int, C.c_double, _f64p, _f64p]
        L.or_kernel.restype = C.c_double
        L.or_quantize_block.argtypes = [C.c_int, C.c_int64, _f64p]
        L.or_round_bf16.argtypes = [C.c_double]
        L.or_round_bf16.restype = C.c_double
        L.or_build.argtypes = [_f64p, C.c_int64, C.c_int, C.c_int, C.c_int, C.c_double, C.c_double,
                               C.c_int, C.c_int, C.c_int, C.POINTER(C.c_void_p)]
        L.or_build.restype = C.c_int
        L.or_free.argtypes = [C.c_void_p]
        L.or_sizes.argtypes = [C.c_void_p, _i64p]
        L.or_perm.argtypes = [C.c_void_p, _i64p]
        L.or_ranges.argtypes = [C.c_void_p, _i64p, _i64p]
        L.or_boxes.argtypes = [C.c_void_p, _f64p, _f64p]
        L.or_coupling_count.argtypes = [C.c_void_p, C.c_int]
        L.or_coupling_count.restype = C.c_int64
        L.or_coupling_bsr.argtypes = [C.c_void_p, C.c_int, _i32p, _i32p]
        L.or_dense_count.argtypes = [C.c_void_p]
        L.or_dense_count.restype = C.c_int64
        L.or_dense_bsr.argtypes = [C.c_void_p, _i32p, _i32p]
        L.or_near_ties.argtypes = [C.c_void_p]
        L.or_near_ties.restype = C.c_int64
        L.or_flat_tree.argtypes = [C.c_void_p, _i64p, _i64p, _i64p, _i64p]
        L.or_bsr_assemble.argtypes = [C.c_int32, C.c_int64, _i32p, _i32p, _i32p, _i32p, _i64p]
        L.or_leaf_basis.argtypes = [C.c_void_p, C.c_int64, _f64p]
        L.or_transfer.argtypes = [C.c_void_p, C.c_int64, _f64p]
        L.or_coupling_block.argtypes = [C.c_void_p, C.c_int, C.c_int64, _f64p]
        L.or_dense_block.argtypes = [C.c_void_p, C.c_int64, _f64p]
        L.or_explicit_basis.argtypes = [C.c_void_p, C.c_int64, C.c_int, _f64p]
        L.or_matvec.argtypes = [C.c_void_p, _f64p, _f64p]
        L.or_matvec_leaves.argtypes = [C.c_void_p, _f64p, C.c_int64, _i64p, _f64p]
        L.or_matvec_parts.argtypes = [C.c_void_p, _f64p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
        L.or_dense_expand.argtypes = [C.c_void_p, _f64p]
        L.or_kernel_matvec.argtypes = [_f64p, C.c_int64, C.c_int, C.c_double, C.c_int, _f64p,
                                       C.c_int64, _i64p, _f64p]
        vp = C.c_void_p
        L.or_arrays_matvec.argtypes = [C.c_int64, C.c_int, _i32p, _i64p, _i64p, vp, vp, vp, vp,
                                       C.POINTER(vp), C.POINTER(vp), C.POINTER(vp), _i32p, vp, vp, _f64p, _f64p]
        L.or_arrays_matvec.restype = C.c_int
        _lib = L
    return _lib


def cheb_nodes(p: int) -> np.ndarray:
    t = np.zeros(p)
    lib().or_cheb_nodes(p, t)
    return t


def lagrange_1d(t: np.ndarray, a: int, s: float) -> float:
    return lib().or_lagrange_1d(len(t), np.ascontiguousarray(t, dtype=np.float64), a, s)


def quantize(storage: int, vals: np.ndarray) -> np.ndarray:
    v = np.array(vals, dtype=np.float64, copy=True).ravel()
    lib().or_quantize_block(storage, v.size, v)
    return v.reshape(np.shape(vals))


def kernel_matvec(pts, x, ell, rows=None, kernel=KERNEL_EXP) -> np.ndarray:
    pts = np.ascontiguousarray(pts, dtype=np.float64)
    n, d = pts.shape
    rows = np.arange(n, dtype=np.int64) if rows is None else np.ascontiguousarray(rows, dtype=np.int64)
    y = np.zeros(len(rows))
    lib().or_kernel_matvec(pts, n, d, ell, kernel, np.ascontiguousarray(x, dtype=np.float64),
                           len(rows), rows, y)
    return y


class OracleH2:
    """An H^2 matrix built by the oracle from points; see h2oracle.h."""

    def __init__(self, pts, leaf, cheb_p, eta, corr_len, kernel=KERNEL_EXP,
                 storage=STORE_FP64, keep_blocks=True):
        pts = np.ascontiguousarray(pts, dtype=np.float64)
        n, d = pts.shape
        h = C.c_void_p()
        rc = lib().or_build(pts, n, d, leaf, cheb_p, eta, corr_len, kernel, storage,
                            1 if keep_blocks else 0, C.byref(h))
        if rc != 0:
            raise ValueError(f"oracle build rejected its arguments (rc={rc})")
        self._h = h
        s = np.zeros(9, dtype=np.int64)
        lib().or_sizes(h, s)
        (self.n, self.d, self.m, self.p, self.k, self.q, self.lmin, self.nnodes,
         self.n_coupling) = (int(v) for v in s)
        self.eta, self.corr_len, self.storage = eta, corr_len, storage

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.or_free(h)
            self._h = None

    # structure
    def perm(self):
        p = np.zeros(self.n, dtype=np.int64)
        lib().or_perm(self._h, p)
        return p

    def ranges(self):
        b = np.zeros(self.nnodes, dtype=np.int64)
        e = np.zeros(self.nnodes, dtype=np.int64)
        lib().or_ranges(self._h, b, e)
        return b, e

    def boxes(self):
        lo = np.zeros((self.nnodes, self.d))
        hi = np.zeros((self.nnodes, self.d))
        lib().or_boxes(self._h, lo, hi)
        return lo, hi

    def coupling_bsr(self, level):
        cnt = lib().or_coupling_count(self._h, level)
        rp = np.zeros((1 << level) + 1, dtype=np.int32)
        ci = np.zeros(max(cnt, 1), dtype=np.int32)
        lib().or_coupling_bsr(self._h, level, rp, ci)
        return rp, ci[:cnt]

    def dense_bsr(self):
        cnt = lib().or_dense_count(self._h)
        rp = np.zeros((1 << self.q) + 1, dtype=np.int32)
        ci = np.zeros(max(cnt, 1), dtype=np.int32)
        lib().or_dense_bsr(self._h, rp, ci)
        return rp, ci[:cnt]

    def near_ties(self):
        return int(lib().or_near_ties(self._h))

    def flat_tree(self):
        lp = np.zeros(self.q + 2, dtype=np.int64)
        par = np.zeros(self.nnodes, dtype=np.int64)
        head = np.zeros(self.nnodes, dtype=np.int64)
        nxt = np.zeros(self.nnodes, dtype=np.int64)
        lib().or_flat_tree(self._h, lp, par, head, nxt)
        return lp, par, head, nxt

    def leaf_nodes(self):
        f = (1 << self.q) - 1
        return np.arange(f, f + (1 << self.q), dtype=np.int64)

    # data
    def node_size(self, v):
        b, e = self.ranges()
        return int(e[v] - b[v])

    def leaf_basis(self, node):
        U = np.zeros(self.node_size(node) * self.k)
        lib().or_leaf_basis(self._h, node, U)
        return U.reshape(self.k, -1).T          # column-major m_i x k

    def transfer(self, node):
        E = np.zeros(self.k * self.k)
        lib().or_transfer(self._h, node, E)
        return E.reshape(self.k, self.k).T

    def coupling_block(self, level, idx):
        S = np.zeros(self.k * self.k)
        lib().or_coupling_block(self._h, level, idx, S)
        return S.reshape(self.k, self.k).T

    def dense_block(self, idx, rows, cols):
        D = np.zeros(rows * cols)
        lib().or_dense_block(self._h, idx, D)
        return D.reshape(cols, rows).T

    def explicit_basis(self, node, method):
        U = np.zeros(self.node_size(node) * self.k)
        lib().or_explicit_basis(self._h, node, method, U)
        return U.reshape(self.k, -1).T

    # products (tree order)
    def matvec(self, x_tree):
        y = np.zeros(self.n)
        lib().or_matvec(self._h, np.ascontiguousarray(x_tree, dtype=np.float64), y)
        return y

    def matvec_parts(self, x_tree):
        xh = np.zeros((self.nnodes, self.k))
        yh = np.zeros((self.nnodes, self.k))
        yn = np.zeros(self.n)
        yf = np.zeros(self.n)
        lib().or_matvec_parts(self._h, np.ascontiguousarray(x_tree, dtype=np.float64),
                              xh.ctypes.data, yh.ctypes.data, yn.ctypes.data, yf.ctypes.data)
        return xh, yh, yn, yf

    def matvec_leaves(self, x_tree, leaves):
        leaves = np.ascontiguousarray(leaves, dtype=np.int64)
        b, e = self.ranges()
        y = np.zeros(int(np.sum(e[leaves] - b[leaves])))
        lib().or_matvec_leaves(self._h, np.ascontiguousarray(x_tree, dtype=np.float64),
                               len(leaves), leaves, y)
        return y

    def leaf_rows(self, leaves):
        """Tree positions of the rows of the listed leaves, in matvec_leaves order."""
        b, e = self.ranges()
        return np.concatenate([np.arange(b[v], e[v]) for v in leaves]).astype(np.int64)

    def export_arrays(self):
        """The representation as flattened arrays (column-major blocks; see
        arrays_matvec), FP64 values as stored (dequantized in reduced modes)."""
        q, k = self.q, self.k
        b, e = self.ranges()
        lf = (1 << q) - 1
        U = np.concatenate([self.leaf_basis(v).ravel(order="F") for v in range(lf, 2 * lf + 1)])
        E = np.concatenate([self.transfer(c).ravel(order="F") for c in range(1, self.nnodes)]) \
            if q > 0 else np.zeros(0)
        S_rowptr, S_colidx, S = [], [], []
        for l in range(q + 1):
            rp, ci = self.coupling_bsr(l)
            S_rowptr.append(rp)
            S_colidx.append(ci)
            S.append(np.concatenate([self.coupling_block(l, i).ravel(order="F") for i in range(len(ci))])
                     if len(ci) else np.zeros(0))
        drp, dci = self.dense_bsr()
        sizes = e - b
        blocks = []
        for i in range(1 << q):
            for t in range(drp[i], drp[i + 1]):
                blocks.append(self.dense_block(t, int(sizes[lf + i]), int(sizes[lf + dci[t]])).ravel(order="F"))
        return {"n": self.n, "q": q, "level_rank": np.full(q + 1, k, dtype=np.int32), "begin": b, "end": e,
                "U": U, "V": U, "E": E, "F": E, "S_rowptr": S_rowptr, "S_colidx": S_colidx, "S": S,
                "D_rowptr": drp, "D_colidx": dci, "D": np.concatenate(blocks) if blocks else np.zeros(0)}

    def dense_expand(self):
        A = np.zeros((self.n, self.n))
        lib().or_dense_expand(self._h, A)
        return A


def _ptr(a):
    return None if a is None or a.size == 0 else a.ctypes.data


def arrays_matvec(arr, x):
    """y = A x for an H^2 matrix given by its arrays (dict with n, q,
    level_rank, begin, end, U, V, E, F, S_rowptr, S_colidx, S (lists over
    levels), D_rowptr, D_colidx, D; layout as in or_arrays_matvec)."""
    q = int(arr["q"])
    keep = []

    def f64(a):
        a = np.ascontiguousarray(a, dtype=np.float64)
        keep.append(a)
        return a

    def i32(a):
        a = np.ascontiguousarray(a, dtype=np.int32)
        keep.append(a)
        return a
    VP = C.c_void_p * (q + 1)
    rp = VP(*[_ptr(i32(r)) for r in arr["S_rowptr"]])
    ci = VP(*[_ptr(i32(c)) for c in arr["S_colidx"]])
    sv = VP(*[_ptr(f64(v)) for v in arr["S"]])
    y = np.zeros(int(arr["n"]))
    rc = lib().or_arrays_matvec(int(arr["n"]), q, i32(arr["level_rank"]),
                                np.ascontiguousarray(arr["begin"], dtype=np.int64),
                                np.ascontiguousarray(arr["end"], dtype=np.int64),
                                _ptr(f64(arr["U"])), _ptr(f64(arr["V"])), _ptr(f64(arr["E"])), _ptr(f64(arr["F"])),
                                rp, ci, sv, i32(arr["D_rowptr"]), _ptr(i32(arr["D_colidx"])), _ptr(f64(arr["D"])),
                                np.ascontiguousarray(x, dtype=np.float64), y)
    if rc != 0:
        raise ValueError("or_arrays_matvec rejected the arrays")
    return y


def bsr_assemble(nrows, rows, cols):
    rows = np.ascontiguousarray(rows, dtype=np.int32)
    cols = np.ascontiguousarray(cols, dtype=np.int32)
    rp = np.zeros(nrows + 1, dtype=np.int32)
    ci = np.zeros(max(len(rows), 1), dtype=np.int32)
    order = np.zeros(max(len(rows), 1), dtype=np.int64)
    lib().or_bsr_assemble(nrows, len(rows), rows, cols, rp, ci, order)
    return rp, ci[:len(rows)], order[:len(rows)]


def rel_err(y, ref) -> float:
    """Relative 2-norm error |y - ref| / |ref| (the error measure of Sec. 4.6)."""
    ref = np.asarray(ref)
    return float(np.linalg.norm(np.asarray(y) - ref) / np.linalg.norm(ref))


def _qr_positive(M):
    """Thin QR with a non-negative diagonal of R (the unique factorization of
    a full-column-rank M); numpy's Householder QR, signs normalized."""
    Q, R = np.linalg.qr(M, mode="reduced")
    d = np.where(np.diag(R) < 0.0, -1.0, 1.0)
    return Q * d[None, :], R * d[:, None]


def orthogonalize_arrays(arr):
    """Basis orthogonalization and projection of the coupling blocks (Sec. 5.1,
    Alg. 6 and Alg. 7) of a symmetric H^2 matrix given by its arrays (V = U,
    F = E; see arrays_matvec for the layout).  Leaves: U_j = Q_j T_j (QR), Q_j
    the new leaf basis.  Levels q .. l_min + 1, parent p with children c1, c2:
    Z = [T_c1 E_c1; T_c2 E_c2] = Q T_p, the two k_l x k_(l-1) blocks of Q the
    new transfers.  Every coupling block S_ij <- T_i S_ij T_j^T.  Transfers of
    levels at or above l_min are not used by the product and are left as they
    are.  Requires leaves with at least k_q rows and 2 k_l >= k_(l-1).
    Returns (new arrays, {node: T})."""
    q = int(arr["q"])
    kr = [int(k) for k in arr["level_rank"]]
    b, e = arr["begin"], arr["end"]
    lf = (1 << q) - 1
    lmin = next((l for l in range(q + 1) if int(arr["S_rowptr"][l][1 << l]) > 0), q + 1)
    out = dict(arr)
    T = {}
    if lmin > q:
        return out, T
    U = np.array(arr["U"], dtype=np.float64, copy=True)
    off = 0
    for j in range(1 << q):
        m = int(e[lf + j] - b[lf + j])
        if m < kr[q]:
            raise ValueError("a leaf holds fewer rows than the rank")
        Uj = U[off:off + m * kr[q]].reshape(kr[q], m).T
        Qj, T[lf + j] = _qr_positive(Uj)
        U[off:off + m * kr[q]] = Qj.ravel(order="F")
        off += m * kr[q]
    E = np.array(arr["E"], dtype=np.float64, copy=True)
    eo, off = {}, 0
    for l in range(1, q + 1):
        for c in range((1 << l) - 1, (2 << l) - 1):
            eo[c] = off
            off += kr[l] * kr[l - 1]
    for l in range(q, lmin, -1):
        kc, kp = kr[l], kr[l - 1]
        if 2 * kc < kp:
            raise ValueError("a level's rank exceeds twice its children's")
        for p in range((1 << (l - 1)) - 1, (1 << l) - 1):
            c1, c2 = 2 * p + 1, 2 * p + 2
            E1 = E[eo[c1]:eo[c1] + kc * kp].reshape(kp, kc).T
            E2 = E[eo[c2]:eo[c2] + kc * kp].reshape(kp, kc).T
            Q, T[p] = _qr_positive(np.vstack([T[c1] @ E1, T[c2] @ E2]))
            E[eo[c1]:eo[c1] + kc * kp] = Q[:kc].ravel(order="F")
            E[eo[c2]:eo[c2] + kc * kp] = Q[kc:].ravel(order="F")
    S = []
    for l in range(q + 1):
        Sl = np.array(arr["S"][l], dtype=np.float64, copy=True)
        k, f = kr[l], (1 << l) - 1
        rp, ci = arr["S_rowptr"][l], arr["S_colidx"][l]
        for i in range(1 << l):
            for t in range(rp[i], rp[i + 1]):
                Sb = Sl[t * k * k:(t + 1) * k * k].reshape(k, k).T
                Sl[t * k * k:(t + 1) * k * k] = (T[f + i] @ Sb @ T[f + int(ci[t])].T).ravel(order="F")
        S.append(Sl)
    out.update(U=U, V=U, E=E, F=E, S=S)
    return out, T


def _leaf_offsets(arr):
    """Element offset of every leaf's m_j x k_q block in U (and V)."""
    q, kq = int(arr["q"]), int(arr["level_rank"][int(arr["q"])])
    b, e = arr["begin"], arr["end"]
    lf = (1 << q) - 1
    off, out = 0, {}
    for j in range(1 << q):
        m = int(e[lf + j] - b[lf + j])
        out[lf + j] = (off, m)
        off += m * kq
    return out


def _transfer_offsets(kr, q):
    """Element offset of every node's k_l x k_(l-1) transfer in E (and F), levels 1 .. q."""
    eo, off = {}, 0
    for l in range(1, q + 1):
        for c in range((1 << l) - 1, (2 << l) - 1):
            eo[c] = off
            off += kr[l] * kr[l - 1]
    return eo, off


def coupling_is_symmetric(arr):
    """Whether every coupling block has a mirror block with S_ji = S_ij^T
    exactly (then A = A^T when V = U, F = E and D is symmetric)."""
    q = int(arr["q"])
    for l in range(q + 1):
        k = int(arr["level_rank"][l])
        rp, ci, Sl = arr["S_rowptr"][l], arr["S_colidx"][l], arr["S"][l]
        where = {}
        for i in range(1 << l):
            for t in range(int(rp[i]), int(rp[i + 1])):
                where[(i, int(ci[t]))] = t
        for (i, j), t in where.items():
            u = where.get((j, i))
            if u is None:
                return False
            if not np.array_equal(Sl[t * k * k:(t + 1) * k * k].reshape(k, k),
                                  Sl[u * k * k:(u + 1) * k * k].reshape(k, k).T):
                return False
    return True


def basis_generation(arr, columns=None):
    """The tree R of Sec. 5.2 (Alg. 8 and 9) for an H^2 matrix with one
    orthonormal nested basis tree for rows and columns (V = U, F = E), given by
    its arrays.  For node i of level l, with parent i+ and coupling blocks
    S_ij1 .. S_ijb in its block row,
        Sbar_i = [R_i+ E_i^T; S_ij1^T; ...; S_ijb^T]
    and R_i is the triangular factor of the QR factorization of Sbar_i (Q is
    not formed).  When the coupling blocks are not symmetric (S_ji != S_ij^T
    for some block), the basis also carries block column i, so the blocks
    S_j1i .. S_jci of that column are stacked below as well (the rows of the
    column's blocks restricted to node i's columns).  The parent term is absent
    on the coarsest level with blocks, l_min (every level above it has no
    blocks, so its R is 0).  R_i is returned as a k_l x k_l matrix (rows past
    the number of rows of Sbar_i are zero).  Returns {node: R_i} for the nodes
    of levels l_min .. q.  columns: stack the block columns (None: when the
    coupling blocks of arr are not exactly symmetric)."""
    if columns is None:
        columns = not coupling_is_symmetric(arr)
    return _basis_generation_tree(arr, "E", True, columns)


def _basis_generation_tree(arr, tkey, rows, cols):
    """R tree of one basis tree (tkey "E": the row tree, "F": the column
    tree): Sbar_i stacks R_i+ X_i^T (X = E or F), then the blocks of block row
    i transposed (rows) and the blocks of block column i as they are (cols)."""
    q = int(arr["q"])
    kr = [int(k) for k in arr["level_rank"]]
    lmin = next((l for l in range(q + 1) if int(arr["S_rowptr"][l][1 << l]) > 0), q + 1)
    eo, _ = _transfer_offsets(kr, q)
    R = {}
    for l in range(lmin, q + 1):
        k, f = kr[l], (1 << l) - 1
        rp, ci, S = arr["S_rowptr"][l], arr["S_colidx"][l], arr["S"][l]
        in_column = [[] for _ in range(1 << l)]   # blocks of each block column, by row
        for i in range(1 << l):
            for t in range(int(rp[i]), int(rp[i + 1])):
                in_column[int(ci[t])].append(t)
        for i in range(1 << l):
            node = f + i
            parts = []
            if l > lmin:
                kp = kr[l - 1]
                Xi = arr[tkey][eo[node]:eo[node] + k * kp].reshape(kp, k).T     # k_l x k_(l-1)
                parts.append(R[(node - 1) // 2] @ Xi.T)
            if rows:
                for t in range(int(rp[i]), int(rp[i + 1])):
                    parts.append(S[t * k * k:(t + 1) * k * k].reshape(k, k))      # S_ij^T (column-major S_ij read row-major)
            if cols:
                for t in in_column[i]:
                    parts.append(S[t * k * k:(t + 1) * k * k].reshape(k, k).T)   # S_ji
            Ri = np.zeros((k, k))
            if parts:
                r = np.linalg.qr(np.vstack(parts), mode="r")
                Ri[:r.shape[0], :] = r
            R[node] = Ri
    return R


def compress_arrays(arr, eps):
    """Algebraic compression of an H^2 matrix given by its arrays (Sec. 5);
    matrices with different row and column trees go to compress_two_trees,
    the rest (one basis tree, V = U, F = E) follow here: orthogonalization
    (Sec. 5.1), basis generation (Sec. 5.2, block columns included when the
    coupling blocks are not symmetric), basis
    truncation (Sec. 5.3, Alg. 10) with relative threshold eps, and projection
    of the coupling blocks into the truncated bases.

    Leaves: W_i = U_i R_i^T, SVD W_i = Q S Y^T; node i keeps the singular
    vectors whose singular value is at least eps times its largest, and the
    level keeps the largest such count over its nodes (at least 1): k~_q.  The
    new leaf basis is the first k~_q columns of Q, T_i = Q^T U_i.  Levels q ..
    l_min + 1, parent p with children c1, c2: Z_p = [T_c1 E_c1; T_c2 E_c2]
    (2 k~_l x k_(l-1)), W_p = Z_p R_p^T, the same truncated SVD gives k~_(l-1)
    and Q; its two k~_l x k~_(l-1) blocks are the new transfers of c1 and c2,
    T_p = Q^T Z_p.  Every coupling block S_ij <- T_i S_ij T_j^T (k~_l x k~_l);
    dense blocks are unchanged.  Levels above l_min take rank k~_(l_min) with
    zero transfers (the product does not use them).

    Returns (new arrays, info) with info = {"rank": k~ per level, "sigma":
    {node: singular values of W}, "count": {node: kept count}, "R": R tree,
    "T": {node: T}}."""
    if not shares_one_tree(arr):
        return compress_two_trees(arr, eps)
    # symmetry is decided on the input: the projection keeps S_ji = S_ij^T in
    # exact arithmetic but not bit for bit
    columns = not coupling_is_symmetric(arr)
    orth, _ = orthogonalize_arrays(arr)
    q = int(arr["q"])
    kr = [int(k) for k in orth["level_rank"]]
    lmin = next((l for l in range(q + 1) if int(orth["S_rowptr"][l][1 << l]) > 0), q + 1)
    if lmin > q:
        return orth, {"rank": kr, "sigma": {}, "count": {}, "R": {}, "T": {}}
    R = basis_generation(orth, columns)
    eo, _ = _transfer_offsets(kr, q)
    lo = _leaf_offsets(orth)
    lf = (1 << q) - 1

    def kept(s):
        return int(np.count_nonzero(s >= eps * s[0])) if s.size and s[0] > 0.0 else 0

    sigma, count, T, kt = {}, {}, {}, list(kr)
    Ul, left = {}, {}
    for v in range(lf, 2 * lf + 1):   # leaves
        off, m = lo[v]
        Ul[v] = orth["U"][off:off + m * kr[q]].reshape(kr[q], m).T
        Qv, s, _ = np.linalg.svd(Ul[v] @ R[v].T, full_matrices=False)
        left[v], sigma[v], count[v] = Qv, s, kept(s)
    kt[q] = max(1, max(count[v] for v in range(lf, 2 * lf + 1)))
    newU = []
    for v in range(lf, 2 * lf + 1):
        Qv = left[v][:, :kt[q]]
        T[v] = Qv.T @ Ul[v]
        newU.append(Qv.ravel(order="F"))
    newE = {}
    for l in range(q, lmin, -1):
        kc, kp = kr[l], kr[l - 1]
        Z, left = {}, {}
        for p in range((1 << (l - 1)) - 1, (1 << l) - 1):
            halves = []
            for c in (2 * p + 1, 2 * p + 2):
                Ec = orth["E"][eo[c]:eo[c] + kc * kp].reshape(kp, kc).T
                halves.append(T[c] @ Ec)
            Z[p] = np.vstack(halves)
            Qp, s, _ = np.linalg.svd(Z[p] @ R[p].T, full_matrices=False)
            left[p], sigma[p], count[p] = Qp, s, kept(s)
        kt[l - 1] = max(1, max(count[p] for p in Z))
        for p in Z:
            Qp = left[p][:, :kt[l - 1]]
            newE[2 * p + 1] = Qp[:kt[l]]
            newE[2 * p + 2] = Qp[kt[l]:]
            T[p] = Qp.T @ Z[p]
    for l in range(lmin):
        kt[l] = kt[lmin]
    E = []
    for l in range(1, q + 1):
        for c in range((1 << l) - 1, (2 << l) - 1):
            E.append(newE[c].ravel(order="F") if c in newE else np.zeros(kt[l] * kt[l - 1]))
    S = []
    for l in range(q + 1):
        k, kn, f = kr[l], kt[l], (1 << l) - 1
        rp, ci, Sl = orth["S_rowptr"][l], orth["S_colidx"][l], orth["S"][l]
        blocks = []
        for i in range(1 << l):
            for t in range(int(rp[i]), int(rp[i + 1])):
                Sb = Sl[t * k * k:(t + 1) * k * k].reshape(k, k).T
                blocks.append((T[f + i] @ Sb @ T[f + int(ci[t])].T).ravel(order="F"))
        S.append(np.concatenate(blocks) if blocks else np.zeros(0))
    out = dict(orth)
    Uc = np.concatenate(newU)
    Ec = np.concatenate(E) if E else np.zeros(0)
    out.update(level_rank=np.array(kt, dtype=np.int32), U=Uc, V=Uc, E=Ec, F=Ec, S=S)
    return out, {"rank": kt, "sigma": sigma, "count": count, "R": R, "T": T}


def transpose_arrays(arr):
    """The arrays of A^T for an H^2 matrix A = sum_l U S^l V^T + D given by
    its arrays (Sec. 2.2): the row and column trees exchange roles (U <-> V,
    E <-> F), every coupling block S_ij of level l becomes block (j, i) of
    A^T with value S_ij^T, and every dense block D_ij becomes block (j, i)
    with value D_ij^T.  Block rows of A^T list their columns in increasing
    order."""
    q = int(arr["q"])
    kr = [int(k) for k in arr["level_rank"]]
    b, e = arr["begin"], arr["end"]
    lf = (1 << q) - 1

    def transpose_bsr(nrows, rp, ci, blocks):
        # blocks[t]: the t-th block as a dense matrix; returns rowptr, colidx, blocks of the transpose
        rows = [[] for _ in range(nrows)]
        for i in range(nrows):
            for t in range(int(rp[i]), int(rp[i + 1])):
                rows[int(ci[t])].append((i, blocks[t].T))
        nrp = np.zeros(nrows + 1, dtype=np.int32)
        nci, nbl = [], []
        for jrow in range(nrows):
            for i, blk in sorted(rows[jrow], key=lambda z: z[0]):
                nci.append(i)
                nbl.append(blk)
            nrp[jrow + 1] = len(nci)
        return nrp, np.array(nci, dtype=np.int32), nbl

    S_rowptr, S_colidx, S = [], [], []
    for l in range(q + 1):
        k = kr[l]
        rp, ci, Sl = arr["S_rowptr"][l], arr["S_colidx"][l], arr["S"][l]
        blocks = [Sl[t * k * k:(t + 1) * k * k].reshape(k, k).T for t in range(len(ci))]
        nrp, nci, nbl = transpose_bsr(1 << l, rp, ci, blocks)
        S_rowptr.append(nrp)
        S_colidx.append(nci)
        S.append(np.concatenate([m.ravel(order="F") for m in nbl]) if nbl else np.zeros(0))
    drp, dci = arr["D_rowptr"], arr["D_colidx"]
    dblocks, off = [], 0
    for i in range(1 << q):
        for t in range(int(drp[i]), int(drp[i + 1])):
            ms, mt = int(e[lf + i] - b[lf + i]), int(e[lf + int(dci[t])] - b[lf + int(dci[t])])
            dblocks.append(arr["D"][off:off + ms * mt].reshape(mt, ms).T)
            off += ms * mt
    nrp, nci, nbl = transpose_bsr(1 << q, drp, dci, dblocks)
    out = dict(arr)
    out.update(U=arr["V"], V=arr["U"], E=arr["F"], F=arr["E"], S_rowptr=S_rowptr, S_colidx=S_colidx, S=S,
               D_rowptr=nrp, D_colidx=nci,
               D=np.concatenate([m.ravel(order="F") for m in nbl]) if nbl else np.zeros(0))
    return out


def shares_one_tree(arr):
    """V = U and F = E value by value: one basis tree for rows and columns."""
    return np.array_equal(arr["U"], arr["V"]) and np.array_equal(arr["E"], arr["F"])


def _orthogonalize_tree(arr, bkey, tkey):
    """Sec. 5.1 up one basis tree (bkey "U" / tkey "E", or "V" / "F"):
    returns the new leaf bases and transfers (flattened) and {node: T}."""
    q = int(arr["q"])
    kr = [int(k) for k in arr["level_rank"]]
    b, e = arr["begin"], arr["end"]
    lf = (1 << q) - 1
    lmin = next((l for l in range(q + 1) if int(arr["S_rowptr"][l][1 << l]) > 0), q + 1)
    B = np.array(arr[bkey], dtype=np.float64, copy=True)
    X = np.array(arr[tkey], dtype=np.float64, copy=True)
    T = {}
    off = 0
    for j in range(1 << q):
        m = int(e[lf + j] - b[lf + j])
        if m < kr[q]:
            raise ValueError("a leaf holds fewer rows than the rank")
        Q, T[lf + j] = _qr_positive(B[off:off + m * kr[q]].reshape(kr[q], m).T)
        B[off:off + m * kr[q]] = Q.ravel(order="F")
        off += m * kr[q]
    eo, _ = _transfer_offsets(kr, q)
    for l in range(q, lmin, -1):
        kc, kp = kr[l], kr[l - 1]
        if 2 * kc < kp:
            raise ValueError("a level's rank exceeds twice its children's")
        for p in range((1 << (l - 1)) - 1, (1 << l) - 1):
            c1, c2 = 2 * p + 1, 2 * p + 2
            X1 = X[eo[c1]:eo[c1] + kc * kp].reshape(kp, kc).T
            X2 = X[eo[c2]:eo[c2] + kc * kp].reshape(kp, kc).T
            Q, T[p] = _qr_positive(np.vstack([T[c1] @ X1, T[c2] @ X2]))
            X[eo[c1]:eo[c1] + kc * kp] = Q[:kc].ravel(order="F")
            X[eo[c2]:eo[c2] + kc * kp] = Q[kc:].ravel(order="F")
    return B, X, T


def orthogonalize_two_trees(arr):
    """Basis orthogonalization (Sec. 5.1) of an H^2 matrix whose row and
    column trees differ (V != U or F != E): each tree as in
    orthogonalize_arrays (U = Q T up the row tree, V = Q' T' up the column
    tree), then every coupling block S_ij <- T_i S_ij T'_j^T.  Returns (new
    arrays, T of the row tree, T' of the column tree)."""
    q = int(arr["q"])
    kr = [int(k) for k in arr["level_rank"]]
    lmin = next((l for l in range(q + 1) if int(arr["S_rowptr"][l][1 << l]) > 0), q + 1)
    out = dict(arr)
    if lmin > q:
        return out, {}, {}
    U, E, Tr = _orthogonalize_tree(arr, "U", "E")
    V, F, Tc = _orthogonalize_tree(arr, "V", "F")
    S = []
    for l in range(q + 1):
        Sl = np.array(arr["S"][l], dtype=np.float64, copy=True)
        k, f = kr[l], (1 << l) - 1
        rp, ci = arr["S_rowptr"][l], arr["S_colidx"][l]
        for i in range(1 << l):
            for t in range(int(rp[i]), int(rp[i + 1])):
                Sb = Sl[t * k * k:(t + 1) * k * k].reshape(k, k).T
                Sl[t * k * k:(t + 1) * k * k] = (Tr[f + i] @ Sb @ Tc[f + int(ci[t])].T).ravel(order="F")
        S.append(Sl)
    out.update(U=U, V=V, E=E, F=F, S=S)
    return out, Tr, Tc


def compress_two_trees(arr, eps):
    """Algebraic compression (Sec. 5) with different row and column trees:
    orthogonalize both (orthogonalize_two_trees); the row tree's R from the
    block rows (S_ij^T) under R_i+ E_i^T, the column tree's R' from the block
    columns (S_ji) under R'_i+ F_i^T (Sec. 5.2 for each tree); truncation
    (Sec. 5.3) of each tree with its own R, the rank of a level being the
    largest kept count over the nodes of both trees (the blocks stay square,
    one rank per level); S_ij <- T_i S_ij T'_j^T.  Returns (new arrays, info)
    with info["sigma"], info["count"] for the row tree and info["sigma_col"],
    info["count_col"] for the column tree."""
    orth, _, _ = orthogonalize_two_trees(arr)
    q = int(arr["q"])
    kr = [int(k) for k in orth["level_rank"]]
    lmin = next((l for l in range(q + 1) if int(orth["S_rowptr"][l][1 << l]) > 0), q + 1)
    if lmin > q:
        return orth, {"rank": kr, "sigma": {}, "count": {}, "sigma_col": {}, "count_col": {}}
    Rr = _basis_generation_tree(orth, "E", True, False)
    Rc = _basis_generation_tree(orth, "F", False, True)
    eo, _ = _transfer_offsets(kr, q)
    lo = _leaf_offsets(orth)
    lf = (1 << q) - 1

    def kept(sv):
        return int(np.count_nonzero(sv >= eps * sv[0])) if sv.size and sv[0] > 0.0 else 0

    trees = {"row": ("U", "E", Rr), "col": ("V", "F", Rc)}
    sigma = {"row": {}, "col": {}}
    count = {"row": {}, "col": {}}
    T = {"row": {}, "col": {}}
    left = {"row": {}, "col": {}}
    leafb = {"row": {}, "col": {}}
    kt = list(kr)
    for name, (bkey, _, R) in trees.items():
        for v in range(lf, 2 * lf + 1):
            off, m = lo[v]
            leafb[name][v] = orth[bkey][off:off + m * kr[q]].reshape(kr[q], m).T
            Qv, sv, _ = np.linalg.svd(leafb[name][v] @ R[v].T, full_matrices=False)
            left[name][v], sigma[name][v], count[name][v] = Qv, sv, kept(sv)
    kt[q] = max(1, max(max(count[t][v] for v in range(lf, 2 * lf + 1)) for t in trees))
    newb = {"row": [], "col": []}
    for name in trees:
        for v in range(lf, 2 * lf + 1):
            Qv = left[name][v][:, :kt[q]]
            T[name][v] = Qv.T @ leafb[name][v]
            newb[name].append(Qv.ravel(order="F"))
    newx = {"row": {}, "col": {}}
    for l in range(q, lmin, -1):
        kc, kp = kr[l], kr[l - 1]
        Z = {"row": {}, "col": {}}
        for name, (_, tkey, R) in trees.items():
            for p in range((1 << (l - 1)) - 1, (1 << l) - 1):
                halves = []
                for c in (2 * p + 1, 2 * p + 2):
                    Xc = orth[tkey][eo[c]:eo[c] + kc * kp].reshape(kp, kc).T
                    halves.append(T[name][c] @ Xc)
                Z[name][p] = np.vstack(halves)
                Qp, sv, _ = np.linalg.svd(Z[name][p] @ R[p].T, full_matrices=False)
                left[name][p], sigma[name][p], count[name][p] = Qp, sv, kept(sv)
        kt[l - 1] = max(1, max(max(count[t][p] for p in Z[t]) for t in trees))
        for name in trees:
            for p in Z[name]:
                Qp = left[name][p][:, :kt[l - 1]]
                newx[name][2 * p + 1] = Qp[:kt[l]]
                newx[name][2 * p + 2] = Qp[kt[l]:]
                T[name][p] = Qp.T @ Z[name][p]
    for l in range(lmin):
        kt[l] = kt[lmin]
    flat = {}
    for name in trees:
        X = []
        for l in range(1, q + 1):
            for c in range((1 << l) - 1, (2 << l) - 1):
                X.append(newx[name][c].ravel(order="F") if c in newx[name] else np.zeros(kt[l] * kt[l - 1]))
        flat[name] = np.concatenate(X) if X else np.zeros(0)
    S = []
    for l in range(q + 1):
        k, f = kr[l], (1 << l) - 1
        rp, ci, Sl = orth["S_rowptr"][l], orth["S_colidx"][l], orth["S"][l]
        blocks = []
        for i in range(1 << l):
            for t in range(int(rp[i]), int(rp[i + 1])):
                Sb = Sl[t * k * k:(t + 1) * k * k].reshape(k, k).T
                blocks.append((T["row"][f + i] @ Sb @ T["col"][f + int(ci[t])].T).ravel(order="F"))
        S.append(np.concatenate(blocks) if blocks else np.zeros(0))
    out = dict(orth)
    out.update(level_rank=np.array(kt, dtype=np.int32), U=np.concatenate(newb["row"]), V=np.concatenate(newb["col"]),
               E=flat["row"], F=flat["col"], S=S)
    return out, {"rank": kt, "sigma": sigma["row"], "count": count["row"], "sigma_col": sigma["col"],
                 "count_col": count["col"], "R": Rr, "R_col": Rc, "T": T["row"], "T_col": T["col"]}
