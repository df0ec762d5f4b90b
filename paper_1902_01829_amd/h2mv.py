"""Thin ctypes binding of libh2mv (include/h2mv.h).

Argument marshalling only: every step of the product runs in the library's
HIP kernels.  Device buffers and streams come from PyTorch; the functions
take raw device pointers and hipStream_t handles (ints), like the C ABI.
Loading fails loudly if the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

# H2MV_LIBRARY names another build of the library (the sanitizer test's)
LIB_PATH = os.environ.get("H2MV_LIBRARY") or os.path.join(os.path.dirname(os.path.abspath(__file__)), "libh2mv.so")

H2_OK, H2_ERR_INVALID_ARG, H2_ERR_OOM, H2_ERR_DEVICE, H2_ERR_UNSUPPORTED, H2_ERR_INTERNAL = range(6)
H2_FP64, H2_FP32, H2_BF16_SCALED = 0, 1, 2
H2_FLAG_STRUCTURE_ONLY = 1
H2_HALF_STORAGE = 16   # OR-ed into a storage value: blocks stored by halves (symmetric matrices)
STORAGE_NAMES = {H2_FP64: "fp64", H2_FP32: "fp32", H2_BF16_SCALED: "bf16"}
H2_SCHEDULE_MERGED, H2_SCHEDULE_STREAMED = 0, 1

# Every function declared in include/h2mv.h.
EXPORTS = ("h2_build_from_points", "h2_build_from_arrays", "h2_export_arrays", "h2_orthogonalize", "h2_compress", "h2_transpose", "h2_matvec", "h2_matvec_noalloc", "h2_matmat", "h2_free", "h2_get_info", "h2_get_perm",
           "h2_get_level_bsr", "h2_profile", "h2_profile_read", "h2_batch_create", "h2_batch_matmat",
           "h2_batch_tuning", "h2_batch_set_tuning", "h2_matmat_tuning", "h2_matmat_set_tuning", "h2_batch_free", "h2_read_probe", "h2_set_schedule",
           "h2_last_error")


class h2_params(C.Structure):
    _fields_ = [("dim", C.c_int), ("leaf_size", C.c_int), ("cheb_p", C.c_int), ("eta", C.c_double),
                ("corr_len", C.c_double), ("storage", C.c_int), ("flags", C.c_uint)]


class h2_arrays(C.Structure):
    _fields_ = [("n", C.c_int64), ("q", C.c_int), ("level_rank", C.c_void_p), ("node_begin", C.c_void_p),
                ("node_end", C.c_void_p), ("U", C.c_void_p), ("V", C.c_void_p), ("E", C.c_void_p),
                ("F", C.c_void_p), ("S_rowptr", C.c_void_p), ("S_colidx", C.c_void_p), ("S", C.c_void_p),
                ("D_rowptr", C.c_void_p), ("D_colidx", C.c_void_p), ("D", C.c_void_p)]


class h2_arrays_out(C.Structure):
    _fields_ = [("level_rank", C.c_void_p), ("node_begin", C.c_void_p), ("node_end", C.c_void_p),
                ("U", C.c_void_p), ("V", C.c_void_p), ("E", C.c_void_p), ("F", C.c_void_p),
                ("S_rowptr", C.c_void_p), ("S_colidx", C.c_void_p), ("S", C.c_void_p),
                ("D_rowptr", C.c_void_p), ("D_colidx", C.c_void_p), ("D", C.c_void_p)]


class h2_info(C.Structure):
    _fields_ = [("n", C.c_int64), ("dim", C.c_int), ("leaf_size", C.c_int), ("cheb_p", C.c_int),
                ("rank", C.c_int), ("levels_q", C.c_int), ("lmin", C.c_int), ("storage", C.c_int),
                ("nnodes", C.c_int64), ("coupling_blocks", C.c_int64), ("dense_blocks", C.c_int64),
                ("bytes_coupling", C.c_int64), ("bytes_dense", C.c_int64), ("bytes_leaf_bases", C.c_int64),
                ("bytes_transfers", C.c_int64), ("bytes_device_total", C.c_int64), ("near_ties", C.c_int64),
                ("partial_slots", C.c_int64)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class H2Error(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"h2mv error {code}: {msg}")
        self.code = code


_lib = None


def lib():
    """The loaded library; raises if libh2mv.so has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1902_01829_amd.build` (there is no fallback path)")
        L = C.CDLL(LIB_PATH)
        vp, i64, i32 = C.c_void_p, C.c_int64, C.c_int32
        L.h2_build_from_points.argtypes = [vp, i64, C.POINTER(h2_params), vp, C.POINTER(vp)]
        L.h2_build_from_arrays.argtypes = [C.POINTER(h2_arrays), C.c_int, vp, C.POINTER(vp)]
        L.h2_export_arrays.argtypes = [vp, C.POINTER(h2_arrays_out), vp]
        L.h2_orthogonalize.argtypes = [vp, vp]
        L.h2_compress.argtypes = [vp, C.c_double, vp, vp]
        L.h2_transpose.argtypes = [vp, vp, C.POINTER(vp)]
        L.h2_matvec.argtypes = [vp, vp, vp, vp]
        L.h2_matvec_noalloc.argtypes = [vp, vp, vp, vp]
        L.h2_matmat.argtypes = [vp, vp, i64, vp, i64, C.c_int, vp]
        L.h2_free.argtypes = [vp]
        L.h2_free.restype = None
        L.h2_get_info.argtypes = [vp, C.POINTER(h2_info)]
        L.h2_get_perm.argtypes = [vp, vp]
        L.h2_get_level_bsr.argtypes = [vp, C.c_int, C.POINTER(i64), vp, vp]
        L.h2_profile.argtypes = [vp, C.c_int]
        L.h2_profile_read.argtypes = [vp, vp, C.POINTER(i64)]
        L.h2_batch_create.argtypes = [vp, C.c_int, C.c_int, vp, C.POINTER(vp)]
        L.h2_batch_matmat.argtypes = [vp, vp, vp, vp, vp, vp]
        L.h2_batch_tuning.argtypes = [vp, C.POINTER(C.c_int), C.POINTER(i64), C.POINTER(C.c_int),
                                      C.POINTER(C.c_double)]
        L.h2_batch_set_tuning.argtypes = [vp, C.c_int, i64, C.c_int]
        L.h2_matmat_tuning.argtypes = [vp, C.c_int, C.POINTER(C.c_int), C.POINTER(i64), C.POINTER(C.c_int),
                                       C.POINTER(C.c_double)]
        L.h2_matmat_set_tuning.argtypes = [vp, C.c_int, C.c_int, i64, C.c_int]
        L.h2_read_probe.argtypes = [vp, i64, C.c_int, vp, vp]
        L.h2_batch_free.argtypes = [vp]
        L.h2_batch_free.restype = None
        L.h2_last_error.argtypes = []
        L.h2_last_error.restype = C.c_char_p
        for name in EXPORTS:
            if name not in ("h2_free", "h2_batch_free", "h2_last_error"):
                getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def _check(code):
    if code != H2_OK:
        raise H2Error(code, lib().h2_last_error().decode())


def h2_last_error() -> str:
    return lib().h2_last_error().decode()


def h2_build_from_points(points, dim, leaf_size, cheb_p, eta, corr_len, storage=H2_FP64, flags=0,
                         stream=0):
    """points: host array n x dim (float64).  Returns the handle (an int)."""
    pts = np.ascontiguousarray(points, dtype=np.float64)
    n = pts.shape[0] if pts.ndim == 2 else 0
    prm = h2_params(dim, leaf_size, cheb_p, eta, corr_len, storage, flags)
    h = C.c_void_p()
    _check(lib().h2_build_from_points(pts.ctypes.data if pts.size else None, n, C.byref(prm),
                                      C.c_void_p(stream), C.byref(h)))
    return h.value


def h2_build_from_arrays(arr, storage=H2_FP64, stream=0):
    """arr: dict with n, q, level_rank, begin, end, U, V, E, F, S_rowptr,
    S_colidx, S (lists over levels), D_rowptr, D_colidx, D (host arrays,
    column-major blocks; see include/h2mv.h).  Returns the handle (an int)."""
    keep = []

    def arr_of(a, dtype):
        if a is None:
            return None
        a = np.ascontiguousarray(a, dtype=dtype)
        keep.append(a)
        return a.ctypes.data if a.size else None
    q = int(arr["q"])
    nl = max(1, len(arr["S_rowptr"]))
    rp = (C.c_void_p * nl)(*[arr_of(r, np.int32) for r in arr["S_rowptr"]])
    ci = (C.c_void_p * nl)(*[arr_of(c, np.int32) for c in arr["S_colidx"]])
    sv = (C.c_void_p * nl)(*[arr_of(v, np.float64) for v in arr["S"]])
    a = h2_arrays(int(arr["n"]), q, arr_of(arr["level_rank"], np.int32), arr_of(arr["begin"], np.int64),
                  arr_of(arr["end"], np.int64), arr_of(arr.get("U"), np.float64), arr_of(arr.get("V"), np.float64),
                  arr_of(arr.get("E"), np.float64), arr_of(arr.get("F"), np.float64),
                  C.cast(rp, C.c_void_p), C.cast(ci, C.c_void_p), C.cast(sv, C.c_void_p),
                  arr_of(arr["D_rowptr"], np.int32), arr_of(arr["D_colidx"], np.int32),
                  arr_of(arr["D"], np.float64))
    h = C.c_void_p()
    _check(lib().h2_build_from_arrays(C.byref(a), storage, C.c_void_p(stream), C.byref(h)))
    return h.value


def h2_export_arrays(h, stream=0):
    """The representation read back as a dict in the layout h2_build_from_arrays
    takes (numpy arrays)."""
    info = h2_get_info(h)
    q = info.levels_q
    nn = (2 << q) - 1
    lr = np.zeros(q + 1, dtype=np.int32)
    b = np.zeros(nn, dtype=np.int64)
    e = np.zeros(nn, dtype=np.int64)
    _check(lib().h2_export_arrays(C.c_void_p(h), C.byref(h2_arrays_out(lr.ctypes.data, b.ctypes.data,
                                                                         e.ctypes.data)), C.c_void_p(stream)))
    lf = (1 << q) - 1
    m = e[lf:] - b[lf:]
    nU = int(m.sum()) * int(lr[q])
    nE = sum(int(lr[l]) * int(lr[l - 1]) << l for l in range(1, q + 1))
    U, V, E, F = (np.zeros(max(nU, 1)), np.zeros(max(nU, 1)), np.zeros(max(nE, 1)), np.zeros(max(nE, 1)))
    S_rowptr, S_colidx, S = [], [], []
    for l in range(q + 1):
        rp, ci = h2_get_level_bsr(h, l, 1 << l)
        S_rowptr.append(rp)
        S_colidx.append(np.ascontiguousarray(ci))
        S.append(np.zeros(max(len(ci), 1) * int(lr[l]) ** 2))
    drp, dci = h2_get_level_bsr(h, -1, 1 << q)
    dci = np.ascontiguousarray(dci)
    nD = sum(int(m[i]) * int(m[dci[t]]) for i in range(1 << q) for t in range(drp[i], drp[i + 1]))
    D = np.zeros(max(nD, 1))
    P = C.c_void_p * (q + 1)
    rpp = P(*[a.ctypes.data for a in S_rowptr])
    cip = P(*[a.ctypes.data if a.size else None for a in S_colidx])
    sp = P(*[a.ctypes.data for a in S])
    out = h2_arrays_out(None, None, None, U.ctypes.data, V.ctypes.data, E.ctypes.data, F.ctypes.data,
                        C.cast(rpp, C.c_void_p), C.cast(cip, C.c_void_p), C.cast(sp, C.c_void_p),
                        None, None, D.ctypes.data)
    _check(lib().h2_export_arrays(C.c_void_p(h), C.byref(out), C.c_void_p(stream)))
    return {"n": info.n, "q": q, "level_rank": lr, "begin": b, "end": e, "U": U[:nU], "V": V[:nU],
            "E": E[:nE], "F": F[:nE], "S_rowptr": S_rowptr, "S_colidx": S_colidx,
            "S": [S[l][:len(S_colidx[l]) * int(lr[l]) ** 2] for l in range(q + 1)],
            "D_rowptr": drp, "D_colidx": dci, "D": D[:nD]}


def h2_orthogonalize(h, stream=0):
    _check(lib().h2_orthogonalize(C.c_void_p(h), C.c_void_p(stream)))


def h2_transpose(h, stream=0):
    """A new handle for the transposed matrix."""
    out = C.c_void_p()
    _check(lib().h2_transpose(C.c_void_p(h), C.c_void_p(stream), C.byref(out)))
    return out.value


def h2_compress(h, eps, stream=0):
    """Compresses in place; returns the new rank of every level (numpy int32)."""
    q = h2_get_info(h).levels_q
    ranks = np.zeros(q + 1, dtype=np.int32)
    _check(lib().h2_compress(C.c_void_p(h), C.c_double(eps), C.c_void_p(ranks.ctypes.data), C.c_void_p(stream)))
    return ranks


def h2_matvec(h, x_ptr, y_ptr, stream=0):
    _check(lib().h2_matvec(C.c_void_p(h), C.c_void_p(x_ptr), C.c_void_p(y_ptr), C.c_void_p(stream)))


def h2_matvec_noalloc(h, x_ptr, y_ptr, stream=0):
    _check(lib().h2_matvec_noalloc(C.c_void_p(h), C.c_void_p(x_ptr), C.c_void_p(y_ptr), C.c_void_p(stream)))


def h2_set_schedule(h, schedule, near_wg_per_cu=0, near_early=1.0):
    _check(lib().h2_set_schedule(C.c_void_p(h), int(schedule), int(near_wg_per_cu), C.c_double(near_early)))


def h2_matmat(h, X_ptr, ldx, Y_ptr, ldy, nrhs, stream=0):
    _check(lib().h2_matmat(C.c_void_p(h), C.c_void_p(X_ptr), ldx, C.c_void_p(Y_ptr), ldy, nrhs,
                           C.c_void_p(stream)))


def h2_free(h):
    lib().h2_free(C.c_void_p(h))


def h2_get_info(h) -> h2_info:
    info = h2_info()
    _check(lib().h2_get_info(C.c_void_p(h), C.byref(info)))
    return info


def h2_get_perm(h, n) -> np.ndarray:
    perm = np.zeros(n, dtype=np.int64)
    _check(lib().h2_get_perm(C.c_void_p(h), perm.ctypes.data))
    return perm


def h2_get_level_bsr(h, level, nrows):
    """(rowptr, colidx) of one level of the matrix tree; level -1 = dense blocks."""
    cnt = C.c_int64()
    _check(lib().h2_get_level_bsr(C.c_void_p(h), level, C.byref(cnt), None, None))
    rp = np.zeros(nrows + 1, dtype=np.int32)
    ci = np.zeros(max(cnt.value, 1), dtype=np.int32)
    _check(lib().h2_get_level_bsr(C.c_void_p(h), level, C.byref(cnt), rp.ctypes.data, ci.ctypes.data))
    return rp, ci[:cnt.value]


def h2_profile(h, enable):
    _check(lib().h2_profile(C.c_void_p(h), 1 if enable else 0))


def h2_profile_read(h):
    """(ms per phase [up, stream, down, leaf, whole call], calls)."""
    ms = np.zeros(8)
    calls = C.c_int64()
    _check(lib().h2_profile_read(C.c_void_p(h), ms.ctypes.data, C.byref(calls)))
    return ms[:5], calls.value


def h2_batch_create(handles, nrhs, stream=0):
    arr = (C.c_void_p * len(handles))(*handles)
    b = C.c_void_p()
    _check(lib().h2_batch_create(arr, len(handles), nrhs, C.c_void_p(stream), C.byref(b)))
    return b.value


def h2_batch_matmat(batch, X_ptrs, ldx, Y_ptrs, ldy, stream=0):
    n = len(X_ptrs)
    xa = (C.c_void_p * n)(*X_ptrs)
    ya = (C.c_void_p * n)(*Y_ptrs)
    lx = (C.c_int64 * n)(*ldx)
    ly = (C.c_int64 * n)(*ldy)
    _check(lib().h2_batch_matmat(C.c_void_p(batch), xa, lx, ya, ly, C.c_void_p(stream)))


def h2_batch_tuning(batch):
    p, g, nt, ms = C.c_int(), C.c_int64(), C.c_int(), C.c_double()
    _check(lib().h2_batch_tuning(C.c_void_p(batch), C.byref(p), C.byref(g), C.byref(nt), C.byref(ms)))
    return {"pipelined": p.value, "grid": g.value, "tile_width": nt.value, "tuned_ms": ms.value}


def h2_batch_set_tuning(batch, pipelined, grid, tile_width):
    _check(lib().h2_batch_set_tuning(C.c_void_p(batch), pipelined, grid, tile_width))


def h2_matmat_set_tuning(h, narrow, pipelined, grid, tile_width):
    _check(lib().h2_matmat_set_tuning(C.c_void_p(h), narrow, pipelined, grid, tile_width))


def h2_matmat_tuning(h, narrow):
    p, g, nt, ms = C.c_int(), C.c_int64(), C.c_int(), C.c_double()
    _check(lib().h2_matmat_tuning(C.c_void_p(h), narrow, C.byref(p), C.byref(g), C.byref(nt), C.byref(ms)))
    return {"pipelined": p.value, "grid": g.value, "tile_width": nt.value, "tuned_ms": ms.value}


def h2_read_probe(buf_ptr, nbytes, grid, sink_ptr, stream=0):
    _check(lib().h2_read_probe(C.c_void_p(buf_ptr), nbytes, grid, C.c_void_p(sink_ptr), C.c_void_p(stream)))


def h2_batch_free(batch):
    lib().h2_batch_free(C.c_void_p(batch))


class H2Batch:
    """Many H2Matrix members (same storage, FP32 or BF16) multiplied together."""

    def __init__(self, members, nrhs):
        import torch
        self._torch = torch
        self.members = list(members)
        self.nrhs = nrhs
        self.handle = h2_batch_create([m.handle for m in self.members], nrhs,
                                      torch.cuda.current_stream().cuda_stream)

    def close(self):
        if getattr(self, "handle", None):
            h2_batch_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def matmat(self, Xs, outs=None):
        """Xs: list of float64 CUDA tensors (nrhs, n_b), each row one right-hand side."""
        torch = self._torch
        Ys = outs if outs is not None else [torch.empty_like(X) for X in Xs]
        for X, m in zip(Xs, self.members):
            assert X.dtype == torch.float64 and X.is_cuda and X.is_contiguous() and X.shape == (self.nrhs, m.n)
        h2_batch_matmat(self.handle, [X.data_ptr() for X in Xs], [m.n for m in self.members],
                        [Y.data_ptr() for Y in Ys], [m.n for m in self.members],
                        torch.cuda.current_stream().cuda_stream)
        return Ys

    def tuning(self):
        return h2_batch_tuning(self.handle)

    def set_tuning(self, pipelined, grid, tile_width):
        h2_batch_set_tuning(self.handle, pipelined, grid, tile_width)


class H2Matrix:
    """Owns one handle; products take and return torch tensors on the GPU."""

    def __init__(self, points, dim, leaf_size, cheb_p, eta, corr_len, storage=H2_FP64, flags=0,
                 stream=None):
        import torch
        self._torch = torch
        st = stream if stream is not None else (torch.cuda.current_stream().cuda_stream
                                                if torch.cuda.is_available() else 0)
        self.handle = h2_build_from_points(points, dim, leaf_size, cheb_p, eta, corr_len, storage, flags, st)
        self.info = h2_get_info(self.handle)
        self.n = self.info.n

    @classmethod
    def from_arrays(cls, arr, storage=H2_FP64, stream=None):
        """A matrix given by its arrays (h2_build_from_arrays); vectors are in
        the order of arr's node ranges."""
        import torch
        self = cls.__new__(cls)
        self._torch = torch
        st = stream if stream is not None else (torch.cuda.current_stream().cuda_stream
                                                if torch.cuda.is_available() else 0)
        self.handle = h2_build_from_arrays(arr, storage, st)
        self.info = h2_get_info(self.handle)
        self.n = self.info.n
        return self

    def close(self):
        if getattr(self, "handle", None):
            h2_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def perm(self):
        return h2_get_perm(self.handle, self.n)

    def level_bsr(self, level):
        nrows = (1 << self.info.levels_q) if level < 0 else (1 << level)
        return h2_get_level_bsr(self.handle, level, nrows)

    def _stream(self):
        return self._torch.cuda.current_stream().cuda_stream

    def orthogonalize(self):
        h2_orthogonalize(self.handle, self._stream())

    def transpose(self):
        """A new H2Matrix for the transposed matrix (same tree order)."""
        import torch
        t = type(self).__new__(type(self))
        t._torch = torch
        t.handle = h2_transpose(self.handle, self._stream())
        t.info = h2_get_info(t.handle)
        t.n = t.info.n
        return t

    def compress(self, eps):
        """Algebraic compression in place (h2_compress); returns the new rank of every level."""
        ranks = h2_compress(self.handle, eps, self._stream())
        self.info = h2_get_info(self.handle)
        return ranks

    def matvec(self, x, out=None):
        """x: float64 CUDA tensor (n,), tree order."""
        torch = self._torch
        assert x.dtype == torch.float64 and x.is_cuda and x.is_contiguous() and x.numel() == self.n
        y = out if out is not None else torch.empty_like(x)
        h2_matvec(self.handle, x.data_ptr(), y.data_ptr(), self._stream())
        return y

    def matmat_tuning(self, narrow=0):
        return h2_matmat_tuning(self.handle, narrow)

    def set_schedule(self, schedule, near_wg_per_cu=0, near_early=1.0):
        h2_set_schedule(self.handle, schedule, near_wg_per_cu, near_early)

    def set_matmat_tuning(self, narrow, pipelined, tile_width, grid=0):
        h2_matmat_set_tuning(self.handle, narrow, pipelined, grid, tile_width)

    def matmat(self, X, out=None):
        """X: float64 CUDA tensor (nrhs, n) (each row one right-hand side, i.e.
        column-major n x nrhs with leading dimension n)."""
        torch = self._torch
        assert X.dtype == torch.float64 and X.is_cuda and X.is_contiguous() and X.shape[1] == self.n
        Y = out if out is not None else torch.empty_like(X)
        h2_matmat(self.handle, X.data_ptr(), self.n, Y.data_ptr(), self.n, X.shape[0], self._stream())
        return Y
