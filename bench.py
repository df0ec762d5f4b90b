"""Benchmark of the H^2 matrix-vector product on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME] [--storage fp64|fp32|bf16]

A step is one whole product y = A x (leaf projection, upsweep, coupling and
dense streaming, downsweep, leaf expansion and sum) on a resident matrix and
vector.  The default workload is the 2-D covariance of 2^20 uniform points
(exponential kernel, correlation length 0.1, leaf size 64, 8x8 Chebyshev
bases: rank 64, eta 0.9), FP64.  value = algorithmic bytes per product / time
(GB/s): the bytes of D, S, U, V, E, F, x and y.

Prints one JSON line.  Besides the headline it reports the dominant kernel
(coupling + dense streaming) against the HBM roofline, the FP64 CPU oracle
timed on a bounded sample of the same workload, the reduced-storage modes of
the 3-D workload with their speedup over FP64 and their error against the FP64
oracle, the 32-right-hand-side product on the matrix cores, and a batch of 64
uneven matrices with 8 right-hand sides each.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_1902_01829_amd import workloads as W  # noqa: E402

HBM_PEAK_GBS = 8000.0
STORAGE = {"fp64": 0, "fp32": 1, "bf16": 2}
DTYPE = {"fp64": "f64", "fp32": "f32", "bf16": "bf16xf32scale"}
# HBM bytes per launch of the streaming kernel from rocprofv3 FETCH_SIZE and
# WRITE_SIZE (KiB per dispatch, scaled by the factors a 1 GiB device copy
# gives: x2.0 for FETCH_SIZE, x1.0 for WRITE_SIZE).  Keyed by workload and
# storage; valid for the kernel as measured (drop the entry when it changes).
MEASURED_TRAFFIC = {
    ("2d-n1048576-m64-k64", "fp64"): (21552975.0 * 2.0 + 24568.0) * 1024,
}


# The paper's own figure for this product, on other hardware (context, not a
# target): above 550 GB/s on an NVIDIA P100, up to 78 % of its peak bandwidth
# with the dense and low-rank phases overlapped (Sec. 1 and Sec. 4.6).
PAPER_CONTEXT = {"hmv_GB_per_s": "> 550", "fraction_of_peak": "up to 0.78 (streamed version)",
                 "hardware": "NVIDIA P100 (Pascal)", "source": "Sec. 1 and Sec. 4.6",
                 "note": "other hardware and precision; context only"}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def read_ceiling(gib=8.0, reps=10):
    """HBM read ceiling measured on this GPU: the library's plain streaming
    read (h2_read_probe: the product kernels' 16-byte non-temporal loads, one
    contiguous kilobyte per wavefront load) over a buffer far larger than the
    caches, timed with events for a few grid sizes; the best rate is kept."""
    import torch
    from paper_1902_01829_amd import h2mv
    nbytes = int(gib * (1 << 30)) // 16 * 16
    buf = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    sink = torch.zeros(65536, dtype=torch.int64, device="cuda")
    st = torch.cuda.current_stream().cuda_stream
    best, best_grid, rates = 0.0, 0, {}
    for grid in (4096, 8192, 16384, 32768, 65536):
        for _ in range(2):
            h2mv.h2_read_probe(buf.data_ptr(), nbytes, grid, sink.data_ptr(), st)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            h2mv.h2_read_probe(buf.data_ptr(), nbytes, grid, sink.data_ptr(), st)
        e1.record()
        torch.cuda.synchronize()
        gbs = nbytes * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
        rates[str(grid)] = round(gbs, 1)
        if gbs > best:
            best, best_grid = gbs, grid
    del buf, sink
    torch.cuda.empty_cache()
    log(f"read ceiling: {best:.1f} GB/s ({rates})")
    return {"GB_per_s": round(best, 1), "frac_of_8TB_peak": round(best / HBM_PEAK_GBS, 4), "bytes": nbytes,
            "grid": best_grid, "GB_per_s_by_grid": rates, "kernel": "read_probe_kernel (h2_read_probe)",
            "timing": f"HIP events around {reps} launches after 2 warm-ups"}


def algorithmic_bytes(info, n, nrhs=1):
    """D + S + U + V + E + F, plus x read and y written (FP64)."""
    rep = info.bytes_coupling + info.bytes_dense + info.bytes_leaf_bases + info.bytes_transfers
    return rep + 16 * n * nrhs


def stream_kernel_bytes(info, n, storage):
    """Algorithmic bytes of one launch of the streaming kernel: every coupling
    and dense block once, x read once (FP64) and the near field written."""
    vb = 8 if storage == 0 else 4
    return info.bytes_coupling + info.bytes_dense + 8 * n + vb * n


def run_matvec(w, storage, steps, warmup):
    """Builds the workload, times `steps` products after `warmup`, returns a dict."""
    import torch
    from paper_1902_01829_amd import h2mv
    stream = torch.cuda.current_stream()
    t0 = time.perf_counter()
    A = h2mv.H2Matrix(W.points(w), w.dim, w.leaf, w.cheb_p, w.eta, w.corr_len, storage=storage)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    info = A.info
    perm = A.perm()
    xt = W.rhs(w, 1)[perm]
    x = torch.from_numpy(xt).cuda()
    y = torch.empty_like(x)
    log(f"{w.name} storage={storage}: built in {build_s:.1f} s, {info.coupling_blocks} coupling + "
        f"{info.dense_blocks} dense blocks, {info.bytes_device_total / 1e9:.2f} GB on device")
    for _ in range(warmup):
        A.matvec(x, out=y)
    torch.cuda.synchronize()
    h2mv.h2_profile(A.handle, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        h2mv.h2_matvec(A.handle, x.data_ptr(), y.data_ptr(), stream.cuda_stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    phase_ms, calls = h2mv.h2_profile_read(A.handle)
    h2mv.h2_profile(A.handle, False)
    y_host = y.cpu().numpy()
    A.close()
    del x, y
    torch.cuda.empty_cache()
    ms = (t1 - t0) * 1e3 / steps
    return {"ms": ms, "phase_ms": phase_ms / max(calls, 1), "info": info, "perm": perm, "xt": xt,
            "y": y_host, "build_s": build_s}


def oracle_sample(w, perm, xt, nleaves, storage=0, seed=7):
    """FP64 oracle rows of a seeded sample of leaves (matrix-free)."""
    from oracle import oracle as O
    o = O.OracleH2(W.points(w), w.leaf, w.cheb_p, w.eta, w.corr_len, storage=storage, keep_blocks=False)
    assert np.array_equal(perm, o.perm())
    rng = np.random.Generator(np.random.PCG64(seed))
    leaves = np.sort(rng.choice(o.leaf_nodes(), size=min(nleaves, 1 << o.q), replace=False))
    return o.leaf_rows(leaves), o.matvec_leaves(xt, leaves)


def cpu_baseline(w, perm, xt, budget_s=20.0):
    """FP64 oracle (matrix-free, all host threads) on a sample of leaves: the
    full upsweep plus the rows of the sampled leaves (their dense blocks and
    the coupling rows of their ancestors).  Reported in GB/s of the blocks,
    bases and transfers that sample touches, counted at their stored size."""
    from oracle import oracle as O
    t0 = time.perf_counter()
    o = O.OracleH2(W.points(w), w.leaf, w.cheb_p, w.eta, w.corr_len, keep_blocks=False)
    build_s = time.perf_counter() - t0
    assert np.array_equal(perm, o.perm())
    k, q = o.k, o.q
    eb = 8
    rps = [o.coupling_bsr(l)[0] for l in range(q + 1)]
    drp, dci = o.dense_bsr()
    b, e = o.ranges()
    sizes = e - b
    lf = (1 << q) - 1
    rng = np.random.Generator(np.random.PCG64(11))
    leaves_all = rng.permutation(o.leaf_nodes())

    def touched_bytes(leaves):
        ntransfer = max(0, (1 << (q + 1)) - (1 << (o.lmin + 1)))     # nodes of levels lmin+1 .. q
        tot = (k * int(sizes[lf:].sum()) + k * k * ntransfer) * eb   # upsweep: V and F
        for v in leaves:
            j = v - lf
            cols = dci[drp[j]:drp[j + 1]]
            tot += int(sizes[v]) * int(sizes[lf + cols].sum()) * eb   # dense row
            tot += int(sizes[v]) * k * eb                              # U of the leaf
            a = v
            for l in range(q, o.lmin - 1, -1):
                i = a - ((1 << l) - 1)
                tot += int(rps[l][i + 1] - rps[l][i]) * k * k * eb     # coupling row of the ancestor
                if l > o.lmin:
                    tot += k * k * eb                                  # its E
                a = (a - 1) // 2
        return tot

    # sample size from two calibration runs: t(nl) = fixed (upsweep) + nl * per-leaf
    def timed(count):
        t0 = time.perf_counter()
        o.matvec_leaves(xt, np.sort(leaves_all[:count]))
        return time.perf_counter() - t0
    n_small, n_large = 4, min(64, len(leaves_all))
    t_small, t_large = timed(n_small), timed(n_large)
    per_leaf = max((t_large - t_small) / max(n_large - n_small, 1), 1e-6)
    fixed = max(t_small - n_small * per_leaf, 0.0)
    nl = int(max(4, min(len(leaves_all), (budget_s - fixed) / per_leaf)))
    leaves = np.sort(leaves_all[:nl])
    t0 = time.perf_counter()
    y_ref = o.matvec_leaves(xt, leaves)
    t = time.perf_counter() - t0
    nbytes = touched_bytes(leaves)
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    model = "unknown CPU"
    try:
        with open("/proc/cpuinfo") as f:
            model = next(line.split(":", 1)[1].strip() for line in f if line.startswith("model name"))
    except (OSError, StopIteration):
        pass
    return {
        "value": round(nbytes / t / 1e9, 3), "unit": "GB/s", "cores": cores, "kind": "oracle",
        "sample": f"FP64 oracle, matrix-free (blocks regenerated from the kernel), full upsweep + rows of "
                  f"{nl} of {1 << q} leaves ({len(o.leaf_rows(leaves))} rows): {t:.1f} s for "
                  f"{nbytes / 1e9:.2f} GB of blocks, bases and transfers touched (at FP64 stored size); "
                  f"oracle build {build_s:.1f} s; {cores} threads of {os.cpu_count()} on {model}",
    }, o.leaf_rows(leaves), y_ref


def small_case(reps=200):
    """The 4096-point 2-D workload (rank 16, leaf 32), cache-resident, so a
    latency figure: microseconds per product, eager and replayed from a HIP
    graph, and its error against the FP64 oracle (the same H^2) and against
    the exact kernel product (the approximation error)."""
    import torch
    from oracle import oracle as O
    from paper_1902_01829_amd import h2mv
    w = W.C1
    A = h2mv.H2Matrix(W.points(w), w.dim, w.leaf, w.cheb_p, w.eta, w.corr_len, storage=0)
    perm = A.perm()
    x_in = W.rhs(w, 1)
    x = torch.from_numpy(x_in[perm]).cuda()
    y = torch.empty_like(x)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        for _ in range(10):
            A.matvec(x, out=y)
        s.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            A.matvec(x, out=y)
        s.synchronize()
        eager_us = (time.perf_counter() - t0) * 1e6 / reps
    torch.cuda.current_stream().wait_stream(s)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        A.matvec(x, out=y)
    for _ in range(10):
        g.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        g.replay()
    torch.cuda.synchronize()
    graph_us = (time.perf_counter() - t0) * 1e6 / reps
    yt = y.cpu().numpy()
    del g
    A.close()
    o = O.OracleH2(W.points(w), w.leaf, w.cheb_p, w.eta, w.corr_len)
    rel_oracle = float(np.linalg.norm(yt - o.matvec(x_in[perm])) / np.linalg.norm(o.matvec(x_in[perm])))
    y_in = np.empty_like(yt)
    y_in[perm] = yt
    exact = O.kernel_matvec(W.points(w), x_in, w.corr_len)
    rel_exact = float(np.linalg.norm(y_in - exact) / np.linalg.norm(exact))
    log(f"{w.name}: {eager_us:.1f} us eager, {graph_us:.1f} us graph replay, rel err vs oracle {rel_oracle:.1e}, "
        f"vs exact kernel product {rel_exact:.1e}")
    return {"workload": w.name, "us_eager": round(eager_us, 2), "us_graph": round(graph_us, 2),
            "rel_err_vs_fp64_oracle": rel_oracle, "rel_err_vs_exact_kernel_product": rel_exact,
            "reps": reps}


_ONE_THREAD_SCRIPT = r"""
import json, sys, time
import numpy as np
sys.path.insert(0, sys.argv[1])
from oracle import oracle as O
from paper_1902_01829_amd import workloads as W
out = {}
w = W.C1
o = O.OracleH2(W.points(w), w.leaf, w.cheb_p, w.eta, w.corr_len, keep_blocks=True)
x = W.rhs(w, 1)[o.perm()]
ts = []
for _ in range(3):
    t0 = time.perf_counter(); o.matvec(x); ts.append(time.perf_counter() - t0)
out[w.name] = {"ms_per_product_median_of_3": round(1e3 * sorted(ts)[1], 3), "mode": "stored blocks, all rows"}
w = W.C2
o = O.OracleH2(W.points(w), w.leaf, w.cheb_p, w.eta, w.corr_len, keep_blocks=False)
x = W.rhs(w, 1)[o.perm()]
leaves = np.sort(np.random.Generator(np.random.PCG64(11)).permutation(o.leaf_nodes())[:64])
t0 = time.perf_counter(); o.matvec_leaves(x, leaves); t = time.perf_counter() - t0
out[w.name] = {"s_for_sample": round(t, 3), "mode": "matrix-free, full upsweep + rows of 64 seeded leaves"}
print(json.dumps(out))
"""


def oracle_one_thread():
    """The oracle on one host thread (a child process with OMP_NUM_THREADS=1):
    the whole 4096-point product (median of 3), and the 2^20-point workload's
    upsweep plus 64 sampled leaf rows."""
    import subprocess
    env = dict(os.environ, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, "-c", _ONE_THREAD_SCRIPT, ROOT], env=env, capture_output=True,
                       text=True, timeout=600)
    if r.returncode != 0:
        return {"error": r.stderr[-400:]}
    return json.loads(r.stdout.strip().splitlines()[-1])


def orthogonalize_section(reps=3):
    """Basis orthogonalization and projection of the coupling blocks (Sec. 5.1)
    of the 2-D 2^20-point workload, FP64, on the GPU: time per call (a fresh
    matrix each time), algorithmic flops (Householder QR with Q formed:
    4 M N^2 - 4 N^3 / 3 per factorization; T_c E_c: k^3 per child; projection
    with triangular T: 2 k^3 per coupling block), the bytes of the blocks,
    bases and transfers read and written, and the change of A x."""
    import torch
    from paper_1902_01829_amd import h2mv
    w = W.C2
    ms = []
    for rep in range(reps):
        A = h2mv.H2Matrix(W.points(w), w.dim, w.leaf, w.cheb_p, w.eta, w.corr_len, storage=0)
        info = A.info
        x = torch.from_numpy(W.rhs(w, 1)[A.perm()]).cuda()
        y0 = A.matvec(x)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h2mv.h2_orthogonalize(A.handle)   # returns when the device work is done
        ms.append((time.perf_counter() - t0) * 1e3)
        y1 = A.matvec(x)
        rel = float(((y1 - y0).norm() / y0.norm()).item())
        A.close()
        del x, y0, y1
        torch.cuda.empty_cache()
        time.sleep(SETTLE_S)
    k, q, lmin = info.rank, info.levels_q, info.lmin
    nleaves, m = 1 << q, w.leaf
    qr = lambda M, N: 4.0 * M * N * N - 4.0 * N ** 3 / 3.0
    nparents = sum(1 << (l - 1) for l in range(lmin + 1, q + 1))
    flops = nleaves * qr(m, k) + nparents * (2 * k ** 3 + qr(2 * k, k)) + info.coupling_blocks * 2.0 * k ** 3
    nbytes = 2 * (info.bytes_coupling + info.bytes_leaf_bases + info.bytes_transfers)
    best = min(ms)
    log(f"orthogonalize {w.name}: {best:.1f} ms (of {[round(v, 1) for v in ms]}), {flops / best / 1e6:.0f} GFLOP/s, "
        f"A x change {rel:.1e}")
    return {"workload": w.name, "ms": round(best, 3), "ms_all": [round(v, 3) for v in ms],
            "flops": flops, "GFLOP_per_s": round(flops / (best * 1e-3) / 1e9, 1),
            "bytes_read_written": nbytes, "GB_per_s": round(nbytes / (best * 1e-3) / 1e9, 1),
            "rel_change_of_Ax": rel, "fp64_vector_peak_TFLOP_per_s": 78.6}


def _time_matvec(A, x, y, steps):
    import torch
    from paper_1902_01829_amd import h2mv
    stream = torch.cuda.current_stream()
    for _ in range(2):
        h2mv.h2_matvec(A.handle, x.data_ptr(), y.data_ptr(), stream.cuda_stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        h2mv.h2_matvec(A.handle, x.data_ptr(), y.data_ptr(), stream.cuda_stream)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / steps


# Seconds waited, outside the timed region, after releasing a matrix (the
# orthogonalization, compression and transpose sections) and after building
# the matrix a compression call is timed on: the HIP runtime's hipMalloc of
# tens of GB right after freeing or allocating as much has taken 0.8-4.6 s
# (HIP API trace), which is the driver returning the previous allocation,
# not the call.
SETTLE_S = 2.0


def compress_section(steps=10, reps=3, nrows=256):
    """Algebraic compression (Sec. 5) on the GPU, FP64: the 2-D 2^20-point
    workload at the paper's 2-D threshold 1e-7 and the 3-D 2^19-point one at
    its 3-D threshold 1e-3 (Tables 2 and 3).  Time per call (a fresh matrix
    each time, orthogonalization included), the new rank of every level, the
    bytes of the representation before and after, the change of A x, the
    error against the exact kernel on sampled rows before and after (the
    columns of Tables 2 and 3), and the time of the product before and after
    (per-level ranks)."""
    import torch
    from oracle import oracle as O
    from paper_1902_01829_amd import h2mv
    out = {}
    for w, eps in ((W.C2, 1e-7), (W.C3, 1e-3)):
        ms = []
        for rep in range(reps):
            A = h2mv.H2Matrix(W.points(w), w.dim, w.leaf, w.cheb_p, w.eta, w.corr_len, storage=0)
            if rep == 0:
                info0, perm = A.info, A.perm()
                x_in = W.rhs(w, 1)
                x = torch.from_numpy(x_in[perm]).cuda()
                y = torch.empty_like(x)
                mv0 = _time_matvec(A, x, y, steps)
                y0 = y.cpu().numpy()
            torch.cuda.synchronize()
            time.sleep(SETTLE_S)   # after the construction's allocations, as after a release
            t0 = time.perf_counter()
            ranks = A.compress(eps)   # returns when the device work is done
            ms.append((time.perf_counter() - t0) * 1e3)
            if rep + 1 < reps:
                A.close()
                torch.cuda.empty_cache()
                time.sleep(SETTLE_S)
        info1 = A.info
        mv1 = _time_matvec(A, x, y, steps)
        y1 = y.cpu().numpy()
        A.close()
        del x, y
        torch.cuda.empty_cache()
        rows = np.sort(np.random.Generator(np.random.PCG64(17)).choice(w.n, size=nrows, replace=False))
        exact = O.kernel_matvec(W.points(w), x_in, w.corr_len, rows=perm[rows])
        err = lambda yy: float(np.linalg.norm(yy[rows] - exact) / np.linalg.norm(exact))
        lowrank = lambda i: i.bytes_coupling + i.bytes_leaf_bases + i.bytes_transfers
        change = float(np.linalg.norm(y1 - y0) / np.linalg.norm(y0))
        med = float(np.median(ms))
        log(f"compress {w.name} eps {eps:g}: median {med:.1f} ms (of {[round(v, 1) for v in ms]}), ranks "
            f"{[int(r) for r in ranks]}, low-rank bytes {lowrank(info0) / 1e9:.2f} -> {lowrank(info1) / 1e9:.2f} GB, "
            f"A x change {change:.1e}, matvec {mv0:.3f} -> {mv1:.3f} ms")
        out[w.name] = {
            "eps": eps, "ms": round(med, 2), "ms_statistic": f"median of {reps} calls",
            "ms_all": [round(v, 2) for v in ms],
            "level_rank_before": info0.rank, "level_rank_after": [int(r) for r in ranks],
            "lowrank_bytes_before": int(lowrank(info0)), "lowrank_bytes_after": int(lowrank(info1)),
            "dense_bytes": int(info0.bytes_dense),
            "rel_change_of_Ax": change,
            "rel_err_vs_exact_kernel_before": err(y0), "rel_err_vs_exact_kernel_after": err(y1),
            "error_sample": f"{nrows} seeded rows against the dense kernel (brute force)",
            "matvec_ms_before": round(mv0, 4), "matvec_ms_after": round(mv1, 4),
            "matvec_speedup": round(mv0 / mv1, 3)}
    return out


def transpose_section(reps=5):
    """The transposed matrix (h2_transpose) of the 2-D 2^20-point FP64 matrix:
    time per call (device transposition of every block, basis and transfer
    plus the new work lists), the bytes read and written, and A^T x against
    A x (the covariance matrix is symmetric)."""
    import torch
    from paper_1902_01829_amd import h2mv
    w = W.C2
    A = h2mv.H2Matrix(W.points(w), w.dim, w.leaf, w.cheb_p, w.eta, w.corr_len, storage=0)
    info = A.info
    x = torch.from_numpy(W.rhs(w, 1)[A.perm()]).cuda()
    y = A.matvec(x)
    ms, free_ms = [], []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        At = A.transpose()   # returns when the device work is done
        ms.append((time.perf_counter() - t0) * 1e3)
        yt = At.matvec(x)
        rel = float(((yt - y).norm() / y.norm()).item())
        del yt
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        At.close()   # hipFree of its ~47 GB
        free_ms.append((time.perf_counter() - t0) * 1e3)
        torch.cuda.empty_cache()
        time.sleep(SETTLE_S)
    A.close()
    nbytes = 2 * (info.bytes_coupling + info.bytes_dense + info.bytes_leaf_bases + info.bytes_transfers)
    med = float(np.median(ms))
    log(f"transpose {w.name}: median {med:.1f} ms (of {[round(v, 1) for v in ms]}), "
        f"{nbytes / (med * 1e-3) / 1e9:.0f} GB/s read + written, A^T x vs A x {rel:.1e}")
    return {"workload": w.name, "ms": round(med, 2), "ms_statistic": f"median of {reps} calls",
            "ms_all": [round(v, 2) for v in ms],
            "release_ms_all": [round(v, 2) for v in free_ms],
            "bytes_read_written": int(nbytes), "GB_per_s": round(nbytes / (med * 1e-3) / 1e9, 1),
            "rel_diff_AT_x_vs_A_x": rel}


HALF = 16   # storage modifier: blocks stored by halves


def half_partial_bytes(info, vb):
    """Partial sums of the transposed products (slots of 64 values in the
    vector type, vb bytes each: one per column segment and row group, as the
    library reports them), written once and read once."""
    return 2 * vb * 64 * info.partial_slots


HALF_CASES = ((W.C2, "fp64"), (W.C3, "fp64"), (W.C3, "fp32"), (W.C3, "bf16"))


def half_section(steps, warmup, full_ms=None, nleaves=16, cases=HALF_CASES):
    """Blocks stored by halves (symmetric matrices): the 2-D 2^20-point FP64
    matrix and the 3-D 2^19-point matrix in its three storage modes.  Time per
    product, stored bytes, the streaming phase (stored blocks read once for
    both products, partial sums, their addition per segment) as GB/s of the
    bytes it moves, the product's GB/s of the bytes it stores, the speedup
    over full storage, and the error
    against the FP64 oracle on sampled leaves.  full_ms: full-storage times
    by (workload, storage) already measured; the others are measured here.
    cases: the (workload, storage) pairs to run."""
    full_ms = dict(full_ms or {})
    out = {}
    for w, name in cases:
        r = run_matvec(w, STORAGE[name] | HALF, steps, warmup)
        info = r["info"]
        key = (w.name, name)
        if key not in full_ms:
            rf = run_matvec(w, STORAGE[name], steps, warmup)
            full_ms[key] = (rf["ms"], algorithmic_bytes(rf["info"], w.n))
        ms_full = full_ms[key][0]
        rows, ref = oracle_sample(w, r["perm"], r["xt"], nleaves)
        rel = float(np.linalg.norm(r["y"][rows] - ref) / np.linalg.norm(ref))
        vb = 8 if name == "fp64" else 4
        phase_bytes = info.bytes_coupling + info.bytes_dense + 8 * w.n + 2 * vb * w.n + half_partial_bytes(info, vb)
        stream_ms = float(r["phase_ms"][1])
        out[f"{w.name}/{name}"] = {
            "ms": round(r["ms"], 4), "ms_full_storage": round(ms_full, 4),
            "speedup_vs_full_storage": round(ms_full / r["ms"], 3),
            "stored_block_bytes": int(info.bytes_coupling + info.bytes_dense),
            "algorithmic_bytes": int(algorithmic_bytes(info, w.n)),
            "GB_per_s": round(algorithmic_bytes(info, w.n) / (r["ms"] * 1e-3) / 1e9, 1),
            "stream_phase_ms": round(stream_ms, 4), "stream_phase_bytes": int(phase_bytes),
            "partial_slots": int(info.partial_slots),
            "stream_phase_GB_per_s": round(phase_bytes / (stream_ms * 1e-3) / 1e9, 1),
            "rel_err_vs_fp64_oracle": rel}
        log(f"half {w.name} {name}: {r['ms']:.3f} ms (full {ms_full:.3f} ms, x{ms_full / r['ms']:.2f}), stream "
            f"phase {stream_ms:.3f} ms = {phase_bytes / (stream_ms * 1e-3) / 1e9:.0f} GB/s, rel err {rel:.2e}")
    out["error_sample"] = f"all rows of {nleaves} seeded leaves vs the FP64 oracle"
    return out


def storage_modes(steps, warmup, nleaves=16):
    """The 3-D workload (2^19 points, rank 64) in FP64, FP32 and BF16 storage."""
    w = W.C3
    out = {}
    for name in ("fp64", "fp32", "bf16"):
        r = run_matvec(w, STORAGE[name], steps, warmup)
        rows, ref = oracle_sample(w, r["perm"], r["xt"], nleaves)
        rel = float(np.linalg.norm(r["y"][rows] - ref) / np.linalg.norm(ref))
        nbytes = algorithmic_bytes(r["info"], w.n)
        out[name] = {"ms": round(r["ms"], 4), "GB_per_s": round(nbytes / (r["ms"] * 1e-3) / 1e9, 1),
                     "algorithmic_bytes": nbytes, "rel_err_vs_fp64_oracle": rel,
                     "stream_ms": round(float(r["phase_ms"][1]), 4)}
        log(f"{w.name} {name}: {r['ms']:.3f} ms, rel err {rel:.2e}")
    for name in ("fp32", "bf16"):
        out[name]["speedup_vs_fp64"] = round(out["fp64"]["ms"] / out[name]["ms"], 3)
    out["workload"] = w.name
    out["error_sample"] = f"all rows of {nleaves} seeded leaves vs the FP64 oracle"
    return out


def matmat_modes(steps, warmup, fp64_matvec_ms, nleaves=8):
    """The 2^20-point 2-D workload with 32 right-hand sides on the matrix cores,
    FP32 and BF16 storage, against 32 single-vector FP64 products."""
    import torch
    from paper_1902_01829_amd import h2mv
    w = W.C4
    out = {"workload": w.name, "nrhs": w.nrhs,
           "fp64_32_matvecs_ms": None if fp64_matvec_ms is None else round(32 * fp64_matvec_ms, 3)}
    for name in ("fp32", "bf16"):
        A = h2mv.H2Matrix(W.points(w), w.dim, w.leaf, w.cheb_p, w.eta, w.corr_len, storage=STORAGE[name])
        info, perm = A.info, A.perm()
        Xt = np.ascontiguousarray(W.rhs(w).T[:, perm])
        X = torch.from_numpy(Xt).cuda()
        Y = torch.empty_like(X)
        for _ in range(warmup):
            A.matmat(X, out=Y)
        torch.cuda.synchronize()
        h2mv.h2_profile(A.handle, True)
        t0 = time.perf_counter()
        for _ in range(steps):
            A.matmat(X, out=Y)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        phase_ms, calls = h2mv.h2_profile_read(A.handle)
        h2mv.h2_profile(A.handle, False)
        tuning = A.matmat_tuning(0)
        Yh = Y.cpu().numpy()
        A.close()
        del X, Y
        torch.cuda.empty_cache()
        nbytes = algorithmic_bytes(info, w.n, w.nrhs)
        entries = (info.bytes_coupling + info.bytes_dense + info.bytes_leaf_bases + info.bytes_transfers) / \
            (4 if name == "fp32" else 1)
        if name == "bf16":   # blocks are 2 bytes (+4 per block scale), bases 4 bytes
            entries = (info.bytes_coupling - 4 * info.coupling_blocks + info.bytes_dense - 4 * info.dense_blocks) / 2 \
                + (info.bytes_leaf_bases + info.bytes_transfers) / 4
        flops = 2.0 * entries * w.nrhs
        errs = []
        for j in (0, 31):
            rows, ref = oracle_sample(w, perm, Xt[j], nleaves, seed=13)
            errs.append(float(np.linalg.norm(Yh[j][rows] - ref) / np.linalg.norm(ref)))
        # roof = min(matrix-core peak, intensity x HBM peak); the useful products of BF16 blocks
        # are issued as three exact BF16 MFMAs each, so their matrix-core roof is 1/3 of the BF16 peak
        peak = 157.3 if name == "fp32" else 2500.0 / 3
        roof = min(peak, flops / nbytes * HBM_PEAK_GBS / 1e3)
        tflops = flops / (ms * 1e-3) / 1e12
        out[name] = {"ms": round(ms, 4), "GB_per_s": round(nbytes / (ms * 1e-3) / 1e9, 1),
                     "TFLOP_per_s": round(tflops, 2), "roof_TFLOP_per_s": round(roof, 1),
                     "frac_of_roof": round(tflops / roof, 4), "algorithmic_bytes": nbytes,
                     "flops": flops, "stream_ms": round(float(phase_ms[1] / max(calls, 1)), 4),
                     "speedup_vs_32_fp64_matvecs": None if fp64_matvec_ms is None
                     else round(32 * fp64_matvec_ms / ms, 2),
                     "rel_err_vs_fp64_oracle_max": max(errs), "tuning": tuning}
        log(f"{w.name} matmat {name}: {ms:.3f} ms, {out[name]['GB_per_s']} GB/s, "
            f"{out[name]['TFLOP_per_s']} TFLOP/s, rel err {max(errs):.2e}, tuning {tuning}")
    out["error_sample"] = f"columns 0 and 31, all rows of {nleaves} seeded leaves vs the FP64 oracle"
    return out


def batch_modes(steps, warmup, nleaves=4):
    """64 uneven H^2 matrices (2-D and 3-D, ranks 16, 27 and 64, leaf sizes 32
    and 64), 8 right-hand sides each, FP32 storage: one batched product (one
    launch per level slot, replayed from a HIP graph, launch shape chosen by
    the autotuner) against the same members multiplied one after another, and
    against 8 FP64 single-vector products per member."""
    import torch
    from paper_1902_01829_amd import h2mv
    members = W.batch_members()
    nrhs = members[0].nrhs
    t0 = time.perf_counter()
    mats = [h2mv.H2Matrix(W.points(w), w.dim, w.leaf, w.cheb_p, w.eta, w.corr_len, storage=1) for w in members]
    perms = [m.perm() for m in mats]
    Xt = [np.ascontiguousarray(W.rhs(w).T[:, p]) for w, p in zip(members, perms)]
    Xs = [torch.from_numpy(x).cuda() for x in Xt]
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    infos = [m.info for m in mats]
    nbytes = sum(algorithmic_bytes(i, w.n, nrhs) for i, w in zip(infos, members))
    log(f"batch: {len(members)} members, {sum(w.n for w in members)} points, "
        f"{sum(i.bytes_device_total for i in infos) / 1e9:.2f} GB on device, built in {build_s:.1f} s")
    batch = h2mv.H2Batch(mats, nrhs)
    Ys = batch.matmat(Xs)            # tunes the launch shape and captures the graph
    for _ in range(warmup):
        batch.matmat(Xs, outs=Ys)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        batch.matmat(Xs, outs=Ys)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    tuning = batch.tuning()
    # the same members, one many-right-hand-side product after another
    Rs = [m.matmat(X) for m, X in zip(mats, Xs)]
    for _ in range(warmup):
        for m, X, R in zip(mats, Xs, Rs):
            m.matmat(X, out=R)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        for m, X, R in zip(mats, Xs, Rs):
            m.matmat(X, out=R)
    torch.cuda.synchronize()
    seq_ms = (time.perf_counter() - t0) * 1e3 / steps
    diff = max(float(((Y - R).norm() / R.norm()).item()) for Y, R in zip(Ys, Rs))
    Yh = [Y.cpu().numpy() for Y in Ys]
    batch.close()
    for m in mats:
        m.close()
    del Ys, Rs, mats, batch
    torch.cuda.empty_cache()
    # 8 FP64 single-vector products per member, members built one at a time
    fp64_ms = 0.0
    reps = 5
    for w, X in zip(members, Xs):
        A = h2mv.H2Matrix(W.points(w), w.dim, w.leaf, w.cheb_p, w.eta, w.corr_len, storage=0)
        cols = [X[j].contiguous() for j in range(nrhs)]
        y = torch.empty_like(cols[0])
        for c in cols:
            A.matvec(c, out=y)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            for c in cols:
                A.matvec(c, out=y)
        torch.cuda.synchronize()
        fp64_ms += (time.perf_counter() - t0) * 1e3 / reps
        A.close()
        del cols, y
        torch.cuda.empty_cache()
    # error of a few members against the FP64 oracle
    order = np.argsort([w.n for w in members])
    picks = sorted({int(order[0]), int(order[len(order) // 2]), int(order[-1]),
                    max(range(len(members)), key=lambda b: (members[b].dim, members[b].rank, members[b].n))})
    errs = []
    for b in picks:
        for j in (0, nrhs - 1):
            rows, ref = oracle_sample(members[b], perms[b], Xt[b][j], nleaves, seed=17)
            errs.append(float(np.linalg.norm(Yh[b][j][rows] - ref) / np.linalg.norm(ref)))
    out = {"members": len(members), "nrhs": nrhs, "points_total": int(sum(w.n for w in members)),
           "storage": "fp32", "ms": round(ms, 4), "GB_per_s": round(nbytes / (ms * 1e-3) / 1e9, 1),
           "algorithmic_bytes": nbytes, "unbatched_members_ms": round(seq_ms, 4),
           "speedup_vs_unbatched": round(seq_ms / ms, 2),
           "fp64_8_matvecs_per_member_ms": round(fp64_ms, 3),
           "speedup_vs_fp64_matvecs": round(fp64_ms / ms, 2),
           "max_rel_diff_vs_member_products": diff,
           "rel_err_vs_fp64_oracle_max": max(errs), "tuning": tuning,
           "error_sample": f"members {picks}, columns 0 and {nrhs - 1}, all rows of {nleaves} seeded leaves "
                           "vs the FP64 oracle"}
    log(f"batch fp32: {ms:.3f} ms ({out['GB_per_s']} GB/s), unbatched {seq_ms:.3f} ms, "
        f"FP64 matvecs {fp64_ms:.2f} ms, rel err {max(errs):.2e}, tuning {tuning}")
    return out


SCHEDULES = (("merged", 0, 0, 1.0), ("streamed", 1, 0, 1.0), ("streamed-cap3", 1, 3, 1.0),
             ("streamed-cap2", 1, 2, 1.0), ("streamed-cap3-half-late", 1, 3, 0.5),
             ("streamed-cap3-late", 1, 3, 0.0))
SCHEDULE_CASES = (W.C1, W.C1.with_(name="2d-n16384-m64-k64", n=1 << 14, leaf=64, cheb_p=8, seed=1011),
                  W.C1.with_(name="2d-n65536-m64-k64", n=1 << 16, leaf=64, cheb_p=8, seed=1012),
                  W.C1.with_(name="2d-n262144-m64-k64", n=1 << 18, leaf=64, cheb_p=8, seed=1013),
                  W.C2, W.C3)


def schedule_section(trials=5, cases=SCHEDULE_CASES):
    """The merged schedule (coupling and near field in one launch after the
    upsweep) against the streamed one (near field on a second stream, Sec.
    4.5) at sizes from 4096 to 2^20 points, FP64: time per product (median of
    `trials` runs of many products each, the schedules interleaved), and the
    same products replayed from a HIP graph at the smallest size.  All
    schedules give bitwise the same product (checked here too)."""
    import torch
    from paper_1902_01829_amd import h2mv
    out = {}
    for w in cases:
        A = h2mv.H2Matrix(W.points(w), w.dim, w.leaf, w.cheb_p, w.eta, w.corr_len, storage=0)
        x = torch.from_numpy(np.ascontiguousarray(W.rhs(w)[A.perm()])).cuda()
        y = torch.empty_like(x)
        y0 = A.matvec(x)
        reps = max(5, min(400, int(2e5 / max(1, w.n) * 40)))
        times = {name: [] for name, *_ in SCHEDULES}
        for _ in range(trials):
            for name, sched, cap, early in SCHEDULES:
                A.set_schedule(sched, cap, early)
                times[name].append(_time_matvec(A, x, y, reps))
                if not torch.equal(y, y0):
                    raise RuntimeError(f"{w.name}: schedule {name} changed the product")
        med = {k: float(np.median(v)) for k, v in times.items()}
        res = {"n": w.n, "reps": reps, "trials": trials,
               "ms": {k: round(v, 5) for k, v in med.items()},
               "speedup_vs_merged": {k: round(med["merged"] / v, 4) for k, v in med.items() if k != "merged"}}
        if w.n <= 1 << 14:
            g_us = {}
            for name in ("merged", "streamed-cap3"):
                _, sched, cap, early = next(s for s in SCHEDULES if s[0] == name)
                A.set_schedule(sched, cap, early)
                A.matvec(x, out=y)
                torch.cuda.synchronize()
                g = torch.cuda.CUDAGraph()
                with torch.cuda.graph(g):
                    A.matvec(x, out=y)
                for _ in range(10):
                    g.replay()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(reps):
                    g.replay()
                torch.cuda.synchronize()
                g_us[name] = round((time.perf_counter() - t0) * 1e6 / reps, 2)
                del g
                if not torch.equal(y, y0):
                    raise RuntimeError(f"{w.name}: graph replay of {name} changed the product")
            res["graph_us"] = g_us
        best = min(med, key=med.get)
        log(f"schedule {w.name}: " + ", ".join(f"{k} {v:.4f}" for k, v in med.items()) + f" ms; best {best}"
            + (f"; graph us {res['graph_us']}" if "graph_us" in res else ""))
        out[w.name] = res
        A.close()
        del x, y, y0
        torch.cuda.empty_cache()
    return out


SECTIONS = ("small", "modes", "matmat", "batch", "orthogonalize", "compress", "transpose", "half", "read",
            "schedule")


def run_section(name, args):
    """One section alone (--only), its JSON on one line."""
    if name == "small":
        out = small_case()
    elif name == "modes":
        out = storage_modes(args.steps, args.warmup)
    elif name == "matmat":
        out = matmat_modes(args.steps, args.warmup, None)
    elif name == "orthogonalize":
        out = orthogonalize_section()
    elif name == "compress":
        out = compress_section()
    elif name == "transpose":
        out = transpose_section()
    elif name == "read":
        out = read_ceiling()
    elif name == "schedule":
        out = schedule_section()
    elif name == "half":
        cases = HALF_CASES
        if args.half_case:
            cases = tuple((W.WORKLOADS[c.split("/")[0]], c.split("/")[1]) for c in args.half_case)
        out = half_section(args.steps, args.warmup, cases=cases)
    else:
        out = batch_modes(args.steps, args.warmup)
    print(json.dumps({"section": name, **out}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default=W.C2.name, choices=sorted(W.WORKLOADS))
    ap.add_argument("--storage", default="fp64", choices=sorted(STORAGE))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-modes", action="store_true",
                    help="skip the storage-mode, many-right-hand-side and batch sections")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--only", default=None,
                    help="run these sections alone, in this order (comma-separated: " + ", ".join(SECTIONS) +
                         ") and print one JSON line per section (for profiling runs); the headline line is "
                         "not printed")
    ap.add_argument("--half-case", action="append", default=None, metavar="WORKLOAD/STORAGE",
                    help="with --only half: run only these cases (e.g. 2d-n1048576-m64-k64/fp64)")
    ap.add_argument("--calibrate-copy-gib", type=float, default=0.0,
                    help="first run one device-to-device copy of this many GiB (a known-size "
                         "reference for hardware byte counters)")
    args = ap.parse_args()
    only = [] if args.only is None else args.only.split(",")
    for name in only:
        if name not in SECTIONS:
            ap.error(f"--only: unknown section {name!r} (sections: {', '.join(SECTIONS)})")
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(the per-GPU kernel at its real shape is what one GPU shows).", file=sys.stderr)
        sys.exit(2)

    import torch
    torch.cuda.set_device(0)
    if args.calibrate_copy_gib > 0:
        nel = int(args.calibrate_copy_gib * (1 << 30)) // 8
        src = torch.ones(nel, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"calibration copy: {nel * 8} bytes read, {nel * 8} bytes written")
        del src, dst

    for name in only:
        run_section(name, args)
    if only:
        return

    ceiling = read_ceiling()
    w = W.WORKLOADS[args.workload]
    log(f"building {w.name} storage={args.storage}")
    r = run_matvec(w, STORAGE[args.storage], args.steps, args.warmup)
    info, ms, phase = r["info"], r["ms"], r["phase_ms"]
    nbytes = algorithmic_bytes(info, w.n)
    value = nbytes / (ms * 1e-3) / 1e9
    sk_bytes = stream_kernel_bytes(info, w.n, STORAGE[args.storage])
    achieved = sk_bytes / (phase[1] * 1e-3) / 1e9
    log(f"{ms:.3f} ms/step, {value:.1f} GB/s; phases ms/call up {phase[0]:.3f} stream {phase[1]:.3f} "
        f"down {phase[2]:.3f} leaf {phase[3]:.3f}")
    traffic = MEASURED_TRAFFIC.get((w.name, args.storage))
    result = {
        "metric": "H2 matvec GB/s & % HBM peak; BF16/FP32/batched vs FP64 speedup at rel err",
        "value": round(value, 2), "unit": "GB/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": DTYPE[args.storage], "data": "synthetic",
        "config": {"workload": w.name, "n": w.n, "dim": w.dim, "leaf_size": w.leaf, "rank": w.rank,
                   "corr_len": w.corr_len, "eta": w.eta, "nrhs": 1, "storage": args.storage,
                   "coupling_blocks": info.coupling_blocks, "dense_blocks": info.dense_blocks,
                   "algorithmic_bytes": nbytes, "pct_hbm_peak": round(100 * value / HBM_PEAK_GBS, 2),
                   "build_s": round(r["build_s"], 2)},
        "phases_ms": {"upsweep": round(float(phase[0]), 4), "stream": round(float(phase[1]), 4),
                      "downsweep": round(float(phase[2]), 4), "leaf_expand": round(float(phase[3]), 4),
                      "call": round(float(phase[4]), 4)},
        "roofline": {"bound": "hbm", "kernel": "stream_kernel (coupling blocks of all levels + dense blocks)",
                     "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": None if traffic is None else int(traffic),
                     "algorithmic_bytes": int(sk_bytes),
                     "timing": "mean duration of the stream phase over the timed steps, from HIP events the "
                               "library records on the call's stream around it",
                     "measured_read_ceiling_GB_per_s": ceiling["GB_per_s"],
                     "frac_of_measured_read_ceiling": round(achieved / ceiling["GB_per_s"], 4)},
        "hbm_read_ceiling": ceiling,
        "paper_context": PAPER_CONTEXT,
    }
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a sample")
        cb, rows, y_ref = cpu_baseline(w, r["perm"], r["xt"], args.cpu_budget)
        cb["one_thread"] = oracle_one_thread()
        result["cpu_baseline"] = cb
        result["rel_err_vs_oracle_sample"] = float(np.linalg.norm(r["y"][rows] - y_ref) / np.linalg.norm(y_ref))
    if not args.no_modes:
        result["small"] = small_case()
        result["storage_modes"] = modes = storage_modes(args.steps, args.warmup)
        fp64_ms = ms if (w.name == W.C2.name and args.storage == "fp64") else None
        if fp64_ms is not None:
            result["matmat"] = matmat_modes(max(3, args.steps // 4), 1, fp64_ms)
        result["batch"] = batch_modes(max(3, args.steps // 2), 1)
        result["orthogonalize"] = orthogonalize_section()
        result["compress"] = compress_section()
        result["transpose"] = transpose_section()
        full = {(W.C3.name, m): (modes[m]["ms"], modes[m]["algorithmic_bytes"]) for m in ("fp64", "fp32", "bf16")}
        if w.name == W.C2.name and args.storage == "fp64":
            full[(w.name, "fp64")] = (ms, nbytes)
        result["half_storage"] = half_section(args.steps, args.warmup, full)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
