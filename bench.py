"""Benchmark of the H^2 matrix-vector product on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME] [--storage fp64|fp32|bf16]

A step is one whole product y = A x (leaf projection, upsweep, coupling and
dense streaming, downsweep, leaf expansion and sum) on a resident matrix and
vector.  The default workload is the 2-D covariance of 2^20 uniform points
(exponential kernel, correlation length 0.1, leaf size 64, 8x8 Chebyshev
bases: rank 64, eta 0.9), FP64.  value = algorithmic bytes per product / time
(GB/s): the bytes of D, S, U, V, E, F, x and y.

Prints one JSON line.  Also reports the dominant kernel (coupling + dense
streaming) against the HBM roofline, and the FP64 CPU oracle timed on a
bounded sample of the same workload.
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
# Fraction of HBM traffic per algorithmic byte of the streaming kernel, from
# rocprofv3 FETCH_SIZE/WRITE_SIZE counters; None until measured for the
# current kernel.
MEASURED_TRAFFIC = {}


def algorithmic_bytes(info, n, nrhs=1):
    """D + S + U + V + E + F, plus x read and y written (FP64)."""
    rep = info.bytes_coupling + info.bytes_dense + info.bytes_leaf_bases + info.bytes_transfers
    return rep + 16 * n * nrhs


def stream_kernel_bytes(info, n, storage):
    """Algorithmic bytes of one launch of the streaming kernel: every coupling
    and dense block once, x read once (FP64) and the near field written."""
    vb = 8 if storage == 0 else 4
    return info.bytes_coupling + info.bytes_dense + 8 * n + vb * n


def cpu_baseline(w, perm, xt, budget_s=20.0):
    """FP64 oracle (matrix-free, all host threads) on a sample of leaves: the
    full upsweep plus the rows of the sampled leaves (their dense blocks and
    the coupling rows of their ancestors).  Reported in GB/s of the blocks,
    bases and transfers that sample touches, as if they were stored."""
    from oracle import oracle as O
    t0 = time.perf_counter()
    o = O.OracleH2(W.points(w), w.leaf, w.cheb_p, w.eta, w.corr_len, keep_blocks=False)
    build_s = time.perf_counter() - t0
    assert np.array_equal(perm, o.perm())
    k, q = o.k, o.q
    eb = 8
    rps = [o.coupling_bsr(l)[0] for l in range(q + 1)]
    drp, _ = o.dense_bsr()
    b, e = o.ranges()
    sizes = e - b
    rng = np.random.Generator(np.random.PCG64(11))
    leaves_all = rng.permutation(o.leaf_nodes())

    def touched_bytes(leaves):
        up = (2 * k * int(sizes[(1 << q) - 1:].sum()) + 2 * k * k * max(0, (1 << (q + 1)) - (1 << (o.lmin + 1)))) * eb
        tot = up
        for v in leaves:
            j = v - ((1 << q) - 1)
            tot += int(drp[j + 1] - drp[j]) * int(sizes[v]) * w.leaf * eb   # dense row (approx. leaf size cols)
            a = v
            for l in range(q, o.lmin - 1, -1):
                i = a - ((1 << l) - 1)
                tot += int(rps[l][i + 1] - rps[l][i]) * k * k * eb
                a = (a - 1) // 2
        return tot

    # calibrate on a few leaves, then size the sample to the budget
    nl = 4
    t0 = time.perf_counter()
    o.matvec_leaves(xt, leaves_all[:nl])
    t_cal = time.perf_counter() - t0
    nl = int(max(4, min(len(leaves_all), nl * budget_s / max(t_cal, 1e-3))))
    leaves = np.sort(leaves_all[:nl])
    t0 = time.perf_counter()
    y_ref = o.matvec_leaves(xt, leaves)
    t = time.perf_counter() - t0
    nbytes = touched_bytes(leaves)
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {
        "value": round(nbytes / t / 1e9, 3), "unit": "GB/s", "cores": cores, "kind": "oracle",
        "sample": f"FP64 oracle, matrix-free (blocks regenerated), full upsweep + rows of {nl} of "
                  f"{1 << q} leaves ({len(o.leaf_rows(leaves))} rows); {t:.1f} s for "
                  f"{nbytes / 1e9:.2f} GB of blocks touched; oracle build {build_s:.1f} s",
    }, leaves, o.leaf_rows(leaves), y_ref


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default=W.C2.name, choices=sorted(W.WORKLOADS))
    ap.add_argument("--storage", default="fp64", choices=sorted(STORAGE))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(the per-GPU kernel at its real shape is what one GPU shows).", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1902_01829_amd import h2mv

    w = W.WORKLOADS[args.workload]
    storage = STORAGE[args.storage]
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    print(f"[bench] building {w.name} storage={args.storage}", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    A = h2mv.H2Matrix(W.points(w), w.dim, w.leaf, w.cheb_p, w.eta, w.corr_len, storage=storage)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    info = A.info
    perm = A.perm()
    xt = W.rhs(w, 1)[perm]
    x = torch.from_numpy(xt).cuda()
    y = torch.empty_like(x)
    print(f"[bench] built in {build_s:.1f} s: {info.coupling_blocks} coupling, {info.dense_blocks} dense blocks, "
          f"{info.bytes_device_total / 1e9:.2f} GB on device", file=sys.stderr, flush=True)

    for _ in range(args.warmup):
        A.matvec(x, out=y)
    torch.cuda.synchronize()
    h2mv.h2_profile(A.handle, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        h2mv.h2_matvec(A.handle, x.data_ptr(), y.data_ptr(), stream.cuda_stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    phase_ms, calls = h2mv.h2_profile_read(A.handle)
    h2mv.h2_profile(A.handle, False)
    ms = (t1 - t0) * 1e3 / args.steps
    nbytes = algorithmic_bytes(info, w.n)
    value = nbytes / (ms * 1e-3) / 1e9
    stream_ms = phase_ms[1] / max(calls, 1)
    sk_bytes = stream_kernel_bytes(info, w.n, storage)
    achieved = sk_bytes / (stream_ms * 1e-3) / 1e9
    y_host = y.cpu().numpy()
    print(f"[bench] {ms:.3f} ms/step, {value:.1f} GB/s; phases ms/call up {phase_ms[0] / calls:.3f} "
          f"stream {stream_ms:.3f} down {phase_ms[2] / calls:.3f} leaf {phase_ms[3] / calls:.3f}",
          file=sys.stderr, flush=True)

    result = {
        "metric": "H2 matvec GB/s & % HBM peak; BF16/FP32/batched vs FP64 speedup at rel err",
        "value": round(value, 2), "unit": "GB/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": DTYPE[args.storage], "data": "synthetic",
        "config": {"workload": w.name, "n": w.n, "dim": w.dim, "leaf_size": w.leaf, "rank": w.rank,
                   "corr_len": w.corr_len, "eta": w.eta, "nrhs": 1, "storage": args.storage,
                   "coupling_blocks": info.coupling_blocks, "dense_blocks": info.dense_blocks,
                   "algorithmic_bytes": nbytes, "pct_hbm_peak": round(100 * value / HBM_PEAK_GBS, 2),
                   "build_s": round(build_s, 2)},
        "phases_ms": {"upsweep": round(phase_ms[0] / calls, 4), "stream": round(stream_ms, 4),
                      "downsweep": round(phase_ms[2] / calls, 4), "leaf_expand": round(phase_ms[3] / calls, 4),
                      "call": round(phase_ms[4] / calls, 4)},
        "roofline": {"bound": "hbm", "kernel": "blockrow_kernel (coupling all levels + dense)",
                     "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": MEASURED_TRAFFIC.get((w.name, args.storage))},
    }
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle on a sample", file=sys.stderr, flush=True)
        cb, leaves, rows, y_ref = cpu_baseline(w, perm, xt, args.cpu_budget)
        result["cpu_baseline"] = cb
        result["rel_err_vs_oracle_sample"] = float(np.linalg.norm(y_host[rows] - y_ref) / np.linalg.norm(y_ref))
    print(json.dumps(result), flush=True)
    A.close()


if __name__ == "__main__":
    main()
