"""Seeded synthetic inputs for the H^2 matrix-vector product.

This module only draws random numbers: points, right-hand sides and the
parameters of batch members.  It holds none of the method's arithmetic, and it
is the one module that both the HIP path's tests and the oracle's tests use.

The workloads stand in for the covariance matrices of the paper's Sec. 4.6
(Gaussian-process covariances of points in [0,1]^2 and [0,1]^3 with an
isotropic exponential kernel, correlation length 0.1 in 2-D and 0.2 in 3-D).
The paper places its points on randomly perturbed grids of unstated
perturbation; here they are uniform in the unit square / cube.
"""
from __future__ import annotations

from dataclasses import dataclass, replace

import numpy as np


@dataclass(frozen=True)
class Workload:
    name: str
    n: int
    dim: int
    leaf: int          # leaf size m
    cheb_p: int        # Chebyshev points per axis (rank k = p^dim)
    corr_len: float
    eta: float = 0.9
    nrhs: int = 1
    seed: int = 0      # points seed; the right-hand side uses seed + 1000

    @property
    def rank(self) -> int:
        return self.cheb_p ** self.dim

    def with_(self, **kw) -> "Workload":
        return replace(self, **kw)


# The workloads of the benchmark, small to large.
C1 = Workload("2d-n4096-m32-k16", 4096, 2, 32, 4, 0.1, seed=1001)
C2 = Workload("2d-n1048576-m64-k64", 1 << 20, 2, 64, 8, 0.1, seed=1002)
C3 = Workload("3d-n524288-m64-k64", 1 << 19, 3, 64, 4, 0.2, seed=1003)
C4 = Workload("2d-n1048576-m64-k64-r32", 1 << 20, 2, 64, 8, 0.1, nrhs=32, seed=1004)
WORKLOADS = {w.name: w for w in (C1, C2, C3, C4)}


def points(w: Workload) -> np.ndarray:
    """n x dim points, uniform in the unit square / cube (float64, C order)."""
    rng = np.random.Generator(np.random.PCG64(w.seed))
    return np.ascontiguousarray(rng.random((w.n, w.dim)))


def rhs(w: Workload, nrhs: int | None = None) -> np.ndarray:
    """Right-hand side(s), N(0,1): shape (n,) for one vector, (n, r) otherwise."""
    r = w.nrhs if nrhs is None else nrhs
    rng = np.random.Generator(np.random.PCG64(w.seed + 1000))
    if r == 1:
        return rng.standard_normal(w.n)
    return np.ascontiguousarray(rng.standard_normal((w.n, r)))


def batch_members(count: int = 64, seed: int = 5000, nmin_log2: float = 12.0,
                  nmax_log2: float = 17.0, nrhs: int = 8) -> list[Workload]:
    """Uneven batch: n log-uniform in [2^nmin, 2^nmax]; the first half 2-D
    (p in {4, 8}: ranks 16 or 64), the second half 3-D (p in {3, 4}: ranks 27
    or 64); correlation length uniform in [0.05, 0.3]; leaf size 32 or 64."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for b in range(count):
        dim = 2 if b < count // 2 else 3
        n = int(round(2.0 ** rng.uniform(nmin_log2, nmax_log2)))
        p = int(rng.choice([4, 8])) if dim == 2 else int(rng.choice([3, 4]))
        leaf = int(rng.choice([32, 64]))
        ell = float(rng.uniform(0.05, 0.3))
        out.append(Workload(f"batch{b}-{dim}d-n{n}-m{leaf}-p{p}", n, dim, leaf, p, ell,
                            nrhs=nrhs, seed=seed + 1 + b))
    return out


def random_h2_values(seed: int, sizes_leaf: np.ndarray, level_rank: np.ndarray, coupling_counts: list,
                     dense_shapes: list) -> dict:
    """Random N(0,1) entries for an H^2 matrix whose structure is given:
    leaf sizes m_j (leaf order), ranks k_l per level, the number of coupling
    blocks per level, and the (rows, cols) of every dense block in order.
    Returns the value arrays in the column-major layout of h2_arrays (U, V,
    E, F, S per level, D).  Bases and transfers are scaled by 1/sqrt(rank)
    so that products keep unit size."""
    rng = np.random.Generator(np.random.PCG64(seed))
    q = len(level_rank) - 1
    kq = int(level_rank[q])
    nU = int(np.sum(sizes_leaf)) * kq
    nE = sum(int(level_rank[l]) * int(level_rank[l - 1]) << l for l in range(1, q + 1))
    U = rng.standard_normal(nU) / np.sqrt(kq)
    V = rng.standard_normal(nU) / np.sqrt(kq)
    E = np.concatenate([rng.standard_normal((int(level_rank[l]) * int(level_rank[l - 1])) << l)
                        / np.sqrt(level_rank[l - 1]) for l in range(1, q + 1)]) if q > 0 else np.zeros(0)
    F = np.concatenate([rng.standard_normal((int(level_rank[l]) * int(level_rank[l - 1])) << l)
                        / np.sqrt(level_rank[l - 1]) for l in range(1, q + 1)]) if q > 0 else np.zeros(0)
    assert E.size == nE
    S = [rng.standard_normal(int(c) * int(level_rank[l]) ** 2) for l, c in enumerate(coupling_counts)]
    D = np.concatenate([rng.standard_normal(r * c) for r, c in dense_shapes]) if dense_shapes else np.zeros(0)
    return {"U": U, "V": V, "E": E, "F": F, "S": S, "D": D}
