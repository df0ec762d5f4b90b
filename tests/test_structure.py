"""Host logic of the library against the oracle (CPU only, no device calls).

The library's own tree, partition and block-sparse-row lists (built by its
C++ code, compiled into libh2mv) must equal the oracle's exactly: both follow
the same construction rules, and an H^2 built from the same points with the
same rules is then the same representation, which is what makes the FP64
parity of the products meaningful at 1e-12.
"""
import numpy as np
import pytest

from paper_1902_01829_amd import h2mv
from paper_1902_01829_amd import workloads as W

CASES = [
    W.C1,
    W.C1.with_(name="3d-n3000-m24-p3", n=3000, dim=3, leaf=24, cheb_p=3, corr_len=0.2, seed=77),
    W.C1.with_(name="2d-n5000-m32-p4-ragged", n=5000, seed=78),
    W.C1.with_(name="2d-n1-m32", n=1, seed=79),
    W.C1.with_(name="3d-n65536-m64-p4", n=1 << 16, dim=3, leaf=64, cheb_p=4, corr_len=0.2, seed=80),
    W.C1.with_(name="2d-n999-m7-p2-eta2", n=999, leaf=7, cheb_p=2, eta=2.0, seed=81),
]


@pytest.mark.parametrize("w", CASES, ids=lambda w: w.name)
def test_structure_identical_to_oracle(oracle_mod, w):
    P = W.points(w)
    h = h2mv.h2_build_from_points(P, w.dim, w.leaf, w.cheb_p, w.eta, w.corr_len,
                                  flags=h2mv.H2_FLAG_STRUCTURE_ONLY)
    try:
        info = h2mv.h2_get_info(h)
        o = oracle_mod.OracleH2(P, w.leaf, w.cheb_p, w.eta, w.corr_len, keep_blocks=False)
        assert (info.n, info.levels_q, info.lmin, info.rank) == (o.n, o.q, o.lmin, o.k)
        assert np.array_equal(h2mv.h2_get_perm(h, w.n), o.perm())
        for l in range(o.q + 1):
            rp, ci = h2mv.h2_get_level_bsr(h, l, 1 << l)
            orp, oci = o.coupling_bsr(l)
            assert np.array_equal(rp, orp) and np.array_equal(ci, oci), l
        rp, ci = h2mv.h2_get_level_bsr(h, -1, 1 << o.q)
        orp, oci = o.dense_bsr()
        assert np.array_equal(rp, orp) and np.array_equal(ci, oci)
        assert info.near_ties == o.near_ties() == 0
        assert info.coupling_blocks == o.n_coupling and info.dense_blocks == len(oci)
    finally:
        h2mv.h2_free(h)
