// Transformations of a built representation in place or into a new handle:
// basis orthogonalization (Sec. 4), compression (Sec. 5) and the transpose.
#include "h2_internal.h"

namespace h2i {

namespace {

// S_ji = S_ij^T, bit for bit, for every coupling block (FP64 storage): the
// mirror of each block is found by binary search in its mirror row (sorted
// per row on the host), and the pairs are compared on the device.
bool coupling_symmetric(h2_matrix_ &A, hipStream_t st) {
    const Structure &s = A.st;
    std::vector<h2::MirrorDesc> pairs;
    {
        int64_t total = 0;
        for (const auto &B : s.coupling) total += B.blocks();
        pairs.reserve(size_t(total / 2 + s.nnodes));
    }
    int64_t fi = 0;
    for (int l = 0; l <= s.q; ++l) {
        const h2::Bsr &B = s.coupling[l];
        const int64_t rows = int64_t(1) << l, f0 = fi;
        // each row's (column, fill index) pairs sorted by column (rows are short)
        std::vector<std::pair<int32_t, int64_t>> key(size_t(B.blocks()));
        for (int64_t i = 0; i < rows; ++i) {
            for (int32_t b = B.rowptr[i]; b < B.rowptr[i + 1]; ++b) key[size_t(b)] = {B.colidx[b], f0 + b};
            std::sort(key.begin() + B.rowptr[i], key.begin() + B.rowptr[i + 1]);
        }
        for (int64_t i = 0; i < rows; ++i)
            for (int32_t b = B.rowptr[i]; b < B.rowptr[i + 1]; ++b) {
                const int64_t j = B.colidx[b];
                if (j < i) continue;   // each pair once (i <= j)
                const auto lo = key.begin() + B.rowptr[j], hi = key.begin() + B.rowptr[j + 1];
                const auto it = std::lower_bound(lo, hi, std::make_pair(int32_t(i), int64_t(-1)));
                if (it == hi || it->first != int32_t(i)) return false;   // no mirror block
                pairs.push_back({A.off_blk[size_t(f0 + b)], A.off_blk[size_t(it->second)], s.lrank[l], 0});
            }
        fi += B.blocks();
    }
    if (pairs.empty()) return true;
    DeviceArena scratch;
    int32_t *flag = static_cast<int32_t *>(scratch.alloc(4));
    check_hip(hipMemsetAsync(flag, 0, 4, st), "hipMemsetAsync");
    check_hip(h2::launch_symmetry_check(static_cast<const double *>(A.blocks), scratch.upload(pairs, st),
                                        int64_t(pairs.size()), flag, st),
              "symmetry check launch");
    int32_t h = 0;
    check_hip(hipMemcpyAsync(&h, flag, 4, hipMemcpyDeviceToHost, st), "hipMemcpyAsync");
    check_hip(hipStreamSynchronize(st), "symmetry check");
    return h == 0;
}

// Moves the representation of B (structure, layout, device memory, work
// lists) into A; B receives A's old one and frees it when destroyed.
void adopt(h2_matrix_ &A, h2_matrix_ &B) {
    std::swap(A.st, B.st);
    A.mem.swap(B.mem);
    std::swap(A.basis, B.basis);
    std::swap(A.blocks, B.blocks);
    std::swap(A.scales, B.scales);
    std::swap(A.xh, B.xh);
    std::swap(A.yh, B.yh);
    std::swap(A.ynear, B.ynear);
    std::swap(A.lists, B.lists);
    std::swap(A.mm_lists, B.mm_lists);
    std::swap(A.mm_host_rows, B.mm_host_rows);
    std::swap(A.mm_host_blks, B.mm_host_blks);
    std::swap(A.nscales, B.nscales);
    std::swap(A.tile_slot, B.tile_slot);
    std::swap(A.d_leaf_begin, B.d_leaf_begin);
    std::swap(A.d_leaf_end, B.d_leaf_end);
    std::swap(A.t_xh, B.t_xh);
    std::swap(A.t_yh, B.t_yh);
    std::swap(A.t_x, B.t_x);
    std::swap(A.t_ynear, B.t_ynear);
    for (int w = 0; w < 2; ++w) {
        std::swap(A.mm_cfg[w], B.mm_cfg[w]);
        std::swap(A.mm_tuned[w], B.mm_tuned[w]);
    }
    std::swap(A.bytes_coupling, B.bytes_coupling);
    std::swap(A.bytes_dense, B.bytes_dense);
    std::swap(A.bytes_leaf, B.bytes_leaf);
    std::swap(A.bytes_transfer, B.bytes_transfer);
    std::swap(A.off_U, B.off_U);
    std::swap(A.off_VT, B.off_VT);
    std::swap(A.off_E, B.off_E);
    std::swap(A.off_FT, B.off_FT);
    std::swap(A.off_blk, B.off_blk);
    std::swap(A.basis_elems, B.basis_elems);
    std::swap(A.block_elems, B.block_elems);
}

}  // namespace

// Basis orthogonalization and projection of the coupling blocks in place
// (one basis tree, or a row and a column tree of their own).
void orthogonalize(h2_matrix_ &A, hipStream_t st) {
    const Structure &s = A.st;
    const int q = s.q;
    if (A.storage != H2_FP64) fail(H2_ERR_UNSUPPORTED, "orthogonalization needs FP64 storage");
    if (A.half) fail(H2_ERR_UNSUPPORTED, "orthogonalization of a matrix stored by halves");
    if (s.lmin > q) return;   // no coupling block: nothing to orthogonalize
    const int64_t nleaves = int64_t(1) << q, lf = Structure::first(q);
    for (int64_t j = 0; j < nleaves; ++j)
        if (s.size(lf + j) < s.lrank[q]) fail(H2_ERR_UNSUPPORTED, "a leaf holds fewer rows than the rank");
    for (int l = q; l > s.lmin; --l)
        if (2 * s.lrank[l] < s.lrank[l - 1]) fail(H2_ERR_UNSUPPORTED, "a level's rank exceeds twice its children's");
    std::vector<h2::ProjDesc> proj;
    {
        int64_t total = 0;
        for (const auto &B : s.coupling) total += B.blocks();
        proj.reserve(size_t(total));
    }
    int64_t fi = 0;
    for (int l = 0; l <= q; ++l) {
        const h2::Bsr &B = s.coupling[l];
        const int64_t f = Structure::first(l);
        for (int64_t i = 0; i < (int64_t(1) << l); ++i)
            for (int32_t b = B.rowptr[i]; b < B.rowptr[i + 1]; ++b, ++fi)
                proj.push_back({A.off_blk[fi], A.off_blk[fi], f + i, f + B.colidx[b], s.lrank[l], s.lrank[l]});
    }
    DeviceArena scratch;
    const int kmax = s.rank;
    h2::OrthLaunch L;
    L.basis = static_cast<double *>(A.basis);
    L.blocks = static_cast<double *>(A.blocks);
    L.T = static_cast<double *>(scratch.alloc((s.nnodes * int64_t(kmax) * kmax + h2::PROJ_T_PAD) * 8));
    if (!A.symmetric)
        L.T_col = static_cast<double *>(scratch.alloc((s.nnodes * int64_t(kmax) * kmax + h2::PROJ_T_PAD) * 8));
    L.off_U = scratch.upload(A.off_U, st);
    L.off_VT = scratch.upload(A.off_VT, st);
    L.off_E = scratch.upload(A.off_E, st);
    L.off_FT = scratch.upload(A.off_FT, st);
    L.leaf_begin = A.d_leaf_begin;
    L.leaf_end = A.d_leaf_end;
    L.proj = scratch.upload(proj, st);
    L.nleaves = nleaves;
    L.first_leaf = lf;
    L.nproj = int64_t(proj.size());
    L.level_rank = s.lrank.data();
    L.q = q;
    L.lmin = s.lmin;
    L.kmax = kmax;
    check_hip(h2::launch_orthogonalize(L, st), "orthogonalization launch");
    check_hip(hipStreamSynchronize(st), "orthogonalization");
}

// The transposed matrix as a new handle: A^T = sum over levels of V S^T U^T
// plus D^T (Sec. 2.2), i.e. the row and column trees exchange roles.  The
// tree, ranks and permutation are A's; every level's block-sparse rows are
// transposed (block (i, j) of A becomes block (j, i), rows listing their
// columns in increasing order); blocks, bases and transfers are copied
// transposed on the device (U'_j = V_j, V'_j = U_j, E'_c = F_c, F'_c = E_c),
// values unchanged (BF16 codes and scales included).
h2_matrix_ *transpose_matrix(h2_matrix_ &A, hipStream_t st) {
    if (A.half) fail(H2_ERR_UNSUPPORTED, "a matrix stored by halves is symmetric: it is its own transpose");
    const Structure &s = A.st;
    const int q = s.q;
    const std::vector<int> &kl = s.lrank;
    const int64_t nleaves = int64_t(1) << q, lf = Structure::first(q);
    std::unique_ptr<h2_matrix_> B(new h2_matrix_());
    B->st = s;
    B->storage = A.storage;
    B->basis_kind = A.basis_kind;
    B->block_kind = A.block_kind;
    B->vec_f64 = A.vec_f64;
    B->symmetric = A.symmetric;
    // transposed rows; for block t of B (fill order): the block of A it copies and that block's size
    int64_t total = s.dense.blocks();
    for (int l = 0; l <= q; ++l) total += s.coupling[l].blocks();
    const size_t nblk = size_t(total);
    std::vector<int64_t> src_fill(nblk);
    std::vector<int32_t> src_R(nblk), src_C(nblk);
    // out = in^T (rows: block columns of in); from[pos] = the block of in that block pos of out mirrors
    auto transpose_bsr = [](const h2::Bsr &in, int64_t rows, h2::Bsr &out, std::vector<int32_t> &from) {
        out.rowptr.assign(size_t(rows + 1), 0);
        for (int32_t c : in.colidx) ++out.rowptr[size_t(c) + 1];
        for (int64_t i = 0; i < rows; ++i) out.rowptr[i + 1] += out.rowptr[i];
        out.colidx.assign(in.colidx.size(), 0);
        from.assign(in.colidx.size(), 0);
        std::vector<int32_t> next(out.rowptr.begin(), out.rowptr.end() - 1);
        for (int64_t i = 0; i < rows; ++i)
            for (int32_t t = in.rowptr[i]; t < in.rowptr[i + 1]; ++t) {
                const int32_t pos = next[in.colidx[t]]++;
                out.colidx[pos] = int32_t(i);
                from[pos] = t;
            }
    };
    std::vector<int32_t> from;
    int64_t fill0 = 0;
    for (int l = 0; l <= q; ++l) {
        transpose_bsr(s.coupling[l], int64_t(1) << l, B->st.coupling[l], from);
        for (size_t pos = 0; pos < from.size(); ++pos) {
            src_fill[size_t(fill0) + pos] = fill0 + from[pos];
            src_R[size_t(fill0) + pos] = src_C[size_t(fill0) + pos] = kl[l];
        }
        fill0 += s.coupling[l].blocks();
    }
    {
        // dense block t of A: rows of leaf i (its BSR row), columns of leaf colidx[t]
        std::vector<int32_t> row_of(s.dense.colidx.size());
        for (int64_t i = 0; i < nleaves; ++i)
            for (int32_t t = s.dense.rowptr[i]; t < s.dense.rowptr[i + 1]; ++t) row_of[t] = int32_t(i);
        transpose_bsr(s.dense, nleaves, B->st.dense, from);
        for (size_t pos = 0; pos < from.size(); ++pos) {
            const int32_t t = from[pos];
            src_fill[size_t(fill0) + pos] = fill0 + t;
            src_R[size_t(fill0) + pos] = int32_t(s.size(lf + row_of[t]));
            src_C[size_t(fill0) + pos] = int32_t(s.size(lf + s.dense.colidx[t]));
        }
    }
    int64_t ncoupling = 0;
    const std::vector<h2::FillDesc> fill = make_layout(*B, ncoupling);
    DeviceArena scratch;
    std::vector<h2::TransDesc> tb(fill.size()), tbas;
    h2::parallel_ranges(int64_t(fill.size()), 1 << 16, [&](int64_t f0, int64_t f1) {
        for (int64_t fb = f0; fb < f1; ++fb)
            tb[fb] = {A.off_blk[size_t(src_fill[fb])], B->off_blk[fb], src_R[fb], src_C[fb]};
    });
    if (s.lmin <= q) {
        tbas.reserve(size_t(2 * s.nnodes));
        for (int64_t j = 0; j < nleaves; ++j) {
            const int m = int(s.size(lf + j));
            tbas.push_back({A.off_VT[j], B->off_U[j], kl[q], m});   // U'_j = (V_j^T)^T
            tbas.push_back({A.off_U[j], B->off_VT[j], m, kl[q]});   // V'_j^T = U_j^T
        }
        for (int l = s.lmin + 1; l <= q; ++l)
            for (int64_t c = Structure::first(l); c < Structure::first(l + 1); ++c) {
                tbas.push_back({A.off_FT[c], B->off_E[c], kl[l - 1], kl[l]});   // E'_c = (F_c^T)^T
                tbas.push_back({A.off_E[c], B->off_FT[c], kl[l], kl[l - 1]});   // F'_c^T = E_c^T
            }
    }
    check_hip(h2::launch_transpose_blocks(A.block_kind, A.blocks, B->blocks, scratch.upload(tb, st),
                                          int64_t(tb.size()), st),
              "transpose launch");
    check_hip(h2::launch_transpose_blocks(A.basis_kind, A.basis, B->basis, scratch.upload(tbas, st),
                                          int64_t(tbas.size()), st),
              "transpose launch");
    if (A.block_kind == h2::ELEM_BF16 && A.nscales > 0) {
        std::vector<float> sa(size_t(A.nscales)), sb(fill.size());
        check_hip(hipMemcpyAsync(sa.data(), A.scales, sa.size() * 4, hipMemcpyDeviceToHost, st), "hipMemcpyAsync");
        check_hip(hipStreamSynchronize(st), "transpose scales");
        for (size_t fb = 0; fb < fill.size(); ++fb) sb[fb] = sa[size_t(src_fill[fb])];
        check_hip(hipMemcpyAsync(B->scales, sb.data(), sb.size() * 4, hipMemcpyHostToDevice, st), "hipMemcpyAsync");
    }
    check_hip(hipStreamSynchronize(st), "transpose");
    build_lists(*B, fill, ncoupling, st);
    return B.release();
}

// Algebraic compression (Sec. 5): orthogonalization, basis generation,
// truncation with relative threshold eps (rank of a level: the largest count
// of kept singular values over its nodes, of both trees when rows and columns
// have their own), projection of the coupling blocks into the truncated bases;
// the representation is rebuilt with the new ranks.
void compress(h2_matrix_ &A, double eps, hipStream_t st, int *ranks_out) {
    if (!(eps >= 0.0) || !std::isfinite(eps)) fail(H2_ERR_INVALID_ARG, "eps must be finite and >= 0");
    if (A.batch_refs > 0) fail(H2_ERR_INVALID_ARG, "the matrix belongs to a batch (free the batch first)");
    if (A.storage != H2_FP64) fail(H2_ERR_UNSUPPORTED, "compression needs FP64 storage");
    if (A.half) fail(H2_ERR_UNSUPPORTED, "compression of a matrix stored by halves");
    // One basis tree for rows and columns (V = U, F = E): whether S_ji = S_ij^T
    // for every coupling block, decided before the orthogonalization (which
    // keeps the symmetry only up to rounding); if not, the one tree also serves
    // block columns that differ from the block rows, and the basis generation
    // stacks both.  Two trees: each from its own blocks (rows / columns).
    const bool two = !A.symmetric;
    const bool sym = !two && coupling_symmetric(A, st);
    orthogonalize(A, st);
    const Structure &s = A.st;
    const int q = s.q, lmin = s.lmin, kmax = s.rank;
    const std::vector<int> kr = s.lrank;
    std::vector<int> kt = kr;
    if (lmin <= q) {
        const int64_t nleaves = int64_t(1) << q, lf = Structure::first(q);
        // coupling blocks in BSR order (all levels) and the first block of every node's row
        std::vector<h2::ProjDesc> blk;
        std::vector<int64_t> row_start(s.nnodes + 1);
        {
            int64_t total = 0;
            for (const auto &B : s.coupling) total += B.blocks();
            blk.reserve(size_t(total));
            int64_t fi = 0;
            for (int l = 0; l <= q; ++l) {
                const h2::Bsr &B = s.coupling[l];
                const int64_t f = Structure::first(l);
                for (int64_t i = 0; i < (int64_t(1) << l); ++i) {
                    row_start[f + i] = int64_t(blk.size());
                    for (int32_t b = B.rowptr[i]; b < B.rowptr[i + 1]; ++b, ++fi)
                        blk.push_back({A.off_blk[fi], 0, f + i, f + B.colidx[b], kr[l], 0});
                }
            }
            row_start[s.nnodes] = int64_t(blk.size());
        }
        // blocks of every block column (by column, rows increasing)
        std::vector<int64_t> col_blk, col_start(s.nnodes + 1, 0);
        if (!sym) {
            int64_t fi = 0;
            std::vector<std::vector<int64_t>> per_col;
            for (int l = 0; l <= q; ++l) {
                const h2::Bsr &B = s.coupling[l];
                const int64_t f = Structure::first(l), rows = int64_t(1) << l;
                per_col.assign(size_t(rows), {});
                for (int64_t i = 0; i < rows; ++i)
                    for (int32_t b = B.rowptr[i]; b < B.rowptr[i + 1]; ++b, ++fi)
                        per_col[size_t(B.colidx[b])].push_back(A.off_blk[size_t(fi)]);
                for (int64_t jc = 0; jc < rows; ++jc) {
                    col_start[f + jc] = int64_t(col_blk.size());
                    col_blk.insert(col_blk.end(), per_col[size_t(jc)].begin(), per_col[size_t(jc)].end());
                }
            }
            col_start[s.nnodes] = int64_t(col_blk.size());
        }
        DeviceArena scratch;
        const int64_t tree = s.nnodes * int64_t(kmax) * kmax;
        const int64_t maxlevel = std::max<int64_t>(nleaves, 1);
        // the launch of one tree: its bases, R, T, new bases and SVD buffers
        auto tree_launch = [&](bool column_tree) {
            h2::CompLaunch L{};
            L.basis = static_cast<const double *>(A.basis);
            L.blocks = static_cast<const double *>(A.blocks);
            L.off_U = scratch.upload(column_tree ? A.off_VT : A.off_U, st);
            L.off_E = scratch.upload(column_tree ? A.off_FT : A.off_E, st);
            L.b_t = L.x_t = column_tree ? 1 : 0;
            L.leaf_begin = A.d_leaf_begin;
            L.leaf_end = A.d_leaf_end;
            L.blk = scratch.upload(blk, st);
            L.row_start = scratch.upload(row_start, st);
            L.use_rows = column_tree ? 0 : 1;
            L.columns = (column_tree || (!two && !sym)) ? 1 : 0;
            L.col_blk = scratch.upload(col_blk, st);
            L.col_start = scratch.upload(col_start, st);
            L.R = static_cast<double *>(scratch.alloc(tree * 8));
            L.T = static_cast<double *>(scratch.alloc((tree + h2::PROJ_T_PAD) * 8));
            L.Enew = static_cast<double *>(scratch.alloc(tree * 8));
            L.X = static_cast<double *>(scratch.alloc(maxlevel * h2::COMP_XSLOT * 8));
            L.sigma = static_cast<double *>(scratch.alloc(maxlevel * 64 * 8));
            L.count = static_cast<int32_t *>(scratch.alloc(maxlevel * 4));
            L.Unew = static_cast<double *>(scratch.alloc(nleaves * h2::COMP_USLOT * 8));
            L.first_leaf = lf;
            L.nleaves = nleaves;
            L.kmax = kmax;
            return L;
        };
        std::vector<h2::CompLaunch> trees{tree_launch(false)};
        if (two) trees.push_back(tree_launch(true));
        // basis generation, top-down (Sec. 5.2)
        for (const h2::CompLaunch &L : trees)
            for (int l = lmin; l <= q; ++l)
                check_hip(h2::launch_basis_generation(L, l, kr[l], l > lmin ? kr[l - 1] : 0, l > lmin, st),
                          "basis generation launch");
        // truncation, bottom-up (Sec. 5.3); a level's rank is the largest kept count over its nodes
        // (of both trees)
        std::vector<int32_t> cnt;
        auto level_rank = [&](int64_t nodes, int bound) {
            int r = 1;
            for (const h2::CompLaunch &L : trees) {
                cnt.resize(size_t(nodes));
                check_hip(hipMemcpyAsync(cnt.data(), L.count, size_t(nodes) * 4, hipMemcpyDeviceToHost, st),
                          "hipMemcpyAsync");
                check_hip(hipStreamSynchronize(st), "truncation");
                for (int32_t c : cnt) r = std::max(r, int(c));
            }
            return std::min(r, bound);
        };
        for (const h2::CompLaunch &L : trees)
            check_hip(h2::launch_truncate_leaves(L, kr[q], eps, st), "truncation launch");
        kt[q] = level_rank(nleaves, kr[q]);
        for (const h2::CompLaunch &L : trees)
            check_hip(h2::launch_truncate_leaves_apply(L, kr[q], kt[q], st), "truncation launch");
        for (int l = q; l > lmin; --l) {
            for (const h2::CompLaunch &L : trees)
                check_hip(h2::launch_truncate_level(L, l, kr[l], kt[l], kr[l - 1], eps, st), "truncation launch");
            kt[l - 1] = level_rank(int64_t(1) << (l - 1), std::min(kr[l - 1], 2 * kt[l]));
            for (const h2::CompLaunch &L : trees)
                check_hip(h2::launch_truncate_level_apply(L, l, kr[l], kt[l], kr[l - 1], kt[l - 1], st),
                          "truncation launch");
        }
        for (int l = 0; l < lmin; ++l) kt[l] = kt[lmin];
        const h2::CompLaunch &Lr = trees.front(), &Lc = trees.back();
        // the representation with the new ranks
        std::unique_ptr<h2_matrix_> B(new h2_matrix_());
        B->st = s;
        B->st.lrank = kt;
        B->st.rank = *std::max_element(kt.begin(), kt.end());
        B->storage = A.storage;
        B->basis_kind = A.basis_kind;
        B->block_kind = A.block_kind;
        B->vec_f64 = A.vec_f64;
        B->symmetric = A.symmetric;
        int64_t ncoupling = 0;
        const std::vector<h2::FillDesc> fill = make_layout(*B, ncoupling);
        std::vector<h2::PlaceDesc> pu, pv, pe, pf;
        for (int64_t j = 0; j < nleaves; ++j) {
            const int m = int(s.size(lf + j));
            pu.push_back({j * h2::COMP_USLOT, B->off_U[j], m, kt[q], 64, 0});
            pv.push_back({j * h2::COMP_USLOT, B->off_VT[j], kt[q], m, 64, 1});
        }
        for (int l = lmin + 1; l <= q; ++l)
            for (int64_t c = Structure::first(l); c < Structure::first(l + 1); ++c) {
                pe.push_back({c * kmax * kmax, B->off_E[c], kt[l], kt[l - 1], kmax, 0});
                pf.push_back({c * kmax * kmax, B->off_FT[c], kt[l - 1], kt[l], kmax, 1});
            }
        double *nbasis = static_cast<double *>(B->basis);
        check_hip(h2::launch_place(Lr.Unew, nbasis, scratch.upload(pu, st), int64_t(pu.size()), st), "place launch");
        check_hip(h2::launch_place(Lc.Unew, nbasis, scratch.upload(pv, st), int64_t(pv.size()), st), "place launch");
        check_hip(h2::launch_place(Lr.Enew, nbasis, scratch.upload(pe, st), int64_t(pe.size()), st), "place launch");
        check_hip(h2::launch_place(Lc.Enew, nbasis, scratch.upload(pf, st), int64_t(pf.size()), st), "place launch");
        for (int l = 0; l <= q; ++l)   // the blocks of level l: rows first(l) .. first(l + 1) - 1
            for (int64_t i = row_start[Structure::first(l)]; i < row_start[Structure::first(l + 1)]; ++i) {
                blk[size_t(i)].out = B->off_blk[size_t(i)];
                blk[size_t(i)].kout = kt[l];
            }
        check_hip(h2::launch_project(static_cast<const double *>(A.blocks), static_cast<double *>(B->blocks),
                                     scratch.upload(blk, st), int64_t(blk.size()), Lr.T, Lc.T, kmax, st, false),
                  "projection launch");
        if (int64_t(fill.size()) > ncoupling) {   // dense blocks: same sizes and order
            const int64_t from = A.off_blk[size_t(ncoupling)], to = B->off_blk[size_t(ncoupling)];
            check_hip(hipMemcpyAsync(static_cast<double *>(B->blocks) + to, static_cast<const double *>(A.blocks) + from,
                                     size_t(A.block_elems - from) * 8, hipMemcpyDeviceToDevice, st),
                      "hipMemcpyAsync");
        }
        check_hip(hipStreamSynchronize(st), "compression");
        build_lists(*B, fill, ncoupling, st);
        adopt(A, *B);
    }
    if (ranks_out)
        for (int l = 0; l <= q; ++l) ranks_out[l] = kt[l];
}

}  // namespace h2i

using namespace h2i;

extern "C" {

h2_status h2_transpose(h2_handle A, void *stream, h2_handle *out) {
    if (out) *out = nullptr;
    try {
        if (!A || !out) fail(H2_ERR_INVALID_ARG, "NULL argument");
        if (A->structure_only) fail(H2_ERR_INVALID_ARG, "structure-only handle");
        *out = transpose_matrix(*A, static_cast<hipStream_t>(stream));
        return H2_OK;
    } catch (const Failure &f) {
        g_last_error = f.what;
        return f.code;
    } catch (const std::bad_alloc &) {
        g_last_error = "host allocation failed";
        return H2_ERR_OOM;
    } catch (...) {
        g_last_error = "internal error";
        return H2_ERR_INTERNAL;
    }
}

h2_status h2_compress(h2_handle A, double eps, int *level_rank, void *stream) {
    try {
        if (!A) fail(H2_ERR_INVALID_ARG, "NULL handle");
        if (A->structure_only) fail(H2_ERR_INVALID_ARG, "structure-only handle");
        compress(*A, eps, static_cast<hipStream_t>(stream), level_rank);
        return H2_OK;
    } catch (const Failure &f) {
        g_last_error = f.what;
        return f.code;
    } catch (const std::bad_alloc &) {
        g_last_error = "host allocation failed";
        return H2_ERR_OOM;
    } catch (...) {
        g_last_error = "internal error";
        return H2_ERR_INTERNAL;
    }
}

h2_status h2_orthogonalize(h2_handle A, void *stream) {
    try {
        if (!A) fail(H2_ERR_INVALID_ARG, "NULL handle");
        if (A->structure_only) fail(H2_ERR_INVALID_ARG, "structure-only handle");
        orthogonalize(*A, static_cast<hipStream_t>(stream));
        return H2_OK;
    } catch (const Failure &f) {
        g_last_error = f.what;
        return f.code;
    } catch (const std::bad_alloc &) {
        g_last_error = "host allocation failed";
        return H2_ERR_OOM;
    } catch (...) {
        g_last_error = "internal error";
        return H2_ERR_INTERNAL;
    }
}

}  // extern "C"
