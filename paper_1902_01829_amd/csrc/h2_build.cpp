// Construction of the H^2 representation on the device (from points, or
// from the arrays of an existing representation), its work lists, and the
// export of its stored arrays.
#include "h2_internal.h"

#include <future>
#include <numeric>
#include <unordered_map>
#include <unordered_set>

namespace h2i {

namespace {

// Host conversion of a column-major FP64 block (R x C, leading dimension R)
// into the device layout of its element kind: 16-byte column groups (see
// block_elems), transposed on request, FP32 rounded to nearest even, BF16
// with one FP32 scale (max |fp32(a)|) and codes rounded to nearest even --
// the same rules as the device fill kernels.
uint16_t host_bf16_rne(float f) {
    uint32_t u;
    std::memcpy(&u, &f, 4);
    return uint16_t((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

}  // namespace

// Wavefront items of a tile list in dispatch order (see h2::MmLaunch): one
// item per 32-row half of each row, the list cut into MM_XCDS contiguous
// ranges of about equal work (per block: its columns rounded up to the
// 16-column MFMA step, plus a fixed cost), each range padded to whole
// workgroups, and range x's l-th workgroup placed at workgroup l * MM_XCDS + x.
namespace {

// Cost of a row's block loop (columns rounded to the MFMA step, plus a
// constant per block).
double row_work(const h2::RowDesc &r, const std::vector<h2::BlkDesc> &blks) {
    double w = 0.0;
    for (int32_t b = r.b0; b < r.b1; ++b) w += double((blks[b].C + 15) / 16 * 16 + 8);
    return w;
}

// Dispatch order of work units (usize items each, in list order): the list
// is cut into MM_XCDS contiguous ranges of about equal work, and range x's
// units fill workgroups wg = l * MM_XCDS + x (per_wg items each) in order, so
// that the workgroups of XCD x (wg % MM_XCDS == x) walk range x.
std::vector<int32_t> layout_units(const std::vector<int32_t> &units, int usize, const std::vector<double> &work,
                                  int per_wg) {
    constexpr int X = h2::MM_XCDS;
    const size_t n = work.size(), upw = size_t(per_wg / usize);
    double total = 0.0;
    for (double w : work) total += w;
    std::vector<size_t> cut(X + 1, n);   // range x = units [cut[x], cut[x+1])
    cut[0] = 0;
    double acc = 0.0;
    int x = 1;
    for (size_t i = 0; i < n && x < X; ++i) {
        while (x < X && acc >= total * x / X) cut[x++] = i;
        acc += work[i];
    }
    size_t per = 0;   // workgroups per XCD
    for (int r = 0; r < X; ++r) per = std::max(per, (cut[r + 1] - cut[r] + upw - 1) / upw);
    std::vector<int32_t> out(per * X * size_t(per_wg), -1);
    for (int r = 0; r < X; ++r)
        for (size_t i = cut[r]; i < cut[r + 1]; ++i) {
            const size_t l = (i - cut[r]) / upw, v = (i - cut[r]) % upw;
            for (int e = 0; e < usize; ++e) out[(l * X + r) * size_t(per_wg) + v * usize + e] = units[i * usize + e];
        }
    return out;
}

}  // namespace

std::vector<int32_t> wave_items(const std::vector<h2::RowDesc> &rows, const std::vector<h2::BlkDesc> &blks) {
    if (rows.size() >= (size_t(1) << 30)) fail(H2_ERR_UNSUPPORTED, "too many rows in one tile list");
    std::vector<int32_t> items;
    std::vector<double> work;
    for (size_t r = 0; r < rows.size(); ++r) {
        const double w = row_work(rows[r], blks);
        for (int mt = 0; mt * 32 < std::max(rows[r].R, 1); ++mt) {
            items.push_back(int32_t(r << 1) | mt);
            work.push_back(w);
        }
    }
    return layout_units(items, 1, work, 4);
}

std::vector<int32_t> pair_items(const std::vector<h2::RowDesc> &rows, const std::vector<h2::BlkDesc> &blks) {
    if (rows.size() >= (size_t(1) << 30)) fail(H2_ERR_UNSUPPORTED, "too many rows in one tile list");
    std::vector<int32_t> units;
    std::vector<double> work;
    int32_t single = -1;   // a row of at most 32 rows waiting for a partner
    double single_w = 0.0;
    for (size_t r = 0; r < rows.size(); ++r) {
        const double w = row_work(rows[r], blks);
        if (rows[r].R > 32) {
            units.push_back(int32_t(r << 1));
            units.push_back(int32_t(r << 1) | 1);
            work.push_back(2 * w);
        } else if (single < 0) {
            single = int32_t(r << 1);
            single_w = w;
        } else {
            units.push_back(single);
            units.push_back(int32_t(r << 1));
            work.push_back(single_w + w);
            single = -1;
        }
    }
    if (single >= 0) {
        units.push_back(single);
        units.push_back(-1);
        work.push_back(single_w);
    }
    return layout_units(units, 2, work, 2);
}

void convert_block(const double *src, int R, int C, bool transpose, int kind, void *dst, float *scale) {
    // element (r, c) of the stored block: src[r + c * R] (or src[c + r * C] transposed)
    auto val = [&](int r, int c) { return transpose ? src[c + int64_t(r) * C] : src[r + int64_t(c) * R]; };
    const int W = 16 / h2::elem_bytes(kind);
    const int64_t ne = h2::block_elems(R, C, kind);
    float s = 0.0f;
    if (kind == h2::ELEM_BF16)
        for (int c = 0; c < C; ++c)
            for (int r = 0; r < R; ++r) s = std::max(s, std::fabs(float(val(r, c))));
    for (int64_t e = 0; e < ne; ++e) {
        const int w = int(e % W);
        const int64_t t = e / W;
        const int r = int(t % R), c = int(t / R) * W + w;
        const double v = c < C ? val(r, c) : 0.0;
        if (kind == h2::ELEM_F64) static_cast<double *>(dst)[e] = v;
        else if (kind == h2::ELEM_F32) static_cast<float *>(dst)[e] = float(v);
        else static_cast<uint16_t *>(dst)[e] = s == 0.0f ? uint16_t(0) : host_bf16_rne(float(v) / s);
    }
    if (scale) *scale = s;
}

// Uploads converted blocks through a bounded host staging buffer.
struct Stager {
    char *dev;
    int64_t elem;
    hipStream_t st;
    std::vector<char> buf;
    int64_t buf_off = 0;   // element offset of buf[0] on the device
    int64_t used = 0;      // bytes in buf
    static constexpr int64_t kCap = int64_t(64) << 20;
    Stager(void *d, int kind, hipStream_t s) : dev(static_cast<char *>(d)), elem(h2::elem_bytes(kind)), st(s) {
        buf.resize(kCap);
    }
    void flush() {
        if (used > 0) {
            check_hip(hipMemcpyAsync(dev + buf_off * elem, buf.data(), size_t(used), hipMemcpyHostToDevice, st),
                      "hipMemcpyAsync");
            check_hip(hipStreamSynchronize(st), "upload blocks");
        }
        buf_off += used / elem;
        used = 0;
    }
    // Room for a block of ne elements placed at element offset off (blocks arrive in offset order).
    void *place(int64_t off, int64_t ne) {
        const int64_t bytes = ne * elem;
        if (off * elem != buf_off * elem + used || used + bytes > kCap) {
            flush();
            buf_off = off;
        }
        if (bytes > kCap) fail(H2_ERR_INTERNAL, "block larger than the staging buffer");
        void *p = buf.data() + used;
        used += bytes;
        return p;
    }
};

// The device representation's layout for the structure's level ranks: sets
// the offsets and byte counts of A, allocates its regions (basis, blocks,
// scales) and returns the fill list (coupling blocks level by level in BSR
// order, then dense blocks; stored by halves, only the blocks with column >=
// row, A.blk_store mapping every block of the lists to its stored block);
// ncoupling receives the number of stored coupling blocks.
std::vector<h2::FillDesc> make_layout(h2_matrix_ &A, int64_t &ncoupling) {
    const Structure &s = A.st;
    const int q = s.q;
    const std::vector<int> &kl = s.lrank;
    const int64_t nleaves = int64_t(1) << q, lf = Structure::first(q);
    const bool lowrank = s.lmin <= q;
    const int bk = A.basis_kind, sk = A.block_kind;

    // basis region: U_j, V_j^T per leaf; E_c, F_c^T per node of levels lmin+1..q
    std::vector<int64_t> off_U(nleaves), off_VT(nleaves);
    std::vector<int64_t> off_E(s.nnodes, -1), off_FT(s.nnodes, -1);
    int64_t nb = 0;
    for (int64_t j = 0; j < nleaves; ++j) {
        const int m = int(s.size(lf + j));
        off_U[j] = nb;
        nb += h2::block_elems(m, kl[q], bk);
        off_VT[j] = nb;
        nb += h2::block_elems(kl[q], m, bk);
    }
    const int64_t leaf_elems = nb;
    if (lowrank)
        for (int l = s.lmin + 1; l <= q; ++l)
            for (int64_t c = Structure::first(l); c < Structure::first(l + 1); ++c) {
                off_E[c] = nb;
                nb += h2::block_elems(kl[l], kl[l - 1], bk);
                off_FT[c] = nb;
                nb += h2::block_elems(kl[l - 1], kl[l], bk);
            }
    const int64_t eb = h2::elem_bytes(bk), sb = h2::elem_bytes(sk);
    A.bytes_leaf = lowrank ? leaf_elems * eb : 0;
    A.bytes_transfer = (nb - leaf_elems) * eb;

    // block region: coupling blocks level by level in BSR order, then dense
    // blocks; stored by halves, only the blocks with column >= row
    std::vector<h2::FillDesc> fill;
    std::vector<int64_t> store;   // per block of the lists: stored index, or -1 until linked
    {
        int64_t total = s.dense.blocks();
        for (int l = 0; l <= q; ++l) total += s.coupling[l].blocks();
        fill.reserve(size_t(total));
        store.reserve(size_t(total));
    }
    int64_t ns = 0;
    // Stored by halves: each block below the diagonal takes the index of its
    // mirror; the pattern must be symmetric, with every pair listed once.
    auto link_mirrors = [&](const h2::Bsr &B, int64_t nrows, size_t base) {
        std::unordered_set<uint64_t> seen;
        std::unordered_map<uint64_t, int64_t> upper;
        for (int64_t i = 0; i < nrows; ++i)
            for (int32_t b = B.rowptr[i]; b < B.rowptr[i + 1]; ++b) {
                const uint64_t key = (uint64_t(i) << 32) | uint32_t(B.colidx[b]);
                if (!seen.insert(key).second) fail(H2_ERR_INVALID_ARG, "half storage: a block pair listed twice");
                if (B.colidx[b] >= i) upper.emplace(key, store[base + size_t(b)]);
            }
        for (int64_t i = 0; i < nrows; ++i)
            for (int32_t b = B.rowptr[i]; b < B.rowptr[i + 1]; ++b)
                if (B.colidx[b] < i) {
                    const auto it = upper.find((uint64_t(uint32_t(B.colidx[b])) << 32) | uint64_t(i));
                    if (it == upper.end()) fail(H2_ERR_INVALID_ARG, "half storage: block pattern not symmetric");
                    store[base + size_t(b)] = -(it->second + 1);
                }
    };
    for (int l = 0; l <= q; ++l) {
        const h2::Bsr &B = s.coupling[l];
        const int64_t f = Structure::first(l);
        const size_t base = store.size();
        for (int64_t i = 0; i < (int64_t(1) << l); ++i)
            for (int32_t b = B.rowptr[i]; b < B.rowptr[i + 1]; ++b) {
                if (A.half && B.colidx[b] < i) {
                    store.push_back(-1);
                    continue;
                }
                store.push_back(int64_t(fill.size()));
                fill.push_back({ns, int32_t(f + i), int32_t(f + B.colidx[b]), int32_t(fill.size()),
                                h2::FILL_COUPLING});
                ns += h2::block_elems(kl[l], kl[l], sk);
            }
        if (A.half) link_mirrors(B, int64_t(1) << l, base);
    }
    const int64_t coupling_elems = ns;
    ncoupling = int64_t(fill.size());
    {
        const size_t base = store.size();
        for (int64_t i = 0; i < nleaves; ++i)
            for (int32_t b = s.dense.rowptr[i]; b < s.dense.rowptr[i + 1]; ++b) {
                if (A.half && s.dense.colidx[b] < i) {
                    store.push_back(-1);
                    continue;
                }
                const int64_t t = lf + s.dense.colidx[b];
                store.push_back(int64_t(fill.size()));
                fill.push_back({ns, int32_t(lf + i), int32_t(t), int32_t(fill.size()), h2::FILL_DENSE});
                ns += h2::block_elems(int(s.size(lf + i)), int(s.size(t)), sk);
            }
        if (A.half) link_mirrors(s.dense, nleaves, base);
    }
    if (A.half)
        A.blk_store = std::move(store);
    else
        A.blk_store.clear();
    const int64_t scale_bytes = sk == h2::ELEM_BF16 ? 4 : 0;
    A.off_U = std::move(off_U);
    A.off_VT = std::move(off_VT);
    A.off_E = std::move(off_E);
    A.off_FT = std::move(off_FT);
    A.off_blk.resize(fill.size());
    for (size_t i = 0; i < fill.size(); ++i) A.off_blk[i] = fill[i].a;
    A.bytes_coupling = coupling_elems * sb + scale_bytes * ncoupling;
    A.bytes_dense = (ns - coupling_elems) * sb + scale_bytes * (int64_t(fill.size()) - ncoupling);

    A.basis_elems = nb;
    A.block_elems = ns;
    A.basis = A.mem.alloc(nb * eb);
    A.blocks = A.mem.alloc(ns * sb);
    A.scales = static_cast<float *>(A.mem.alloc(std::max<int64_t>(1, int64_t(fill.size())) * 4));
    A.nscales = int64_t(fill.size());
    return fill;
}

// Layout of the representation, generation on the device (from points) or
// conversion of caller arrays (src), and the work lists of one product in
// launch order.  Ranks may differ per level (k_l); vectors and tiles use the
// largest rank as their node stride.
void build_device(h2_matrix_ &A, const h2_arrays *src, hipStream_t stream) {
    const Structure &s = A.st;
    const int k = s.rank, q = s.q;   // k: largest level rank
    const std::vector<int> &kl = s.lrank;
    const int64_t nleaves = int64_t(1) << q, lf = Structure::first(q);
    const bool lowrank = s.lmin <= q;
    const int bk = A.basis_kind, sk = A.block_kind;
    int64_t ncoupling = 0;
    const std::vector<h2::FillDesc> fill = make_layout(A, ncoupling);
    const std::vector<int64_t> &off_U = A.off_U, &off_VT = A.off_VT, &off_E = A.off_E, &off_FT = A.off_FT;
    std::vector<int64_t> leaf_node(nleaves);
    for (int64_t j = 0; j < nleaves; ++j) leaf_node[j] = lf + j;
    if (!src) {
        // generation of the representation on the device (Sec. 4.6)
        std::vector<double> cheb(s.cheb_p);
        for (int a = 0; a < s.cheb_p; ++a) cheb[a] = std::cos((2.0 * a + 1.0) * M_PI / (2.0 * s.cheb_p));
        DeviceArena scratch;   // geometry and fill lists, freed after the build
        if (A.mem.cap >= 0) scratch.cap = std::max<int64_t>(0, A.mem.cap - A.mem.bytes);
        h2::Geometry g;
        g.pts = scratch.upload(s.pts, stream);
        g.lo = scratch.upload(s.lo, stream);
        g.hi = scratch.upload(s.hi, stream);
        g.begin = scratch.upload(s.begin, stream);
        g.end = scratch.upload(s.end, stream);
        g.cheb = scratch.upload(cheb, stream);
        g.dim = s.dim;
        g.cheb_p = s.cheb_p;
        g.rank = k;
        g.corr_len = s.corr_len;
        const int64_t *d_leaf = scratch.upload(leaf_node, stream);
        const int64_t *d_offU = scratch.upload(off_U, stream);
        const int64_t *d_offVT = scratch.upload(off_VT, stream);
        const int64_t *d_offE = scratch.upload(off_E, stream);
        const int64_t *d_offFT = scratch.upload(off_FT, stream);
        const h2::FillDesc *d_fill = scratch.upload(fill, stream);
        check_hip(h2::launch_fill_bases(g, bk, A.basis, d_leaf, d_offU, d_offVT, nleaves, d_offE, d_offFT,
                                        lowrank ? s.nnodes : 0, stream),
                  "fill bases");
        check_hip(h2::launch_fill_blocks(g, sk, A.blocks, A.scales, d_fill, int64_t(fill.size()), stream),
                  "fill blocks");
        check_hip(hipStreamSynchronize(stream), "fill");
    } else {
        // caller arrays (column-major FP64) converted to the device layout
        {
            Stager up(A.basis, bk, stream);
            const int kq = kl[q];
            int64_t uoff = 0;   // offset of leaf j's m_j x k_q block in U and V
            for (int64_t j = 0; j < nleaves && lowrank; ++j) {
                const int m = int(s.size(lf + j));
                convert_block(src->U + uoff, m, kq, false, bk, up.place(off_U[j], h2::block_elems(m, kq, bk)),
                              nullptr);
                convert_block(src->V + uoff, kq, m, true, bk, up.place(off_VT[j], h2::block_elems(kq, m, bk)),
                              nullptr);
                uoff += int64_t(m) * kq;
            }
            int64_t eoff = 0;   // offset of node c's k_l x k_(l-1) block in E and F
            for (int l = 1; l <= q; ++l)
                for (int64_t c = Structure::first(l); c < Structure::first(l + 1); ++c) {
                    if (off_E[c] >= 0) {
                        convert_block(src->E + eoff, kl[l], kl[l - 1], false, bk,
                                      up.place(off_E[c], h2::block_elems(kl[l], kl[l - 1], bk)), nullptr);
                        convert_block(src->F + eoff, kl[l - 1], kl[l], true, bk,
                                      up.place(off_FT[c], h2::block_elems(kl[l - 1], kl[l], bk)), nullptr);
                    }
                    eoff += int64_t(kl[l]) * kl[l - 1];
                }
            up.flush();
        }
        {
            // every block of the lists: its source values and shape
            std::vector<const double *> bsrc;
            std::vector<int> bR, bC;
            for (int l = 0; l <= q; ++l) {
                const int64_t kk = int64_t(kl[l]) * kl[l];
                for (int64_t b = 0; b < s.coupling[l].blocks(); ++b) {
                    bsrc.push_back(src->S[l] + b * kk);
                    bR.push_back(kl[l]);
                    bC.push_back(kl[l]);
                }
            }
            int64_t doff = 0;
            for (int64_t i = 0; i < nleaves; ++i)
                for (int32_t b = s.dense.rowptr[i]; b < s.dense.rowptr[i + 1]; ++b) {
                    const int R = int(s.size(lf + i)), C = int(s.size(lf + s.dense.colidx[b]));
                    bsrc.push_back(src->D + doff);
                    bR.push_back(R);
                    bC.push_back(C);
                    doff += int64_t(R) * C;
                }
            if (A.half) {
                // stored by halves: V = U, F = E, and every block below the
                // diagonal the transpose of its mirror, value by value
                if (!A.symmetric) fail(H2_ERR_INVALID_ARG, "half storage needs V = U and F = E");
                std::vector<size_t> stored_at(fill.size());
                for (size_t b = 0; b < bsrc.size(); ++b)
                    if (A.blk_store[b] >= 0) stored_at[size_t(A.blk_store[b])] = b;
                for (size_t b = 0; b < bsrc.size(); ++b) {
                    if (A.blk_store[b] >= 0) continue;
                    const size_t m = stored_at[size_t(-A.blk_store[b] - 1)];
                    const int R = bR[b], C = bC[b];
                    bool same = bR[m] == C && bC[m] == R;
                    for (int c = 0; c < C && same; ++c)
                        for (int r = 0; r < R && same; ++r)
                            same = std::memcmp(bsrc[b] + r + int64_t(c) * R, bsrc[m] + c + int64_t(r) * C, 8) == 0;
                    if (!same) fail(H2_ERR_INVALID_ARG, "half storage: a block differs from its mirror's transpose");
                }
            }
            Stager up(A.blocks, sk, stream);
            std::vector<float> scales(fill.size(), 1.0f);
            for (size_t b = 0; b < bsrc.size(); ++b) {
                const int64_t fi = A.blk_store.empty() ? int64_t(b) : A.blk_store[b];
                if (fi < 0) continue;   // mirror of a stored block
                convert_block(bsrc[b], bR[b], bC[b], false, sk,
                              up.place(fill[size_t(fi)].a, h2::block_elems(bR[b], bC[b], sk)), &scales[size_t(fi)]);
            }
            up.flush();
            if (sk == h2::ELEM_BF16 && !scales.empty()) {
                check_hip(hipMemcpyAsync(A.scales, scales.data(), scales.size() * 4, hipMemcpyHostToDevice, stream),
                          "hipMemcpyAsync");
                check_hip(hipStreamSynchronize(stream), "upload scales");
            }
        }
    }
    build_lists(A, fill, ncoupling, stream);
}

// Vector workspace and work lists of the product for the layout of A.
void build_lists(h2_matrix_ &A, const std::vector<h2::FillDesc> &fill, int64_t ncoupling, hipStream_t stream) {
    const Structure &s = A.st;
    const int k = s.rank, q = s.q;
    const std::vector<int> &kl = s.lrank;
    const int64_t nleaves = int64_t(1) << q, lf = Structure::first(q);
    const bool lowrank = s.lmin <= q;
    const int bk = A.basis_kind, sk = A.block_kind;
    const std::vector<int64_t> &off_U = A.off_U, &off_VT = A.off_VT, &off_E = A.off_E, &off_FT = A.off_FT;

    // workspace: vector trees x^ and y^ (nnodes x k) and the near field (n)
    const int64_t vb = A.vec_f64 ? 8 : 4;
    A.xh = A.mem.alloc(s.nnodes * k * vb);
    A.yh = A.mem.alloc(s.nnodes * k * vb);
    A.ynear = A.mem.alloc(s.n * vb);

    // Work lists in launch order.  Rows are first built logically: each
    // operand names either a tree node's vector (x^ / y^) or a leaf's segment of
    // the point vectors (x, y_near, y); they are then encoded twice, with
    // single-vector offsets and with tile offsets for many right-hand sides.
    // A row's blocks are a range of one pool shared by the rows of a list
    // (a list of the 2^20-point matrix holds ~1.3M blocks: one allocation,
    // reused from list to list, instead of one per row).
    struct LBlk {
        int64_t a;
        int32_t C, sidx;
        bool point;
        int64_t id;
        int32_t slot;   // stored by halves: partial slot of the transposed product
    };
    struct LRow {
        bool point;      // output is a leaf segment (else a tree node)
        int64_t id;      // leaf index or node id
        bool has_init;   // add the current value (downsweep: y^; leaf phase: y_near)
        int R, sel;
        size_t b0, b1;   // its blocks: pool[b0, b1)
        size_t nb() const { return b1 - b0; }
    };
    std::vector<LBlk> pool;
    std::vector<LRow> L;
    auto add_row = [&](bool point, int64_t id, bool has_init, int R, int sel) {
        L.push_back({point, id, has_init, R, sel, pool.size(), pool.size()});
    };
    auto add_blk = [&](int64_t a, int32_t C, int32_t sidx, bool point, int64_t id) {
        pool.push_back({a, C, sidx, point, id, -1});
        L.back().b1 = pool.size();
    };
    const int64_t kp = (k + 15) / 16 * 16;
    int64_t mmax = 0;
    for (int64_t j = 0; j < nleaves; ++j) mmax = std::max(mmax, s.size(lf + j));
    A.tile_slot = (mmax + 15) / 16 * 16 * h2::MM_TILE;
    auto mv_off = [&](bool point, int64_t id) { return point ? s.begin[lf + id] : id * k; };
    auto mm_off = [&](bool point, int64_t id) { return point ? id * A.tile_slot : id * kp * h2::MM_TILE; };
    // enc 0: single-vector offsets into A.lists; enc 1: tile offsets into A.mm_lists.
    // Rows in the order of `order` (indices into L), else in L's order.
    // encode only reads L and the pool (two encodings may run at once);
    // commit uploads and records the list.
    struct Encoded {
        std::vector<RowDesc> rows;
        std::vector<BlkDesc> blks;
        std::vector<int32_t> items, pitems;   // tile lists
    };
    auto encode = [&](int enc, Phase ph, const std::vector<size_t> *order) {
        const size_t nr = order ? order->size() : L.size();
        size_t nblk = 0;
        for (size_t o = 0; o < nr; ++o) nblk += L[order ? (*order)[o] : o].nb();
        Encoded e;
        e.rows.reserve(nr);
        e.blks.reserve(nblk);
        for (size_t o = 0; o < nr; ++o) {
            const LRow &r = L[order ? (*order)[o] : o];
            RowDesc d;
            if (ph == PH_LEAF) {   // out: rows of y; init: y_near
                d.out = s.begin[lf + r.id];
                d.init = enc == 0 ? mv_off(true, r.id) : mm_off(true, r.id);
            } else {
                d.out = enc == 0 ? mv_off(r.point, r.id) : mm_off(r.point, r.id);
                d.init = !r.has_init ? -1 : enc == 0 ? mv_off(r.point, r.id) : mm_off(r.point, r.id);
            }
            d.b0 = int32_t(e.blks.size());
            for (size_t i = r.b0; i < r.b1; ++i) {
                const LBlk &b = pool[i];
                e.blks.push_back({b.a, enc == 0 ? mv_off(b.point, b.id) : mm_off(b.point, b.id), b.C, b.sidx});
            }
            d.b1 = int32_t(e.blks.size());
            d.R = r.R;
            d.sel = r.sel;
            e.rows.push_back(d);
        }
        if (enc == 1) {
            e.items = wave_items(e.rows, e.blks);
            e.pitems = pair_items(e.rows, e.blks);
        }
        return e;
    };
    auto commit = [&](int enc, Phase ph, int kind, const void *data, Encoded &&e) {
        WorkList w;
        w.phase = ph;
        w.kind = kind;
        w.data = data;
        w.nrows = int64_t(e.rows.size());
        w.rows = A.mem.upload(e.rows, stream);
        w.blks = A.mem.upload(e.blks, stream);
        if (enc == 1) {
            w.items = A.mem.upload(e.items, stream);
            w.nitems = int64_t(e.items.size());
            w.pitems = A.mem.upload(e.pitems, stream);
            w.npitems = int64_t(e.pitems.size());
        }
        (enc == 0 ? A.lists : A.mm_lists).push_back(w);
        if (enc == 1) {
            A.mm_host_rows.push_back(std::move(e.rows));
            A.mm_host_blks.push_back(std::move(e.blks));
        }
    };
    auto emit_one = [&](int enc, Phase ph, int kind, const void *data, const std::vector<size_t> *order) {
        commit(enc, ph, kind, data, encode(enc, ph, order));
    };
    auto clear = [&]() {
        L.clear();
        pool.clear();
    };
    auto emit = [&](Phase ph, int kind, const void *data) {
        emit_one(0, ph, kind, data, nullptr);
        emit_one(1, ph, kind, data, nullptr);
        clear();
    };
    if (lowrank) {
        // leaf projection x^_j = V_j^T x(j)   (Sec. 4.2)
        for (int64_t j = 0; j < nleaves; ++j) {
            const int64_t v = lf + j;
            add_row(false, v, false, kl[q], h2::ROW_IN_X);
            add_blk(off_VT[j], int32_t(s.size(v)), 0, true, j);
        }
        emit(PH_UP, bk, A.basis);
        // upsweep x^_p = F_c1^T x^_c1 + F_c2^T x^_c2 for levels q .. lmin+1   (Sec. 4.2)
        for (int l = q; l > s.lmin; --l) {
            for (int64_t p = Structure::first(l - 1); p < Structure::first(l); ++p) {
                add_row(false, p, false, kl[l - 1], 0);
                add_blk(off_FT[2 * p + 1], kl[l], 0, false, 2 * p + 1);
                add_blk(off_FT[2 * p + 2], kl[l], 0, false, 2 * p + 2);
            }
            emit(PH_UP, bk, A.basis);
        }
    }
    // tree multiplication y^_i = sum_j S_ij x^_j on all levels (Sec. 4.3) and the
    // dense near field y_near(i) = sum_j D_ij x(j) (Sec. 4.1) in one launch
    {
        // blocks by their index in the lists (coupling levels, then dense);
        // stored by halves, the mirrors of stored blocks are left out
        int64_t li = 0, total = s.dense.blocks();
        auto stored = [&](int64_t b) { return A.blk_store.empty() ? b : A.blk_store[size_t(b)]; };
        for (int l = 0; l <= q; ++l) total += s.coupling[l].blocks();
        pool.reserve(size_t(total));
        for (int l = 0; l < s.lmin && lowrank; ++l) li += s.coupling[l].blocks();
        if (lowrank)
            for (int l = s.lmin; l <= q; ++l) {
                const h2::Bsr &B = s.coupling[l];
                const int64_t f = Structure::first(l);
                for (int64_t i = 0; i < (int64_t(1) << l); ++i) {
                    add_row(false, f + i, false, kl[l], 0);
                    for (int32_t b = B.rowptr[i]; b < B.rowptr[i + 1]; ++b, ++li) {
                        const int64_t fi = stored(li);
                        if (fi >= 0) add_blk(fill[fi].a, kl[l], fill[fi].sidx, false, f + B.colidx[b]);
                    }
                }
            }
        li = 0;
        for (int l = 0; l <= q; ++l) li += s.coupling[l].blocks();
        for (int64_t i = 0; i < nleaves; ++i) {
            add_row(true, i, false, int(s.size(lf + i)), h2::ROW_IN_X | h2::ROW_OUT_P);
            for (int32_t b = s.dense.rowptr[i]; b < s.dense.rowptr[i + 1]; ++b, ++li) {
                const int64_t t = s.dense.colidx[b], fi = stored(li);
                if (fi >= 0) add_blk(fill[fi].a, int32_t(s.size(lf + t)), fill[fi].sidx, true, t);
            }
        }
        if (A.half) {
            // One launch reads every stored block once for both of its
            // products.  Its wavefronts take groups of up to HALF_GROUP_ROWS
            // consecutive block rows of one kind (the list's spatial order:
            // coupling rows level by level, then leaf rows), whose transposed
            // products of one column segment are added in LDS, rows in order,
            // and written to one partial slot per segment and group (when a
            // group has more segments than HALF_LDS_SLOTS, the most shared
            // ones get LDS slots and the blocks of the others slots of their
            // own).  Slots are numbered by segment, and a second launch adds
            // each segment's slots to its row sum, in order (deterministic).
            struct Col {
                bool point;
                int64_t id;
                int32_t C;
            };
            struct Grp {
                size_t r0, r1;
                std::vector<Col> cols;   // merged segments, first appearance first
                int64_t nblk;
            };
            auto off_diagonal = [&](const LRow &r, const LBlk &b) { return b.point != r.point || b.id != r.id; };
            auto find_col = [](const std::vector<Col> &cols, const LBlk &b) {
                for (size_t c = 0; c < cols.size(); ++c)
                    if (cols[c].point == b.point && cols[c].id == b.id) return int(c);
                return -1;
            };
            // Rows per group: at most HALF_GROUP_ROWS, and few enough that the
            // groups fill the wavefronts the device holds at least three times
            // over (with fewer rounds the last one leaves compute units idle:
            // measured on the 3-D 2^19-point matrix, whose 24,544 block rows
            // in groups of four made the FP32 and BF16 products 6-12 %
            // slower, 1.5 rounds, while the FP64 ones, at half the
            // wavefronts per CU, gained 1-4 % in 2-D (6 rounds) and 3-D (3)).
            size_t group_rows = 1;
            {
                int dev = 0, cus = 0, per_cu = 0;
                check_hip(hipGetDevice(&dev), "hipGetDevice");
                check_hip(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev), "device attribute");
                check_hip(h2::stream_half_workgroups_per_cu(sk, A.vec_f64, &per_cu), "occupancy query");
                const size_t waves = size_t(std::max(1, cus)) * size_t(std::max(1, per_cu)) * 4;
                group_rows = std::min(size_t(h2::HALF_GROUP_ROWS), std::max(size_t(1), L.size() / (3 * waves)));
                // test-only override (environment variable H2MV_HALF_GROUP_ROWS,
                // 1 .. HALF_GROUP_ROWS), so that small matrices run the grouped path
                if (const char *e = std::getenv("H2MV_HALF_GROUP_ROWS")) {
                    const long v = std::atol(e);
                    if (v >= 1 && v <= h2::HALF_GROUP_ROWS) group_rows = size_t(v);
                }
            }
            std::vector<Grp> groups;
            std::vector<Col> all;   // a group's segments, first appearance first
            std::vector<int> mult;  // and how many of its blocks fall in each
            std::vector<size_t> ord;
            for (size_t r = 0; r < L.size();) {
                Grp G{r, r, {}, 0};
                while (G.r1 < L.size() && G.r1 - G.r0 < group_rows && L[G.r1].point == L[G.r0].point) {
                    G.nblk += int64_t(L[G.r1].nb());
                    ++G.r1;
                }
                all.clear();
                mult.clear();
                for (size_t q = G.r0; q < G.r1; ++q)
                    for (size_t b = L[q].b0; b < L[q].b1; ++b) {
                        if (!off_diagonal(L[q], pool[b])) continue;
                        const int c = find_col(all, pool[b]);
                        if (c >= 0) {
                            ++mult[size_t(c)];
                        } else {
                            all.push_back({pool[b].point, pool[b].id, pool[b].C});
                            mult.push_back(1);
                        }
                    }
                // LDS slots: every segment if they fit, else the most shared
                // ones (a segment of a single block gains nothing from one)
                ord.resize(all.size());
                std::iota(ord.begin(), ord.end(), size_t(0));
                std::stable_sort(ord.begin(), ord.end(), [&](size_t x, size_t y) { return mult[x] > mult[y]; });
                const bool fit = all.size() <= size_t(h2::HALF_LDS_SLOTS);
                for (size_t i = 0; i < ord.size() && i < size_t(h2::HALF_LDS_SLOTS); ++i)
                    if (fit || mult[ord[i]] > 1) G.cols.push_back(all[ord[i]]);
                for (size_t q = G.r0; q < G.r1; ++q)
                    for (size_t b = L[q].b0; b < L[q].b1; ++b) {
                        LBlk &lb = pool[b];
                        if (!off_diagonal(L[q], lb)) {
                            lb.slot = -1;
                            continue;
                        }
                        const int c = find_col(G.cols, lb);
                        lb.slot = c >= 0 ? c : -2;   // -2: a slot of its own, numbered below
                    }
                groups.push_back(std::move(G));
                r = groups.back().r1;
            }
            // longest groups first, so the wavefronts that start last are the short ones
            std::stable_sort(groups.begin(), groups.end(), [](const Grp &x, const Grp &y) { return x.nblk > y.nblk; });
            // partial slots: one per merged segment of a group, one per block without an LDS slot
            struct Ent {
                bool point;
                int64_t id;
                int32_t C;
                size_t gslot_pos;   // merged: position in gslot; else SIZE_MAX
                size_t blk;         // own slot: the block's pool index
            };
            std::vector<Ent> ents;
            std::vector<int32_t> gslot;
            std::vector<h2::HalfGroup> hg;
            std::vector<RowDesc> rows;
            std::vector<BlkDesc> blks;
            std::vector<int32_t> slots;
            rows.reserve(L.size());
            blks.reserve(pool.size());
            slots.reserve(pool.size());
            for (const Grp &G : groups) {
                h2::HalfGroup d;
                d.r0 = int32_t(rows.size());
                d.s0 = int32_t(gslot.size());
                for (const Col &c : G.cols) {
                    ents.push_back({c.point, c.id, c.C, gslot.size(), 0});
                    gslot.push_back(-1);
                }
                for (size_t r = G.r0; r < G.r1; ++r) {
                    const LRow &row = L[r];
                    RowDesc rd;
                    rd.out = mv_off(row.point, row.id);
                    rd.init = -1;
                    rd.R = row.R;
                    rd.sel = row.sel;
                    rd.b0 = int32_t(blks.size());
                    for (size_t i = row.b0; i < row.b1; ++i) {
                        const LBlk &b = pool[i];
                        if (b.slot == -2) ents.push_back({b.point, b.id, b.C, SIZE_MAX, blks.size()});
                        blks.push_back({b.a, mv_off(b.point, b.id), b.C, b.sidx});
                        slots.push_back(b.slot);
                    }
                    rd.b1 = int32_t(blks.size());
                    rows.push_back(rd);
                }
                d.r1 = int32_t(rows.size());
                d.s1 = int32_t(gslot.size());
                hg.push_back(d);
            }
            std::stable_sort(ents.begin(), ents.end(), [](const Ent &x, const Ent &y) {
                return x.point != y.point ? x.point < y.point : x.id < y.id;
            });
            if (ents.size() >= (size_t(1) << 30)) fail(H2_ERR_UNSUPPORTED, "too many blocks stored by halves");
            std::vector<h2::ReduceDesc> red;
            for (size_t k = 0; k < ents.size(); ++k) {
                const Ent &e = ents[k];
                if (e.gslot_pos != SIZE_MAX)
                    gslot[e.gslot_pos] = int32_t(k);
                else
                    slots[e.blk] = -(int32_t(k) + 2);
                if (k == 0 || e.point != ents[k - 1].point || e.id != ents[k - 1].id)
                    red.push_back({mv_off(e.point, e.id), int32_t(k), int32_t(k), e.C, e.point ? 1 : 0});
                red.back().c1 = int32_t(k + 1);
            }
            WorkList w;
            w.phase = PH_STREAM;
            w.kind = sk;
            w.data = A.blocks;
            w.nrows = int64_t(rows.size());
            w.rows = A.mem.upload(rows, stream);
            w.blks = A.mem.upload(blks, stream);
            w.slot = A.mem.upload(slots, stream);
            w.groups = A.mem.upload(hg, stream);
            w.ngroups = int64_t(hg.size());
            w.gslot = A.mem.upload(gslot, stream);
            w.red = A.mem.upload(red, stream);
            w.nred = int64_t(red.size());
            w.partials_bytes = int64_t(ents.size()) * 64 * (A.vec_f64 ? 8 : 4);
            w.partials = A.mem.alloc(w.partials_bytes);
            A.lists.push_back(w);
            clear();
        }
    }
    if (!A.half) {
        // Tile lists (many right-hand sides): the input tiles (k x 32 per node)
        // outgrow the last-level cache, so rows stay in spatial order -- leaf rows
        // (dense) first, then coupling rows from the finest level up, each by
        // index -- and concurrently running rows share their input tiles.
        std::vector<size_t> spatial;
        spatial.reserve(L.size());
        for (size_t r = 0; r < L.size(); ++r)
            if (L[r].point) spatial.push_back(r);
        for (int l = q; l >= s.lmin && lowrank; --l)
            for (size_t r = 0; r < L.size(); ++r)
                if (!L[r].point && L[r].id >= Structure::first(l) && L[r].id < Structure::first(l + 1))
                    spatial.push_back(r);
        // (encoded on a second host thread while this one orders and encodes
        // the single-vector list)
        auto tiles = std::async(std::launch::async | std::launch::deferred,
                                [&] { return encode(1, PH_STREAM, &spatial); });
        // Single right-hand side: the vector trees fit in the caches; longest
        // rows first, so the wavefronts that start last are the short ones.
        std::vector<size_t> by_len(L.size());
        std::iota(by_len.begin(), by_len.end(), size_t(0));
        std::stable_sort(by_len.begin(), by_len.end(), [&](size_t a, size_t b) { return L[a].nb() > L[b].nb(); });
        const int64_t nblk = int64_t(pool.size());
        const bool split = int64_t(L.size()) < kSplitRows && nblk > int64_t(L.size());
        Encoded single;
        if (!split) single = encode(0, PH_STREAM, &by_len);
        commit(1, PH_STREAM, sk, A.blocks, tiles.get());
        {
            std::vector<LRow> sorted;
            sorted.reserve(L.size());
            for (size_t r : by_len) sorted.push_back(L[r]);
            L.swap(sorted);
        }
        // the streamed schedule's order: coupling rows, then near-field rows
        std::vector<size_t> order;
        for (size_t r = 0; r < L.size(); ++r)
            if (!L[r].point) order.push_back(r);
        const int64_t ncoup = int64_t(order.size());
        for (size_t r = 0; r < L.size(); ++r)
            if (L[r].point) order.push_back(r);
        std::vector<int64_t> near_cum{0};
        if (split) {
            // few rows: every row cut into chunks of `chunk` blocks, one wavefront
            // each, writing FP64 partial sums that a second launch adds up per row
            const int chunk = int(std::max<int64_t>(1, (nblk + kSplitWaves - 1) / kSplitWaves));
            std::vector<RowDesc> rows;
            std::vector<BlkDesc> blks;
            std::vector<h2::ReduceDesc> red;
            std::vector<size_t> first_chunk;   // per row of L: its first chunk in rows
            for (const LRow &r : L) {
                first_chunk.push_back(rows.size());
                const int nb = int(r.nb()), nc = std::max(1, (nb + chunk - 1) / chunk);
                red.push_back({mv_off(r.point, r.id), int32_t(rows.size()), int32_t(rows.size() + nc), r.R,
                               r.point ? 1 : 0});
                for (int c = 0; c < nc; ++c) {
                    RowDesc d;
                    d.out = int64_t(rows.size()) * 64;
                    d.init = -1;
                    d.R = r.R;
                    d.sel = (r.sel & h2::ROW_IN_X) | h2::ROW_OUT_P;
                    d.b0 = int32_t(blks.size());
                    for (int b = c * chunk; b < std::min(nb, (c + 1) * chunk); ++b) {
                        const LBlk &lb = pool[r.b0 + size_t(b)];
                        blks.push_back({lb.a, mv_off(lb.point, lb.id), lb.C, lb.sidx});
                    }
                    d.b1 = int32_t(blks.size());
                    rows.push_back(d);
                }
            }
            WorkList w;
            w.phase = PH_STREAM;
            w.kind = sk;
            w.data = A.blocks;
            w.nrows = int64_t(rows.size());
            w.rows = A.mem.upload(rows, stream);
            w.blks = A.mem.upload(blks, stream);
            w.red = A.mem.upload(red, stream);
            w.nred = int64_t(red.size());
            w.partials_bytes = w.nrows * 64 * 8;
            w.partials = A.mem.alloc(w.partials_bytes);
            first_chunk.push_back(rows.size());
            std::vector<RowDesc> srows;
            std::vector<h2::ReduceDesc> sred;
            for (size_t o = 0; o < order.size(); ++o) {
                const size_t r = order[o];
                for (size_t c = first_chunk[r]; c < first_chunk[r + 1]; ++c) {
                    srows.push_back(rows[c]);
                    if (int64_t(o) >= ncoup) near_cum.push_back(near_cum.back() + (rows[c].b1 - rows[c].b0));
                }
                sred.push_back(red[r]);
                if (int64_t(o) + 1 == ncoup) w.nsrows_coupling = int64_t(srows.size());
            }
            w.srows = A.mem.upload(srows, stream);
            w.sred = A.mem.upload(sred, stream);
            w.nsred_coupling = ncoup;
            w.near_cum = std::move(near_cum);
            A.lists.push_back(w);
        } else {
            commit(0, PH_STREAM, sk, A.blocks, std::move(single));
            std::vector<int64_t> b0(L.size() + 1, 0);
            for (size_t r = 0; r < L.size(); ++r) b0[r + 1] = b0[r] + int64_t(L[r].nb());
            std::vector<RowDesc> srows;
            srows.reserve(L.size());
            for (size_t o = 0; o < order.size(); ++o) {
                const LRow &r = L[order[o]];
                RowDesc d;
                d.out = mv_off(r.point, r.id);
                d.init = -1;
                d.b0 = int32_t(b0[order[o]]);
                d.b1 = int32_t(b0[order[o] + 1]);
                d.R = r.R;
                d.sel = r.sel;
                srows.push_back(d);
                if (int64_t(o) >= ncoup) near_cum.push_back(near_cum.back() + int64_t(r.nb()));
            }
            WorkList &w = A.lists.back();
            w.srows = A.mem.upload(srows, stream);
            w.nsrows_coupling = ncoup;
            w.near_cum = std::move(near_cum);
        }
        clear();
    }
    if (lowrank) {
        // downsweep y^_c += E_c y^_parent for levels lmin+1 .. q   (Sec. 4.4)
        for (int l = s.lmin + 1; l <= q; ++l) {
            for (int64_t c = Structure::first(l); c < Structure::first(l + 1); ++c) {
                add_row(false, c, true, kl[l], 0);
                add_blk(off_E[c], kl[l - 1], 0, false, (c - 1) / 2);
            }
            emit(PH_DOWN, bk, A.basis);
        }
    }
    // leaf expansion and sum: y(i) = y_near(i) + U_i y^_i   (Sec. 4.4, Sec. 4.1)
    for (int64_t j = 0; j < nleaves; ++j) {
        add_row(true, j, true, int(s.size(lf + j)), h2::ROW_OUT_P);
        if (lowrank) add_blk(off_U[j], kl[q], 0, false, lf + j);
    }
    emit(PH_LEAF, bk, A.basis);
    std::vector<int64_t> lb(nleaves), le(nleaves);
    for (int64_t j = 0; j < nleaves; ++j) {
        lb[j] = s.begin[lf + j];
        le[j] = s.end[lf + j];
    }
    A.d_leaf_begin = A.mem.upload(lb, stream);
    A.d_leaf_end = A.mem.upload(le, stream);
    check_hip(hipStreamSynchronize(stream), "upload work lists");
}

void validate_params(const double *points, int64_t n, const h2_params *prm) {
    if (!points || !prm) fail(H2_ERR_INVALID_ARG, "NULL points or params");
    if (n < 1 || n >= (int64_t(1) << 31)) fail(H2_ERR_INVALID_ARG, "n must be in [1, 2^31)");
    if (prm->dim != 2 && prm->dim != 3) fail(H2_ERR_INVALID_ARG, "dim must be 2 or 3");
    if (prm->leaf_size < 2) fail(H2_ERR_INVALID_ARG, "leaf_size must be >= 2");
    if (prm->cheb_p < 1) fail(H2_ERR_INVALID_ARG, "cheb_p must be >= 1");
    if (!(prm->eta > 0.0) || !std::isfinite(prm->eta)) fail(H2_ERR_INVALID_ARG, "eta must be > 0");
    if (!(prm->corr_len > 0.0) || !std::isfinite(prm->corr_len))
        fail(H2_ERR_INVALID_ARG, "corr_len must be > 0");
    const int prec = prm->storage & ~H2_HALF_STORAGE;
    if (prec < H2_FP64 || prec > H2_BF16_SCALED) fail(H2_ERR_INVALID_ARG, "bad storage");
    if (prm->flags & ~unsigned(H2_FLAG_STRUCTURE_ONLY)) fail(H2_ERR_INVALID_ARG, "unknown flags");
    for (int64_t i = 0; i < n * prm->dim; ++i)
        if (!std::isfinite(points[i])) fail(H2_ERR_INVALID_ARG, "non-finite coordinate");
    int64_t k = 1;
    for (int a = 0; a < prm->dim; ++a) {
        k *= prm->cheb_p;
        if (k > 64) fail(H2_ERR_UNSUPPORTED, "rank cheb_p^dim above 64");
    }
    if (prm->leaf_size > 64) fail(H2_ERR_UNSUPPORTED, "leaf_size above 64");
}

// Checks the arrays and fills the host structure from them.
void structure_from_arrays(const h2_arrays *a, h2::Structure &s) {
    if (!a) fail(H2_ERR_INVALID_ARG, "NULL arrays");
    if (a->n < 1 || a->n >= (int64_t(1) << 31)) fail(H2_ERR_INVALID_ARG, "n out of range");
    if (a->q < 0) fail(H2_ERR_INVALID_ARG, "q < 0");
    if (a->q > 29) fail(H2_ERR_UNSUPPORTED, "q above 29");
    if ((int64_t(1) << a->q) > a->n) fail(H2_ERR_INVALID_ARG, "more leaves than rows");
    if (!a->level_rank || !a->node_begin || !a->node_end || !a->S_rowptr || !a->S_colidx || !a->S ||
        !a->D_rowptr || (!a->D_colidx && a->D_rowptr[int64_t(1) << a->q] > 0) ||
        (!a->D && a->D_rowptr[int64_t(1) << a->q] > 0))
        fail(H2_ERR_INVALID_ARG, "NULL array");
    s = h2::Structure();
    s.n = a->n;
    s.q = a->q;
    s.nnodes = (int64_t(2) << a->q) - 1;
    s.lrank.resize(a->q + 1);
    s.rank = 0;
    for (int l = 0; l <= a->q; ++l) {
        const int k = a->level_rank[l];
        if (k < 1) fail(H2_ERR_INVALID_ARG, "level rank < 1");
        if (k > 64) fail(H2_ERR_UNSUPPORTED, "level rank above 64");
        s.lrank[l] = k;
        s.rank = std::max(s.rank, k);
    }
    s.begin.assign(a->node_begin, a->node_begin + s.nnodes);
    s.end.assign(a->node_end, a->node_end + s.nnodes);
    if (s.begin[0] != 0 || s.end[0] != a->n) fail(H2_ERR_INVALID_ARG, "root must hold rows [0, n)");
    for (int64_t v = 0; v < s.nnodes; ++v) {
        if (s.end[v] <= s.begin[v]) fail(H2_ERR_INVALID_ARG, "empty node");
        if (2 * v + 2 < s.nnodes) {
            const int64_t c1 = 2 * v + 1, c2 = 2 * v + 2;
            if (s.begin[c1] != s.begin[v] || s.end[c1] != s.begin[c2] || s.end[c2] != s.end[v])
                fail(H2_ERR_INVALID_ARG, "children must split their parent into consecutive ranges");
        } else {
            s.leaf = int(std::max<int64_t>(s.leaf, s.size(v)));
        }
    }
    if (s.leaf > 64) fail(H2_ERR_UNSUPPORTED, "leaf above 64 rows");
    auto take_bsr = [&](int64_t rows, const int32_t *rp, const int32_t *ci, h2::Bsr &B) {
        if (rp[0] != 0) fail(H2_ERR_INVALID_ARG, "BSR offsets must start at 0");
        B.rowptr.assign(rp, rp + rows + 1);
        for (int64_t i = 0; i < rows; ++i)
            if (B.rowptr[i + 1] < B.rowptr[i]) fail(H2_ERR_INVALID_ARG, "BSR offsets must not decrease");
        B.colidx.assign(ci, ci + B.rowptr[rows]);
        for (int32_t c : B.colidx)
            if (c < 0 || c >= rows) fail(H2_ERR_INVALID_ARG, "BSR column out of range");
    };
    s.coupling.resize(a->q + 1);
    s.lmin = a->q + 1;
    for (int l = a->q; l >= 0; --l) {
        if (!a->S_rowptr[l]) fail(H2_ERR_INVALID_ARG, "NULL S_rowptr");
        if (a->S_rowptr[l][int64_t(1) << l] > 0 && (!a->S_colidx[l] || !a->S[l]))
            fail(H2_ERR_INVALID_ARG, "NULL S_colidx / S for a level with blocks");
        take_bsr(int64_t(1) << l, a->S_rowptr[l], a->S_colidx[l], s.coupling[l]);
        if (s.coupling[l].blocks() > 0) s.lmin = l;
    }
    take_bsr(int64_t(1) << a->q, a->D_rowptr, a->D_colidx, s.dense);
    if (s.lmin <= a->q && (!a->U || !a->V)) fail(H2_ERR_INVALID_ARG, "NULL U / V with coupling blocks");
    if (s.lmin < a->q && (!a->E || !a->F)) fail(H2_ERR_INVALID_ARG, "NULL E / F with coupling blocks above the leaves");
    s.perm.resize(a->n);
    for (int64_t i = 0; i < a->n; ++i) s.perm[i] = i;
}

// Reads blocks of a device region in offset order through a bounded host
// window, converting each to column-major FP64 (the inverse of convert_block;
// BF16 values are code x scale in FP32, as stored).
struct Reader {
    const char *dev;
    int kind;
    int64_t elem, total;   // element size, region length in elements
    hipStream_t st;
    std::vector<char> buf;
    int64_t win = 0, len = 0;   // window [win, win + len) in elements
    static constexpr int64_t kCap = int64_t(64) << 20;
    Reader(const void *d, int k, int64_t n, hipStream_t s)
        : dev(static_cast<const char *>(d)), kind(k), elem(h2::elem_bytes(k)), total(n), st(s) {}
    const char *at(int64_t off, int64_t ne) {
        if (off < 0 || off + ne > total) fail(H2_ERR_INTERNAL, "block outside its region");
        if (off < win || off + ne > win + len) {
            len = std::min<int64_t>(std::max<int64_t>(ne, kCap / elem), total - off);
            buf.resize(size_t(len * elem));
            check_hip(hipMemcpyAsync(buf.data(), dev + off * elem, size_t(len * elem), hipMemcpyDeviceToHost, st),
                      "hipMemcpyAsync");
            check_hip(hipStreamSynchronize(st), "export");
            win = off;
        }
        return buf.data() + (off - win) * elem;
    }
    void block(int64_t off, int R, int C, bool transpose, float scale, double *dst) {
        const int W = 16 / int(elem);
        const int64_t ne = h2::block_elems(R, C, kind);
        const char *p = at(off, ne);
        for (int64_t e = 0; e < ne; ++e) {
            const int w = int(e % W);
            const int64_t t = e / W;
            const int r = int(t % R), c = int(t / R) * W + w;
            if (c >= C) continue;
            double v;
            if (kind == h2::ELEM_F64) v = reinterpret_cast<const double *>(p)[e];
            else if (kind == h2::ELEM_F32) v = reinterpret_cast<const float *>(p)[e];
            else {
                const uint32_t u = uint32_t(reinterpret_cast<const uint16_t *>(p)[e]) << 16;
                float f;
                std::memcpy(&f, &u, 4);
                v = double(f * scale);
            }
            if (transpose) dst[c + int64_t(r) * C] = v;   // stored R x C is the transpose of a C x R block
            else dst[r + int64_t(c) * R] = v;
        }
    }
};

void export_arrays(h2_matrix_ &A, const h2_arrays_out *o, hipStream_t st) {
    const Structure &s = A.st;
    const int q = s.q;
    const std::vector<int> &kl = s.lrank;
    const int64_t nleaves = int64_t(1) << q, lf = Structure::first(q);
    if (o->level_rank)
        for (int l = 0; l <= q; ++l) o->level_rank[l] = kl[l];
    if (o->node_begin) std::copy(s.begin.begin(), s.begin.end(), o->node_begin);
    if (o->node_end) std::copy(s.end.begin(), s.end.end(), o->node_end);
    const bool lowrank = s.lmin <= q;
    if (o->U || o->V || o->E || o->F) {
        Reader rd(A.basis, A.basis_kind, A.basis_elems, st);
        int64_t uoff = 0;
        for (int64_t j = 0; j < nleaves; ++j) {
            const int m = int(s.size(lf + j));
            const int64_t len = int64_t(m) * kl[q];
            if (!lowrank) {
                if (o->U) std::fill(o->U + uoff, o->U + uoff + len, 0.0);
                if (o->V) std::fill(o->V + uoff, o->V + uoff + len, 0.0);
            } else {
                if (o->U) rd.block(A.off_U[j], m, kl[q], false, 1.0f, o->U + uoff);
                if (o->V) rd.block(A.off_VT[j], kl[q], m, true, 1.0f, o->V + uoff);
            }
            uoff += len;
        }
        int64_t eoff = 0;
        for (int l = 1; l <= q; ++l)
            for (int64_t c = Structure::first(l); c < Structure::first(l + 1); ++c) {
                const int64_t len = int64_t(kl[l]) * kl[l - 1];
                if (A.off_E[c] < 0) {   // not stored: not used by the product
                    if (o->E) std::fill(o->E + eoff, o->E + eoff + len, 0.0);
                    if (o->F) std::fill(o->F + eoff, o->F + eoff + len, 0.0);
                } else {
                    if (o->E) rd.block(A.off_E[c], kl[l], kl[l - 1], false, 1.0f, o->E + eoff);
                    if (o->F) rd.block(A.off_FT[c], kl[l - 1], kl[l], true, 1.0f, o->F + eoff);
                }
                eoff += len;
            }
    }
    std::vector<float> scales;
    if (A.block_kind == h2::ELEM_BF16 && A.nscales > 0) {
        scales.resize(size_t(A.nscales));
        check_hip(hipMemcpyAsync(scales.data(), A.scales, scales.size() * 4, hipMemcpyDeviceToHost, st),
                  "hipMemcpyAsync");
        check_hip(hipStreamSynchronize(st), "export scales");
    }
    auto scale_of = [&](int64_t i) { return scales.empty() ? 1.0f : scales[size_t(i)]; };
    Reader rd(A.blocks, A.block_kind, A.block_elems, st);
    // Stored by halves, a block below the diagonal is its mirror transposed;
    // those are read after the stored ones, in storage order.
    struct Mirror {
        int64_t m;
        int R, C;
        double *dst;
    };
    std::vector<Mirror> mirrors;
    auto read_block = [&](int64_t li, int R, int C, double *dst) {
        const int64_t si = A.blk_store.empty() ? li : A.blk_store[size_t(li)];
        if (si >= 0)
            rd.block(A.off_blk[size_t(si)], R, C, false, scale_of(si), dst);
        else
            mirrors.push_back({-si - 1, R, C, dst});
    };
    int64_t fi = 0;
    for (int l = 0; l <= q; ++l) {
        const h2::Bsr &B = s.coupling[l];
        if (o->S_rowptr && o->S_rowptr[l]) std::copy(B.rowptr.begin(), B.rowptr.end(), o->S_rowptr[l]);
        if (o->S_colidx && o->S_colidx[l]) std::copy(B.colidx.begin(), B.colidx.end(), o->S_colidx[l]);
        const int64_t kk = int64_t(kl[l]) * kl[l];
        for (int64_t b = 0; b < B.blocks(); ++b, ++fi)
            if (o->S && o->S[l]) read_block(fi, kl[l], kl[l], o->S[l] + b * kk);
    }
    if (o->D_rowptr) std::copy(s.dense.rowptr.begin(), s.dense.rowptr.end(), o->D_rowptr);
    if (o->D_colidx) std::copy(s.dense.colidx.begin(), s.dense.colidx.end(), o->D_colidx);
    if (o->D) {
        int64_t doff = 0;
        for (int64_t i = 0; i < nleaves; ++i)
            for (int32_t b = s.dense.rowptr[i]; b < s.dense.rowptr[i + 1]; ++b, ++fi) {
                const int R = int(s.size(lf + i)), C = int(s.size(lf + s.dense.colidx[b]));
                read_block(fi, R, C, o->D + doff);
                doff += int64_t(R) * C;
            }
    }
    std::stable_sort(mirrors.begin(), mirrors.end(), [](const Mirror &x, const Mirror &y) { return x.m < y.m; });
    for (const Mirror &mi : mirrors)   // the stored block is C x R
        rd.block(A.off_blk[size_t(mi.m)], mi.C, mi.R, true, scale_of(mi.m), mi.dst);
}

}  // namespace h2i

using namespace h2i;

extern "C" {

h2_status h2_build_from_points(const double *points, int64_t n, const h2_params *prm, void *stream,
                               h2_handle *out) {
    if (out) *out = nullptr;
    h2_matrix_ *A = nullptr;
    try {
        if (!out) fail(H2_ERR_INVALID_ARG, "NULL out");
        validate_params(points, n, prm);
        A = new h2_matrix_();
        const int prec = prm->storage & ~H2_HALF_STORAGE;
        A->storage = prec;
        A->half = (prm->storage & H2_HALF_STORAGE) != 0;
        A->structure_only = (prm->flags & H2_FLAG_STRUCTURE_ONLY) != 0;
        A->basis_kind = prec == H2_FP64 ? h2::ELEM_F64 : h2::ELEM_F32;
        A->block_kind = prec == H2_FP64 ? h2::ELEM_F64 : prec == H2_FP32 ? h2::ELEM_F32 : h2::ELEM_BF16;
        A->vec_f64 = prec == H2_FP64;
        std::string err = h2::build_structure(points, n, prm->dim, prm->leaf_size, prm->cheb_p, prm->eta,
                                              prm->corr_len, A->st);
        if (!err.empty()) fail(H2_ERR_UNSUPPORTED, err);
        if (!A->structure_only) build_device(*A, nullptr, static_cast<hipStream_t>(stream));
        *out = A;
        g_last_error.clear();
        return H2_OK;
    } catch (const Failure &f) {
        delete A;
        g_last_error = f.what;
        return f.code;
    } catch (const std::bad_alloc &) {
        delete A;
        g_last_error = "host allocation failed";
        return H2_ERR_OOM;
    } catch (...) {
        delete A;
        g_last_error = "internal error";
        return H2_ERR_INTERNAL;
    }
}

h2_status h2_build_from_arrays(const h2_arrays *arrays, int storage, void *stream, h2_handle *out) {
    if (out) *out = nullptr;
    h2_matrix_ *A = nullptr;
    try {
        if (!out) fail(H2_ERR_INVALID_ARG, "NULL out");
        const int prec = storage & ~H2_HALF_STORAGE;
        if (prec < H2_FP64 || prec > H2_BF16_SCALED) fail(H2_ERR_INVALID_ARG, "storage out of range");
        A = new h2_matrix_();
        structure_from_arrays(arrays, A->st);
        A->storage = prec;
        A->half = (storage & H2_HALF_STORAGE) != 0;
        A->basis_kind = prec == H2_FP64 ? h2::ELEM_F64 : h2::ELEM_F32;
        A->block_kind = prec == H2_FP64 ? h2::ELEM_F64 : prec == H2_FP32 ? h2::ELEM_F32 : h2::ELEM_BF16;
        A->vec_f64 = prec == H2_FP64;
        {
            // V = U and F = E (value by value): the symmetric case orthogonalization handles
            const h2::Structure &st = A->st;
            const int64_t lf = h2::Structure::first(st.q);
            int64_t nu = 0, ne = 0;
            for (int64_t v = lf; v < st.nnodes; ++v) nu += st.size(v) * st.lrank[st.q];
            for (int l = 1; l <= st.q; ++l) ne += (int64_t(st.lrank[l]) * st.lrank[l - 1]) << l;
            const bool su = arrays->U == arrays->V || (arrays->U && arrays->V &&
                                                         std::memcmp(arrays->U, arrays->V, size_t(nu) * 8) == 0);
            const bool se = arrays->E == arrays->F || (arrays->E && arrays->F &&
                                                         std::memcmp(arrays->E, arrays->F, size_t(ne) * 8) == 0);
            A->symmetric = su && se;
        }
        build_device(*A, arrays, static_cast<hipStream_t>(stream));
        *out = A;
        g_last_error.clear();
        return H2_OK;
    } catch (const Failure &f) {
        delete A;
        g_last_error = f.what;
        return f.code;
    } catch (const std::bad_alloc &) {
        delete A;
        g_last_error = "host allocation failed";
        return H2_ERR_OOM;
    } catch (...) {
        delete A;
        g_last_error = "internal error";
        return H2_ERR_INTERNAL;
    }
}

h2_status h2_export_arrays(h2_handle A, const h2_arrays_out *out, void *stream) {
    try {
        if (!A || !out) fail(H2_ERR_INVALID_ARG, "NULL argument");
        if (A->structure_only && (out->U || out->V || out->E || out->F || out->S || out->D))
            fail(H2_ERR_INVALID_ARG, "structure-only handle holds no values");
        export_arrays(*A, out, static_cast<hipStream_t>(stream));
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
