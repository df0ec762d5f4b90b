// C ABI of libh2mv (include/h2mv.h): builds the H^2 representation on the
// device from points and runs the product y = A x as a fixed sequence of
// block-row launches over work lists built once at construction (the paper's
// per-call marshaling of pointer batches, Sec. 3.2, becomes static lists).
#include "h2mv.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <memory>
#include <new>
#include <mutex>
#include <string>
#include <vector>

#include "h2_device.h"
#include "h2_structure.h"

namespace {

thread_local std::string g_last_error;

struct Failure {
    h2_status code;
    std::string what;
};

[[noreturn]] void fail(h2_status code, const std::string &what) { throw Failure{code, what}; }

void check_hip(hipError_t e, const char *where) {
    if (e != hipSuccess) fail(H2_ERR_DEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

// Device allocations of one owner; a test-only cap (environment variable
// H2MV_DEVICE_BYTE_CAP, bytes) turns any allocation past it into H2_ERR_OOM.
struct DeviceArena {
    std::vector<void *> ptrs;
    int64_t bytes = 0;
    int64_t cap = -1;

    DeviceArena() {
        if (const char *c = std::getenv("H2MV_DEVICE_BYTE_CAP")) cap = std::atoll(c);
    }
    DeviceArena(const DeviceArena &) = delete;
    DeviceArena &operator=(const DeviceArena &) = delete;
    ~DeviceArena() {
        for (void *p : ptrs) (void)hipFree(p);
    }
    void swap(DeviceArena &o) {
        std::swap(ptrs, o.ptrs);
        std::swap(bytes, o.bytes);
        std::swap(cap, o.cap);
    }
    void *alloc(int64_t nbytes) {
        if (nbytes <= 0) nbytes = 16;
        nbytes = (nbytes + 255) / 256 * 256;
        if (cap >= 0 && bytes + nbytes > cap) fail(H2_ERR_OOM, "device byte cap exceeded");
        void *p = nullptr;
        hipError_t e = hipMalloc(&p, size_t(nbytes));
        if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) {
            (void)hipGetLastError();
            fail(H2_ERR_OOM, "hipMalloc of " + std::to_string(nbytes) + " bytes failed");
        }
        check_hip(e, "hipMalloc");
        ptrs.push_back(p);
        bytes += nbytes;
        return p;
    }
    template <typename T>
    // Copies v to new device memory; returns once v may be released (set-up
    // only, never inside a product).
    T *upload(const std::vector<T> &v, hipStream_t st) {
        T *d = static_cast<T *>(alloc(int64_t(v.size() * sizeof(T))));
        if (!v.empty()) {
            check_hip(hipMemcpyAsync(d, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, st),
                      "hipMemcpyAsync");
            check_hip(hipStreamSynchronize(st), "upload");
        }
        return d;
    }
};

enum Phase { PH_UP = 0, PH_STREAM = 1, PH_DOWN = 2, PH_LEAF = 3, PH_COUNT = 4 };

struct WorkList {
    Phase phase;
    int kind;   // element kind of its data
    const void *data;
    const h2::RowDesc *rows;
    int64_t nrows;
    const h2::BlkDesc *blks;
    const int32_t *items = nullptr;   // tile lists: wavefront items in dispatch order
    int64_t nitems = 0;
    // split stream list (single vector, small matrices): the rows are chunks
    // writing FP64 partial sums, added up by a second launch
    const h2::ReduceDesc *red = nullptr;
    int64_t nred = 0;
    double *partials = nullptr;
};

// A single-vector stream list with fewer block rows than this is split into
// chunks: one wavefront per row would leave most of the machine idle.
constexpr int64_t kSplitRows = 4096;
constexpr int64_t kSplitWaves = 4096;   // target number of chunks (about 16 per CU)

// Wavefront items of a tile list in dispatch order (see h2::MmLaunch): one
// item per 32-row half of each row, the list cut into MM_XCDS contiguous
// ranges of about equal work (per block: its columns rounded up to the
// 16-column MFMA step, plus a fixed cost), each range padded to whole
// workgroups, and range x's l-th workgroup placed at workgroup l * MM_XCDS + x.
std::vector<int32_t> wave_items(const std::vector<h2::RowDesc> &rows, const std::vector<h2::BlkDesc> &blks) {
    constexpr int X = h2::MM_XCDS;
    if (rows.size() >= (size_t(1) << 30)) fail(H2_ERR_UNSUPPORTED, "too many rows in one tile list");
    std::vector<int32_t> items;
    std::vector<double> work;
    double total = 0.0;
    for (size_t r = 0; r < rows.size(); ++r) {
        double w = 0.0;
        for (int32_t b = rows[r].b0; b < rows[r].b1; ++b) w += double((blks[b].C + 15) / 16 * 16 + 8);
        for (int mt = 0; mt * 32 < std::max(rows[r].R, 1); ++mt) {
            items.push_back(int32_t(r << 1) | mt);
            work.push_back(w);
            total += w;
        }
    }
    // cut points: range x = [cut[x], cut[x+1])
    std::vector<size_t> cut(X + 1, items.size());
    cut[0] = 0;
    double acc = 0.0;
    int x = 1;
    for (size_t i = 0; i < items.size() && x < X; ++i) {
        while (x < X && acc >= total * x / X) cut[x++] = i;
        acc += work[i];
    }
    size_t per = 0;   // workgroups per XCD
    for (int r = 0; r < X; ++r) per = std::max(per, (cut[r + 1] - cut[r] + 3) / 4);
    std::vector<int32_t> out(per * X * 4, -1);
    for (int r = 0; r < X; ++r)
        for (size_t i = cut[r]; i < cut[r + 1]; ++i) {
            const size_t l = (i - cut[r]) / 4, v = (i - cut[r]) % 4;
            out[(l * X + r) * 4 + v] = items[i];
        }
    return out;
}

}  // namespace

struct h2_matrix_ {
    h2::Structure st;
    int storage = H2_FP64;
    bool structure_only = false;
    int basis_kind = h2::ELEM_F64, block_kind = h2::ELEM_F64;
    bool vec_f64 = true;
    DeviceArena mem;
    void *basis = nullptr, *blocks = nullptr;
    float *scales = nullptr;
    void *xh = nullptr, *yh = nullptr, *ynear = nullptr;
    std::vector<WorkList> lists;      // single right-hand side (vector offsets)
    std::vector<WorkList> mm_lists;   // tiles of MM_TILE right-hand sides (tile offsets)
    std::vector<std::vector<h2::RowDesc>> mm_host_rows;   // host copies of mm_lists (for batches)
    std::vector<std::vector<h2::BlkDesc>> mm_host_blks;
    int64_t nscales = 0;
    int64_t tile_slot = 0;            // elements per leaf in point tiles
    int64_t *d_leaf_begin = nullptr, *d_leaf_end = nullptr;
    float *t_xh = nullptr, *t_yh = nullptr, *t_x = nullptr, *t_ynear = nullptr;   // tile workspace (lazy)
    // block loop chosen at the first pass of each tile width (32, or 16 for
    // passes of at most 16 right-hand sides)
    h2::MmConfig mm_cfg[2] = {{1, 0}, {1, 0}};
    bool mm_tuned[2] = {false, false};
    int64_t bytes_coupling = 0, bytes_dense = 0, bytes_leaf = 0, bytes_transfer = 0;
    // layout: element offsets of U_j, V_j^T (per leaf), E_c, F_c^T (per node,
    // -1 where not stored) in basis, and of every block in blocks (coupling
    // blocks level by level in BSR order, then dense blocks)
    std::vector<int64_t> off_U, off_VT, off_E, off_FT, off_blk;
    int64_t basis_elems = 0, block_elems = 0;   // lengths of the two regions
    bool symmetric = true;                      // V = U and F = E
    int batch_refs = 0;                         // batches holding addresses into this matrix
    // profiling: PH_COUNT + 1 events per recorded call
    bool prof = false;
    std::vector<hipEvent_t> pending, spare;
    double prof_ms[8] = {0};
    int64_t prof_calls = 0;

    ~h2_matrix_() {
        for (hipEvent_t e : pending) (void)hipEventDestroy(e);
        for (hipEvent_t e : spare) (void)hipEventDestroy(e);
    }
};

namespace {

using h2::BlkDesc;
using h2::RowDesc;
using h2::Structure;

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

// Layout of the representation, generation on the device (from points) or
// conversion of caller arrays (src), and the work lists of one product in
// launch order.  Ranks may differ per level (k_l); vectors and tiles use the
// largest rank as their node stride.
// The device representation's layout for the structure's level ranks: sets
// the offsets and byte counts of A, allocates its regions (basis, blocks,
// scales) and returns the fill list (coupling blocks level by level in BSR
// order, then dense blocks); ncoupling receives the number of coupling blocks.
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

    // block region: coupling blocks level by level in BSR order, then dense blocks
    std::vector<h2::FillDesc> fill;
    int64_t ns = 0;
    for (int l = 0; l <= q; ++l) {
        const h2::Bsr &B = s.coupling[l];
        const int64_t f = Structure::first(l);
        for (int64_t i = 0; i < (int64_t(1) << l); ++i)
            for (int32_t b = B.rowptr[i]; b < B.rowptr[i + 1]; ++b) {
                fill.push_back({ns, int32_t(f + i), int32_t(f + B.colidx[b]), int32_t(fill.size()),
                                h2::FILL_COUPLING});
                ns += h2::block_elems(kl[l], kl[l], sk);
            }
    }
    const int64_t coupling_elems = ns;
    ncoupling = int64_t(fill.size());
    for (int64_t i = 0; i < nleaves; ++i)
        for (int32_t b = s.dense.rowptr[i]; b < s.dense.rowptr[i + 1]; ++b) {
            const int64_t t = lf + s.dense.colidx[b];
            fill.push_back({ns, int32_t(lf + i), int32_t(t), int32_t(fill.size()), h2::FILL_DENSE});
            ns += h2::block_elems(int(s.size(lf + i)), int(s.size(t)), sk);
        }
    const int64_t scale_bytes = sk == h2::ELEM_BF16 ? 4 : 0;
    A.off_U = off_U;
    A.off_VT = off_VT;
    A.off_E = off_E;
    A.off_FT = off_FT;
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

void build_lists(h2_matrix_ &A, const std::vector<h2::FillDesc> &fill, int64_t ncoupling, hipStream_t stream);

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
            Stager up(A.blocks, sk, stream);
            std::vector<float> scales(fill.size(), 1.0f);
            int64_t fi = 0;
            for (int l = 0; l <= q; ++l) {
                const h2::Bsr &B = s.coupling[l];
                const int64_t kk = int64_t(kl[l]) * kl[l];
                for (int64_t b = 0; b < B.blocks(); ++b, ++fi)
                    convert_block(src->S[l] + b * kk, kl[l], kl[l], false, sk,
                                  up.place(fill[fi].a, h2::block_elems(kl[l], kl[l], sk)), &scales[fi]);
            }
            int64_t doff = 0;
            for (int64_t i = 0; i < nleaves; ++i)
                for (int32_t b = s.dense.rowptr[i]; b < s.dense.rowptr[i + 1]; ++b, ++fi) {
                    const int R = int(s.size(lf + i)), C = int(s.size(lf + s.dense.colidx[b]));
                    convert_block(src->D + doff, R, C, false, sk, up.place(fill[fi].a, h2::block_elems(R, C, sk)),
                                  &scales[fi]);
                    doff += int64_t(R) * C;
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
    struct LBlk {
        int64_t a;
        int32_t C, sidx;
        bool point;
        int64_t id;
    };
    struct LRow {
        bool point;      // output is a leaf segment (else a tree node)
        int64_t id;      // leaf index or node id
        bool has_init;   // add the current value (downsweep: y^; leaf phase: y_near)
        int R, sel;
        std::vector<LBlk> b;
    };
    const int64_t kp = (k + 15) / 16 * 16;
    int64_t mmax = 0;
    for (int64_t j = 0; j < nleaves; ++j) mmax = std::max(mmax, s.size(lf + j));
    A.tile_slot = (mmax + 15) / 16 * 16 * h2::MM_TILE;
    auto mv_off = [&](bool point, int64_t id) { return point ? s.begin[lf + id] : id * k; };
    auto mm_off = [&](bool point, int64_t id) { return point ? id * A.tile_slot : id * kp * h2::MM_TILE; };
    // enc 0: single-vector offsets into A.lists; enc 1: tile offsets into A.mm_lists
    auto emit_one = [&](int enc, Phase ph, int kind, const void *data, const std::vector<LRow> &L) {
        std::vector<RowDesc> rows;
        std::vector<BlkDesc> blks;
        for (const LRow &r : L) {
            RowDesc d;
            if (ph == PH_LEAF) {   // out: rows of y; init: y_near
                d.out = s.begin[lf + r.id];
                d.init = enc == 0 ? mv_off(true, r.id) : mm_off(true, r.id);
            } else {
                d.out = enc == 0 ? mv_off(r.point, r.id) : mm_off(r.point, r.id);
                d.init = !r.has_init ? -1 : enc == 0 ? mv_off(r.point, r.id) : mm_off(r.point, r.id);
            }
            d.b0 = int32_t(blks.size());
            for (const LBlk &b : r.b)
                blks.push_back({b.a, enc == 0 ? mv_off(b.point, b.id) : mm_off(b.point, b.id), b.C, b.sidx});
            d.b1 = int32_t(blks.size());
            d.R = r.R;
            d.sel = r.sel;
            rows.push_back(d);
        }
        WorkList w;
        w.phase = ph;
        w.kind = kind;
        w.data = data;
        w.nrows = int64_t(rows.size());
        w.rows = A.mem.upload(rows, stream);
        w.blks = A.mem.upload(blks, stream);
        if (enc == 1) {
            const std::vector<int32_t> it = wave_items(rows, blks);
            w.items = A.mem.upload(it, stream);
            w.nitems = int64_t(it.size());
        }
        (enc == 0 ? A.lists : A.mm_lists).push_back(w);
        if (enc == 1) {
            A.mm_host_rows.push_back(std::move(rows));
            A.mm_host_blks.push_back(std::move(blks));
        }
    };
    auto emit = [&](Phase ph, int kind, const void *data, std::vector<LRow> &L) {
        emit_one(0, ph, kind, data, L);
        emit_one(1, ph, kind, data, L);
        L.clear();
    };
    std::vector<LRow> L;
    if (lowrank) {
        // leaf projection x^_j = V_j^T x(j)   (Sec. 4.2)
        for (int64_t j = 0; j < nleaves; ++j) {
            const int64_t v = lf + j;
            L.push_back({false, v, false, kl[q], h2::ROW_IN_X, {{off_VT[j], int32_t(s.size(v)), 0, true, j}}});
        }
        emit(PH_UP, bk, A.basis, L);
        // upsweep x^_p = F_c1^T x^_c1 + F_c2^T x^_c2 for levels q .. lmin+1   (Sec. 4.2)
        for (int l = q; l > s.lmin; --l) {
            for (int64_t p = Structure::first(l - 1); p < Structure::first(l); ++p)
                L.push_back({false, p, false, kl[l - 1], 0,
                             {{off_FT[2 * p + 1], kl[l], 0, false, 2 * p + 1},
                              {off_FT[2 * p + 2], kl[l], 0, false, 2 * p + 2}}});
            emit(PH_UP, bk, A.basis, L);
        }
    }
    // tree multiplication y^_i = sum_j S_ij x^_j on all levels (Sec. 4.3) and the
    // dense near field y_near(i) = sum_j D_ij x(j) (Sec. 4.1) in one launch
    {
        int64_t fi = 0;
        if (lowrank)
            for (int l = s.lmin; l <= q; ++l) {
                const h2::Bsr &B = s.coupling[l];
                const int64_t f = Structure::first(l);
                for (int64_t i = 0; i < (int64_t(1) << l); ++i) {
                    LRow r{false, f + i, false, kl[l], 0, {}};
                    for (int32_t b = B.rowptr[i]; b < B.rowptr[i + 1]; ++b, ++fi)
                        r.b.push_back({fill[fi].a, kl[l], fill[fi].sidx, false, f + B.colidx[b]});
                    L.push_back(std::move(r));
                }
            }
        fi = ncoupling;
        for (int64_t i = 0; i < nleaves; ++i) {
            LRow r{true, i, false, int(s.size(lf + i)), h2::ROW_IN_X | h2::ROW_OUT_P, {}};
            for (int32_t b = s.dense.rowptr[i]; b < s.dense.rowptr[i + 1]; ++b, ++fi) {
                const int64_t t = s.dense.colidx[b];
                r.b.push_back({fill[fi].a, int32_t(s.size(lf + t)), fill[fi].sidx, true, t});
            }
            L.push_back(std::move(r));
        }
        // Tile lists (many right-hand sides): the input tiles (k x 32 per node)
        // outgrow the last-level cache, so rows stay in spatial order -- leaf rows
        // (dense) first, then coupling rows from the finest level up, each by
        // index -- and concurrently running rows share their input tiles.
        std::vector<LRow> spatial;
        for (const LRow &r : L)
            if (r.point) spatial.push_back(r);
        for (int l = q; l >= s.lmin && lowrank; --l)
            for (const LRow &r : L)
                if (!r.point && r.id >= Structure::first(l) && r.id < Structure::first(l + 1)) spatial.push_back(r);
        emit_one(1, PH_STREAM, sk, A.blocks, spatial);
        // Single right-hand side: the vector trees fit in the caches; longest
        // rows first, so the wavefronts that start last are the short ones.
        std::stable_sort(L.begin(), L.end(), [](const LRow &a, const LRow &b) { return a.b.size() > b.b.size(); });
        int64_t nblk = 0;
        for (const LRow &r : L) nblk += int64_t(r.b.size());
        if (int64_t(L.size()) < kSplitRows && nblk > int64_t(L.size())) {
            // few rows: every row cut into chunks of `chunk` blocks, one wavefront
            // each, writing FP64 partial sums that a second launch adds up per row
            const int chunk = int(std::max<int64_t>(1, (nblk + kSplitWaves - 1) / kSplitWaves));
            std::vector<RowDesc> rows;
            std::vector<BlkDesc> blks;
            std::vector<h2::ReduceDesc> red;
            for (const LRow &r : L) {
                const int nb = int(r.b.size()), nc = std::max(1, (nb + chunk - 1) / chunk);
                red.push_back({mv_off(r.point, r.id), int32_t(rows.size()), int32_t(rows.size() + nc), r.R,
                               r.point ? 1 : 0});
                for (int c = 0; c < nc; ++c) {
                    RowDesc d;
                    d.out = int64_t(rows.size()) * 64;
                    d.init = -1;
                    d.R = r.R;
                    d.sel = (r.sel & h2::ROW_IN_X) | h2::ROW_OUT_P;
                    d.b0 = int32_t(blks.size());
                    for (int b = c * chunk; b < std::min(nb, (c + 1) * chunk); ++b)
                        blks.push_back({r.b[b].a, mv_off(r.b[b].point, r.b[b].id), r.b[b].C, r.b[b].sidx});
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
            w.partials = static_cast<double *>(A.mem.alloc(w.nrows * 64 * 8));
            A.lists.push_back(w);
        } else {
            emit_one(0, PH_STREAM, sk, A.blocks, L);
        }
        L.clear();
    }
    if (lowrank) {
        // downsweep y^_c += E_c y^_parent for levels lmin+1 .. q   (Sec. 4.4)
        for (int l = s.lmin + 1; l <= q; ++l) {
            for (int64_t c = Structure::first(l); c < Structure::first(l + 1); ++c)
                L.push_back({false, c, true, kl[l], 0, {{off_E[c], kl[l - 1], 0, false, (c - 1) / 2}}});
            emit(PH_DOWN, bk, A.basis, L);
        }
    }
    // leaf expansion and sum: y(i) = y_near(i) + U_i y^_i   (Sec. 4.4, Sec. 4.1)
    for (int64_t j = 0; j < nleaves; ++j) {
        LRow r{true, j, true, int(s.size(lf + j)), h2::ROW_OUT_P, {}};
        if (lowrank) r.b.push_back({off_U[j], kl[q], 0, false, lf + j});
        L.push_back(std::move(r));
    }
    emit(PH_LEAF, bk, A.basis, L);
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
    if (prm->storage < H2_FP64 || prm->storage > H2_BF16_SCALED) fail(H2_ERR_INVALID_ARG, "bad storage");
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

hipEvent_t take_event(h2_matrix_ &A) {
    if (!A.spare.empty()) {
        hipEvent_t e = A.spare.back();
        A.spare.pop_back();
        return e;
    }
    hipEvent_t e;
    check_hip(hipEventCreate(&e), "hipEventCreate");
    return e;
}

// Enqueues the lists in order, with profiling events at phase boundaries
// when enabled; launch(w) enqueues one list.
template <class Launch>
void run_lists(h2_matrix_ &A, const std::vector<WorkList> &lists, hipStream_t st, Launch launch) {
    hipEvent_t ev[PH_COUNT + 1] = {};
    if (A.prof)
        for (auto &e : ev) e = take_event(A);
    int next_phase = 0;   // lists are in phase order; each phase's event precedes its lists
    for (const WorkList &w : lists) {
        while (A.prof && next_phase <= int(w.phase))
            check_hip(hipEventRecord(ev[next_phase++], st), "hipEventRecord");
        launch(w);
    }
    if (A.prof) {
        while (next_phase <= PH_COUNT) check_hip(hipEventRecord(ev[next_phase++], st), "hipEventRecord");
        A.pending.insert(A.pending.end(), ev, ev + PH_COUNT + 1);
    }
}

// Enqueues the whole single-vector product on st.
void run_product(h2_matrix_ &A, const double *x, double *y, hipStream_t st) {
    run_lists(A, A.lists, st, [&](const WorkList &w) {
        h2::RowLaunch L;
        L.rows = w.rows;
        L.nrows = w.nrows;
        L.blks = w.blks;
        L.data = w.data;
        L.scales = A.scales;
        L.in1 = x;
        L.init = nullptr;
        L.out1 = nullptr;
        switch (w.phase) {
            case PH_UP:
                L.in0 = A.xh;
                L.out0 = A.xh;
                break;
            case PH_STREAM:
                L.in0 = A.xh;
                L.out0 = A.yh;
                L.out1 = A.ynear;
                if (w.red) {   // chunks of a split list: partial sums, then their sums per row
                    L.out0 = L.out1 = w.partials;
                    check_hip(h2::launch_blockrow(L, w.kind, A.vec_f64, int(w.phase), st, 1), "blockrow launch");
                    check_hip(h2::launch_reduce_chunks(w.red, w.nred, w.partials, A.yh, A.ynear, A.vec_f64, st),
                              "chunk sum launch");
                    return;
                }
                break;
            case PH_DOWN:
                L.in0 = A.yh;
                L.init = A.yh;
                L.out0 = A.yh;
                break;
            default:
                L.in0 = A.yh;
                L.init = A.ynear;
                L.out0 = A.yh;
                L.out1 = y;
                break;
        }
        check_hip(h2::launch_blockrow(L, w.kind, A.vec_f64, int(w.phase), st), "blockrow launch");
    });
}

// Tile workspace of the many-right-hand-side product, allocated at first use.
void ensure_tiles(h2_matrix_ &A) {
    if (A.t_xh) return;
    const int64_t kp = (A.st.rank + 15) / 16 * 16;
    const int64_t tree = A.st.nnodes * kp * h2::MM_TILE, pts = (int64_t(1) << A.st.q) * A.tile_slot;
    A.t_xh = static_cast<float *>(A.mem.alloc(tree * 4));
    A.t_yh = static_cast<float *>(A.mem.alloc(tree * 4));
    A.t_x = static_cast<float *>(A.mem.alloc(pts * 4));
    A.t_ynear = static_cast<float *>(A.mem.alloc(pts * 4));
}

// One pass of up to MM_TILE right-hand sides on the matrix cores.
void run_tile_pass(h2_matrix_ &A, const double *X, int64_t ldx, double *Y, int64_t ldy, int nrhs, int j0,
                   const h2::MmConfig &cfg, hipStream_t st) {
    const int64_t nleaves = int64_t(1) << A.st.q;
    {
        check_hip(h2::launch_pack(X, ldx, j0, nrhs, A.d_leaf_begin, A.d_leaf_end, nleaves, A.tile_slot, A.t_x, st),
                  "pack launch");
        run_lists(A, A.mm_lists, st, [&](const WorkList &w) {
            h2::MmLaunch L;
            L.rows = w.rows;
            L.items = w.items;
            L.nitems = w.nitems;
            L.blks = w.blks;
            L.data = w.data;
            L.scales = A.scales;
            L.in_tree = nullptr;
            L.in_pts = A.t_x;
            L.init = nullptr;
            L.out_tree = nullptr;
            L.out_pts = nullptr;
            L.Y = Y + int64_t(j0) * ldy;
            L.ldy = ldy;
            L.ncols = std::min(h2::MM_TILE, nrhs - j0);
            switch (w.phase) {
                case PH_UP:
                    L.in_tree = A.t_xh;
                    L.out_tree = A.t_xh;
                    break;
                case PH_STREAM:
                    L.in_tree = A.t_xh;
                    L.out_tree = A.t_yh;
                    L.out_pts = A.t_ynear;
                    break;
                case PH_DOWN:
                    L.in_tree = A.t_yh;
                    L.init = A.t_yh;
                    L.out_tree = A.t_yh;
                    break;
                default:
                    L.in_tree = A.t_yh;
                    L.init = A.t_ynear;
                    break;
            }
            check_hip(h2::launch_mm(L, w.kind, int(w.phase), cfg, st), "mfma launch");
        });
    }
}

// Chooses the block loop (pipelined or not) for this matrix and the tile
// width of pass j0 by timing both on that pass, unless cached.
void tune_tiles(h2_matrix_ &A, const double *X, int64_t ldx, double *Y, int64_t ldy, int nrhs, int j0,
                hipStream_t st);

// Y = A X on the matrix cores, MM_TILE right-hand sides per pass.
void run_tiles(h2_matrix_ &A, const double *X, int64_t ldx, double *Y, int64_t ldy, int nrhs, hipStream_t st) {
    ensure_tiles(A);
    for (int j0 = 0; j0 < nrhs; j0 += h2::MM_TILE) {
        const int w = std::min(h2::MM_TILE, nrhs - j0) <= 16 ? 1 : 0;
        if (!A.mm_tuned[w]) tune_tiles(A, X, ldx, Y, ldy, nrhs, j0, st);
        run_tile_pass(A, X, ldx, Y, ldy, nrhs, j0, A.mm_cfg[w], st);
    }
}

// ---------------------------------------------------------------- batches
// Many H^2 matrices of uneven size and rank per launch: the members' tile
// lists are concatenated per "level slot" -- upsweep lists aligned by their
// distance from the leaves, downsweep lists aligned at their end (the leaf
// level), one streaming slot and one leaf slot -- so every slot is one
// grid-strided launch over all members.  Tiles of all members live in one
// pool; block operands are absolute addresses into the members' storage.
struct BatchSlot {
    Phase phase;
    int kind;
    h2::RowDesc *rows;
    int64_t nrows;
    h2::BlkDesc *blks;
    int32_t *items;
    int64_t nitems;
};

struct BatchConfigCache {
    std::mutex mu;   // handles may be tuned from several host threads
    std::vector<std::pair<std::string, h2::MmConfig>> entries;
};
BatchConfigCache &config_cache() {
    static BatchConfigCache c;
    return c;
}

}  // namespace

struct h2_batch_ {
    std::vector<h2_matrix_ *> mats;
    int nrhs = 0;
    DeviceArena mem;
    float *pool = nullptr;
    float *scales = nullptr;
    std::vector<BatchSlot> slots;
    h2::PackEntry *pack = nullptr;
    int64_t npack = 0;
    double **d_Xtab = nullptr, **d_Ytab = nullptr;
    int64_t *d_ldx = nullptr, *d_ldy = nullptr;
    hipStream_t own = nullptr;
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    // pinned host copy of the per-call tables (X, Y pointers, ldx, ldy), and
    // the event after their upload: the next call waits for it before rewriting
    int64_t *h_tables = nullptr;
    hipEvent_t ev_tables = nullptr;
    bool tables_pending = false;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    h2::MmConfig cfg{1, 0};
    bool tuned = false;
    double tuned_ms = 0.0;
    std::string signature;
    int64_t cu_count = 256;
    bool counted = false;   // the members' batch_refs include this batch

    ~h2_batch_() {
        if (counted)
            for (h2_matrix_ *m : mats) --m->batch_refs;
        if (ev_tables) {
            if (tables_pending) (void)hipEventSynchronize(ev_tables);
            (void)hipEventDestroy(ev_tables);
        }
        if (h_tables) (void)hipHostFree(h_tables);
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (ev_in) (void)hipEventDestroy(ev_in);
        if (ev_out) (void)hipEventDestroy(ev_out);
        if (own) (void)hipStreamDestroy(own);
    }
};

namespace {

// Enqueues one batched product (tables already set) with configuration cfg.
void batch_enqueue(h2_batch_ &B, const h2::MmConfig &cfg, hipStream_t st) {
    check_hip(h2::launch_batch_pack(B.pack, B.npack, B.d_Xtab, B.d_ldx, B.nrhs, B.pool,
                                    cfg.grid > 0 ? cfg.grid : 0, st),
              "batch pack");
    for (const BatchSlot &sl : B.slots) {
        h2::MmBatchLaunch L{sl.rows, sl.items, sl.nitems, sl.blks, B.scales, B.pool, B.d_Ytab, B.d_ldy, B.nrhs};
        check_hip(h2::launch_mm_batch(L, sl.kind, int(sl.phase), cfg, st), "batch launch");
    }
}

std::string config_file() {
    const char *p = std::getenv("H2MV_AUTOTUNE_CACHE");
    return p ? std::string(p) : std::string();
}

// The cache file holds one "signature pipelined grid" line per entry.
bool cached_config(const std::string &sig, h2::MmConfig &cfg) {
    std::lock_guard<std::mutex> lock(config_cache().mu);
    for (auto &e : config_cache().entries)
        if (e.first == sig) {
            cfg = e.second;
            return true;
        }
    const std::string f = config_file();
    if (f.empty()) return false;
    FILE *fp = std::fopen(f.c_str(), "r");
    if (!fp) return false;
    char line[512];
    bool found = false;
    while (std::fgets(line, sizeof line, fp)) {
        char key[400];
        int pipe = 0;
        long long grid = 0;
        if (std::sscanf(line, "%399s %d %lld", key, &pipe, &grid) == 3 && sig == key) {
            cfg = {pipe, grid};
            found = true;
        }
    }
    std::fclose(fp);
    if (found) config_cache().entries.push_back({sig, cfg});
    return found;
}

void store_config(const std::string &sig, const h2::MmConfig &cfg) {
    std::lock_guard<std::mutex> lock(config_cache().mu);
    config_cache().entries.push_back({sig, cfg});
    const std::string f = config_file();
    if (f.empty()) return;
    if (FILE *fp = std::fopen(f.c_str(), "a")) {
        std::fprintf(fp, "%s %d %lld\n", sig.c_str(), cfg.pipelined, static_cast<long long>(cfg.grid));
        std::fclose(fp);
    }
}

// Times every candidate configuration on the batch (tables set) and keeps the
// fastest: pipelined block loop or not, times persistent grids of 2, 4 and 8
// workgroups per compute unit or one workgroup per two rows.
void batch_autotune(h2_batch_ &B) {
    h2::MmConfig best{1, 0};
    if (cached_config(B.signature, best)) {
        B.cfg = best;
        B.tuned = true;
        return;
    }
    hipEvent_t t0, t1;
    check_hip(hipEventCreate(&t0), "hipEventCreate");
    check_hip(hipEventCreate(&t1), "hipEventCreate");
    double best_ms = 1e30;
    const int64_t cu = (B.cu_count + h2::MM_XCDS - 1) / h2::MM_XCDS * h2::MM_XCDS;
    const int64_t grids[4] = {0, 2 * cu, 4 * cu, 8 * cu};
    for (int pipe = 0; pipe < 2; ++pipe)
        for (int64_t grid : grids) {
            const h2::MmConfig c{pipe, grid};
            batch_enqueue(B, c, B.own);   // warm-up
            float ms_best = 1e30f;
            for (int rep = 0; rep < 2; ++rep) {
                check_hip(hipEventRecord(t0, B.own), "hipEventRecord");
                batch_enqueue(B, c, B.own);
                check_hip(hipEventRecord(t1, B.own), "hipEventRecord");
                check_hip(hipEventSynchronize(t1), "hipEventSynchronize");
                float ms = 0.0f;
                check_hip(hipEventElapsedTime(&ms, t0, t1), "hipEventElapsedTime");
                ms_best = std::min(ms_best, ms);
            }
            if (ms_best < best_ms) {
                best_ms = ms_best;
                best = c;
            }
        }
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    B.cfg = best;
    B.tuned = true;
    B.tuned_ms = best_ms;
    store_config(B.signature, best);
}

void tune_tiles(h2_matrix_ &A, const double *X, int64_t ldx, double *Y, int64_t ldy, int nrhs, int j0,
                hipStream_t st) {
    const int w = std::min(h2::MM_TILE, nrhs - j0) <= 16 ? 1 : 0;
    int64_t nblocks = 0;
    for (const auto &hb : A.mm_host_blks) nblocks += int64_t(hb.size());
    const std::string sig = "single-k" + std::to_string(A.block_kind) + "-n" + std::to_string(A.st.n) + "-r" +
                            std::to_string(A.st.rank) + "-blocks" + std::to_string(nblocks) + "-nt" +
                            std::to_string(w ? 16 : 32);
    h2::MmConfig best{1, 0};
    if (!cached_config(sig, best)) {
        const bool prof = A.prof;   // tuning runs stay out of the profile
        A.prof = false;
        hipEvent_t t0, t1;
        check_hip(hipEventCreate(&t0), "hipEventCreate");
        check_hip(hipEventCreate(&t1), "hipEventCreate");
        float best_ms = 1e30f;
        for (int pipe = 0; pipe < 2; ++pipe) {
            const h2::MmConfig c{pipe, 0};
            run_tile_pass(A, X, ldx, Y, ldy, nrhs, j0, c, st);   // warm-up
            check_hip(hipEventRecord(t0, st), "hipEventRecord");
            run_tile_pass(A, X, ldx, Y, ldy, nrhs, j0, c, st);
            check_hip(hipEventRecord(t1, st), "hipEventRecord");
            check_hip(hipEventSynchronize(t1), "hipEventSynchronize");
            float ms = 0.0f;
            check_hip(hipEventElapsedTime(&ms, t0, t1), "hipEventElapsedTime");
            if (ms < best_ms) {
                best_ms = ms;
                best = c;
            }
        }
        (void)hipEventDestroy(t0);
        (void)hipEventDestroy(t1);
        A.prof = prof;
        store_config(sig, best);
    }
    A.mm_cfg[w] = best;
    A.mm_tuned[w] = true;
}

void build_batch(h2_batch_ &B, hipStream_t stream) {
    const int nm = int(B.mats.size());
    const int kind_basis = B.mats[0]->basis_kind, kind_block = B.mats[0]->block_kind;
    for (h2_matrix_ *M : B.mats) {
        if (M->structure_only) fail(H2_ERR_INVALID_ARG, "structure-only member");
        if (M->storage == H2_FP64) fail(H2_ERR_UNSUPPORTED, "batches need FP32 or BF16 storage");
        if (M->basis_kind != kind_basis || M->block_kind != kind_block)
            fail(H2_ERR_UNSUPPORTED, "all batch members need the same storage");
    }
    // pool layout and scale concatenation
    std::vector<int64_t> xh(nm), yh(nm), xp(nm), yn(nm), sb(nm);
    int64_t pool = 0, nsc = 0;
    for (int b = 0; b < nm; ++b) {
        const h2_matrix_ &M = *B.mats[b];
        const int64_t kp = (M.st.rank + 15) / 16 * 16;
        const int64_t tree = M.st.nnodes * kp * h2::MM_TILE, pts = (int64_t(1) << M.st.q) * M.tile_slot;
        xh[b] = pool; pool += tree;
        yh[b] = pool; pool += tree;
        xp[b] = pool; pool += pts;
        yn[b] = pool; pool += pts;
        sb[b] = nsc; nsc += M.nscales;
    }
    B.pool = static_cast<float *>(B.mem.alloc(pool * 4));
    B.scales = static_cast<float *>(B.mem.alloc(std::max<int64_t>(1, nsc) * 4));
    for (int b = 0; b < nm; ++b)
        if (B.mats[b]->nscales > 0)
            check_hip(hipMemcpyAsync(B.scales + sb[b], B.mats[b]->scales, B.mats[b]->nscales * 4,
                                     hipMemcpyDeviceToDevice, stream),
                      "copy scales");
    // per-member list indices by phase
    std::vector<std::vector<int>> up(nm), down(nm);
    std::vector<int> strm(nm, -1), leaf(nm, -1);
    size_t nu = 0, nd = 0;
    for (int b = 0; b < nm; ++b) {
        const auto &L = B.mats[b]->mm_lists;
        for (int li = 0; li < int(L.size()); ++li) {
            if (L[li].phase == PH_UP) up[b].push_back(li);
            if (L[li].phase == PH_DOWN) down[b].push_back(li);
            if (L[li].phase == PH_STREAM) strm[b] = li;
            if (L[li].phase == PH_LEAF) leaf[b] = li;
        }
        nu = std::max(nu, up[b].size());
        nd = std::max(nd, down[b].size());
    }
    // translates member b's list li into the slot's rows/blocks
    auto append = [&](int b, int li, std::vector<h2::RowDesc> &rows, std::vector<h2::BlkDesc> &blks) {
        const h2_matrix_ &M = *B.mats[b];
        const WorkList &w = M.mm_lists[li];
        const int64_t es = h2::elem_bytes(w.kind);
        const int64_t base = int64_t(reinterpret_cast<uintptr_t>(w.data));
        const auto &hr = M.mm_host_rows[li];
        const auto &hb = M.mm_host_blks[li];
        for (const h2::RowDesc &r0 : hr) {
            h2::RowDesc r = r0;
            const bool in_x = (r.sel & h2::ROW_IN_X) != 0, out_p = (r.sel & h2::ROW_OUT_P) != 0;
            int64_t in_base = 0;
            switch (w.phase) {
                case PH_UP:
                    r.out += xh[b];
                    in_base = in_x ? xp[b] : xh[b];
                    break;
                case PH_STREAM:
                    r.out += out_p ? yn[b] : yh[b];
                    in_base = in_x ? xp[b] : xh[b];
                    break;
                case PH_DOWN:
                    r.out += yh[b];
                    if (r.init >= 0) r.init += yh[b];
                    in_base = yh[b];
                    break;
                default:
                    r.init += yn[b];
                    r.sel |= b << 8;
                    in_base = yh[b];
                    break;
            }
            const int32_t b0 = int32_t(blks.size());
            for (int32_t k = r0.b0; k < r0.b1; ++k) {
                h2::BlkDesc d = hb[k];
                d.a = base + d.a * es;
                d.in += in_base;
                d.sidx += int32_t(sb[b]);
                blks.push_back(d);
            }
            r.b0 = b0;
            r.b1 = int32_t(blks.size());
            rows.push_back(r);
        }
    };
    auto add_slot = [&](Phase ph, int kind, std::vector<h2::RowDesc> &rows, std::vector<h2::BlkDesc> &blks) {
        if (rows.empty()) return;
        const std::vector<int32_t> it = wave_items(rows, blks);
        BatchSlot sl{ph, kind, B.mem.upload(rows, stream), int64_t(rows.size()), B.mem.upload(blks, stream),
                     B.mem.upload(it, stream), int64_t(it.size())};
        B.slots.push_back(sl);
    };
    std::vector<h2::RowDesc> rows;
    std::vector<h2::BlkDesc> blks;
    for (size_t j = 0; j < nu; ++j) {
        rows.clear(); blks.clear();
        for (int b = 0; b < nm; ++b)
            if (j < up[b].size()) append(b, up[b][j], rows, blks);
        add_slot(PH_UP, kind_basis, rows, blks);
    }
    rows.clear(); blks.clear();
    for (int b = 0; b < nm; ++b) append(b, strm[b], rows, blks);
    add_slot(PH_STREAM, kind_block, rows, blks);
    for (size_t j = 0; j < nd; ++j) {
        rows.clear(); blks.clear();
        for (int b = 0; b < nm; ++b) {
            const int64_t k = int64_t(j) - int64_t(nd - down[b].size());
            if (k >= 0) append(b, down[b][k], rows, blks);
        }
        add_slot(PH_DOWN, kind_basis, rows, blks);
    }
    rows.clear(); blks.clear();
    for (int b = 0; b < nm; ++b) append(b, leaf[b], rows, blks);
    add_slot(PH_LEAF, kind_basis, rows, blks);
    // point-tile pack entries
    std::vector<h2::PackEntry> pe;
    int64_t total_rows = 0, total_blocks = 0;
    for (int b = 0; b < nm; ++b) {
        const h2_matrix_ &M = *B.mats[b];
        const int64_t nl = int64_t(1) << M.st.q, lf = Structure::first(M.st.q);
        for (int64_t j = 0; j < nl; ++j)
            pe.push_back({xp[b] + j * M.tile_slot, M.st.begin[lf + j], int32_t(M.st.size(lf + j)), b});
    }
    for (const BatchSlot &sl : B.slots) total_rows += sl.nrows;
    for (h2_matrix_ *M : B.mats)
        for (const auto &hb : M->mm_host_blks) total_blocks += int64_t(hb.size());
    B.pack = B.mem.upload(pe, stream);
    B.npack = int64_t(pe.size());
    B.d_Xtab = static_cast<double **>(B.mem.alloc(nm * 8));
    B.d_Ytab = static_cast<double **>(B.mem.alloc(nm * 8));
    B.d_ldx = static_cast<int64_t *>(B.mem.alloc(nm * 8));
    B.d_ldy = static_cast<int64_t *>(B.mem.alloc(nm * 8));
    int dev = 0, cus = 256;
    check_hip(hipGetDevice(&dev), "hipGetDevice");
    check_hip(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev), "device attribute");
    B.cu_count = cus;
    B.signature = "batch-k" + std::to_string(kind_block) + "-r" + std::to_string(B.nrhs) + "-m" + std::to_string(nm) +
                  "-rows" + std::to_string(total_rows) + "-blocks" + std::to_string(total_blocks) + "-cu" +
                  std::to_string(cus);
    check_hip(hipStreamCreateWithFlags(&B.own, hipStreamNonBlocking), "hipStreamCreate");
    check_hip(hipEventCreateWithFlags(&B.ev_in, hipEventDisableTiming), "hipEventCreate");
    check_hip(hipEventCreateWithFlags(&B.ev_out, hipEventDisableTiming), "hipEventCreate");
    check_hip(hipEventCreateWithFlags(&B.ev_tables, hipEventDisableTiming), "hipEventCreate");
    check_hip(hipHostMalloc(reinterpret_cast<void **>(&B.h_tables), size_t(4 * nm) * 8, hipHostMallocDefault),
              "hipHostMalloc");
    check_hip(hipStreamSynchronize(stream), "batch build");
}

}  // namespace

extern "C" {

const char *h2_last_error(void) { return g_last_error.c_str(); }

h2_status h2_build_from_points(const double *points, int64_t n, const h2_params *prm, void *stream,
                               h2_handle *out) {
    if (out) *out = nullptr;
    h2_matrix_ *A = nullptr;
    try {
        if (!out) fail(H2_ERR_INVALID_ARG, "NULL out");
        validate_params(points, n, prm);
        A = new h2_matrix_();
        A->storage = prm->storage;
        A->structure_only = (prm->flags & H2_FLAG_STRUCTURE_ONLY) != 0;
        A->basis_kind = prm->storage == H2_FP64 ? h2::ELEM_F64 : h2::ELEM_F32;
        A->block_kind = prm->storage == H2_FP64   ? h2::ELEM_F64
                        : prm->storage == H2_FP32 ? h2::ELEM_F32
                                                  : h2::ELEM_BF16;
        A->vec_f64 = prm->storage == H2_FP64;
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

// Checks the arrays and fills the host structure from them.
}  // extern "C"

namespace {

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
    int64_t fi = 0;
    for (int l = 0; l <= q; ++l) {
        const h2::Bsr &B = s.coupling[l];
        if (o->S_rowptr && o->S_rowptr[l]) std::copy(B.rowptr.begin(), B.rowptr.end(), o->S_rowptr[l]);
        if (o->S_colidx && o->S_colidx[l]) std::copy(B.colidx.begin(), B.colidx.end(), o->S_colidx[l]);
        const int64_t kk = int64_t(kl[l]) * kl[l];
        for (int64_t b = 0; b < B.blocks(); ++b, ++fi)
            if (o->S && o->S[l]) rd.block(A.off_blk[fi], kl[l], kl[l], false, scale_of(fi), o->S[l] + b * kk);
    }
    if (o->D_rowptr) std::copy(s.dense.rowptr.begin(), s.dense.rowptr.end(), o->D_rowptr);
    if (o->D_colidx) std::copy(s.dense.colidx.begin(), s.dense.colidx.end(), o->D_colidx);
    if (o->D) {
        int64_t doff = 0;
        for (int64_t i = 0; i < nleaves; ++i)
            for (int32_t b = s.dense.rowptr[i]; b < s.dense.rowptr[i + 1]; ++b, ++fi) {
                const int R = int(s.size(lf + i)), C = int(s.size(lf + s.dense.colidx[b]));
                rd.block(A.off_blk[fi], R, C, false, scale_of(fi), o->D + doff);
                doff += int64_t(R) * C;
            }
    }
}

}  // namespace

extern "C" {

h2_status h2_build_from_arrays(const h2_arrays *arrays, int storage, void *stream, h2_handle *out) {
    if (out) *out = nullptr;
    h2_matrix_ *A = nullptr;
    try {
        if (!out) fail(H2_ERR_INVALID_ARG, "NULL out");
        if (storage < H2_FP64 || storage > H2_BF16_SCALED) fail(H2_ERR_INVALID_ARG, "storage out of range");
        A = new h2_matrix_();
        structure_from_arrays(arrays, A->st);
        A->storage = storage;
        A->basis_kind = storage == H2_FP64 ? h2::ELEM_F64 : h2::ELEM_F32;
        A->block_kind = storage == H2_FP64 ? h2::ELEM_F64 : storage == H2_FP32 ? h2::ELEM_F32 : h2::ELEM_BF16;
        A->vec_f64 = storage == H2_FP64;
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

}  // extern "C"

namespace {

// Basis orthogonalization and projection of the coupling blocks in place
// (one basis tree, or a row and a column tree of their own).
void orthogonalize(h2_matrix_ &A, hipStream_t st) {
    const Structure &s = A.st;
    const int q = s.q;
    if (A.storage != H2_FP64) fail(H2_ERR_UNSUPPORTED, "orthogonalization needs FP64 storage");
    if (s.lmin > q) return;   // no coupling block: nothing to orthogonalize
    const int64_t nleaves = int64_t(1) << q, lf = Structure::first(q);
    for (int64_t j = 0; j < nleaves; ++j)
        if (s.size(lf + j) < s.lrank[q]) fail(H2_ERR_UNSUPPORTED, "a leaf holds fewer rows than the rank");
    for (int l = q; l > s.lmin; --l)
        if (2 * s.lrank[l] < s.lrank[l - 1]) fail(H2_ERR_UNSUPPORTED, "a level's rank exceeds twice its children's");
    std::vector<h2::ProjDesc> proj;
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
    L.T = static_cast<double *>(scratch.alloc(s.nnodes * int64_t(kmax) * kmax * 8));
    if (!A.symmetric) L.T_col = static_cast<double *>(scratch.alloc(s.nnodes * int64_t(kmax) * kmax * 8));
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
    std::vector<int64_t> src_fill;
    std::vector<int32_t> src_R, src_C;
    auto transpose_bsr = [&](const h2::Bsr &in, int64_t rows, int64_t fill0, h2::Bsr &out,
                             const std::function<void(int64_t, int64_t)> &dims) {
        out.rowptr.assign(size_t(rows + 1), 0);
        for (int32_t c : in.colidx) ++out.rowptr[size_t(c) + 1];
        for (int64_t i = 0; i < rows; ++i) out.rowptr[i + 1] += out.rowptr[i];
        out.colidx.assign(in.colidx.size(), 0);
        std::vector<int32_t> next(out.rowptr.begin(), out.rowptr.end() - 1);
        std::vector<int64_t> from(in.colidx.size());
        for (int64_t i = 0; i < rows; ++i)
            for (int32_t t = in.rowptr[i]; t < in.rowptr[i + 1]; ++t) {
                const int32_t pos = next[in.colidx[t]]++;
                out.colidx[pos] = int32_t(i);
                from[pos] = t;
            }
        for (size_t pos = 0; pos < from.size(); ++pos) {
            src_fill.push_back(fill0 + from[pos]);
            dims(from[pos], int64_t(pos));
        }
    };
    int64_t fill0 = 0;
    for (int l = 0; l <= q; ++l) {
        transpose_bsr(s.coupling[l], int64_t(1) << l, fill0, B->st.coupling[l], [&](int64_t, int64_t) {
            src_R.push_back(kl[l]);
            src_C.push_back(kl[l]);
        });
        fill0 += s.coupling[l].blocks();
    }
    {
        // dense block t of A: rows of leaf i (its BSR row), columns of leaf colidx[t]
        std::vector<int32_t> row_of(s.dense.colidx.size());
        for (int64_t i = 0; i < nleaves; ++i)
            for (int32_t t = s.dense.rowptr[i]; t < s.dense.rowptr[i + 1]; ++t) row_of[t] = int32_t(i);
        transpose_bsr(s.dense, nleaves, fill0, B->st.dense, [&](int64_t t, int64_t) {
            src_R.push_back(int32_t(s.size(lf + row_of[t])));
            src_C.push_back(int32_t(s.size(lf + s.dense.colidx[t])));
        });
    }
    int64_t ncoupling = 0;
    const std::vector<h2::FillDesc> fill = make_layout(*B, ncoupling);
    DeviceArena scratch;
    std::vector<h2::TransDesc> tb(fill.size()), tbas;
    for (size_t fb = 0; fb < fill.size(); ++fb)
        tb[fb] = {A.off_blk[size_t(src_fill[fb])], B->off_blk[fb], src_R[fb], src_C[fb]};
    if (s.lmin <= q) {
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

// S_ji = S_ij^T, bit for bit, for every coupling block (FP64 storage): the
// mirror of each block is found by binary search in its mirror row (sorted
// per row on the host), and the pairs are compared on the device.
bool coupling_symmetric(h2_matrix_ &A, hipStream_t st) {
    const Structure &s = A.st;
    std::vector<h2::MirrorDesc> pairs;
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

// Algebraic compression (Sec. 5): orthogonalization, basis generation,
// truncation with relative threshold eps (rank of a level: the largest count
// of kept singular values over its nodes, of both trees when rows and columns
// have their own), projection of the coupling blocks into the truncated bases;
// the representation is rebuilt with the new ranks.
void compress(h2_matrix_ &A, double eps, hipStream_t st, int *ranks_out) {
    if (!(eps >= 0.0) || !std::isfinite(eps)) fail(H2_ERR_INVALID_ARG, "eps must be finite and >= 0");
    if (A.batch_refs > 0) fail(H2_ERR_INVALID_ARG, "the matrix belongs to a batch (free the batch first)");
    if (A.storage != H2_FP64) fail(H2_ERR_UNSUPPORTED, "compression needs FP64 storage");
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
            L.T = static_cast<double *>(scratch.alloc(tree * 8));
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
        for (size_t i = 0; i < blk.size(); ++i) {
            const int l = int(std::floor(std::log2(double(blk[i].row + 1))));
            blk[i].out = B->off_blk[i];
            blk[i].kout = kt[l];
        }
        check_hip(h2::launch_project(static_cast<const double *>(A.blocks), static_cast<double *>(B->blocks),
                                     scratch.upload(blk, st), int64_t(blk.size()), Lr.T, Lc.T, kmax, st),
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

}  // namespace

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

h2_status h2_matvec(h2_handle A, const double *x, double *y, void *stream) {
    try {
        if (!A || !x || !y) fail(H2_ERR_INVALID_ARG, "NULL argument");
        if (A->structure_only) fail(H2_ERR_INVALID_ARG, "structure-only handle");
        run_product(*A, x, y, static_cast<hipStream_t>(stream));
        return H2_OK;
    } catch (const Failure &f) {
        g_last_error = f.what;
        return f.code;
    } catch (...) {
        g_last_error = "internal error";
        return H2_ERR_INTERNAL;
    }
}

h2_status h2_matmat(h2_handle A, const double *X, int64_t ldx, double *Y, int64_t ldy, int nrhs,
                    void *stream) {
    try {
        if (!A || !X || !Y) fail(H2_ERR_INVALID_ARG, "NULL argument");
        if (A->structure_only) fail(H2_ERR_INVALID_ARG, "structure-only handle");
        if (nrhs < 1) fail(H2_ERR_INVALID_ARG, "nrhs must be >= 1");
        if (ldx < A->st.n || ldy < A->st.n) fail(H2_ERR_INVALID_ARG, "leading dimension below n");
        const hipStream_t st = static_cast<hipStream_t>(stream);
        if (A->storage == H2_FP64) {
            // FP64 storage: one single-vector product per column (FP64 arithmetic throughout)
            for (int j = 0; j < nrhs; ++j) run_product(*A, X + int64_t(j) * ldx, Y + int64_t(j) * ldy, st);
        } else {
            run_tiles(*A, X, ldx, Y, ldy, nrhs, st);
        }
        return H2_OK;
    } catch (const Failure &f) {
        g_last_error = f.what;
        return f.code;
    } catch (...) {
        g_last_error = "internal error";
        return H2_ERR_INTERNAL;
    }
}

void h2_free(h2_handle A) { delete A; }

h2_status h2_get_info(h2_handle A, h2_info *info) {
    if (!A || !info) {
        g_last_error = "NULL argument";
        return H2_ERR_INVALID_ARG;
    }
    const h2::Structure &s = A->st;
    h2_info r;
    std::memset(&r, 0, sizeof(r));
    r.n = s.n;
    r.dim = s.dim;
    r.leaf_size = s.leaf;
    r.cheb_p = s.cheb_p;
    r.rank = s.rank;
    r.levels_q = s.q;
    r.lmin = s.lmin;
    r.storage = A->storage;
    r.nnodes = s.nnodes;
    for (const auto &B : s.coupling) r.coupling_blocks += B.blocks();
    r.dense_blocks = s.dense.blocks();
    r.bytes_coupling = A->bytes_coupling;
    r.bytes_dense = A->bytes_dense;
    r.bytes_leaf_bases = A->bytes_leaf;
    r.bytes_transfers = A->bytes_transfer;
    r.bytes_device_total = A->mem.bytes;
    r.near_ties = s.near_ties;
    *info = r;
    return H2_OK;
}

h2_status h2_get_perm(h2_handle A, int64_t *perm) {
    if (!A || !perm) {
        g_last_error = "NULL argument";
        return H2_ERR_INVALID_ARG;
    }
    std::memcpy(perm, A->st.perm.data(), A->st.perm.size() * sizeof(int64_t));
    return H2_OK;
}

h2_status h2_get_level_bsr(h2_handle A, int level, int64_t *count, int32_t *rowptr, int32_t *colidx) {
    if (!A || !count || level < -1 || level > A->st.q) {
        g_last_error = "bad argument";
        return H2_ERR_INVALID_ARG;
    }
    const h2::Bsr &B = level < 0 ? A->st.dense : A->st.coupling[level];
    *count = B.blocks();
    if (rowptr) std::memcpy(rowptr, B.rowptr.data(), B.rowptr.size() * sizeof(int32_t));
    if (colidx) std::memcpy(colidx, B.colidx.data(), B.colidx.size() * sizeof(int32_t));
    return H2_OK;
}

h2_status h2_profile(h2_handle A, int enable) {
    if (!A) {
        g_last_error = "NULL handle";
        return H2_ERR_INVALID_ARG;
    }
    A->prof = enable != 0;
    if (A->prof) {
        std::fill(A->prof_ms, A->prof_ms + 8, 0.0);
        A->prof_calls = 0;
    }
    return H2_OK;
}

h2_status h2_profile_read(h2_handle A, double *ms, int64_t *calls) {
    try {
        if (!A || !ms || !calls) fail(H2_ERR_INVALID_ARG, "NULL argument");
        for (size_t i = 0; i + PH_COUNT < A->pending.size(); i += PH_COUNT + 1) {
            hipEvent_t *ev = &A->pending[i];
            check_hip(hipEventSynchronize(ev[PH_COUNT]), "hipEventSynchronize");
            for (int p = 0; p < PH_COUNT; ++p) {
                float t = 0.0f;
                // end of phase p = start of the next recorded phase
                check_hip(hipEventElapsedTime(&t, ev[p], ev[p + 1]), "hipEventElapsedTime");
                A->prof_ms[p] += t;
            }
            float tot = 0.0f;
            check_hip(hipEventElapsedTime(&tot, ev[0], ev[PH_COUNT]), "hipEventElapsedTime");
            A->prof_ms[PH_COUNT] += tot;
            ++A->prof_calls;
        }
        A->spare.insert(A->spare.end(), A->pending.begin(), A->pending.end());
        A->pending.clear();
        std::copy(A->prof_ms, A->prof_ms + 8, ms);
        *calls = A->prof_calls;
        return H2_OK;
    } catch (const Failure &f) {
        g_last_error = f.what;
        return f.code;
    }
}

h2_status h2_batch_create(const h2_handle *mats, int count, int nrhs, void *stream, h2_batch *out) {
    if (out) *out = nullptr;
    h2_batch_ *B = nullptr;
    try {
        if (!out || !mats || count < 1) fail(H2_ERR_INVALID_ARG, "NULL argument or count < 1");
        if (nrhs < 1) fail(H2_ERR_INVALID_ARG, "nrhs must be >= 1");
        if (nrhs > h2::MM_TILE) fail(H2_ERR_UNSUPPORTED, "batches take at most 32 right-hand sides");
        B = new h2_batch_();
        for (int b = 0; b < count; ++b) {
            if (!mats[b]) fail(H2_ERR_INVALID_ARG, "NULL member");
            B->mats.push_back(mats[b]);
        }
        B->nrhs = nrhs;
        build_batch(*B, static_cast<hipStream_t>(stream));
        for (h2_matrix_ *m : B->mats) ++m->batch_refs;
        B->counted = true;
        *out = B;
        return H2_OK;
    } catch (const Failure &f) {
        delete B;
        g_last_error = f.what;
        return f.code;
    } catch (const std::bad_alloc &) {
        delete B;
        g_last_error = "host allocation failed";
        return H2_ERR_OOM;
    } catch (...) {
        delete B;
        g_last_error = "internal error";
        return H2_ERR_INTERNAL;
    }
}

h2_status h2_batch_matmat(h2_batch B, const double *const *X, const int64_t *ldx, double *const *Y,
                          const int64_t *ldy, void *stream) {
    try {
        if (!B || !X || !ldx || !Y || !ldy) fail(H2_ERR_INVALID_ARG, "NULL argument");
        const int nm = int(B->mats.size());
        for (int b = 0; b < nm; ++b) {
            if (!X[b] || !Y[b]) fail(H2_ERR_INVALID_ARG, "NULL member matrix");
            if (ldx[b] < B->mats[b]->st.n || ldy[b] < B->mats[b]->st.n)
                fail(H2_ERR_INVALID_ARG, "leading dimension below n");
        }
        // pointer tables: written to pinned memory (after the previous call's upload
        // of them has run) and uploaded outside the graph
        if (B->tables_pending) check_hip(hipEventSynchronize(B->ev_tables), "hipEventSynchronize");
        int64_t *tab = B->h_tables;
        for (int b = 0; b < nm; ++b) {
            tab[b] = int64_t(reinterpret_cast<uintptr_t>(X[b]));
            tab[nm + b] = int64_t(reinterpret_cast<uintptr_t>(Y[b]));
            tab[2 * nm + b] = ldx[b];
            tab[3 * nm + b] = ldy[b];
        }
        const hipStream_t user = static_cast<hipStream_t>(stream);
        check_hip(hipEventRecord(B->ev_in, user), "hipEventRecord");
        check_hip(hipStreamWaitEvent(B->own, B->ev_in, 0), "hipStreamWaitEvent");
        check_hip(hipMemcpyAsync(B->d_Xtab, tab, nm * 8, hipMemcpyHostToDevice, B->own), "copy tables");
        check_hip(hipMemcpyAsync(B->d_Ytab, tab + nm, nm * 8, hipMemcpyHostToDevice, B->own), "copy tables");
        check_hip(hipMemcpyAsync(B->d_ldx, tab + 2 * nm, nm * 8, hipMemcpyHostToDevice, B->own), "copy tables");
        check_hip(hipMemcpyAsync(B->d_ldy, tab + 3 * nm, nm * 8, hipMemcpyHostToDevice, B->own), "copy tables");
        check_hip(hipEventRecord(B->ev_tables, B->own), "hipEventRecord");
        B->tables_pending = true;
        if (!B->tuned) batch_autotune(*B);
        if (!B->exec) {
            check_hip(hipStreamBeginCapture(B->own, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
            try {
                batch_enqueue(*B, B->cfg, B->own);
            } catch (...) {
                hipGraph_t aborted = nullptr;   // leave the stream out of capture mode
                (void)hipStreamEndCapture(B->own, &aborted);
                if (aborted) (void)hipGraphDestroy(aborted);
                throw;
            }
            check_hip(hipStreamEndCapture(B->own, &B->graph), "hipStreamEndCapture");
            check_hip(hipGraphInstantiate(&B->exec, B->graph, nullptr, nullptr, 0), "hipGraphInstantiate");
        }
        check_hip(hipGraphLaunch(B->exec, B->own), "hipGraphLaunch");
        check_hip(hipEventRecord(B->ev_out, B->own), "hipEventRecord");
        check_hip(hipStreamWaitEvent(user, B->ev_out, 0), "hipStreamWaitEvent");
        return H2_OK;
    } catch (const Failure &f) {
        g_last_error = f.what;
        return f.code;
    } catch (...) {
        g_last_error = "internal error";
        return H2_ERR_INTERNAL;
    }
}

h2_status h2_batch_tuning(h2_batch B, int *pipelined, int64_t *grid, double *tuned_ms) {
    if (!B || !pipelined || !grid || !tuned_ms) {
        g_last_error = "NULL argument";
        return H2_ERR_INVALID_ARG;
    }
    *pipelined = B->cfg.pipelined;
    *grid = B->cfg.grid;
    *tuned_ms = B->tuned ? B->tuned_ms : -1.0;
    return H2_OK;
}

void h2_batch_free(h2_batch B) { delete B; }

}  // extern "C"
