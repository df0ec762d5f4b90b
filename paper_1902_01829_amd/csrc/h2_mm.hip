// Many right-hand sides on the matrix cores (gfx950 MFMA).
//
// With r right-hand sides every per-node vector of the product becomes a
// k x r tile and every block product a dense contraction (R x C block) x
// (C x r tile).  The phases, work lists and block layout are those of the
// single-vector product; only the arithmetic changes:
//   - tiles hold 32 right-hand sides (one MFMA N dimension), FP32, stored
//     [rhs][row] with a leading dimension rounded up to 16 rows (zero-padded);
//   - v_mfma_f32_32x32x2_f32 does the products on FP32 operands: FP32 blocks
//     as stored, BF16 blocks widened exactly to FP32 (the scale is applied per
//     block).  Splitting the operands into BF16 pieces for the faster BF16
//     MFMA loses accuracy as the tree deepens (measured: 2.5e-6 against 4.7e-7
//     on 2^20 points); the FP32 path matches the single-vector kernels;
//   - one block's products accumulate in FP32, sums over blocks in FP64;
//   - each 32-row half of an output segment has its own wavefront; the two
//     read disjoint halves of every block and share its input tile, which the
//     rows' spatial order keeps in the caches.

#include <hip/hip_runtime.h>

#include <cstdint>

#include "h2_device.h"

namespace h2 {
namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

constexpr int NT = MM_TILE;   // right-hand sides per tile

__device__ inline int round16(int v) { return (v + 15) & ~15; }

// Workgroup -> position in the (spatially ordered) list such that each XCD
// works through one contiguous range: the hardware deals workgroups to the 8
// XCDs round-robin, so workgroup wg runs on XCD wg % 8.
__device__ inline int64_t xcd_local_order(int64_t wg, int64_t nwg) {
    constexpr int64_t kXcds = 8;
    const int64_t x = wg % kXcds, local = wg / kXcds;
    const int64_t base = nwg / kXcds, extra = nwg % kXcds;
    return x * base + (x < extra ? x : extra) + local;
}

// Block operand of one wavefront: 8 column steps of 4 values (FP32 items, or
// raw BF16 words widened at use), and the matching input-tile operand.
template <int KIND> struct BlockA;
template <> struct BlockA<ELEM_F32> {
    f32x4 v[8];
};
template <> struct BlockA<ELEM_BF16> {
    u32x2 v[8];
};
struct TileB {
    f32x4 v[8];
};

// Loads of the block operand with no per-lane condition: lanes past the
// block's last row read its last row (their results are discarded), and
// column groups past the block's width read its last group, which then meets
// the zero padding rows of the input tile.
template <int KIND>
__device__ inline void load_a(const BlkDesc &bd, const void *blk, int R, int ic, int lg, BlockA<KIND> &o) {
    const int C = bd.C, NP = round16(C) >> 3;
#pragma unroll
    for (int p = 0; p < 8; ++p) {
        if (p >= NP) break;   // wave-uniform
        if constexpr (KIND == ELEM_F32) {
            const int CW = (C + 3) >> 2;                      // 4-column groups
            const int cg = 2 * p + lg, cgc = cg < CW ? cg : CW - 1;
            o.v[p] = __builtin_nontemporal_load(
                reinterpret_cast<const f32x4 *>(static_cast<const float *>(blk) + (int64_t(cgc) * R + ic) * 4));
        } else {
            const int CW = (C + 7) >> 3;                      // 8-column groups: half of one per lane
            const int pc = p < CW ? p : CW - 1;
            o.v[p] = __builtin_nontemporal_load(reinterpret_cast<const u32x2 *>(
                static_cast<const uint16_t *>(blk) + (int64_t(pc) * R + ic) * 8 + 4 * lg));
        }
    }
}

__device__ inline void load_b(const BlkDesc &bd, const float *xbase, int li, int lg, TileB &o) {
    const int Cp = round16(bd.C), NP = Cp >> 3;
    const float *xb = xbase + bd.in + li * Cp + 4 * lg;
#pragma unroll
    for (int p = 0; p < 8; ++p) {
        if (p >= NP) break;
        o.v[p] = *reinterpret_cast<const f32x4 *>(xb + 8 * p);
    }
}

// The block's products (K = 2 per MFMA: one column per lane group).
template <int KIND>
__device__ inline f32x16 block_products(const BlockA<KIND> &a_op, const TileB &b_op, int NP) {
    f32x16 acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
#pragma unroll
    for (int p = 0; p < 8; ++p) {
        if (p >= NP) break;
        f32x4 a;
        if constexpr (KIND == ELEM_BF16) {
            const u32x2 w = a_op.v[p];
            a = f32x4{__uint_as_float(w.x << 16), __uint_as_float(w.x & 0xffff0000u),
                      __uint_as_float(w.y << 16), __uint_as_float(w.y & 0xffff0000u)};
        } else {
            a = a_op.v[p];
        }
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a.x, b_op.v[p].x, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a.y, b_op.v[p].y, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a.z, b_op.v[p].z, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a.w, b_op.v[p].w, acc, 0, 0, 0);
    }
    return acc;
}

// Where a work list's operands live.  Single matrix: block offsets are
// element offsets into the matrix's data array, tile offsets index the
// separate tile buffers.  Batch: block "offsets" hold absolute addresses,
// every tile offset indexes one pool, and the leaf phase finds each member's
// result matrix in a device table (member index in RowDesc.sel >> 8).
struct MmArgs {
    const RowDesc *rows;
    int64_t nrows;
    const BlkDesc *blks;
    const void *data;
    const float *scales;
    const float *in_tree, *in_pts, *init;
    float *out_tree, *out_pts;
    double *Y;
    int64_t ldy;
    double *const *Ytab;
    const int64_t *ldytab;
    int ncols;
};

// One output row segment half (mt) of the list, for one wavefront.  Lane l
// owns block row 32*mt + (l % 32) and right-hand side l % 32; for every 8
// block columns 8p .. 8p+7, lane group g = l / 32 supplies columns 8p + 4g + t
// (t = 0..3), one per MFMA.  With PIPE the block loop is software-pipelined:
// the loads of block b + 1 are in flight while block b's products run.
template <int KIND, bool LEAF, bool BATCH, bool PIPE>
__device__ inline void mm_row(const MmArgs &g, int64_t row, int mt, int lane) {
    const RowDesc rd = g.rows[row];
    const int R = rd.R, Rp = round16(R);
    if (32 * mt >= R) return;
    const int li = lane & 31, lg = lane >> 5;
    const int i = 32 * mt + li;   // block row of this lane's A operand
    const int ic = i < R ? i : R - 1;
    const float *xbase = (rd.sel & ROW_IN_X) ? g.in_pts : g.in_tree;
    const void *data = g.data;

    double tot[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) tot[r] = 0.0;

    BlockA<KIND> a_cur, a_nxt;
    TileB b_cur, b_nxt;
    BlkDesc bd_cur, bd_nxt;
    auto block_ptr = [&](const BlkDesc &bd) -> const void * {
        if constexpr (BATCH) return reinterpret_cast<const void *>(bd.a);
        else return static_cast<const char *>(data) + bd.a * (KIND == ELEM_F32 ? 4 : 2);
    };
    if (rd.b0 < rd.b1) {
        bd_cur = g.blks[rd.b0];
        load_a<KIND>(bd_cur, block_ptr(bd_cur), R, ic, lg, a_cur);
        load_b(bd_cur, xbase, li, lg, b_cur);
    }
    for (int b = rd.b0; b < rd.b1; ++b) {
        const bool more = b + 1 < rd.b1;
        if (PIPE && more) {
            bd_nxt = g.blks[b + 1];
            load_a<KIND>(bd_nxt, block_ptr(bd_nxt), R, ic, lg, a_nxt);
            load_b(bd_nxt, xbase, li, lg, b_nxt);
        }
        const f32x16 acc = block_products<KIND>(a_cur, b_cur, round16(bd_cur.C) >> 3);
        const double sc = KIND == ELEM_BF16 ? double(g.scales[bd_cur.sidx]) : 1.0;
#pragma unroll
        for (int r = 0; r < 16; ++r) tot[r] += sc * double(acc[r]);
        if (more) {
            if constexpr (PIPE) {
                a_cur = a_nxt;
                b_cur = b_nxt;
                bd_cur = bd_nxt;
            } else {
                bd_cur = g.blks[b + 1];
                load_a<KIND>(bd_cur, block_ptr(bd_cur), R, ic, lg, a_cur);
                load_b(bd_cur, xbase, li, lg, b_cur);
            }
        }
    }

    // Lane l holds rows 32*mt + 8*q + 4*(l/32) + e (e = 0..3) of right-hand side l % 32.
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int i0 = 32 * mt + 8 * q + 4 * lg;
        if (i0 >= Rp) continue;
        if constexpr (LEAF) {
            // y(i, j) = y_near(i, j) + far part, written to the caller's FP64 matrix
            if (li >= g.ncols) continue;
            const f32x4 yn = *reinterpret_cast<const f32x4 *>(g.init + rd.init + int64_t(li) * Rp + i0);
            const double ynv[4] = {yn.x, yn.y, yn.z, yn.w};
            double *Yb = BATCH ? g.Ytab[rd.sel >> 8] : g.Y;
            const int64_t ldy = BATCH ? g.ldytab[rd.sel >> 8] : g.ldy;
            double *yc = Yb + int64_t(li) * ldy + rd.out;
#pragma unroll
            for (int e = 0; e < 4; ++e)
                if (i0 + e < R) yc[i0 + e] = ynv[e] + tot[4 * q + e];
        } else {
            double v[4];   // rows R .. Rp-1 are the tile's zero padding
#pragma unroll
            for (int e = 0; e < 4; ++e) v[e] = i0 + e < R ? tot[4 * q + e] : 0.0;
            if (rd.init >= 0) {
                const f32x4 t = *reinterpret_cast<const f32x4 *>(g.init + rd.init + int64_t(li) * Rp + i0);
                v[0] += t.x; v[1] += t.y; v[2] += t.z; v[3] += t.w;
            }
            float *o = ((rd.sel & ROW_OUT_P) ? g.out_pts : g.out_tree) + rd.out + int64_t(li) * Rp + i0;
            *reinterpret_cast<f32x4 *>(o) = f32x4{float(v[0]), float(v[1]), float(v[2]), float(v[3])};
        }
    }
}

// Two wavefronts per output row segment (one per 32-row half); a workgroup
// of 4 wavefronts covers 2 segments.  PERSIST: the grid strides over the
// list's workgroup slots (fewer workgroups than slots); otherwise one
// workgroup per slot (no loop, fewer live registers).
template <int KIND, bool LEAF, bool BATCH, bool PIPE, bool PERSIST>
__global__ __launch_bounds__(256) void mm_kernel(MmArgs g) {
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int64_t nslots = (g.nrows + 1) / 2;
    if constexpr (PERSIST) {
        for (int64_t wg = blockIdx.x; wg < nslots; wg += gridDim.x) {
            const int64_t row = xcd_local_order(wg, nslots) * 2 + (wv >> 1);
            if (row < g.nrows) mm_row<KIND, LEAF, BATCH, PIPE>(g, row, wv & 1, lane);
        }
    } else {
        const int64_t row = xcd_local_order(blockIdx.x, nslots) * 2 + (wv >> 1);
        if (row < g.nrows) mm_row<KIND, LEAF, BATCH, PIPE>(g, row, wv & 1, lane);
    }
}

// Copies right-hand sides j0 .. j0+NT-1 of the caller's column-major FP64 X
// into point tiles: leaf j at j * slot, [rhs][row] with a leading dimension of
// its size rounded up to 16, zero-padded (rows and missing right-hand sides).
__global__ __launch_bounds__(256) void pack_kernel(const double *__restrict__ X, int64_t ldx, int j0, int nrhs,
                                                   const int64_t *__restrict__ leaf_begin,
                                                   const int64_t *__restrict__ leaf_end, int64_t slot,
                                                   float *__restrict__ tiles) {
    const int64_t leaf = blockIdx.x;
    const int64_t b = leaf_begin[leaf];
    const int m = int(leaf_end[leaf] - b), mp = round16(m);
    float *t = tiles + leaf * slot;
    for (int e = threadIdx.x; e < NT * mp; e += blockDim.x) {
        const int j = e / mp, c = e - j * mp;
        float v = 0.0f;
        if (c < m && j0 + j < nrhs) v = float(X[(b + c) + int64_t(j0 + j) * ldx]);
        t[e] = v;
    }
}

}  // namespace

hipError_t launch_pack(const double *X, int64_t ldx, int j0, int nrhs, const int64_t *leaf_begin,
                       const int64_t *leaf_end, int64_t nleaves, int64_t slot, float *tiles, hipStream_t st) {
    if (nleaves <= 0) return hipSuccess;
    hipLaunchKernelGGL(pack_kernel, dim3(unsigned(nleaves)), dim3(256), 0, st, X, ldx, j0, nrhs, leaf_begin,
                       leaf_end, slot, tiles);
    return hipGetLastError();
}

template <int KIND, bool LEAF, bool BATCH, bool PIPE, bool PERSIST>
static void launch_one(const MmArgs &g, unsigned grid, hipStream_t st) {
    hipLaunchKernelGGL((mm_kernel<KIND, LEAF, BATCH, PIPE, PERSIST>), dim3(grid), dim3(256), 0, st, g);
}

template <bool BATCH, bool PIPE, bool PERSIST>
static void launch_kind(const MmArgs &g, int kind, bool leaf, unsigned grid, hipStream_t st) {
    if (kind == ELEM_F32) {
        if (leaf) launch_one<ELEM_F32, true, BATCH, PIPE, PERSIST>(g, grid, st);
        else launch_one<ELEM_F32, false, BATCH, PIPE, PERSIST>(g, grid, st);
    } else {
        if (leaf) launch_one<ELEM_BF16, true, BATCH, PIPE, PERSIST>(g, grid, st);
        else launch_one<ELEM_BF16, false, BATCH, PIPE, PERSIST>(g, grid, st);
    }
}

hipError_t launch_mm(const MmLaunch &L, int kind, bool leaf, const MmConfig &cfg, hipStream_t st) {
    if (L.nrows <= 0) return hipSuccess;
    MmArgs g{L.rows, L.nrows, L.blks, L.data, L.scales, L.in_tree, L.in_pts, L.init, L.out_tree, L.out_pts,
             L.Y, L.ldy, nullptr, nullptr, L.ncols};
    const unsigned grid = unsigned((L.nrows + 1) / 2);
    if (cfg.pipelined) launch_kind<false, true, false>(g, kind, leaf, grid, st);
    else launch_kind<false, false, false>(g, kind, leaf, grid, st);
    return hipGetLastError();
}

hipError_t launch_mm_batch(const MmBatchLaunch &L, int kind, bool leaf, const MmConfig &cfg, hipStream_t st) {
    if (L.nrows <= 0) return hipSuccess;
    MmArgs g{L.rows, L.nrows, L.blks, nullptr, L.scales, L.pool, L.pool, L.pool, L.pool, L.pool,
             nullptr, 0, L.Ytab, L.ldytab, L.ncols};
    const int64_t slots = (L.nrows + 1) / 2;
    if (cfg.grid > 0 && cfg.grid < slots) {
        const unsigned grid = unsigned(cfg.grid);
        if (cfg.pipelined) launch_kind<true, true, true>(g, kind, leaf, grid, st);
        else launch_kind<true, false, true>(g, kind, leaf, grid, st);
    } else {
        const unsigned grid = unsigned(slots);
        if (cfg.pipelined) launch_kind<true, true, false>(g, kind, leaf, grid, st);
        else launch_kind<true, false, false>(g, kind, leaf, grid, st);
    }
    return hipGetLastError();
}

// Batch pack: every (member, leaf) entry copies right-hand sides 0 .. MM_TILE-1
// of its member's X (device pointer table) into its point tile in the pool.
__global__ __launch_bounds__(256) void batch_pack_kernel(const PackEntry *__restrict__ entries, int64_t count,
                                                         double const *const *__restrict__ Xtab,
                                                         const int64_t *__restrict__ ldxtab, int nrhs,
                                                         float *__restrict__ pool) {
    for (int64_t k = blockIdx.x; k < count; k += gridDim.x) {
        const PackEntry e = entries[k];
        const double *X = Xtab[e.member];
        const int64_t ldx = ldxtab[e.member];
        const int mp = round16(e.m);
        float *t = pool + e.dst;
        for (int idx = threadIdx.x; idx < NT * mp; idx += blockDim.x) {
            const int j = idx / mp, c = idx - j * mp;
            float v = 0.0f;
            if (c < e.m && j < nrhs) v = float(X[(e.row + c) + int64_t(j) * ldx]);
            t[idx] = v;
        }
    }
}

hipError_t launch_batch_pack(const PackEntry *entries, int64_t count, double const *const *Xtab,
                             const int64_t *ldxtab, int nrhs, float *pool, int64_t grid, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    const int64_t g = grid > 0 && grid < count ? grid : count;
    hipLaunchKernelGGL(batch_pack_kernel, dim3(unsigned(g)), dim3(256), 0, st, entries, count, Xtab, ldxtab, nrhs,
                       pool);
    return hipGetLastError();
}

}  // namespace h2
