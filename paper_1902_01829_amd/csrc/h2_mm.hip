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
__device__ inline void load_a(const BlkDesc &bd, const void *data, int R, int ic, int lg, BlockA<KIND> &o) {
    const int C = bd.C, NP = round16(C) >> 3;
#pragma unroll
    for (int p = 0; p < 8; ++p) {
        if (p >= NP) break;   // wave-uniform
        if constexpr (KIND == ELEM_F32) {
            const int CW = (C + 3) >> 2;                      // 4-column groups
            const int cg = 2 * p + lg, cgc = cg < CW ? cg : CW - 1;
            o.v[p] = __builtin_nontemporal_load(reinterpret_cast<const f32x4 *>(
                static_cast<const float *>(data) + bd.a + (int64_t(cgc) * R + ic) * 4));
        } else {
            const int CW = (C + 7) >> 3;                      // 8-column groups: half of one per lane
            const int pc = p < CW ? p : CW - 1;
            o.v[p] = __builtin_nontemporal_load(reinterpret_cast<const u32x2 *>(
                static_cast<const uint16_t *>(data) + bd.a + (int64_t(pc) * R + ic) * 8 + 4 * lg));
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

// Two wavefronts per output row segment, one per 32-row half (mt); a
// workgroup of 4 wavefronts covers 2 segments.  Lane l owns block row
// 32*mt + (l % 32) and right-hand side l % 32; for every 8 block columns
// 8p .. 8p+7, lane group g = l / 32 supplies columns 8p + 4g + t (t = 0..3),
// one per MFMA.  The block loop is software-pipelined: the loads of block
// b + 1 are in flight while block b's products run.
template <int KIND, bool LEAF>
__global__ __launch_bounds__(256) void mm_kernel(const RowDesc *__restrict__ rows, int64_t nrows,
                                                 const BlkDesc *__restrict__ blks, const void *__restrict__ data,
                                                 const float *__restrict__ scales, const float *__restrict__ in_tree,
                                                 const float *__restrict__ in_pts, const float *__restrict__ init,
                                                 float *__restrict__ out_tree, float *__restrict__ out_pts,
                                                 double *__restrict__ Y, int64_t ldy, int ncols) {
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int64_t row = xcd_local_order(blockIdx.x, gridDim.x) * 2 + (wv >> 1);
    const int mt = wv & 1;
    if (row >= nrows) return;
    const RowDesc rd = rows[row];
    const int R = rd.R, Rp = round16(R);
    if (32 * mt >= R) return;
    const int li = lane & 31, lg = lane >> 5;
    const int i = 32 * mt + li;   // block row of this lane's A operand
    const int ic = i < R ? i : R - 1;
    const float *xbase = (rd.sel & ROW_IN_X) ? in_pts : in_tree;

    double tot[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) tot[r] = 0.0;

    BlockA<KIND> a_cur, a_nxt;
    TileB b_cur, b_nxt;
    BlkDesc bd_cur, bd_nxt;
    if (rd.b0 < rd.b1) {
        bd_cur = blks[rd.b0];
        load_a<KIND>(bd_cur, data, R, ic, lg, a_cur);
        load_b(bd_cur, xbase, li, lg, b_cur);
    }
    for (int b = rd.b0; b < rd.b1; ++b) {
        const bool more = b + 1 < rd.b1;
        if (more) {
            bd_nxt = blks[b + 1];
            load_a<KIND>(bd_nxt, data, R, ic, lg, a_nxt);
            load_b(bd_nxt, xbase, li, lg, b_nxt);
        }
        const f32x16 acc = block_products<KIND>(a_cur, b_cur, round16(bd_cur.C) >> 3);
        const double sc = KIND == ELEM_BF16 ? double(scales[bd_cur.sidx]) : 1.0;
#pragma unroll
        for (int r = 0; r < 16; ++r) tot[r] += sc * double(acc[r]);
        if (more) {
            a_cur = a_nxt;
            b_cur = b_nxt;
            bd_cur = bd_nxt;
        }
    }

    // Lane l holds rows 32*mt + 8*q + 4*(l/32) + e (e = 0..3) of right-hand side l % 32.
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int i0 = 32 * mt + 8 * q + 4 * lg;
        if (i0 >= Rp) continue;
        if constexpr (LEAF) {
            // y(i, j) = y_near(i, j) + far part, written to the caller's FP64 matrix
            if (li >= ncols) continue;
            const f32x4 yn = *reinterpret_cast<const f32x4 *>(init + rd.init + int64_t(li) * Rp + i0);
            const double ynv[4] = {yn.x, yn.y, yn.z, yn.w};
            double *yc = Y + int64_t(li) * ldy + rd.out;
#pragma unroll
            for (int e = 0; e < 4; ++e)
                if (i0 + e < R) yc[i0 + e] = ynv[e] + tot[4 * q + e];
        } else {
            double v[4];   // rows R .. Rp-1 are the tile's zero padding
#pragma unroll
            for (int e = 0; e < 4; ++e) v[e] = i0 + e < R ? tot[4 * q + e] : 0.0;
            if (rd.init >= 0) {
                const f32x4 t = *reinterpret_cast<const f32x4 *>(init + rd.init + int64_t(li) * Rp + i0);
                v[0] += t.x; v[1] += t.y; v[2] += t.z; v[3] += t.w;
            }
            float *o = ((rd.sel & ROW_OUT_P) ? out_pts : out_tree) + rd.out + int64_t(li) * Rp + i0;
            *reinterpret_cast<f32x4 *>(o) = f32x4{float(v[0]), float(v[1]), float(v[2]), float(v[3])};
        }
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

hipError_t launch_mm(const MmLaunch &L, int kind, bool leaf, hipStream_t st) {
    if (L.nrows <= 0) return hipSuccess;
    const dim3 grid(unsigned((L.nrows + 1) / 2)), block(256);
#define H2_MM_ARGS                                                                                           \
    L.rows, L.nrows, L.blks, L.data, L.scales, L.in_tree, L.in_pts, L.init, L.out_tree, L.out_pts, L.Y, L.ldy, \
        L.ncols
    if (kind == ELEM_F32) {
        if (leaf)
            hipLaunchKernelGGL((mm_kernel<ELEM_F32, true>), grid, block, 0, st, H2_MM_ARGS);
        else
            hipLaunchKernelGGL((mm_kernel<ELEM_F32, false>), grid, block, 0, st, H2_MM_ARGS);
    } else {
        if (leaf)
            hipLaunchKernelGGL((mm_kernel<ELEM_BF16, true>), grid, block, 0, st, H2_MM_ARGS);
        else
            hipLaunchKernelGGL((mm_kernel<ELEM_BF16, false>), grid, block, 0, st, H2_MM_ARGS);
    }
#undef H2_MM_ARGS
    return hipGetLastError();
}

}  // namespace h2
