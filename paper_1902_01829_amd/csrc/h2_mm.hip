// Many right-hand sides on the matrix cores (gfx950 MFMA).
//
// With r right-hand sides every per-node vector of the product becomes a
// k x r tile and every block product a dense contraction (R x C block) x
// (C x r tile).  The phases, work lists and block layout are those of the
// single-vector product; only the arithmetic changes:
//   - tiles hold 32 right-hand sides (one MFMA N dimension), FP32, stored
//     [rhs][row] with a leading dimension rounded up to 16 rows (zero-padded);
//   - FP32 blocks: v_mfma_f32_32x32x2_f32 on FP32 operands.  (Splitting both
//     operands into two BF16 pieces each for the faster BF16 MFMA drops bits
//     of the products: measured 2.5e-6 against 4.7e-7 on 2^20 points.)
//   - BF16 blocks are exact BF16 values (the scale is applied per block), so
//     only the FP32 input tile needs splitting: x = hi + mid + lo exactly, each
//     piece a BF16 value (truncation leaves exact residues of 16 and then 8
//     significant bits).  Three v_mfma_f32_32x32x16_bf16 per 16 block columns
//     then form the products exactly and accumulate them in FP32, the accuracy
//     of the FP32 path at a sixth of its matrix-core time;
//   - one block's products accumulate in FP32, sums over blocks in FP64;
//   - each 32-row half of an output segment has its own wavefront; the two
//     read disjoint halves of every block and share its input tile, which the
//     rows' spatial order keeps in the caches.

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "h2_device.h"

namespace h2 {
namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int NT = MM_TILE;   // right-hand sides per tile

__device__ inline int round16(int v) { return (v + 15) & ~15; }

// Non-temporal 16-byte load of block data through a global-address-space
// pointer: batches hold block addresses as integers, and a generic pointer
// made from one would be read with FLAT loads, which the compiler counts
// against both memory counters (it then waits for every load in flight).
template <typename T>
__device__ inline T load_block_item(const T *p) {
    return __builtin_nontemporal_load((const __attribute__((address_space(1))) T *)(p));
}

// Block operand of one wavefront and the matching input-tile operand.
// FP32 blocks: 8 column steps of 4 values (lane group g holds columns
// 8p + 4g + t of step p, one per K = 2 MFMA).  BF16 blocks: 4 steps of 16
// columns, lane group g holding the 8 columns 16s + 8g .. 16s + 8g + 7 (one
// 16-byte item of the block, the K = 16 operand of one BF16 MFMA); the tile
// operand then holds the same 8 columns as two f32x4.
template <int KIND> struct BlockA;
template <> struct BlockA<ELEM_F32> {
    f32x4 v[8];
};
template <> struct BlockA<ELEM_BF16> {
    u32x4 v[4];
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
    const int C = bd.C;
    if constexpr (KIND == ELEM_F32) {
        const int NP = round16(C) >> 3, CW = (C + 3) >> 2;    // 4-column groups
#pragma unroll
        for (int p = 0; p < 8; ++p) {
            if (p >= NP) break;   // wave-uniform
            const int cg = 2 * p + lg, cgc = cg < CW ? cg : CW - 1;
            o.v[p] = load_block_item(
                reinterpret_cast<const f32x4 *>(static_cast<const float *>(blk) + (int64_t(cgc) * R + ic) * 4));
        }
    } else {
        const int NS = round16(C) >> 4, CW = (C + 7) >> 3;    // 8-column groups
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            if (s >= NS) break;
            const int cg = 2 * s + lg, cgc = cg < CW ? cg : CW - 1;
            o.v[s] = load_block_item(reinterpret_cast<const u32x4 *>(
                static_cast<const uint16_t *>(blk) + (int64_t(cgc) * R + ic) * 8));
        }
    }
}

template <int KIND>
__device__ inline void load_b(const BlkDesc &bd, const float *xbase, int li, int lg, TileB &o) {
    const int Cp = round16(bd.C), NP = Cp >> 3;
    const float *xb = xbase + bd.in + li * Cp;
#pragma unroll
    for (int p = 0; p < 8; ++p) {
        if (p >= NP) break;
        // FP32 blocks: columns 8p + 4g .. +3; BF16 blocks: step p/2, half p%2
        const int col = KIND == ELEM_F32 ? 8 * p + 4 * lg : 16 * (p >> 1) + 8 * lg + 4 * (p & 1);
        o.v[p] = *reinterpret_cast<const f32x4 *>(xb + col);
    }
}

// Splits 8 FP32 values into three BF16 vectors with x = hi + mid + lo exactly.
__device__ inline void split3(const f32x4 &x0, const f32x4 &x1, bf16x8 &hi, bf16x8 &mid, bf16x8 &lo) {
    const float x[8] = {x0.x, x0.y, x0.z, x0.w, x1.x, x1.y, x1.z, x1.w};
    unsigned h[8], m[8], l[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        h[e] = __float_as_uint(x[e]) & 0xffff0000u;
        const float r1 = x[e] - __uint_as_float(h[e]);
        m[e] = __float_as_uint(r1) & 0xffff0000u;
        l[e] = __float_as_uint(r1 - __uint_as_float(m[e]));   // at most 8 significant bits: low half zero
    }
    u32x4 ph, pm, pl;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        ph[t] = (h[2 * t] >> 16) | h[2 * t + 1];
        pm[t] = (m[2 * t] >> 16) | m[2 * t + 1];
        pl[t] = (l[2 * t] >> 16) | (l[2 * t + 1] & 0xffff0000u);
    }
    hi = __builtin_bit_cast(bf16x8, ph);
    mid = __builtin_bit_cast(bf16x8, pm);
    lo = __builtin_bit_cast(bf16x8, pl);
}

// The block's products, accumulated in FP32.
template <int KIND>
__device__ inline f32x16 block_products(const BlockA<KIND> &a_op, const TileB &b_op, int C) {
    f32x16 acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
    if constexpr (KIND == ELEM_F32) {
        const int NP = round16(C) >> 3;
#pragma unroll
        for (int p = 0; p < 8; ++p) {
            if (p >= NP) break;
            const f32x4 a = a_op.v[p];
            acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a.x, b_op.v[p].x, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a.y, b_op.v[p].y, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a.z, b_op.v[p].z, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a.w, b_op.v[p].w, acc, 0, 0, 0);
        }
    } else {
        const int NS = round16(C) >> 4;
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            if (s >= NS) break;
            const bf16x8 a = __builtin_bit_cast(bf16x8, a_op.v[s]);
            bf16x8 hi, mid, lo;
            split3(b_op.v[2 * s], b_op.v[2 * s + 1], hi, mid, lo);
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, lo, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, mid, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, hi, acc, 0, 0, 0);
        }
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
    const int32_t *items;
    int64_t nitems;
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

// A row's block descriptors (and BF16 block scales) held one per lane, the
// first 64 blocks of the row, and read with lane reads: one vector load at
// the start of the row instead of a scalar load (and its wait) per block.
// Blocks past the 64th are read from memory.
__device__ inline int64_t readlane64(int64_t v, int j) {
    const uint32_t lo = uint32_t(__builtin_amdgcn_readlane(int(uint32_t(uint64_t(v))), j));
    const uint32_t hi = uint32_t(__builtin_amdgcn_readlane(int(uint32_t(uint64_t(v) >> 32)), j));
    return int64_t((uint64_t(hi) << 32) | lo);
}
template <int KIND>
struct LaneDescs {
    BlkDesc my;
    float sc = 1.0f;
    // nb > 0 blocks in the row
    __device__ void load(const MmArgs &g, const RowDesc &rd, int nb, int lane) {
        my = g.blks[rd.b0 + (lane < nb ? lane : nb - 1)];
        if constexpr (KIND == ELEM_BF16) sc = g.scales[my.sidx];
    }
    // block k of the row (wave-uniform k)
    __device__ BlkDesc get(const MmArgs &g, const RowDesc &rd, int k) const {
        if (k >= 64) return g.blks[rd.b0 + k];
        BlkDesc b;
        b.a = readlane64(my.a, k);
        b.in = readlane64(my.in, k);
        b.C = __builtin_amdgcn_readlane(my.C, k);
        b.sidx = __builtin_amdgcn_readlane(my.sidx, k);
        return b;
    }
    __device__ double scale(const MmArgs &g, int k, const BlkDesc &b) const {
        if constexpr (KIND != ELEM_BF16) return 1.0;
        if (k >= 64) return double(g.scales[b.sidx]);
        return double(__builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, sc), k)));
    }
};

// One output row segment half (mt) of the list, for one wavefront.  Lane l
// owns block row 32*mt + (l % 32) and right-hand side l % 32; for every 8
// block columns 8p .. 8p+7, lane group g = l / 32 supplies columns 8p + 4g + t
// (t = 0..3), one per MFMA.  With PIPE the block loop is software-pipelined:
// the loads of block b + 1 are in flight while block b's products run.
template <bool LEAF, bool BATCH>
__device__ inline void mm_store32(const MmArgs &g, const RowDesc &rd, int mt, int li, int lg, const double (&tot)[16]);
template <bool LEAF, bool BATCH>
__device__ inline void mm_store16(const MmArgs &g, const RowDesc &rd, int mt, int nh, int n, int kq,
                                  const double (&tot)[2][4]);

template <int KIND, bool LEAF, bool BATCH, bool PIPE>
__device__ inline void mm_row(const MmArgs &g, int64_t row, int mt, int lane) {
    const RowDesc rd = g.rows[row];
    const int R = rd.R;
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
    const int nb = rd.b1 - rd.b0;
    LaneDescs<KIND> ld;
    if (nb > 0) {
        ld.load(g, rd, nb, lane);
        bd_cur = ld.get(g, rd, 0);
        load_a<KIND>(bd_cur, block_ptr(bd_cur), R, ic, lg, a_cur);
        load_b<KIND>(bd_cur, xbase, li, lg, b_cur);
    }
    for (int k = 0; k < nb; ++k) {
        const bool more = k + 1 < nb;
        if (PIPE && more) {
            bd_nxt = ld.get(g, rd, k + 1);
            load_a<KIND>(bd_nxt, block_ptr(bd_nxt), R, ic, lg, a_nxt);
            load_b<KIND>(bd_nxt, xbase, li, lg, b_nxt);
        }
        const f32x16 acc = block_products<KIND>(a_cur, b_cur, bd_cur.C);
        const double sc = ld.scale(g, k, bd_cur);
#pragma unroll
        for (int r = 0; r < 16; ++r) tot[r] += sc * double(acc[r]);
        if (more) {
            if constexpr (PIPE) {
                a_cur = a_nxt;
                b_cur = b_nxt;
                bd_cur = bd_nxt;
            } else {
                bd_cur = ld.get(g, rd, k + 1);
                load_a<KIND>(bd_cur, block_ptr(bd_cur), R, ic, lg, a_cur);
                load_b<KIND>(bd_cur, xbase, li, lg, b_cur);
            }
        }
    }

    // Lane l holds rows 32*mt + 8*q + 4*(l/32) + e (e = 0..3) of right-hand side l % 32.
    mm_store32<LEAF, BATCH>(g, rd, mt, li, lg, tot);
}

// Chunks of the 32-wide loop: FP32 blocks have 8 (8 columns, four K = 2
// MFMAs each), BF16 blocks 4 (16 columns, one K = 16 step as three MFMAs).
template <int KIND> constexpr int chunks32() { return KIND == ELEM_F32 ? 8 : 4; }
template <int KIND> __device__ inline int used_chunks32(int C) {
    return KIND == ELEM_F32 ? round16(C) >> 3 : round16(C) >> 4;
}

// Chunk p of the block operand and of the input-tile operand (the loads of
// load_a / load_b restricted to one chunk).  Issued for every chunk, with no
// branch around them, so that the compiler's count of loads in flight stays
// exact (a conditional load makes it wait for all of them): chunks past the
// block's width re-read its last column group and the tile's last columns
// (cache hits; their products are skipped), and with live == false (no block
// left for this slot) the block operand's load reads the first item of the
// input tile instead (a different address from the tile operand's, so the
// compiler cannot fold the two loads into one on that path and branch).
template <int KIND>
__device__ inline void load_chunk32(const BlkDesc &bd, const void *blk, const float *xbase, int R, int ic, int li,
                                    int lg, int p, bool live, BlockA<KIND> &a, TileB &b) {
    const int C = bd.C, Cp = round16(C);
    const float *xb = xbase + bd.in + li * Cp;
    if constexpr (KIND == ELEM_F32) {
        const int CW = (C + 3) >> 2, cg = 2 * p + lg, cgc = cg < CW ? cg : CW - 1;
        const int col = 8 * p + 4 * lg, colc = col < Cp ? col : Cp - 4;
        const f32x4 *bp = reinterpret_cast<const f32x4 *>(xb + colc);
        const f32x4 *ap = live ? reinterpret_cast<const f32x4 *>(static_cast<const float *>(blk) +
                                                                 (int64_t(cgc) * R + ic) * 4)
                               : reinterpret_cast<const f32x4 *>(xbase + bd.in);
        a.v[p] = load_block_item(ap);
        b.v[p] = *bp;
    } else {
        const int CW = (C + 7) >> 3, cg = 2 * p + lg, cgc = cg < CW ? cg : CW - 1;
        const int col = 16 * p + 8 * lg, colc = col < Cp ? col : Cp - 8;
        const f32x4 *bp = reinterpret_cast<const f32x4 *>(xb + colc);
        const u32x4 *ap = live ? reinterpret_cast<const u32x4 *>(static_cast<const uint16_t *>(blk) +
                                                                 (int64_t(cgc) * R + ic) * 8)
                               : reinterpret_cast<const u32x4 *>(xbase + bd.in);
        a.v[p] = load_block_item(ap);
        b.v[2 * p] = bp[0];
        b.v[2 * p + 1] = bp[1];
    }
}

// Products of chunk p accumulated into acc (the steps of block_products).
template <int KIND>
__device__ inline f32x16 chunk_products32(const BlockA<KIND> &a_op, const TileB &b_op, int p, f32x16 acc) {
    if constexpr (KIND == ELEM_F32) {
        const f32x4 a = a_op.v[p];
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a.x, b_op.v[p].x, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a.y, b_op.v[p].y, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a.z, b_op.v[p].z, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a.w, b_op.v[p].w, acc, 0, 0, 0);
    } else {
        const bf16x8 a = __builtin_bit_cast(bf16x8, a_op.v[p]);
        bf16x8 hi, mid, lo;
        split3(b_op.v[2 * p], b_op.v[2 * p + 1], hi, mid, lo);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, lo, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, mid, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, hi, acc, 0, 0, 0);
    }
    return acc;
}

// Epilogue shared by the 32-wide block loops: lane l holds rows
// 32*mt + 8*q + 4*(l/32) + e (e = 0..3) of right-hand side l % 32 in tot.
// The values added to the result (y_near in the leaf phase, the current y^
// in the downsweep) are requested for every row group before any store: one
// memory round trip per row instead of one per group (a load issued after a
// store also waits for that store).  Rows and columns are clamped into the
// tile, so every load is valid; the clamped ones are not used.
template <bool LEAF, bool BATCH>
__device__ inline void mm_store32(const MmArgs &g, const RowDesc &rd, int mt, int li, int lg, const double (&tot)[16]) {
    const int R = rd.R, Rp = round16(R);
    f32x4 t[4] = {};
    if (LEAF || rd.init >= 0) {   // wave-uniform
        const int lic = LEAF && li >= g.ncols ? g.ncols - 1 : li;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int i0 = 32 * mt + 8 * q + 4 * lg, i0c = i0 < Rp ? i0 : Rp - 4;
            t[q] = *reinterpret_cast<const f32x4 *>(g.init + rd.init + int64_t(lic) * Rp + i0c);
        }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int i0 = 32 * mt + 8 * q + 4 * lg;
        if (i0 >= Rp) continue;
        if constexpr (LEAF) {
            if (li >= g.ncols) continue;
            const f32x4 yn = t[q];
            const double ynv[4] = {yn.x, yn.y, yn.z, yn.w};
            double *Yb = BATCH ? g.Ytab[rd.sel >> 8] : g.Y;
            const int64_t ldy = BATCH ? g.ldytab[rd.sel >> 8] : g.ldy;
            double *yc = Yb + int64_t(li) * ldy + rd.out;
#pragma unroll
            for (int e = 0; e < 4; ++e)
                if (i0 + e < R) yc[i0 + e] = ynv[e] + tot[4 * q + e];
        } else {
            double v[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) v[e] = i0 + e < R ? tot[4 * q + e] : 0.0;
            if (rd.init >= 0) {
                v[0] += t[q].x; v[1] += t[q].y; v[2] += t[q].z; v[3] += t[q].w;
            }
            float *o = ((rd.sel & ROW_OUT_P) ? g.out_pts : g.out_tree) + rd.out + int64_t(li) * Rp + i0;
            *reinterpret_cast<f32x4 *>(o) = f32x4{float(v[0]), float(v[1]), float(v[2]), float(v[3])};
        }
    }
}

// Leaf-phase epilogue of a pair wavefront through its LDS buffer (free once
// the block loop's last barrier has passed): the 32 x 32 result half is
// transposed so that each store instruction writes two 256-byte runs of
// rows of two columns of Y, instead of scattering 8-byte values over 32
// columns (the FP64 result matrix is the largest write of the product).
// Same values as mm_store32 (y = y_near + far part, FP64).
template <bool BATCH>
__device__ inline void mm_store32_leaf_lds(const MmArgs &g, const RowDesc &rd, int mt, int lane,
                                           const double (&tot)[16], float *buf) {
    constexpr int LD = 33;   // doubles per right-hand side row (padded)
    double *T = reinterpret_cast<double *>(buf);
    const int li = lane & 31, lg = lane >> 5;
    const int R = rd.R, Rp = round16(R);
    const int r = lane & 31, i = 32 * mt + r;
    // The lane's 16 near-field values, requested together before the
    // transposition (one memory round trip per row instead of one per four
    // columns); row and column are clamped into the tile, so every load is
    // valid (the clamped ones are not used).
    float yn[16];
    {
        const int ic = i < R ? i : R - 1;
#pragma unroll
        for (int c = 0; c < 16; ++c) {
            const int j = 2 * c + lg, jc = j < g.ncols ? j : g.ncols - 1;
            yn[c] = g.init[rd.init + int64_t(jc) * Rp + ic];
        }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int e = 0; e < 4; ++e) T[li * LD + 8 * q + 4 * lg + e] = tot[4 * q + e];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    double *Yb = BATCH ? g.Ytab[rd.sel >> 8] : g.Y;
    const int64_t ldy = BATCH ? g.ldytab[rd.sel >> 8] : g.ldy;
    if (i < R) {
#pragma unroll
        for (int c = 0; c < 16; ++c) {
            const int j = 2 * c + lg;
            if (j < g.ncols) Yb[int64_t(j) * ldy + rd.out + i] = double(yn[c]) + T[j * LD + r];
        }
    }
}

// The 32-wide block loop with a ring of D block slots: slot s holds block
// b = s (mod D).  As each chunk of block b is consumed, the same registers
// are refilled with that chunk of block b + D, so about D blocks of loads
// stay in flight through the row instead of one.  The arithmetic and its
// order are those of mm_row (bitwise the same results).
template <int KIND, bool LEAF, bool BATCH, int D>
__device__ inline void mm_row_ring(const MmArgs &g, int64_t row, int mt, int lane) {
    const RowDesc rd = g.rows[row];
    const int R = rd.R;
    if (32 * mt >= R) return;
    const int li = lane & 31, lg = lane >> 5;
    const int i = 32 * mt + li;
    const int ic = i < R ? i : R - 1;
    const float *xbase = (rd.sel & ROW_IN_X) ? g.in_pts : g.in_tree;
    auto block_ptr = [&](const BlkDesc &bd) -> const void * {
        if constexpr (BATCH) return reinterpret_cast<const void *>(bd.a);
        else return static_cast<const char *>(g.data) + bd.a * (KIND == ELEM_F32 ? 4 : 2);
    };
    constexpr int NCH = chunks32<KIND>();

    double tot[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) tot[r] = 0.0;

    BlockA<KIND> a[D];
    TileB b[D];
    BlkDesc bd[D];
    const int nb = rd.b1 - rd.b0;
    LaneDescs<KIND> ld;
    if (nb > 0) {
        ld.load(g, rd, nb, lane);
#pragma unroll
        for (int s = 0; s < D; ++s) {
            const bool live = s < nb;   // wave-uniform
            bd[s] = ld.get(g, rd, live ? s : 0);
            const void *blk = block_ptr(bd[s]);
#pragma unroll
            for (int p = 0; p < NCH; ++p) load_chunk32<KIND>(bd[s], blk, xbase, R, ic, li, lg, p, live, a[s], b[s]);
        }
    }
    // block k from slot s, whose registers then receive block k + D
    auto step = [&](const int s, const int k) {
        const bool refill = k + D < nb;
        const BlkDesc nx = ld.get(g, rd, refill ? k + D : k);
        const int np = used_chunks32<KIND>(bd[s].C);
        const void *nblk = block_ptr(nx);
        f32x16 acc;
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
#pragma unroll
        for (int p = 0; p < NCH; ++p) {
            if (p < np) acc = chunk_products32<KIND>(a[s], b[s], p, acc);
            load_chunk32<KIND>(nx, nblk, xbase, R, ic, li, lg, p, refill, a[s], b[s]);
        }
        const double sc = ld.scale(g, k, bd[s]);
#pragma unroll
        for (int r = 0; r < 16; ++r) tot[r] += sc * double(acc[r]);
        bd[s] = nx;
    };
    // Whole rounds of D blocks, then the last < D: no branch inside a round
    // reaches the loop's back edge, which keeps the compiler's waits exact.
    int base = 0;
    for (; base + D <= nb; base += D) {
#pragma unroll
        for (int s = 0; s < D; ++s) step(s, base + s);
    }
#pragma unroll
    for (int s = 0; s < D - 1; ++s)
        if (base + s < nb) step(s, base + s);   // wave-uniform
    // The refills of the last D blocks were dead loads: let them land here,
    // so that no load of this row is in flight when a persistent workgroup's
    // loop starts its next row (the compiler's counts stay exact there too).
    __builtin_amdgcn_s_waitcnt(0);
    mm_store32<LEAF, BATCH>(g, rd, mt, li, lg, tot);
}

// ---- 16 right-hand sides (passes of at most 16 columns, batches of <= 16)
// The tiles keep their layout; only their first 16 right-hand sides are
// used.  A wavefront still owns a 32-row half of an output segment, as two
// 16-row MFMA tiles h = 0, 1: lane l owns block row 32*mt + 16*h + (l % 16)
// and right-hand side l % 16, and lane group q = l / 16 supplies K values.
// FP32 blocks: v_mfma_f32_16x16x4_f32; per 16 block columns, lane group q
// loads the 4 columns 16c + 4q .. 16c + 4q + 3 (one 16-byte item) and step t
// uses column 16c + 4q + t.  BF16 blocks: v_mfma_f32_16x16x32_bf16 with the
// exact three-way split of the input tile; per 32 block columns lane group q
// holds columns 32c + 8q .. 32c + 8q + 7 (one 16-byte item).
template <int KIND> struct BlockA16;
template <> struct BlockA16<ELEM_F32> {
    f32x4 v[2][4];   // [row tile][16-column chunk]
};
template <> struct BlockA16<ELEM_BF16> {
    u32x4 v[2][2];   // [row tile][32-column chunk]
};
struct TileB16 {
    f32x4 v[4];      // FP32: one per 16-column chunk; BF16: two per 32-column chunk
};

template <int KIND>
__device__ inline void load_a16(const BlkDesc &bd, const void *blk, int R, const int (&ic)[2], int nh, int kq,
                                BlockA16<KIND> &o) {
    const int C = bd.C;
    if constexpr (KIND == ELEM_F32) {
        const int NC = round16(C) >> 4, CW = (C + 3) >> 2;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            if (c >= NC) break;   // wave-uniform
            const int cg = 4 * c + kq, cgc = cg < CW ? cg : CW - 1;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                if (h >= nh) break;
                o.v[h][c] = load_block_item(reinterpret_cast<const f32x4 *>(
                    static_cast<const float *>(blk) + (int64_t(cgc) * R + ic[h]) * 4));
            }
        }
    } else {
        const int NC = (C + 31) >> 5, CW = (C + 7) >> 3;
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            if (c >= NC) break;
            const int cg = 4 * c + kq, cgc = cg < CW ? cg : CW - 1;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                if (h >= nh) break;
                o.v[h][c] = load_block_item(reinterpret_cast<const u32x4 *>(
                    static_cast<const uint16_t *>(blk) + (int64_t(cgc) * R + ic[h]) * 8));
            }
        }
    }
}

// Input-tile operand.  BF16 chunks may reach past the tile's padded height
// (a multiple of 16): such lanes read the chunk's first columns instead and
// zero them at use.
template <int KIND>
__device__ inline void load_b16(const BlkDesc &bd, const float *xbase, int n, int kq, TileB16 &o) {
    const int Cp = round16(bd.C);
    const float *xb = xbase + bd.in + n * Cp;
    if constexpr (KIND == ELEM_F32) {
        const int NC = Cp >> 4;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            if (c >= NC) break;
            o.v[c] = *reinterpret_cast<const f32x4 *>(xb + 16 * c + 4 * kq);
        }
    } else {
        const int NC = (bd.C + 31) >> 5;
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            if (c >= NC) break;
            const int col = 32 * c + 8 * kq, colc = col < Cp ? col : 32 * c;
            o.v[2 * c] = *reinterpret_cast<const f32x4 *>(xb + colc);
            o.v[2 * c + 1] = *reinterpret_cast<const f32x4 *>(xb + colc + 4);
        }
    }
}

template <int KIND>
__device__ inline void block_products16(const BlockA16<KIND> &a_op, const TileB16 &b_op, int C, int nh, int kq,
                                        f32x4 (&acc)[2]) {
#pragma unroll
    for (int h = 0; h < 2; ++h) acc[h] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    if constexpr (KIND == ELEM_F32) {
        const int NC = round16(C) >> 4;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            if (c >= NC) break;
            const f32x4 b = b_op.v[c];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                if (h >= nh) break;
                const f32x4 a = a_op.v[h][c];
                acc[h] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, b.x, acc[h], 0, 0, 0);
                acc[h] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, b.y, acc[h], 0, 0, 0);
                acc[h] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.z, b.z, acc[h], 0, 0, 0);
                acc[h] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.w, b.w, acc[h], 0, 0, 0);
            }
        }
    } else {
        const int NC = (C + 31) >> 5, Cp = round16(C);
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            if (c >= NC) break;
            bf16x8 hi, mid, lo;
            split3(b_op.v[2 * c], b_op.v[2 * c + 1], hi, mid, lo);
            if (32 * c + 8 * kq >= Cp) {   // past the tile: zero (see load_b16)
                const u32x4 z = {0u, 0u, 0u, 0u};
                hi = mid = lo = __builtin_bit_cast(bf16x8, z);
            }
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                if (h >= nh) break;
                const bf16x8 a = __builtin_bit_cast(bf16x8, a_op.v[h][c]);
                acc[h] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, lo, acc[h], 0, 0, 0);
                acc[h] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, mid, acc[h], 0, 0, 0);
                acc[h] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, hi, acc[h], 0, 0, 0);
            }
        }
    }
}

// One 32-row half (mt) of an output row segment with 16 right-hand sides.
// Accumulator element e of row tile h holds row 32*mt + 16*h + 4*(l/16) + e
// of right-hand side l % 16.
template <int KIND, bool LEAF, bool BATCH, bool PIPE>
__device__ inline void mm_row16(const MmArgs &g, int64_t row, int mt, int lane) {
    const RowDesc rd = g.rows[row];
    const int R = rd.R;
    if (32 * mt >= R) return;
    const int n = lane & 15, kq = lane >> 4;
    const int nh = 32 * mt + 16 < R ? 2 : 1;   // wave-uniform
    int ic[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int i = 32 * mt + 16 * h + n;
        ic[h] = i < R ? i : R - 1;
    }
    const float *xbase = (rd.sel & ROW_IN_X) ? g.in_pts : g.in_tree;
    const void *data = g.data;

    double tot[2][4];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int e = 0; e < 4; ++e) tot[h][e] = 0.0;

    BlockA16<KIND> a_cur, a_nxt;
    TileB16 b_cur, b_nxt;
    BlkDesc bd_cur, bd_nxt;
    auto block_ptr = [&](const BlkDesc &bd) -> const void * {
        if constexpr (BATCH) return reinterpret_cast<const void *>(bd.a);
        else return static_cast<const char *>(data) + bd.a * (KIND == ELEM_F32 ? 4 : 2);
    };
    const int nb = rd.b1 - rd.b0;
    LaneDescs<KIND> ld;
    if (nb > 0) {
        ld.load(g, rd, nb, lane);
        bd_cur = ld.get(g, rd, 0);
        load_a16<KIND>(bd_cur, block_ptr(bd_cur), R, ic, nh, kq, a_cur);
        load_b16<KIND>(bd_cur, xbase, n, kq, b_cur);
    }
    for (int k = 0; k < nb; ++k) {
        const bool more = k + 1 < nb;
        if (PIPE && more) {
            bd_nxt = ld.get(g, rd, k + 1);
            load_a16<KIND>(bd_nxt, block_ptr(bd_nxt), R, ic, nh, kq, a_nxt);
            load_b16<KIND>(bd_nxt, xbase, n, kq, b_nxt);
        }
        f32x4 acc[2];
        block_products16<KIND>(a_cur, b_cur, bd_cur.C, nh, kq, acc);
        const double sc = ld.scale(g, k, bd_cur);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            tot[h][0] += sc * double(acc[h].x);
            tot[h][1] += sc * double(acc[h].y);
            tot[h][2] += sc * double(acc[h].z);
            tot[h][3] += sc * double(acc[h].w);
        }
        if (more) {
            if constexpr (PIPE) {
                a_cur = a_nxt;
                b_cur = b_nxt;
                bd_cur = bd_nxt;
            } else {
                bd_cur = ld.get(g, rd, k + 1);
                load_a16<KIND>(bd_cur, block_ptr(bd_cur), R, ic, nh, kq, a_cur);
                load_b16<KIND>(bd_cur, xbase, n, kq, b_cur);
            }
        }
    }

    mm_store16<LEAF, BATCH>(g, rd, mt, nh, n, kq, tot);
}

// Chunks of the 16-wide loop: FP32 blocks have 4 (16 columns), BF16 blocks 2
// (32 columns).
template <int KIND> constexpr int chunks16() { return KIND == ELEM_F32 ? 4 : 2; }
template <int KIND> __device__ inline int used_chunks16(int C) {
    return KIND == ELEM_F32 ? round16(C) >> 4 : (C + 31) >> 5;
}

// Chunk c of both operands of the 16-wide loop (load_a16 / load_b16 restricted
// to one chunk), issued unconditionally like load_chunk32: a missing second
// row tile re-reads the first's rows (clamped), chunks past the width re-read
// the last column group, and live == false reads the tile's first items (one
// per row tile, at different addresses, as in load_chunk32).
template <int KIND>
__device__ inline void load_chunk16(const BlkDesc &bd, const void *blk, const float *xbase, int R, const int (&ic)[2],
                                    int n, int kq, int c, bool live, BlockA16<KIND> &a, TileB16 &b) {
    const int C = bd.C, Cp = round16(C);
    const float *xb = xbase + bd.in + n * Cp;
    if constexpr (KIND == ELEM_F32) {
        const int CW = (C + 3) >> 2, cg = 4 * c + kq, cgc = cg < CW ? cg : CW - 1;
        const int col = 16 * c + 4 * kq, colc = col < Cp ? col : Cp - 4;
        const f32x4 *bp = reinterpret_cast<const f32x4 *>(xb + colc);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const f32x4 *ap = live ? reinterpret_cast<const f32x4 *>(static_cast<const float *>(blk) +
                                                                     (int64_t(cgc) * R + ic[h]) * 4)
                                   : reinterpret_cast<const f32x4 *>(xbase + bd.in + 4 * h);
            a.v[h][c] = load_block_item(ap);
        }
        b.v[c] = *bp;
    } else {
        const int CW = (C + 7) >> 3, cg = 4 * c + kq, cgc = cg < CW ? cg : CW - 1;
        const int col = 32 * c + 8 * kq, colc = col < Cp ? col : Cp - 8;
        const f32x4 *bp = reinterpret_cast<const f32x4 *>(xb + colc);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const u32x4 *ap = live ? reinterpret_cast<const u32x4 *>(static_cast<const uint16_t *>(blk) +
                                                                     (int64_t(cgc) * R + ic[h]) * 8)
                                   : reinterpret_cast<const u32x4 *>(xbase + bd.in + 4 * h);
            a.v[h][c] = load_block_item(ap);
        }
        b.v[2 * c] = bp[0];
        b.v[2 * c + 1] = bp[1];
    }
}

// Products of chunk c accumulated into acc (the steps of block_products16).
template <int KIND>
__device__ inline void chunk_products16(const BlockA16<KIND> &a_op, const TileB16 &b_op, int c, int Cp, int nh,
                                        int kq, f32x4 (&acc)[2]) {
    if constexpr (KIND == ELEM_F32) {
        const f32x4 b = b_op.v[c];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            if (h >= nh) break;
            const f32x4 a = a_op.v[h][c];
            acc[h] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, b.x, acc[h], 0, 0, 0);
            acc[h] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, b.y, acc[h], 0, 0, 0);
            acc[h] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.z, b.z, acc[h], 0, 0, 0);
            acc[h] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.w, b.w, acc[h], 0, 0, 0);
        }
    } else {
        bf16x8 hi, mid, lo;
        split3(b_op.v[2 * c], b_op.v[2 * c + 1], hi, mid, lo);
        if (32 * c + 8 * kq >= Cp) {   // past the tile: zero (see load_b16)
            const u32x4 z = {0u, 0u, 0u, 0u};
            hi = mid = lo = __builtin_bit_cast(bf16x8, z);
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            if (h >= nh) break;
            const bf16x8 a = __builtin_bit_cast(bf16x8, a_op.v[h][c]);
            acc[h] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, lo, acc[h], 0, 0, 0);
            acc[h] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, mid, acc[h], 0, 0, 0);
            acc[h] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, hi, acc[h], 0, 0, 0);
        }
    }
}

// Epilogue shared by the 16-wide block loops: accumulator element e of row
// tile h holds row 32*mt + 16*h + 4*(l/16) + e of right-hand side l % 16.
template <bool LEAF, bool BATCH>
__device__ inline void mm_store16(const MmArgs &g, const RowDesc &rd, int mt, int nh, int n, int kq,
                                  const double (&tot)[2][4]) {
    const int R = rd.R, Rp = round16(R);
    if constexpr (LEAF) {
        // The leaf phase transposes the wavefront's 32 x 16 FP64 result
        // through its LDS slot, so that each store instruction writes two
        // 256-byte runs of rows of Y (as the pair loop's leaf phase), not
        // 8-byte values scattered over 16 columns; its y_near values are
        // requested first, all together (rows and columns clamped into the
        // tile; the clamped ones are not used).
        constexpr int LD = 33;   // doubles per right-hand side (padded)
        __shared__ double T16[4][16 * LD];
        double *T = T16[__builtin_amdgcn_readfirstlane(threadIdx.x >> 6)];
        const int lane = threadIdx.x & 63, r = lane & 31, jp = lane >> 5, i = 32 * mt + r;
        float yn[8];
        {
            const int ic = i < R ? i : R - 1;
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                const int j = 2 * c + jp, jc = j < g.ncols ? j : g.ncols - 1;
                yn[c] = g.init[rd.init + int64_t(jc) * Rp + ic];
            }
        }
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int e = 0; e < 4; ++e) T[n * LD + 16 * h + 4 * kq + e] = tot[h][e];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
        double *Yb = BATCH ? g.Ytab[rd.sel >> 8] : g.Y;
        const int64_t ldy = BATCH ? g.ldytab[rd.sel >> 8] : g.ldy;
        if (i < R) {
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                const int j = 2 * c + jp;
                if (j < g.ncols) Yb[int64_t(j) * ldy + rd.out + i] = double(yn[c]) + T[j * LD + r];
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
        __builtin_amdgcn_wave_barrier();   // T free again before a persistent wavefront's next row
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
    } else {
        f32x4 t[2] = {};   // requested together, as in mm_store32
        if (rd.init >= 0) {   // wave-uniform
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int i0 = 32 * mt + 16 * h + 4 * kq, i0c = i0 < Rp ? i0 : Rp - 4;
                t[h] = *reinterpret_cast<const f32x4 *>(g.init + rd.init + int64_t(n) * Rp + i0c);
            }
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            if (h >= nh) break;
            const int i0 = 32 * mt + 16 * h + 4 * kq;
            if (i0 >= Rp) continue;
            double v[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) v[e] = i0 + e < R ? tot[h][e] : 0.0;
            if (rd.init >= 0) {
                v[0] += t[h].x; v[1] += t[h].y; v[2] += t[h].z; v[3] += t[h].w;
            }
            float *o = ((rd.sel & ROW_OUT_P) ? g.out_pts : g.out_tree) + rd.out + int64_t(n) * Rp + i0;
            *reinterpret_cast<f32x4 *>(o) = f32x4{float(v[0]), float(v[1]), float(v[2]), float(v[3])};
        }
    }
}

// The 16-wide block loop with a ring of D block slots (as mm_row_ring).
template <int KIND, bool LEAF, bool BATCH, int D>
__device__ inline void mm_row16_ring(const MmArgs &g, int64_t row, int mt, int lane) {
    const RowDesc rd = g.rows[row];
    const int R = rd.R;
    if (32 * mt >= R) return;
    const int n = lane & 15, kq = lane >> 4;
    const int nh = 32 * mt + 16 < R ? 2 : 1;   // wave-uniform
    int ic[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int i = 32 * mt + 16 * h + n;
        ic[h] = i < R ? i : R - 1;
    }
    const float *xbase = (rd.sel & ROW_IN_X) ? g.in_pts : g.in_tree;
    auto block_ptr = [&](const BlkDesc &bd) -> const void * {
        if constexpr (BATCH) return reinterpret_cast<const void *>(bd.a);
        else return static_cast<const char *>(g.data) + bd.a * (KIND == ELEM_F32 ? 4 : 2);
    };
    constexpr int NCH = chunks16<KIND>();

    double tot[2][4];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int e = 0; e < 4; ++e) tot[h][e] = 0.0;

    BlockA16<KIND> a[D];
    TileB16 b[D];
    BlkDesc bd[D];
    const int nb = rd.b1 - rd.b0;
    LaneDescs<KIND> ld;
    if (nb > 0) {
        ld.load(g, rd, nb, lane);
#pragma unroll
        for (int s = 0; s < D; ++s) {
            const bool live = s < nb;   // wave-uniform
            bd[s] = ld.get(g, rd, live ? s : 0);
            const void *blk = block_ptr(bd[s]);
#pragma unroll
            for (int c = 0; c < NCH; ++c) load_chunk16<KIND>(bd[s], blk, xbase, R, ic, n, kq, c, live, a[s], b[s]);
        }
    }
    auto step = [&](const int s, const int k) {
        const bool refill = k + D < nb;
        const BlkDesc nx = ld.get(g, rd, refill ? k + D : k);
        const int np = used_chunks16<KIND>(bd[s].C);
        const int Cp = round16(bd[s].C);
        const void *nblk = block_ptr(nx);
        f32x4 acc[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) acc[h] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            if (c < np) chunk_products16<KIND>(a[s], b[s], c, Cp, nh, kq, acc);
            load_chunk16<KIND>(nx, nblk, xbase, R, ic, n, kq, c, refill, a[s], b[s]);
        }
        const double sc = ld.scale(g, k, bd[s]);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            tot[h][0] += sc * double(acc[h].x);
            tot[h][1] += sc * double(acc[h].y);
            tot[h][2] += sc * double(acc[h].z);
            tot[h][3] += sc * double(acc[h].w);
        }
        bd[s] = nx;
    };
    int base = 0;
    for (; base + D <= nb; base += D) {
#pragma unroll
        for (int s = 0; s < D; ++s) step(s, base + s);
    }
#pragma unroll
    for (int s = 0; s < D - 1; ++s)
        if (base + s < nb) step(s, base + s);   // wave-uniform
    __builtin_amdgcn_s_waitcnt(0);   // the dead refills land (see mm_row_ring)
    mm_store16<LEAF, BATCH>(g, rd, mt, nh, n, kq, tot);
}

// ---- 16-wide loop with a ring of S column chunks instead of S blocks
// The prefetch distance is counted in 16-column chunks (FP32; 32 columns
// for BF16): a row of narrow blocks (rank 16 or 27, leaves of 32) keeps
// S / 2 or more blocks in flight where a block ring would keep D, for the
// registers of S chunks (a quarter of a full-width block each).  The chunks
// of the row's blocks are consumed in order; slot s holds chunk i of the row
// when i = s (mod S), and is refilled with chunk i + S as soon as its
// products are issued.  A block's sum (times its BF16 scale) is added to the
// FP64 totals after its last chunk, so the arithmetic and its order are those
// of mm_row16 (bitwise the same results).
template <int KIND>
struct Chunk16 {
    typename std::conditional<KIND == ELEM_F32, f32x4, u32x4>::type a[2];   // per row tile
    f32x4 b[KIND == ELEM_F32 ? 1 : 2];
};
template <int KIND>
__device__ inline void load_one_chunk16(const BlkDesc &bd, const void *blk, const float *xbase, int R,
                                        const int (&ic)[2], int n, int kq, int c, bool live, Chunk16<KIND> &o) {
    BlockA16<KIND> a;
    TileB16 b;
    load_chunk16<KIND>(bd, blk, xbase, R, ic, n, kq, c, live, a, b);
#pragma unroll
    for (int h = 0; h < 2; ++h) o.a[h] = a.v[h][c];
    if constexpr (KIND == ELEM_F32) {
        o.b[0] = b.v[c];
    } else {
        o.b[0] = b.v[2 * c];
        o.b[1] = b.v[2 * c + 1];
    }
}
template <int KIND>
__device__ inline void one_chunk_products16(const Chunk16<KIND> &o, int c, int Cp, int nh, int kq, f32x4 (&acc)[2]) {
    BlockA16<KIND> a;
    TileB16 b;
#pragma unroll
    for (int h = 0; h < 2; ++h) a.v[h][c] = o.a[h];
    if constexpr (KIND == ELEM_F32) {
        b.v[c] = o.b[0];
    } else {
        b.v[2 * c] = o.b[0];
        b.v[2 * c + 1] = o.b[1];
    }
    chunk_products16<KIND>(a, b, c, Cp, nh, kq, acc);
}

template <int KIND, bool LEAF, bool BATCH, int S>
__device__ inline void mm_row16_cring(const MmArgs &g, int64_t row, int mt, int lane) {
    const RowDesc rd = g.rows[row];
    const int R = rd.R;
    if (32 * mt >= R) return;
    const int n = lane & 15, kq = lane >> 4;
    const int nh = 32 * mt + 16 < R ? 2 : 1;   // wave-uniform
    int ic[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int i = 32 * mt + 16 * h + n;
        ic[h] = i < R ? i : R - 1;
    }
    const float *xbase = (rd.sel & ROW_IN_X) ? g.in_pts : g.in_tree;
    auto block_ptr = [&](const BlkDesc &bd) -> const void * {
        if constexpr (BATCH) return reinterpret_cast<const void *>(bd.a);
        else return static_cast<const char *>(g.data) + bd.a * (KIND == ELEM_F32 ? 4 : 2);
    };

    double tot[2][4];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int e = 0; e < 4; ++e) tot[h][e] = 0.0;

    const int nb = rd.b1 - rd.b0;
    if (nb > 0) {
        LaneDescs<KIND> ld;
        ld.load(g, rd, nb, lane);
        // consumption cursor: chunk c of block k (descriptor bk); refill
        // cursor: chunk c2 of block k2 (descriptor bk2), S chunks ahead
        int k = 0, c = 0, k2 = 0, c2 = 0;
        BlkDesc bk = ld.get(g, rd, 0), bk2 = bk;
        int np = used_chunks16<KIND>(bk.C), np2 = np;
        int total = 0;   // chunks in the row
        for (int j = 0; j < nb; ++j) total += used_chunks16<KIND>(ld.get(g, rd, j).C);
        Chunk16<KIND> ring[S];
        auto refill = [&](int s) {
            const bool live = k2 < nb;   // wave-uniform
            load_one_chunk16<KIND>(bk2, block_ptr(bk2), xbase, R, ic, n, kq, live ? c2 : 0, live, ring[s]);
            if (live && ++c2 == np2) {
                c2 = 0;
                if (++k2 < nb) {
                    bk2 = ld.get(g, rd, k2);
                    np2 = used_chunks16<KIND>(bk2.C);
                }
            }
        };
#pragma unroll
        for (int s = 0; s < S; ++s) refill(s);
        f32x4 acc[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) acc[h] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
        auto step = [&](int s) {
            one_chunk_products16<KIND>(ring[s], c, round16(bk.C), nh, kq, acc);
            refill(s);
            if (++c == np) {   // the block's last chunk: its sum goes to the totals
                const double sc = ld.scale(g, k, bk);
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    tot[h][0] += sc * double(acc[h].x);
                    tot[h][1] += sc * double(acc[h].y);
                    tot[h][2] += sc * double(acc[h].z);
                    tot[h][3] += sc * double(acc[h].w);
                    acc[h] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
                }
                c = 0;
                if (++k < nb) {
                    bk = ld.get(g, rd, k);
                    np = used_chunks16<KIND>(bk.C);
                }
            }
        };
        // whole rounds of S chunks, then the last < S (see mm_row_ring)
        int i = 0;
        for (; i + S <= total; i += S) {
#pragma unroll
            for (int s = 0; s < S; ++s) step(s);
        }
#pragma unroll
        for (int s = 0; s < S - 1; ++s)
            if (i + s < total) step(s);   // wave-uniform
        __builtin_amdgcn_s_waitcnt(0);   // the dead refills land (see mm_row_ring)
    }
    mm_store16<LEAF, BATCH>(g, rd, mt, nh, n, kq, tot);
}

// ---- both halves of a row in one workgroup of two wavefronts, sharing each
// block's input tile through LDS (32-wide tiles)
// Each wavefront loads half of the tile (right-hand sides 16*mt .. 16*mt+15)
// and writes it to the workgroup's LDS buffer; both read the whole tile from
// there, so the tile crosses the memory pipeline once per block instead of
// once per wavefront.  LDS rows are padded to kPairLd floats so that the
// 16-byte reads of consecutive right-hand sides fall in distinct banks.
constexpr int kPairLd = 68;
constexpr int kPairBuf = MM_TILE * kPairLd;   // floats per buffer

// Barrier of the two wavefronts ordering only their LDS accesses: a full
// __syncthreads would also wait for every global load in flight, which would
// drain the block prefetch at every block.
__device__ inline void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// This wavefront's half of the tile of block bd: load t of lane l takes
// right-hand side 16*mt + 4t + l/16 and columns 4*(l % 16) .. + 3, the
// column group clamped to the tile's last one for narrow tiles (duplicates
// of valid items, written to the same LDS place).  With live == false the
// loads re-read the first items.  (Shifts and masks only: this index math
// runs for every block, and the matrix cores leave the vector ALU little
// room.)
struct TileHalf {
    f32x4 v[4];
};
__device__ inline void half_index(int Cp, int mt, int lane, int t, int &r, int &c) {
    const int cg = lane & 15, last = (Cp >> 2) - 1;
    r = 16 * mt + 4 * t + (lane >> 4);
    c = 4 * (cg < last ? cg : last);
}
__device__ inline void load_half(const BlkDesc &bd, const float *xbase, int mt, int lane, bool live, TileHalf &h) {
    const int Cp = round16(bd.C);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        int r, c;
        half_index(Cp, mt, lane, t, r, c);
        const float *p = xbase + bd.in + (live ? r * Cp + c : 4 * t);
        h.v[t] = *reinterpret_cast<const f32x4 *>(p);
    }
}
__device__ inline void store_half(const BlkDesc &bd, int mt, int lane, const TileHalf &h, float *buf) {
    const int Cp = round16(bd.C);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        int r, c;
        half_index(Cp, mt, lane, t, r, c);
        *reinterpret_cast<f32x4 *>(buf + r * kPairLd + c) = h.v[t];
    }
}

// Chunk p of the block operand (the block half's part of load_chunk32).
template <int KIND>
__device__ inline void load_a_chunk(const BlkDesc &bd, const void *blk, const float *xbase, int R, int ic, int lg,
                                    int p, bool live, BlockA<KIND> &a) {
    const int C = bd.C;
    if constexpr (KIND == ELEM_F32) {
        const int CW = (C + 3) >> 2, cg = 2 * p + lg, cgc = cg < CW ? cg : CW - 1;
        const f32x4 *ap = live ? reinterpret_cast<const f32x4 *>(static_cast<const float *>(blk) +
                                                                 (int64_t(cgc) * R + ic) * 4)
                               : reinterpret_cast<const f32x4 *>(xbase + bd.in + 4 * p);
        a.v[p] = load_block_item(ap);
    } else {
        const int CW = (C + 7) >> 3, cg = 2 * p + lg, cgc = cg < CW ? cg : CW - 1;
        const u32x4 *ap = live ? reinterpret_cast<const u32x4 *>(static_cast<const uint16_t *>(blk) +
                                                                 (int64_t(cgc) * R + ic) * 8)
                               : reinterpret_cast<const u32x4 *>(xbase + bd.in + 4 * p);
        a.v[p] = load_block_item(ap);
    }
}

// Products of chunk p with the tile operand read from LDS: lane l supplies
// right-hand side l % 32, columns 8p + 4(l/32) .. + 3 (FP32) or 16p + 8(l/32)
// .. + 7 (BF16).
template <int KIND>
__device__ inline f32x16 chunk_products_lds(const BlockA<KIND> &a_op, const float *buf, int li, int lg, int p,
                                            f32x16 acc) {
    if constexpr (KIND == ELEM_F32) {
        const f32x4 b = *reinterpret_cast<const f32x4 *>(buf + li * kPairLd + 8 * p + 4 * lg);
        const f32x4 a = a_op.v[p];
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a.x, b.x, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a.y, b.y, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a.z, b.z, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a.w, b.w, acc, 0, 0, 0);
    } else {
        const f32x4 *bp = reinterpret_cast<const f32x4 *>(buf + li * kPairLd + 16 * p + 8 * lg);
        const bf16x8 a = __builtin_bit_cast(bf16x8, a_op.v[p]);
        bf16x8 hi, mid, lo;
        split3(bp[0], bp[1], hi, mid, lo);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, lo, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, mid, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, hi, acc, 0, 0, 0);
    }
    return acc;
}

// Half mt of a row whose other half runs on the partner wavefront of the
// workgroup (R > 32).  The block operand uses the ring of mm_row_ring (D
// slots, refilled chunk by chunk); the tile half of block k + D is loaded at
// iteration k into th[k % D] and written to LDS buffer (k + D) % 2 at the end
// of iteration k + D - 1, before the barrier that ends it.  The summation
// order is that of mm_row (bitwise the same results).
template <int KIND, bool LEAF, bool BATCH, int D>
__device__ inline void mm_row_pair(const MmArgs &g, int64_t row, int mt, int lane, float *lds) {
    const RowDesc rd = g.rows[row];
    const int R = rd.R;
    const int li = lane & 31, lg = lane >> 5;
    const int i = 32 * mt + li;
    const int ic = i < R ? i : R - 1;
    const float *xbase = (rd.sel & ROW_IN_X) ? g.in_pts : g.in_tree;
    auto block_ptr = [&](const BlkDesc &bd) -> const void * {
        if constexpr (BATCH) return reinterpret_cast<const void *>(bd.a);
        else return static_cast<const char *>(g.data) + bd.a * (KIND == ELEM_F32 ? 4 : 2);
    };
    constexpr int NCH = chunks32<KIND>();

    double tot[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) tot[r] = 0.0;

    BlockA<KIND> a[D];
    TileHalf th[D];
    BlkDesc bd[D];
    const int nb = rd.b1 - rd.b0;
    LaneDescs<KIND> ld;
    if (nb > 0) {
        ld.load(g, rd, nb, lane);
#pragma unroll
        for (int s = 0; s < D; ++s) {
            const bool live = s < nb;   // wave-uniform
            bd[s] = ld.get(g, rd, live ? s : 0);
            load_half(bd[s], xbase, mt, lane, live, th[s]);
            const void *blk = block_ptr(bd[s]);
#pragma unroll
            for (int p = 0; p < NCH; ++p) load_a_chunk<KIND>(bd[s], blk, xbase, R, ic, lg, p, live, a[s]);
        }
        store_half(bd[0], mt, lane, th[0], lds);
    }
    lds_barrier();
    // block k from slot s and LDS buffer k % 2; then the tile half of block
    // k + 1 goes to the other buffer
    auto step = [&](const int s, const int k) {
        const bool refill = k + D < nb;
        const BlkDesc nx = ld.get(g, rd, refill ? k + D : k);
        load_half(nx, xbase, mt, lane, refill, th[s]);
        const int np = used_chunks32<KIND>(bd[s].C);
        const void *nblk = block_ptr(nx);
        const float *buf = lds + (k & 1) * kPairBuf;
        f32x16 acc;
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
#pragma unroll
        for (int p = 0; p < NCH; ++p) {
            if (p < np) acc = chunk_products_lds<KIND>(a[s], buf, li, lg, p, acc);
            load_a_chunk<KIND>(nx, nblk, xbase, R, ic, lg, p, refill, a[s]);
        }
        const double sc = ld.scale(g, k, bd[s]);
#pragma unroll
        for (int r = 0; r < 16; ++r) tot[r] += sc * double(acc[r]);
        bd[s] = nx;
        if (k + 1 < nb) {   // wave-uniform: the tile half of block k + 1 (slot (s + 1) % D)
            const int s1 = (s + 1) % D;
            store_half(bd[s1], mt, lane, th[s1], lds + ((k + 1) & 1) * kPairBuf);
        }
        lds_barrier();
    };
    int base = 0;
    for (; base + D <= nb; base += D) {
#pragma unroll
        for (int s = 0; s < D; ++s) step(s, base + s);
    }
#pragma unroll
    for (int s = 0; s < D - 1; ++s)
        if (base + s < nb) step(s, base + s);   // wave-uniform (the same on both wavefronts)
    __builtin_amdgcn_s_waitcnt(0);   // the dead refills land (see mm_row_ring)
    if constexpr (LEAF) {
        mm_store32_leaf_lds<BATCH>(g, rd, mt, lane, tot, lds + mt * kPairBuf);
        lds_barrier();   // both buffers free again before a persistent workgroup's next row
    } else {
        mm_store32<LEAF, BATCH>(g, rd, mt, li, lg, tot);
    }
}

// Two wavefronts per workgroup, one work unit (two items) each: both halves
// of one row (R > 32) share their tiles through LDS; otherwise the items are
// independent and each wavefront runs mm_row_ring alone.  The choice is the
// same on both wavefronts (they read the same two items), so the barriers of
// mm_row_pair are met by both.
template <int KIND, bool LEAF, bool BATCH, int D, bool PERSIST>
__device__ inline void mm_pair_body(const MmArgs &g) {
    __shared__ float lds[2 * kPairBuf];
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int64_t nwg = g.nitems >> 1;
    auto unit = [&](int64_t wg) {
        const int32_t it0 = __builtin_amdgcn_readfirstlane(g.items[wg * 2]);
        const int32_t it1 = __builtin_amdgcn_readfirstlane(g.items[wg * 2 + 1]);
        const int32_t it = wv ? it1 : it0;
        if (it0 >= 0 && it1 >= 0 && (it0 >> 1) == (it1 >> 1)) mm_row_pair<KIND, LEAF, BATCH, D>(g, it >> 1, it & 1, lane, lds);
        else if (it >= 0) mm_row_ring<KIND, LEAF, BATCH, D>(g, it >> 1, it & 1, lane);
    };
    if constexpr (PERSIST) {
        for (int64_t wg = blockIdx.x; wg < nwg; wg += gridDim.x) unit(wg);
    } else {
        unit(blockIdx.x);
    }
}

// One wavefront per work item (a 32-row half of an output row segment), 4
// per workgroup, in the dispatch order laid out by the host.  PERSIST: the
// grid strides over the list's workgroups (fewer workgroups than slots; a
// grid that is a multiple of the XCD count keeps each workgroup on its XCD's
// range); otherwise one workgroup per 4 items.
template <int KIND, bool LEAF, bool BATCH, int PIPE, bool PERSIST, int NT>
__device__ inline void mm_body(const MmArgs &g) {
    if constexpr (PIPE >= 4 && PIPE <= 5) {   // 32-wide tiles shared by the two halves of a row
        static_assert(NT == 32, "tile sharing runs 32-wide tiles");
        mm_pair_body<KIND, LEAF, BATCH, PIPE - 3, PERSIST>(g);
        return;
    }
    static_assert(PIPE < 6 || NT == 16, "chunk rings run 16-wide tiles");
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int64_t nwg = g.nitems >> 2;
    auto one = [&](int32_t it) {
        if constexpr (NT == 16) {
            if constexpr (PIPE >= 6) mm_row16_cring<KIND, LEAF, BATCH, PIPE == 6 ? 6 : 8>(g, it >> 1, it & 1, lane);
            else if constexpr (PIPE >= 2) mm_row16_ring<KIND, LEAF, BATCH, PIPE>(g, it >> 1, it & 1, lane);
            else mm_row16<KIND, LEAF, BATCH, PIPE == 1>(g, it >> 1, it & 1, lane);
        } else {
            if constexpr (PIPE >= 2) mm_row_ring<KIND, LEAF, BATCH, PIPE>(g, it >> 1, it & 1, lane);
            else mm_row<KIND, LEAF, BATCH, PIPE == 1>(g, it >> 1, it & 1, lane);
        }
    };
    if constexpr (PERSIST) {
        for (int64_t wg = blockIdx.x; wg < nwg; wg += gridDim.x) {
            // wave-uniform by construction; said explicitly so that the row's
            // descriptors are read with scalar loads (a vector load of a
            // descriptor would make every wait in the row a wait for all loads)
            const int32_t it = __builtin_amdgcn_readfirstlane(g.items[wg * 4 + wv]);
            if (it >= 0) one(it);
        }
    } else {
        const int32_t it = g.items[int64_t(blockIdx.x) * 4 + wv];
        if (it >= 0) one(it);
    }
}

// One kernel name per phase, so that traces attribute time to phases:
// leaf projection + upsweep and downsweep (FP32 bases), coupling + dense
// streaming (block kind), leaf expansion + FP64 sum.
// The descriptor arrays and the block scales also come as __restrict__
// parameters: the kernel never writes them, and saying so lets the compiler
// read them with scalar loads inside a persistent workgroup's loop, whose
// stores it could not otherwise tell apart from them.
#define H2_MM_PHASE_KERNEL(NAME, LEAF)                                                   \
    template <int KIND, bool BATCH, int PIPE, bool PERSIST, int NT>                      \
    __global__ __launch_bounds__(256) void NAME(MmArgs g, const RowDesc *__restrict__ rows, \
                                                const BlkDesc *__restrict__ blks,       \
                                                const int32_t *__restrict__ items,      \
                                                const float *__restrict__ scales) {     \
        g.rows = rows;                                                                   \
        g.blks = blks;                                                                   \
        g.items = items;                                                                 \
        g.scales = scales;                                                               \
        mm_body<KIND, LEAF, BATCH, PIPE, PERSIST, NT>(g);                                \
    }
H2_MM_PHASE_KERNEL(mm_upsweep_kernel, false)
H2_MM_PHASE_KERNEL(mm_stream_kernel, false)
H2_MM_PHASE_KERNEL(mm_downsweep_kernel, false)
H2_MM_PHASE_KERNEL(mm_leafexpand_kernel, true)
#undef H2_MM_PHASE_KERNEL

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
    // thread = (wavefront w, lane c): leaf row c of columns w, w + 4, ...
    // (each load instruction reads one 512-byte run of a column of X; all of
    // a thread's loads are issued before its stores)
    const int c = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (c >= mp) return;
    float v[NT / 4];
#pragma unroll
    for (int k = 0; k < NT / 4; ++k) {
        const int j = w + 4 * k;
        v[k] = c < m && j0 + j < nrhs ? float(X[(b + c) + int64_t(j0 + j) * ldx]) : 0.0f;
    }
#pragma unroll
    for (int k = 0; k < NT / 4; ++k) t[int64_t(w + 4 * k) * mp + c] = v[k];
}

}  // namespace

hipError_t launch_pack(const double *X, int64_t ldx, int j0, int nrhs, const int64_t *leaf_begin,
                       const int64_t *leaf_end, int64_t nleaves, int64_t slot, float *tiles, hipStream_t st) {
    if (nleaves <= 0) return hipSuccess;
    hipLaunchKernelGGL(pack_kernel, dim3(unsigned(nleaves)), dim3(256), 0, st, X, ldx, j0, nrhs, leaf_begin,
                       leaf_end, slot, tiles);
    return hipGetLastError();
}

template <bool BATCH, int PIPE, bool PERSIST, int NT>
static void launch_phase_nt(const MmArgs &g, int kind, int phase, unsigned grid, hipStream_t st) {
    const dim3 gd(grid), bd(PIPE >= MM_FIRST_PAIR && PIPE < MM_FIRST_CRING ? 128 : 256);   // tile sharing: two wavefronts
    switch (phase) {
    case PHASE_UP:
        hipLaunchKernelGGL((mm_upsweep_kernel<ELEM_F32, BATCH, PIPE, PERSIST, NT>), gd, bd, 0, st, g, g.rows, g.blks, g.items, g.scales);
        break;
    case PHASE_DOWN:
        hipLaunchKernelGGL((mm_downsweep_kernel<ELEM_F32, BATCH, PIPE, PERSIST, NT>), gd, bd, 0, st, g, g.rows, g.blks, g.items, g.scales);
        break;
    case PHASE_LEAF:
        hipLaunchKernelGGL((mm_leafexpand_kernel<ELEM_F32, BATCH, PIPE, PERSIST, NT>), gd, bd, 0, st, g, g.rows, g.blks, g.items, g.scales);
        break;
    default:
        if (kind == ELEM_F32)
            hipLaunchKernelGGL((mm_stream_kernel<ELEM_F32, BATCH, PIPE, PERSIST, NT>), gd, bd, 0, st, g, g.rows, g.blks, g.items, g.scales);
        else
            hipLaunchKernelGGL((mm_stream_kernel<ELEM_BF16, BATCH, PIPE, PERSIST, NT>), gd, bd, 0, st, g, g.rows, g.blks, g.items, g.scales);
    }
}

template <bool BATCH, int PIPE, bool PERSIST>
static void launch_phase_p(const MmArgs &g, int kind, int phase, int nt, unsigned grid, hipStream_t st) {
    if (nt == 16) launch_phase_nt<BATCH, PIPE, PERSIST, 16>(g, kind, phase, grid, st);
    else launch_phase_nt<BATCH, PIPE, PERSIST, 32>(g, kind, phase, grid, st);
}

// depth: 0 plain block loop, 1 one block ahead, 2 and 3 rings of that many
// block slots; 4 and 5 the ring of 1 or 2 slots with the two halves of a row
// sharing the tile (workgroups of two wavefronts over the pair list, 32-wide
// tiles); 6 and 7 rings of 6 or 8 column chunks (16-wide tiles).
template <bool BATCH, bool PERSIST>
static void launch_phase(const MmArgs &g, int kind, int phase, int nt, int depth, unsigned grid, hipStream_t st) {
    switch (depth) {
        case 0: launch_phase_p<BATCH, 0, PERSIST>(g, kind, phase, nt, grid, st); break;
        case 1: launch_phase_p<BATCH, 1, PERSIST>(g, kind, phase, nt, grid, st); break;
        case 2: launch_phase_p<BATCH, 2, PERSIST>(g, kind, phase, nt, grid, st); break;
        case 3: launch_phase_p<BATCH, 3, PERSIST>(g, kind, phase, nt, grid, st); break;
        case 4: launch_phase_nt<BATCH, 4, PERSIST, 32>(g, kind, phase, grid, st); break;
        case 5: launch_phase_nt<BATCH, 5, PERSIST, 32>(g, kind, phase, grid, st); break;
        case 6: launch_phase_nt<BATCH, 6, PERSIST, 16>(g, kind, phase, grid, st); break;
        default: launch_phase_nt<BATCH, 7, PERSIST, 16>(g, kind, phase, grid, st); break;
    }
}

hipError_t launch_mm(const MmLaunch &L, int kind, int phase, const MmConfig &cfg, hipStream_t st) {
    if (L.nitems <= 0) return hipSuccess;
    if (L.nitems % (4 * MM_XCDS) != 0) return hipErrorInvalidValue;
    if (phase != PHASE_STREAM && kind != ELEM_F32) return hipErrorInvalidValue;   // bases are FP32
    if (L.ncols < 1 || L.ncols > MM_TILE) return hipErrorInvalidValue;
    const bool pair = cfg.pipelined >= MM_FIRST_PAIR && cfg.pipelined < MM_FIRST_CRING;
    if (pair && (L.npitems <= 0 || L.npitems % (2 * MM_XCDS) != 0)) return hipErrorInvalidValue;
    MmArgs g{L.rows, pair ? L.pitems : L.items, pair ? L.npitems : L.nitems, L.blks, L.data, L.scales, L.in_tree,
             L.in_pts, L.init, L.out_tree, L.out_pts, L.Y, L.ldy, nullptr, nullptr, L.ncols};
    const int nt = cfg.nt == 32 || L.ncols > 16 ? 32 : 16;
    const int64_t slots = pair ? L.npitems / 2 : L.nitems / 4;
    if (cfg.grid > 0 && cfg.grid < slots) launch_phase<false, true>(g, kind, phase, nt, cfg.pipelined, unsigned(cfg.grid), st);
    else launch_phase<false, false>(g, kind, phase, nt, cfg.pipelined, unsigned(slots), st);
    return hipGetLastError();
}

hipError_t launch_mm_batch(const MmBatchLaunch &L, int kind, int phase, const MmConfig &cfg, hipStream_t st) {
    if (L.nitems <= 0) return hipSuccess;
    if (L.nitems % (4 * MM_XCDS) != 0) return hipErrorInvalidValue;
    if (phase != PHASE_STREAM && kind != ELEM_F32) return hipErrorInvalidValue;
    const bool pair = cfg.pipelined >= MM_FIRST_PAIR && cfg.pipelined < MM_FIRST_CRING;
    if (pair && (L.npitems <= 0 || L.npitems % (2 * MM_XCDS) != 0)) return hipErrorInvalidValue;
    MmArgs g{L.rows, pair ? L.pitems : L.items, pair ? L.npitems : L.nitems, L.blks, nullptr, L.scales, L.pool,
             L.pool, L.pool, L.pool, L.pool, nullptr, 0, L.Ytab, L.ldytab, L.ncols};
    if (L.ncols < 1 || L.ncols > MM_TILE) return hipErrorInvalidValue;
    const int nt = cfg.nt == 32 || L.ncols > 16 ? 32 : 16;
    const int64_t slots = pair ? L.npitems / 2 : L.nitems / 4;
    if (cfg.grid > 0 && cfg.grid < slots) launch_phase<true, true>(g, kind, phase, nt, cfg.pipelined, unsigned(cfg.grid), st);
    else launch_phase<true, false>(g, kind, phase, nt, cfg.pipelined, unsigned(slots), st);
    return hipGetLastError();
}

// Batch pack: every (member, leaf) entry copies right-hand sides 0 .. nrhs-1
// of its member's X (device pointer table) into its point tile in the pool,
// with the rows past the leaf's size zero (they meet the clamped block
// columns).  The tile's right-hand sides nrhs .. MM_TILE-1 are not written:
// every product, sum and store keeps the right-hand sides (MFMA columns)
// apart, and the leaf phase writes only the first nrhs, so whatever those
// columns hold never reaches a result.  One wavefront per entry (a leaf
// holds at most 64 points: lane = row), four per workgroup, eight columns'
// loads issued before their stores.
__global__ __launch_bounds__(256) void batch_pack_kernel(const PackEntry *__restrict__ entries, int64_t count,
                                                         double const *const *__restrict__ Xtab,
                                                         const int64_t *__restrict__ ldxtab, int nrhs,
                                                         float *__restrict__ pool) {
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), c = threadIdx.x & 63;
    const int nc = nrhs < NT ? nrhs : NT;
    for (int64_t k = int64_t(blockIdx.x) * 4 + wv; k < count; k += int64_t(gridDim.x) * 4) {
        const PackEntry e = entries[k];
        const double *X = Xtab[e.member];
        const int64_t ldx = ldxtab[e.member];
        const int mp = round16(e.m);
        float *t = pool + e.dst;
        if (c >= mp) continue;
        const double *xr = X + (e.row + (c < e.m ? c : 0));   // rows past the leaf read its first row
        for (int j0 = 0; j0 < nc; j0 += 8) {
            float v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int j = j0 + u < nc ? j0 + u : nc - 1;
                v[u] = float(xr[int64_t(j) * ldx]);
            }
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (j0 + u < nc) t[int64_t(j0 + u) * mp + c] = c < e.m ? v[u] : 0.0f;
        }
    }
}

hipError_t launch_batch_pack(const PackEntry *entries, int64_t count, double const *const *Xtab,
                             const int64_t *ldxtab, int nrhs, float *pool, int64_t grid, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    const int64_t wgs = (count + 3) / 4;
    const int64_t g = grid > 0 && grid < wgs ? grid : wgs;
    hipLaunchKernelGGL(batch_pack_kernel, dim3(unsigned(g)), dim3(256), 0, st, entries, count, Xtab, ldxtab, nrhs,
                       pool);
    return hipGetLastError();
}

}  // namespace h2
