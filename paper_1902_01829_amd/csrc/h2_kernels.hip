// HIP kernels of libh2mv for gfx950 (MI355X): generation of the H^2
// representation on the device, and the block-row streaming kernel that runs
// every phase of the product (Sec. 4): leaf projection and upsweep (Sec. 4.2),
// tree multiplication with all levels in one launch together with the dense
// near field (Sec. 4.3, Sec. 4.1), downsweep and leaf expansion (Sec. 4.4).
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "h2_device.h"

namespace h2 {
namespace {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------- geometry
// 1-D Lagrange polynomial a over the Chebyshev nodes t, at s.
__device__ double lagrange_1d(const double *t, int p, int a, double s) {
    double v = 1.0;
    for (int b = 0; b < p; ++b)
        if (b != a) v *= (s - t[b]) / (t[a] - t[b]);
    return v;
}

// Tensor Lagrange polynomial nu (axis 0 fastest) of node v's box at x.
__device__ double lagrange_box(const Geometry &g, int64_t v, int nu, const double *x) {
    double val = 1.0;
    for (int ax = 0; ax < g.dim; ++ax) {
        const int a = nu % g.cheb_p;
        nu /= g.cheb_p;
        const double lo = g.lo[v * g.dim + ax], hi = g.hi[v * g.dim + ax];
        const double c = 0.5 * (lo + hi), h = 0.5 * (hi - lo);
        val *= lagrange_1d(g.cheb, g.cheb_p, a, (x[ax] - c) / h);
    }
    return val;
}

// Chebyshev interpolation node nu of node v's box.
__device__ void cheb_point(const Geometry &g, int64_t v, int nu, double *xi) {
    for (int ax = 0; ax < g.dim; ++ax) {
        const int a = nu % g.cheb_p;
        nu /= g.cheb_p;
        const double lo = g.lo[v * g.dim + ax], hi = g.hi[v * g.dim + ax];
        xi[ax] = 0.5 * (lo + hi) + 0.5 * (hi - lo) * g.cheb[a];
    }
}

// Exponential covariance exp(-|a - b| / corr_len) (Sec. 4.6).
__device__ double kernel_exp(const double *a, const double *b, int dim, double corr_len) {
    double r2 = 0.0;
    for (int i = 0; i < dim; ++i) r2 += (a[i] - b[i]) * (a[i] - b[i]);
    return exp(-sqrt(r2) / corr_len);
}

// Round-to-nearest-even of an FP32 value to its upper 16 bits (BF16 code).
__device__ uint16_t bf16_rne(float f) {
    const uint32_t u = __float_as_uint(f);
    return uint16_t((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// Element kinds: storage type T, the 16-byte item type V holding W elements,
// and the arithmetic type P of a block's partial sums.
template <int KIND> struct Elem;
template <> struct Elem<ELEM_F64> {
    using T = double;
    using V = f64x2;
    using P = double;
    static constexpr int W = 2;
    __device__ static void unpack(const V &r, double *v) {
        v[0] = r.x;
        v[1] = r.y;
    }
    __device__ static T store(double v) { return v; }
};
template <> struct Elem<ELEM_F32> {
    using T = float;
    using V = f32x4;
    using P = float;
    static constexpr int W = 4;
    __device__ static void unpack(const V &r, float *v) {
        v[0] = r.x;
        v[1] = r.y;
        v[2] = r.z;
        v[3] = r.w;
    }
    __device__ static T store(double v) { return float(v); }
};
template <> struct Elem<ELEM_BF16> {
    using T = uint16_t;
    using V = u32x4;
    using P = float;
    static constexpr int W = 8;
    __device__ static void unpack(const V &r, float *v) {
        v[0] = __uint_as_float(r.x << 16);
        v[1] = __uint_as_float(r.x & 0xffff0000u);
        v[2] = __uint_as_float(r.y << 16);
        v[3] = __uint_as_float(r.y & 0xffff0000u);
        v[4] = __uint_as_float(r.z << 16);
        v[5] = __uint_as_float(r.z & 0xffff0000u);
        v[6] = __uint_as_float(r.w << 16);
        v[7] = __uint_as_float(r.w & 0xffff0000u);
    }
};

// Decodes element index e of an R-row block in 16-byte column groups of W.
__device__ inline void decode(int e, int R, int W, int &r, int &c) {
    const int w = e % W, t = e / W;
    r = t % R;
    c = (t / R) * W + w;
}

// ---------------------------------------------------------------- fill kernels
// Leaf bases: U_j (m_j x k) with U[r, nu] = L^(j)_nu(point r), and V_j^T
// (k x m_j), the same values transposed (V = U: one tree for rows and columns,
// the symmetric case of Sec. 2.2).
template <int KIND>
__global__ __launch_bounds__(256) void fill_leaf_bases_kernel(
    Geometry g, typename Elem<KIND>::T *basis, const int64_t *leaf_node, const int64_t *off_U,
    const int64_t *off_VT, int64_t nleaves) {
    using E = Elem<KIND>;
    constexpr int W = E::W;
    const int64_t j = blockIdx.x;
    if (j >= nleaves) return;
    const int64_t v = leaf_node[j], b = g.begin[v];
    const int m = int(g.end[v] - b), k = g.rank;
    const int nU = m * ((k + W - 1) / W) * W, nVT = k * ((m + W - 1) / W) * W;
    for (int e = threadIdx.x; e < nU; e += blockDim.x) {
        int r, c;
        decode(e, m, W, r, c);
        const double val = c < k ? lagrange_box(g, v, c, g.pts + (b + r) * g.dim) : 0.0;
        basis[off_U[j] + e] = E::store(val);
    }
    for (int e = threadIdx.x; e < nVT; e += blockDim.x) {
        int r, c;
        decode(e, k, W, r, c);
        const double val = c < m ? lagrange_box(g, v, r, g.pts + (b + c) * g.dim) : 0.0;
        basis[off_VT[j] + e] = E::store(val);
    }
}

// Transfers (Eq. (1) of Sec. 2.2): E_c[mu, nu] = L^(parent)_nu(xi^(c)_mu), a
// k x k block with U_parent = [U_c1 E_c1; U_c2 E_c2]; F_c^T = E_c^T is stored
// next to it for the upsweep.
template <int KIND>
__global__ __launch_bounds__(256) void fill_transfers_kernel(
    Geometry g, typename Elem<KIND>::T *basis, const int64_t *off_E, const int64_t *off_FT,
    int64_t nnodes) {
    using E = Elem<KIND>;
    constexpr int W = E::W;
    const int64_t c = int64_t(blockIdx.x) + 1;
    if (c >= nnodes || off_E[c] < 0) return;
    const int64_t par = (c - 1) / 2;
    const int k = g.rank, nE = k * ((k + W - 1) / W) * W;
    for (int e = threadIdx.x; e < nE; e += blockDim.x) {
        int r, col;
        decode(e, k, W, r, col);
        double xi[3];
        double ev = 0.0, fv = 0.0;
        if (col < k) {
            cheb_point(g, c, r, xi);               // E[r, col]
            ev = lagrange_box(g, par, col, xi);
            cheb_point(g, c, col, xi);             // F^T[r, col] = E[col, r]
            fv = lagrange_box(g, par, r, xi);
        }
        basis[off_E[c] + e] = E::store(ev);
        basis[off_FT[c] + e] = E::store(fv);
    }
}

// Coupling blocks S_st[mu, nu] = K(xi^(s)_mu, xi^(t)_nu) and dense blocks
// D_st[a, b] = K(p_a, p_b) (Sec. 4.6), stored as FP64 / FP32 values.
template <int KIND>
__global__ __launch_bounds__(256) void fill_blocks_kernel(Geometry g, typename Elem<KIND>::T *out,
                                                           const FillDesc *desc, int64_t nblocks) {
    using E = Elem<KIND>;
    constexpr int W = E::W;
    const int64_t blk = blockIdx.x;
    if (blk >= nblocks) return;
    const FillDesc d = desc[blk];
    const bool dense = d.kind == FILL_DENSE;
    const int R = dense ? int(g.end[d.s] - g.begin[d.s]) : g.rank;
    const int C = dense ? int(g.end[d.t] - g.begin[d.t]) : g.rank;
    const int ne = R * ((C + W - 1) / W) * W;
    for (int e = threadIdx.x; e < ne; e += blockDim.x) {
        int r, c;
        decode(e, R, W, r, c);
        double val = 0.0;
        if (c < C) {
            if (dense) {
                val = kernel_exp(g.pts + (g.begin[d.s] + r) * g.dim, g.pts + (g.begin[d.t] + c) * g.dim,
                                 g.dim, g.corr_len);
            } else {
                double xs[3], xt[3];
                cheb_point(g, d.s, r, xs);
                cheb_point(g, d.t, c, xt);
                val = kernel_exp(xs, xt, g.dim, g.corr_len);
            }
        }
        out[d.a + e] = E::store(val);
    }
}

// BF16 with one FP32 scale per block: s = max |fp32(a)|, code = bf16(fp32(a) / s).
__global__ __launch_bounds__(256) void fill_blocks_bf16_kernel(Geometry g, uint16_t *out, float *scales,
                                                                const FillDesc *desc, int64_t nblocks) {
    constexpr int W = 8;
    __shared__ float vals[64 * 64];
    __shared__ float wmax[4];
    const int64_t blk = blockIdx.x;
    if (blk >= nblocks) return;
    const FillDesc d = desc[blk];
    const bool dense = d.kind == FILL_DENSE;
    const int R = dense ? int(g.end[d.s] - g.begin[d.s]) : g.rank;
    const int C = dense ? int(g.end[d.t] - g.begin[d.t]) : g.rank;
    const int ne = R * ((C + W - 1) / W) * W;
    float mx = 0.0f;
    for (int e = threadIdx.x; e < ne; e += blockDim.x) {
        int r, c;
        decode(e, R, W, r, c);
        double val = 0.0;
        if (c < C) {
            if (dense) {
                val = kernel_exp(g.pts + (g.begin[d.s] + r) * g.dim, g.pts + (g.begin[d.t] + c) * g.dim,
                                 g.dim, g.corr_len);
            } else {
                double xs[3], xt[3];
                cheb_point(g, d.s, r, xs);
                cheb_point(g, d.t, c, xt);
                val = kernel_exp(xs, xt, g.dim, g.corr_len);
            }
        }
        const float f = float(val);
        vals[e] = f;
        mx = fmaxf(mx, fabsf(f));
    }
    for (int off = 32; off > 0; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off));
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = mx;
    __syncthreads();
    const float s = fmaxf(fmaxf(wmax[0], wmax[1]), fmaxf(wmax[2], wmax[3]));
    for (int e = threadIdx.x; e < ne; e += blockDim.x)
        out[d.a + e] = s == 0.0f ? uint16_t(0) : bf16_rne(vals[e] / s);
    if (threadIdx.x == 0) scales[d.sidx] = s;
}

// ---------------------------------------------------------------- chunk sums
// One wavefront per segment: lane r adds partials[c * 64 + r] (FP64 or FP32)
// over the segment's chunks in order, in FP64, and stores the segment's
// element r; with ADD the sum starts from the element's current value.
template <typename TV, typename TP, bool ADD>
__global__ __launch_bounds__(256) void reduce_chunks_kernel(const ReduceDesc *__restrict__ desc, int64_t n,
                                                            const TP *__restrict__ partials, TV *__restrict__ out0,
                                                            TV *__restrict__ out1) {
    const int64_t i = int64_t(blockIdx.x) * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int r = threadIdx.x & 63;
    if (i >= n) return;
    const ReduceDesc d = desc[i];
    if (r >= d.R) return;
    TV *dst = (d.point ? out1 : out0) + d.out + r;
    double acc = ADD ? double(*dst) : 0.0;
    int c = d.c0;
    for (; c + 8 <= d.c1; c += 8) {   // eight loads in flight, added in order
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = double(partials[int64_t(c + u) * 64 + r]);
#pragma unroll
        for (int u = 0; u < 8; ++u) acc += v[u];
    }
    for (; c < d.c1; ++c) acc += double(partials[int64_t(c) * 64 + r]);
    *dst = TV(acc);
}

// ---------------------------------------------------------------- transposed copies
// One workgroup per block (grid-strided over the list): destination element
// e = ((r / W) * C + c) * W + r % W of the C x R transpose takes source element
// (r, c) at ((c / W) * R + r) * W + c % W; padding columns of the destination's
// last group are written as zero.
template <typename T, int W>
__global__ __launch_bounds__(256) void transpose_blocks_kernel(const T *__restrict__ src, T *__restrict__ dst,
                                                               const TransDesc *__restrict__ desc, int64_t n) {
    for (int64_t b = blockIdx.x; b < n; b += gridDim.x) {
        const TransDesc d = desc[b];
        const int R = d.R, C = d.C;                       // source R x C, destination C x R
        const int64_t ne = int64_t((R + W - 1) / W) * C * W;
        for (int64_t e = threadIdx.x; e < ne; e += blockDim.x) {
            const int w = int(e % W);
            const int64_t g = e / W;
            const int c = int(g % C), r = int(g / C) * W + w;   // destination (c, r) = source (r, c)
            T v = T(0);
            if (r < R) v = src[d.src + (int64_t(c / W) * R + r) * W + c % W];
            dst[d.dst + e] = v;
        }
    }
}

// ---------------------------------------------------------------- block-row product
// One wavefront per output segment.  For every block of the row, the input
// segment (<= 64 values) is staged in the wave's LDS slot; each lane then
// streams its row's 16-byte items of the block with non-temporal loads and
// accumulates the block's dot products.  One block's partial sum is kept in
// the block arithmetic type, sums over blocks in FP64.
// ONE_ROUND (the tree sweeps and the leaf launch, whose rows hold one or two
// blocks): all of a lane's items of a block are requested at once, before
// the input segment, so a block costs one memory round trip instead of one
// per eight items; on the few rows of the levels near the root that chain is
// the launch's whole duration.  The streaming launch's rows hold many blocks
// and keep eight items in flight per round, which leaves room for more
// wavefronts per SIMD.  Both take the same products in the same order.
template <int KIND, typename TV, typename TO1, bool ONE_ROUND>
__device__ __forceinline__ void blockrow_body(
    const RowDesc *__restrict__ rows, int64_t nrows, const BlkDesc *__restrict__ blks,
    const typename Elem<KIND>::T *__restrict__ data, const float *__restrict__ scales,
    const TV *__restrict__ in0, const double *__restrict__ in1, const TV *__restrict__ init,
    TV *__restrict__ out0, TO1 *__restrict__ out1) {
    using E = Elem<KIND>;
    using P = typename E::P;
    constexpr int W = E::W;
    __shared__ __attribute__((aligned(16))) P xs[4][64];
    __shared__ double red[4][64];
    // ONE_ROUND: the wave index made uniform, so that the row and block
    // descriptors come through scalar loads and a block's base address is
    // uniform (its loads then take 32-bit lane offsets)
    const int wv = ONE_ROUND ? __builtin_amdgcn_readfirstlane(threadIdx.x >> 6) : threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const int64_t row = int64_t(blockIdx.x) * 4 + wv;
    if (row >= nrows) return;
    const RowDesc rd = rows[row];
    const int R = rd.R, G = 64 / R, grp = lane / R, rr = lane - grp * R;
    const bool in_x = (rd.sel & ROW_IN_X) != 0;
    double acc = 0.0;
    for (int b = rd.b0; b < rd.b1; ++b) {
        const BlkDesc bd = blks[b];
        const int C = bd.C, CW = (C + W - 1) / W;
        using V = typename E::V;
        P part = P(0);
        bool done = false;
        if constexpr (ONE_ROUND) {
            // Blocks of at most 8 items per lane: N items, a compile-time
            // count (the smallest of 2, 4, 8 covering the block's ceil(CW / G)
            // column groups per lane, a wave-uniform choice), so that they
            // stay in registers.  Item t is column group grp + t G, clamped
            // into the block (every load is valid; the clamped ones are not
            // used).  Larger blocks take the streaming loop below (a fully
            // unrolled round of 16 or 32 items made the kernel's code several
            // times longer and the launches near the root slower).
            auto round = [&](auto n) {
                constexpr int N = decltype(n)::value;
                V raw[N];
                // a wave-uniform base and 32-bit lane offsets (a block is at
                // most 32 KiB), so the loads need no 64-bit address per item
                const char *base = reinterpret_cast<const char *>(data + bd.a);
#pragma unroll
                for (int t = 0; t < N; ++t) {
                    const int cw = grp + t * G;
                    const uint32_t off = uint32_t((cw < CW ? cw : CW - 1) * R + rr) * 16u;
                    raw[t] = __builtin_nontemporal_load(reinterpret_cast<const V *>(base + off));
                }
                P xv = P(0);
                if (lane < C) xv = in_x ? P(in1[bd.in + lane]) : P(in0[bd.in + lane]);
                xs[wv][lane] = xv;
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                P s = P(0);
                if (grp < G) {
#pragma unroll
                    for (int t = 0; t < N; ++t) {
                        const int cw = grp + t * G;
                        if (cw < CW) {
                            P v[W];
                            E::unpack(raw[t], v);
#pragma unroll
                            for (int w = 0; w < W; ++w) s = fma(v[w], xs[wv][cw * W + w], s);
                        }
                    }
                }
                return s;
            };
            const int ni = (CW + G - 1) / G;
            using std::integral_constant;
            done = ni <= 8;
            if (ni <= 0)
                ;   // a block without columns adds nothing
            else if (ni <= 2)
                part = round(integral_constant<int, 2>{});
            else if (ni <= 4)
                part = round(integral_constant<int, 4>{});
            else if (ni <= 8)
                part = round(integral_constant<int, 8>{});
        }
        if (!done) {
            P xv = P(0);
            if (lane < C) xv = in_x ? P(in1[bd.in + lane]) : P(in0[bd.in + lane]);
            xs[wv][lane] = xv;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            if (grp < G) {
                const V *p = reinterpret_cast<const V *>(data + bd.a) + (grp * R + rr);
                const int stride = G * R;
#pragma unroll 8
                for (int cw = grp; cw < CW; cw += G, p += stride) {
                    const V raw = __builtin_nontemporal_load(p);
                    P v[W];
                    E::unpack(raw, v);
#pragma unroll
                    for (int w = 0; w < W; ++w) part = fma(v[w], xs[wv][cw * W + w], part);
                }
            }
        }
        if constexpr (KIND == ELEM_BF16)
            acc += double(part) * double(scales[bd.sidx]);
        else
            acc += double(part);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    if (G > 1) {
        red[wv][lane] = acc;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (lane < R)
            for (int g2 = 1; g2 < G; ++g2) acc += red[wv][g2 * R + lane];
    }
    if (lane < R) {
        const double res = rd.init >= 0 ? double(init[rd.init + lane]) + acc : acc;
        if (rd.sel & ROW_OUT_P)
            out1[rd.out + lane] = TO1(res);
        else
            out0[rd.out + lane] = TV(res);
    }
}

// One kernel name per phase of the product, so that traces and per-kernel
// statistics separate them; all share the block-row body.
#define H2_BLOCKROW_KERNEL(NAME, ONE_ROUND)                                                              \
    template <int KIND, typename TV, typename TO1>                                                      \
    __global__ __launch_bounds__(256) void NAME(                                                        \
        const RowDesc *__restrict__ rows, int64_t nrows, const BlkDesc *__restrict__ blks,              \
        const typename Elem<KIND>::T *__restrict__ data, const float *__restrict__ scales,               \
        const TV *__restrict__ in0, const double *__restrict__ in1, const TV *__restrict__ init,         \
        TV *__restrict__ out0, TO1 *__restrict__ out1) {                                                 \
        blockrow_body<KIND, TV, TO1, ONE_ROUND>(rows, nrows, blks, data, scales, in0, in1, init, out0, out1); \
    }
H2_BLOCKROW_KERNEL(upsweep_kernel, true)
H2_BLOCKROW_KERNEL(stream_kernel, false)
H2_BLOCKROW_KERNEL(downsweep_kernel, true)
H2_BLOCKROW_KERNEL(leafexpand_kernel, true)
#undef H2_BLOCKROW_KERNEL

// ---------------------------------------------------------------- half storage
// Sums of N values per lane across the N lanes that differ in the lane bits
// MASK, MASK / 2, ..., MASK / (N / 2) (v[k] = the lane's value number k): each
// fold pairs lanes across one bit, each partner keeps the half of its live
// values named by that bit and adds the other's copy of it; lane l ends with
// value number (those bits of l, highest first) summed over its N lanes.
template <int H, int MASK, int N, typename P>
__device__ __forceinline__ void fold_half(P (&v)[N], int lane) {
    const bool up = (lane & MASK) != 0;
#pragma unroll
    for (int k = 0; k < H; ++k) {
        const P keep = up ? v[k + H] : v[k];
        const P send = up ? v[k] : v[k + H];
        v[k] = keep + __shfl_xor(send, MASK);
    }
}
template <int N, int MASK, int LIVE = N, typename P>
__device__ __forceinline__ P fold_lanes(P (&v)[N], int lane) {
    if constexpr (LIVE == 1) {
        return v[0];
    } else {
        fold_half<LIVE / 2, MASK>(v, lane);
        return fold_lanes<N, MASK / 2, LIVE / 2>(v, lane);
    }
}

// Stream phase of a matrix stored by halves: block row i holds only its
// blocks with j >= i (S_ji = S_ij^T, D_ji = D_ij^T).  One wavefront per group
// of consecutive block rows (at most HALF_GROUP_ROWS, taken one after the
// other); with TR lanes per column strip, lane l = TR g + a holds, of every
// block, the tile of rows a + TR k (k < 64 / TR) and columns TR g + c
// (c < TR), so each stored block is read once (all of a lane's 16-byte items
// issued together; each load reads 64 / TR runs of TR consecutive rows) and
// gives both of its products from registers: the lane's partial sums of
// S_ij x_j for its rows, accumulated over the row's blocks (FP64 across
// blocks), and of S_ij^T x_i for its columns, summed over the TR lanes of its
// strip (log2 TR folds), after which lane l holds column l of the transposed
// product.  The group's transposed products of one column segment are added
// in the wavefront's LDS slot for that segment, rows in order (slot[b] >= 0;
// lane l only ever touches element l of a slot, so no barrier), and each LDS
// slot is written once, at the end of the group, to its partial slot
// (gslot): adjacent block rows share many columns, so this writes fewer
// partials, whose cost on the read stream exceeds their share of the bytes.
// A block whose column found no LDS slot writes its own partial slot
// -(slot[b] + 2); slot[b] == -1 marks a diagonal block (no transposed
// product).  Partials are in the vector type (FP64, or FP32 in the reduced
// modes).  At the end of each row the row sums are folded over the strip
// bits (lane l: row l).  A second launch adds each segment's slots to its row
// sum.  The row's own input segment has the offset of its output segment
// (x^ and y^ share the node layout, x and y_near the point layout).
template <int KIND, typename TV, int TR>
__global__ __launch_bounds__(256) void stream_half_kernel(
    const HalfGroup *__restrict__ groups, int64_t ngroups, const RowDesc *__restrict__ rows,
    const BlkDesc *__restrict__ blks, const int32_t *__restrict__ slot, const int32_t *__restrict__ gslot,
    const typename Elem<KIND>::T *__restrict__ data, const float *__restrict__ scales, const TV *__restrict__ in0,
    const double *__restrict__ in1, TV *__restrict__ out0, TV *__restrict__ out1, TV *__restrict__ partials) {
    using E = Elem<KIND>;
    using P = typename E::P;
    using V = typename E::V;
    constexpr int W = E::W;
    constexpr int NS = 64 / TR;    // strips, and rows per lane
    constexpr int IPR = TR / W;    // 16-byte items per row of a strip
    static_assert(IPR >= 1 && TR * NS == 64, "strip of whole 16-byte items");
    __shared__ __attribute__((aligned(16))) P xs[4][64];
    __shared__ TV acc[4][HALF_LDS_SLOTS][64];
    // the wave index made uniform: group, row and block descriptors come through scalar loads
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int a = lane % TR, g = lane / TR;
    const int64_t gi = int64_t(blockIdx.x) * 4 + wv;
    if (gi >= ngroups) return;
    const HalfGroup gd = groups[gi];
    const int ns = gd.s1 - gd.s0;
    for (int s = 0; s < ns; ++s) acc[wv][s][lane] = TV(0);
    for (int32_t row = gd.r0; row < gd.r1; ++row) {
        const RowDesc rd = rows[row];
        const int R = rd.R;
        double rp[NS] = {};   // partial sums of the lane's rows, over the row's blocks
        // The block loop is pipelined: block b + 1's descriptor, slot and input
        // are loaded while block b's items are in flight, the next block's
        // input is staged before block b's transposed product is stored, the
        // LDS fences order LDS only, and the input vector is chosen once per
        // row (the row is uniform, so one of two instantiations runs).
        auto blocks = [&](auto input_is_x) {
            constexpr bool IN_X = decltype(input_is_x)::value;
            // element e of the input segment at off, zero from element n on (the
            // load is clamped into the segment, so the loads issue back to back)
            auto input = [&](int64_t off, int e, int n) {
                const int ec = e < n ? e : n - 1;
                P v;
                if constexpr (IN_X) v = P(in1[off + ec]);
                else v = P(in0[off + ec]);
                return e < n ? v : P(0);
            };
            P xi[NS];   // the row's own input at the lane's rows
#pragma unroll
            for (int k = 0; k < NS; ++k) xi[k] = input(rd.out, a + TR * k, R);
            if (rd.b0 >= rd.b1) return;
            P xj[TR];   // the input at the lane's columns of the current block
            auto stage = [&](const P xv) {
                xs[wv][lane] = xv;
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
#pragma unroll
                for (int c = 0; c < TR; ++c) xj[c] = xs[wv][TR * g + c];
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
            };
            BlkDesc bd = blks[rd.b0];
            int32_t sl = slot[rd.b0];
            stage(input(bd.in, lane, bd.C));
            for (int b = rd.b0; b < rd.b1; ++b) {
                const int C = bd.C, CW = (C + W - 1) / W;
                const V *p = reinterpret_cast<const V *>(data + bd.a);   // item (cw, r) at cw * R + r
                V raw[NS][IPR];
#pragma unroll
                for (int k = 0; k < NS; ++k)
#pragma unroll
                    for (int i = 0; i < IPR; ++i) {
                        const int r = a + TR * k, cw = g * IPR + i;
                        raw[k][i] = V{};
                        if (r < R && cw < CW) raw[k][i] = __builtin_nontemporal_load(p + cw * R + r);
                    }
                const bool more = b + 1 < rd.b1;
                const BlkDesc nbd = blks[more ? b + 1 : b];
                const int32_t nsl = slot[more ? b + 1 : b];
                const P nxv = input(nbd.in, lane, nbd.C);   // unused after the last block
                double scale = 1.0;
                if constexpr (KIND == ELEM_BF16) scale = double(scales[bd.sidx]);
                P cp[TR] = {};
#pragma unroll
                for (int k = 0; k < NS; ++k) {
                    P v[TR];
#pragma unroll
                    for (int i = 0; i < IPR; ++i) E::unpack(raw[k][i], v + i * W);
                    P s = P(0);
#pragma unroll
                    for (int c = 0; c < TR; ++c) {
                        s = fma(v[c], xj[c], s);
                        cp[c] = fma(v[c], xi[k], cp[c]);
                    }
                    rp[k] += double(s) * scale;
                }
                P t = P(0);
                if (sl != -1) t = fold_lanes<TR, TR / 2>(cp, lane);   // column TR g + a = lane
                if (more) stage(nxv);
                if (lane < C) {
                    if (sl >= 0)
                        acc[wv][sl][lane] += TV(double(t) * scale);
                    else if (sl <= -2)
                        partials[int64_t(-(sl + 2)) * 64 + lane] = TV(double(t) * scale);
                }
                bd = nbd;
                sl = nsl;
            }
        };
        if (rd.sel & ROW_IN_X)
            blocks(std::true_type{});
        else
            blocks(std::false_type{});
        const double t = fold_lanes<NS, 32>(rp, lane);   // row a + TR g = lane
        if (lane < R) ((rd.sel & ROW_OUT_P) ? out1 : out0)[rd.out + lane] = TV(t);
    }
    for (int s = 0; s < ns; ++s) partials[int64_t(gslot[gd.s0 + s]) * 64 + lane] = acc[wv][s][lane];
}

constexpr int kRowsPerBlock = 4;

template <int KIND, typename TV, typename TO1>
hipError_t run_blockrow(const RowLaunch &L, int phase, hipStream_t st) {
    if (L.nrows <= 0) return hipSuccess;
    const dim3 grid(unsigned((L.nrows + kRowsPerBlock - 1) / kRowsPerBlock)), block(256);
    const auto *data = static_cast<const typename Elem<KIND>::T *>(L.data);
    const auto *in0 = static_cast<const TV *>(L.in0);
    const auto *init = static_cast<const TV *>(L.init);
    auto *out0 = static_cast<TV *>(L.out0);
    auto *out1 = static_cast<TO1 *>(L.out1);
    switch (phase) {
        case PHASE_UP:
            hipLaunchKernelGGL((upsweep_kernel<KIND, TV, TO1>), grid, block, L.lds_bytes, st, L.rows, L.nrows, L.blks, data,
                               L.scales, in0, L.in1, init, out0, out1);
            break;
        case PHASE_STREAM:
            hipLaunchKernelGGL((stream_kernel<KIND, TV, TO1>), grid, block, L.lds_bytes, st, L.rows, L.nrows, L.blks, data,
                               L.scales, in0, L.in1, init, out0, out1);
            break;
        case PHASE_DOWN:
            hipLaunchKernelGGL((downsweep_kernel<KIND, TV, TO1>), grid, block, L.lds_bytes, st, L.rows, L.nrows, L.blks,
                               data, L.scales, in0, L.in1, init, out0, out1);
            break;
        default:
            hipLaunchKernelGGL((leafexpand_kernel<KIND, TV, TO1>), grid, block, L.lds_bytes, st, L.rows, L.nrows, L.blks,
                               data, L.scales, in0, L.in1, init, out0, out1);
            break;
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_fill_bases(const Geometry &g, int basis_kind, void *basis, const int64_t *leaf_node,
                             const int64_t *off_U, const int64_t *off_VT, int64_t nleaves,
                             const int64_t *off_E, const int64_t *off_FT, int64_t nnodes, hipStream_t st) {
    if (nleaves > 0) {
        if (basis_kind == ELEM_F64)
            hipLaunchKernelGGL(fill_leaf_bases_kernel<ELEM_F64>, dim3(unsigned(nleaves)), dim3(256), 0, st, g,
                               static_cast<double *>(basis), leaf_node, off_U, off_VT, nleaves);
        else
            hipLaunchKernelGGL(fill_leaf_bases_kernel<ELEM_F32>, dim3(unsigned(nleaves)), dim3(256), 0, st, g,
                               static_cast<float *>(basis), leaf_node, off_U, off_VT, nleaves);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (nnodes > 1) {
        if (basis_kind == ELEM_F64)
            hipLaunchKernelGGL(fill_transfers_kernel<ELEM_F64>, dim3(unsigned(nnodes - 1)), dim3(256), 0, st, g,
                               static_cast<double *>(basis), off_E, off_FT, nnodes);
        else
            hipLaunchKernelGGL(fill_transfers_kernel<ELEM_F32>, dim3(unsigned(nnodes - 1)), dim3(256), 0, st, g,
                               static_cast<float *>(basis), off_E, off_FT, nnodes);
        return hipGetLastError();
    }
    return hipSuccess;
}

hipError_t launch_fill_blocks(const Geometry &g, int block_kind, void *blocks, float *scales,
                              const FillDesc *desc, int64_t nblocks, hipStream_t st) {
    if (nblocks <= 0) return hipSuccess;
    // launch in chunks: a grid dimension times the block size must stay below 2^32
    const int64_t chunk = int64_t(1) << 22;
    for (int64_t b0 = 0; b0 < nblocks; b0 += chunk) {
        const int64_t nb = nblocks - b0 < chunk ? nblocks - b0 : chunk;
        if (block_kind == ELEM_F64)
            hipLaunchKernelGGL(fill_blocks_kernel<ELEM_F64>, dim3(unsigned(nb)), dim3(256), 0, st, g,
                               static_cast<double *>(blocks), desc + b0, nb);
        else if (block_kind == ELEM_F32)
            hipLaunchKernelGGL(fill_blocks_kernel<ELEM_F32>, dim3(unsigned(nb)), dim3(256), 0, st, g,
                               static_cast<float *>(blocks), desc + b0, nb);
        else
            hipLaunchKernelGGL(fill_blocks_bf16_kernel, dim3(unsigned(nb)), dim3(256), 0, st, g,
                               static_cast<uint16_t *>(blocks), scales, desc + b0, nb);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_reduce_chunks(const ReduceDesc *desc, int64_t n, const void *partials, bool partials_f32, void *out0,
                                void *out1, bool vec_f64, hipStream_t st, bool add) {
    if (n <= 0) return hipSuccess;
    const dim3 grid(unsigned((n + 3) / 4)), block(256);
    auto go = [&](auto tv, auto tp) {   // vector and partial types
        using TV = decltype(tv);
        using TP = decltype(tp);
        auto *o0 = static_cast<TV *>(out0), *o1 = static_cast<TV *>(out1);
        const TP *pp = static_cast<const TP *>(partials);
        if (add)
            hipLaunchKernelGGL((reduce_chunks_kernel<TV, TP, true>), grid, block, 0, st, desc, n, pp, o0, o1);
        else
            hipLaunchKernelGGL((reduce_chunks_kernel<TV, TP, false>), grid, block, 0, st, desc, n, pp, o0, o1);
    };
    if (vec_f64) {
        if (partials_f32) go(double(), float());
        else go(double(), double());
    } else {
        if (partials_f32) go(float(), float());
        else go(float(), double());
    }
    return hipGetLastError();
}

// Lanes per column strip of the half-storage kernel, per element kind (16 and
// 32 measured no faster: 8 x 8 tiles in every storage mode).
constexpr int kHalfStripF64 = 8, kHalfStripF32 = 8, kHalfStripBF16 = 8;

hipError_t stream_half_workgroups_per_cu(int kind, bool vec_f64, int *n) {
    if (vec_f64)
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(n, stream_half_kernel<ELEM_F64, double, kHalfStripF64>, 256, 0);
    if (kind == ELEM_F32)
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(n, stream_half_kernel<ELEM_F32, float, kHalfStripF32>, 256, 0);
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(n, stream_half_kernel<ELEM_BF16, float, kHalfStripBF16>, 256, 0);
}

hipError_t launch_stream_half(const RowLaunch &L, const HalfGroup *groups, int64_t ngroups, const int32_t *slot,
                              const int32_t *gslot, void *partials, int kind, bool vec_f64, hipStream_t st) {
    if (ngroups <= 0) return hipSuccess;
    const dim3 grid(unsigned((ngroups + kRowsPerBlock - 1) / kRowsPerBlock)), block(256);
    if (vec_f64) {
        hipLaunchKernelGGL((stream_half_kernel<ELEM_F64, double, kHalfStripF64>), grid, block, 0, st, groups, ngroups,
                           L.rows, L.blks, slot, gslot, static_cast<const double *>(L.data), L.scales,
                           static_cast<const double *>(L.in0), L.in1, static_cast<double *>(L.out0),
                           static_cast<double *>(L.out1), static_cast<double *>(partials));
    } else if (kind == ELEM_F32) {
        hipLaunchKernelGGL((stream_half_kernel<ELEM_F32, float, kHalfStripF32>), grid, block, 0, st, groups, ngroups,
                           L.rows, L.blks, slot, gslot, static_cast<const float *>(L.data), L.scales,
                           static_cast<const float *>(L.in0), L.in1, static_cast<float *>(L.out0),
                           static_cast<float *>(L.out1), static_cast<float *>(partials));
    } else {
        hipLaunchKernelGGL((stream_half_kernel<ELEM_BF16, float, kHalfStripBF16>), grid, block, 0, st, groups,
                           ngroups, L.rows, L.blks, slot, gslot, static_cast<const uint16_t *>(L.data), L.scales,
                           static_cast<const float *>(L.in0), L.in1, static_cast<float *>(L.out0),
                           static_cast<float *>(L.out1), static_cast<float *>(partials));
    }
    return hipGetLastError();
}

hipError_t launch_transpose_blocks(int kind, const void *src, void *dst, const TransDesc *desc, int64_t n,
                                   hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const dim3 grid(unsigned(n < 65536 ? n : 65536)), block(256);
    if (kind == ELEM_F64)
        hipLaunchKernelGGL((transpose_blocks_kernel<double, 2>), grid, block, 0, st, static_cast<const double *>(src),
                           static_cast<double *>(dst), desc, n);
    else if (kind == ELEM_F32)
        hipLaunchKernelGGL((transpose_blocks_kernel<float, 4>), grid, block, 0, st, static_cast<const float *>(src),
                           static_cast<float *>(dst), desc, n);
    else
        hipLaunchKernelGGL((transpose_blocks_kernel<uint16_t, 8>), grid, block, 0, st,
                           static_cast<const uint16_t *>(src), static_cast<uint16_t *>(dst), desc, n);
    return hipGetLastError();
}

hipError_t launch_blockrow(const RowLaunch &L, int kind, bool vec_f64, int phase, hipStream_t st, int out1_f64_in) {
    const bool out1_f64 = out1_f64_in < 0 ? phase == PHASE_LEAF : out1_f64_in != 0;
    if (vec_f64) return run_blockrow<ELEM_F64, double, double>(L, phase, st);
    if (kind == ELEM_F32)
        return out1_f64 ? run_blockrow<ELEM_F32, float, double>(L, phase, st)
                        : run_blockrow<ELEM_F32, float, float>(L, phase, st);
    return out1_f64 ? run_blockrow<ELEM_BF16, float, double>(L, phase, st)
                    : run_blockrow<ELEM_BF16, float, float>(L, phase, st);
}

namespace {

// A plain streaming read: consecutive lanes take consecutive 16-byte items
// (each wavefront load is one contiguous kilobyte, like the product kernels'),
// non-temporal, eight in flight per lane, grid-strided; one XOR per workgroup
// reaches sink so that the loads stay.
typedef unsigned long long u64x2 __attribute__((ext_vector_type(2)));
__global__ __launch_bounds__(256) void read_probe_kernel(const u64x2 *__restrict__ p, int64_t n16,
                                                         unsigned long long *__restrict__ sink) {
    __shared__ unsigned long long part[256];
    const int64_t stride = int64_t(gridDim.x) * 256;
    int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
    unsigned long long acc = 0;
    for (; i + 7 * stride < n16; i += 8 * stride) {
        u64x2 v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = __builtin_nontemporal_load(p + i + k * stride);
#pragma unroll
        for (int k = 0; k < 8; ++k) acc ^= v[k].x ^ v[k].y;
    }
    for (; i < n16; i += stride) {
        const u64x2 v = __builtin_nontemporal_load(p + i);
        acc ^= v.x ^ v.y;
    }
    part[threadIdx.x] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int k = 0; k < 256; ++k) t ^= part[k];
        sink[blockIdx.x] = t;
    }
}

}  // namespace

hipError_t launch_read_probe(const void *buf, int64_t bytes, int grid, void *sink, hipStream_t st) {
    hipLaunchKernelGGL(read_probe_kernel, dim3(unsigned(grid)), dim3(256), 0, st, static_cast<const u64x2 *>(buf),
                       bytes / 16, static_cast<unsigned long long *>(sink));
    return hipGetLastError();
}

}  // namespace h2
