// Basis orthogonalization and projection of the coupling blocks (Sec. 5.1,
// Alg. 6 and Alg. 7), FP64, for one basis tree serving rows and columns
// (U = V, E = F) or a row and a column tree of their own.
//
// Leaves: U_j = Q_j T_j (thin Householder QR), Q_j the new leaf basis.  Up the
// tree, parent p with children c1, c2: Z = [T_c1 E_c1; T_c2 E_c2] = Q T_p, the
// two blocks of Q the new transfers (the column tree likewise with V and F,
// giving T').  Then every coupling block S_ij becomes T_i S_ij T'_j^T.  The diagonal of every T is made non-negative, which makes
// the factorization unique for full-column-rank inputs.
//
// One workgroup (256 threads) per factorization or per coupling block; the
// matrices are staged column-major in LDS (up to 128 x 64 FP64 for Z).

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "h2_device.h"
#include "h2_lds_la.h"

namespace h2 {
namespace {

using namespace lds;

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));

// A leaf basis is read from `in` (as stored: M x N, or its N x M transpose
// when IN_T) and Q is written to out_n (M x N) and/or out_t (N x M, the
// transpose), either of which may be NULL: one tree for rows and columns
// writes both U_j and V_j^T, a tree of its own only its own.
template <bool IN_T>
__global__ __launch_bounds__(256) void orth_leaf_kernel(double *basis, const int64_t *in,
                                                        const int64_t *out_n, const int64_t *out_t,
                                                        const int64_t *leaf_begin, const int64_t *leaf_end, int kq,
                                                        double *T, int kmax, int64_t first_leaf) {
    __shared__ double A[(64 + QR_PAD) * QR_MAXN], tau[QR_MAXN], sgn[QR_MAXN];
    const int64_t j = blockIdx.x;
    const int M = int(leaf_end[j] - leaf_begin[j]), N = kq;
    const double *B = basis + in[j];
    const int ld = M + QR_PAD;
    for (int i = threadIdx.x; i < M * N; i += blockDim.x) {
        const int c = i / M, r = i - c * M;
        A[c * ld + r] = IN_T ? B[at2(N, c, r)] : B[at2(M, r, c)];
    }
    __syncthreads();
    householder_qr<64>(A, tau, sgn, M, N, T + (first_leaf + j) * kmax * kmax, kmax);
    // the offsets read once: the stores into basis could alias them for all
    // the compiler knows, and would each wait for a reload
    const int64_t on = out_n ? out_n[j] : -1, ot = out_t ? out_t[j] : -1;
    for (int i = threadIdx.x; i < M * N; i += blockDim.x) {
        const int c = i / M, r = i - c * M;
        if (on >= 0) basis[on + at2(M, r, c)] = A[c * ld + r];   // M x N
        if (ot >= 0) basis[ot + at2(N, c, r)] = A[c * ld + r];   // N x M
    }
}

// Parents of level l - 1 (2^(l-1) workgroups): Z = [T_c1 E_c1; T_c2 E_c2].
// Transfers are read from `in` (kc x kp as stored, or its transpose when
// IN_T) and the new ones written to out_n (kc x kp) and/or out_t (kp x kc).
template <bool IN_T>
__global__ __launch_bounds__(256) void orth_level_kernel(double *basis, const int64_t *in,
                                                         const int64_t *out_n, const int64_t *out_t, int kc, int kp,
                                                         double *T, int kmax, int64_t first_parent) {
    __shared__ double A[(QR_MAXM + QR_PAD) * QR_MAXN], tau[QR_MAXN], sgn[QR_MAXN];
    const int64_t p = first_parent + blockIdx.x;
    const int M = 2 * kc, N = kp, ld = M + QR_PAD;
    // Z = [T_c1 E_c1; T_c2 E_c2] on the FP64 matrix cores (the lane layout of
    // the projection below): wavefront w computes rows 16 w .. 16 w + 15 of
    // each half, its T_c operands loaded once, E's one column tile ahead.
    {
        const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63, lr = lane & 15, lk = lane >> 4;
        const int nrt = (kc + 15) >> 4, nct = (kp + 15) >> 4;
        for (int h = 0; h < 2; ++h) {
            const int64_t ch = 2 * p + 1 + h;
            const double *E = basis + in[ch];                       // kc x kp (or its transpose)
            const double *Tc = T + ch * kmax * kmax;                // kc x kc, upper triangular
            if (wv < nrt) {
                const int r0 = 16 * wv;
                double ta[16];
#pragma unroll
                for (int s4 = 0; s4 < 16; ++s4) {
                    const int kk = 4 * s4 + lk, row = r0 + lr;
                    ta[s4] = (row < kc && kk < kc) ? Tc[int64_t(kk) * kmax + row] : 0.0;   // T_c(row, kk)
                }
#pragma unroll
                for (int ct = 0; ct < 4; ++ct) {
                    if (ct >= nct) break;   // wave-uniform
                    const int col = 16 * ct + lr;
                    double eb[16];
#pragma unroll
                    for (int s4 = 0; s4 < 16; ++s4) {
                        const int kk = 4 * s4 + lk;
                        eb[s4] = (kk < kc && col < kp) ? (IN_T ? E[at2(kp, col, kk)] : E[at2(kc, kk, col)])
                                                        : 0.0;   // E(kk, col)
                    }
                    // all 16 steps, with no early exit: the operand arrays keep static
                    // register indices (steps past the rank multiply zeros)
                    f64x4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                    for (int s4 = 0; s4 < 16; ++s4)
                        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(ta[s4], eb[s4], acc, 0, 0, 0);
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int row = r0 + lk + 4 * e;
                        if (row < kc && col < kp) A[col * ld + h * kc + row] = acc[e];
                    }
                }
            }
        }
    }
    __syncthreads();
    householder_qr(A, tau, sgn, M, N, T + p * kmax * kmax, kmax);
    for (int h = 0; h < 2; ++h) {
        const int64_t ch = 2 * p + 1 + h;
        // the offsets read once: the stores into basis could alias them for
        // all the compiler knows, and would each wait for a reload
        const int64_t on = out_n ? out_n[ch] : -1, ot = out_t ? out_t[ch] : -1;
        for (int i = threadIdx.x; i < kc * kp; i += blockDim.x) {
            const int c = i / kc, r = i - c * kc;
            const double v = A[c * ld + h * kc + r];
            if (on >= 0) basis[on + at2(kc, r, c)] = v;   // kc x kp
            if (ot >= 0) basis[ot + at2(kp, c, r)] = v;   // kp x kc
        }
    }
}

// Coupling block b: S' = T_i S T_j^T with T_i, T_j cut to their first kout
// rows (kout = k in the orthogonalization), on the FP64 matrix cores
// (v_mfma_f64_16x16x4_f64: lane l supplies A(l % 16, l / 16) and B(l / 16,
// l % 16) and holds D(l / 16 + 4 e, l % 16), e = 0..3 -- the rows of a lane's
// four results are 4 apart, unlike the FP32 16 x 16 forms).
//
// A wavefront owns one row tile of the output, rows r0 .. r0 + 15, and never
// leaves registers between the two products: it forms W^T = S^T T_i^T one
// 16-column tile of W at a time, and lane (lr, lk) then holds W(r0 + lr,
// 16 ct + lk + 4 e) -- exactly the A operand of step 4 ct + e of
// S'(rows, :) = W T_j^T.  S (column-major) and T_j (row kk of T_j^T
// contiguous) are read from LDS, loaded for the next block while this one's
// products run; the wavefront's rows of T_i (mostly cache hits: consecutive
// blocks share the row) are loaded once its products are done.  The result goes
// out as 16-byte items (two columns of a row) after one exchange between
// neighbouring lanes, written once the next block is staged so that the
// wait for the next loads does not also wait for these stores.  Row tiles
// rotate over the wavefronts from block to block, which evens out the
// triangular case.  Each workgroup takes one contiguous run of the list: the
// blocks of a block row share T_i, which then stays in the caches.
//
// TRI: T_i and T_j are upper triangular (the orthogonalization's R factors,
// stored with explicit zeros), so the K steps that meet only their zeros are
// skipped -- below a row tile's first row in T_i S, before an output column
// tile's first column in W T_j^T (3/8 of the matrix-core work of a rank-64
// block) -- and T_j's zeros are not read.
constexpr int PS_LD = 68;   // LDS leading dimension of S (spread over the banks)
constexpr int PT_LD = 80;   // of T_j^T: rows of the four quarter-waves alternate between bank halves

// The loads below are unconditional: a wave-uniform base (scalar registers)
// plus one 32-bit byte offset per lane.  S items are clamped into the block;
// T_i and T_j are read as a 64 x 64 frame from their node's start, which
// stays inside the array because it is allocated PROJ_T_PAD doubles longer.
// What lies outside the block or the node's T is replaced by zeros where the
// values are staged or used.
__device__ inline const char *proj_at(const void *base, uint32_t off) { return static_cast<const char *>(base) + off; }

// S item j of this thread: column pair g = wavefront + 4 j (wave-uniform),
// row r = lane, valid when r < k and 2 g < k (a 64 x 64 frame: every slot of
// the LDS copy is written, the padding with zeros).
__device__ inline void proj_load(const double *blocks, const ProjDesc &d, int wv, f64x2 (&v)[8]) {
    const int k = d.k;
    const uint32_t off = uint32_t(min(int(threadIdx.x & 63), k - 1)) * 16u;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const int g = min(wv + 4 * j, (k - 1) >> 1);
        v[j] = __builtin_nontemporal_load(reinterpret_cast<const f64x2 *>(proj_at(blocks + d.off + 2 * g * k, off)));
    }
}

// T_j(c, kk) as element kk * 64 + c of 256 threads x 16: one wavefront reads
// one column of T_j (64 consecutive doubles).
__device__ inline void proj_load_t(const double *Tj, int kmax, int wv, double (&v)[16]) {
    const uint32_t off = uint32_t(threadIdx.x & 63) * 8u;
#pragma unroll
    for (int j = 0; j < 16; ++j)
        v[j] = *reinterpret_cast<const double *>(proj_at(Tj + (wv + 4 * j) * kmax, off));
}
template <bool TRI>
__device__ inline bool proj_t_ok(int k, int ko, int j) {
    const int c = threadIdx.x & 63, kk = int(threadIdx.x >> 6) + 4 * j;
    return kk < k && c < ko && (!TRI || c <= kk);
}

// T_i(r0 + lr, 4 s + lk) for row tile rt; the steps a triangular T_i skips
// are not loaded.
template <bool TRI>
__device__ inline void proj_load_ti(const double *Ti, int rt, int kmax, int lr, int lk, double (&o)[16]) {
    const uint32_t off = uint32_t(lk * kmax + 16 * rt + lr) * 8u;
#pragma unroll
    for (int s4 = 0; s4 < 16; ++s4) {
        if (TRI && s4 < 4 * rt) continue;   // wave-uniform
        o[s4] = *reinterpret_cast<const double *>(proj_at(Ti + 4 * s4 * kmax, off));
    }
}

template <bool TRI>
__global__ __launch_bounds__(256, 2) void project_kernel(const double *in, double *outp,
                                                         const ProjDesc *__restrict__ desc, int64_t nblocks,
                                                         const double *__restrict__ T,
                                                         const double *__restrict__ Tcol, int kmax) {
    // (desc, T and Tcol are never written here, so the descriptors are read
    // through the scalar cache and no wait for them waits for the prefetch;
    // in and outp may be the same array)
    __shared__ double S[64 * PS_LD];    // column-major
    __shared__ double Tt[64 * PT_LD];   // T_j(c, kk) at kk * PT_LD + c
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63, lr = lane & 15,
              lk = lane >> 4;
    const int64_t per = (nblocks + gridDim.x - 1) / gridDim.x;
    const int64_t b0 = int64_t(blockIdx.x) * per, b1 = b0 + per < nblocks ? b0 + per : nblocks;
    if (b0 >= b1) return;   // the whole workgroup
    auto row_tile = [&](int64_t b) { return (wv + int(b & 3)) & 3; };
    f64x2 nxt[8];      // the next block's S items
    double nxt_t[16];  // its T_j
    auto prefetch = [&](int64_t b) {
        const ProjDesc d = desc[b];
        proj_load(in, d, wv, nxt);
        proj_load_t(Tcol + d.col * kmax * kmax, kmax, wv, nxt_t);
    };
    double ta[16];     // T_i rows of this wavefront's row tile
    auto load_ta = [&](int64_t b) { proj_load_ti<TRI>(T + desc[b].row * kmax * kmax, row_tile(b), kmax, lr, lk, ta); };
    auto stage = [&](int64_t b) {   // the prefetched block into LDS (its S zero-padded)
        const int k = desc[b].k, ko = desc[b].kout, r = lane;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int g = wv + 4 * j;
            const bool ok = r < k && 2 * g < k;
            S[(2 * g) * PS_LD + r] = ok ? nxt[j].x : 0.0;
            S[(2 * g + 1) * PS_LD + r] = ok && 2 * g + 1 < k ? nxt[j].y : 0.0;
        }
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const int f = threadIdx.x + 256 * j;
            Tt[(f >> 6) * PT_LD + (f & 63)] = proj_t_ok<TRI>(k, ko, j) ? nxt_t[j] : 0.0;
        }
    };
    // block b; NEXT: block b + 1 exists (prefetched, then staged)
    auto block = [&](int64_t b, auto next) {
        constexpr bool NEXT = decltype(next)::value;
        __syncthreads();   // block b staged
        if constexpr (NEXT) prefetch(b + 1);   // in flight during the products
        const ProjDesc d = desc[b];
        const int k = d.k, kp = (k + 15) & ~15, nt = kp >> 4;   // input: k x k, nt column tiles
        const int ko = d.kout, nto = (ko + 15) >> 4;             // output: ko x ko, nto row tiles
        const int rt = row_tile(b), r0 = 16 * rt;
        f64x4 o[4];   // S'(r0 + lk + 4 e, 16 ct + lr)
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) o[ct] = f64x4{0.0, 0.0, 0.0, 0.0};
        if (rt < nto) {
#pragma unroll
            for (int s4 = 0; s4 < 16; ++s4) {   // zeros outside T_i's ko x k block
                const bool ok = (!TRI || s4 >= 4 * rt) && r0 + lr < ko && 4 * s4 + lk < k;
                ta[s4] = ok ? ta[s4] : 0.0;
            }
            f64x4 w[4];   // W(r0 + lr, 16 ct + lk + 4 e)
            // the products with the first K step S0 and the K extent KP (a
            // multiple of 16) as constants, so that each is straight-line code
            auto products = [&](auto s0c, auto kpc) {
                constexpr int S0 = decltype(s0c)::value, KP = decltype(kpc)::value;
#pragma unroll
                for (int ct = 0; ct < KP / 16; ++ct) {
                    w[ct] = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
                    for (int s4 = S0; s4 < KP / 4; ++s4)   // T_i(rows r0 .., kk) = 0 for kk < r0 (TRI)
                        w[ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(S[(16 * ct + lr) * PS_LD + 4 * s4 + lk], ta[s4],
                                                                     w[ct], 0, 0, 0);
                }
#pragma unroll
                for (int ct = 0; ct < 4; ++ct) {
                    if (ct >= nto) break;   // wave-uniform
                    o[ct] = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
                    for (int s4 = TRI ? 4 * ct : 0; s4 < KP / 4; ++s4)   // T_j(cols 16 ct .., kk) = 0 for kk < 16 ct
                        o[ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(w[s4 >> 2][s4 & 3],
                                                                     Tt[(4 * s4 + lk) * PT_LD + 16 * ct + lr], o[ct],
                                                                     0, 0, 0);
                }
            };
            using std::integral_constant;
            auto with_kp = [&](auto kpc) {
                if constexpr (TRI) {
                    switch (rt) {
                    case 0: products(integral_constant<int, 0>{}, kpc); break;
                    case 1: products(integral_constant<int, 4>{}, kpc); break;
                    case 2: products(integral_constant<int, 8>{}, kpc); break;
                    default: products(integral_constant<int, 12>{}, kpc); break;
                    }
                } else {
                    products(integral_constant<int, 0>{}, kpc);
                }
            };
            switch (nt) {
            case 4: with_kp(integral_constant<int, 64>{}); break;
            case 3: with_kp(integral_constant<int, 48>{}); break;
            case 2: with_kp(integral_constant<int, 32>{}); break;
            default: with_kp(integral_constant<int, 16>{}); break;
            }
        }
        if constexpr (NEXT) {
            load_ta(b + 1);    // ta is free: in flight over the barrier and the staging
            __syncthreads();   // every wavefront is done with S and T_j
            stage(b + 1);
        }
        if (rt < nto) {
            // lanes lr = 2 h and 2 h + 1 hold columns 2 h and 2 h + 1 of rows
            // r0 + lk + 4 e; the even lane writes the items of rows e = 0, 2,
            // the odd lane those of e = 1, 3
            double *blk = outp + d.out;
            const bool odd = lr & 1;
#pragma unroll
            for (int ct = 0; ct < 4; ++ct) {
                if (ct >= nto) break;
                const int g = 8 * ct + (lr >> 1);
#pragma unroll
                for (int q = 0; q < 2; ++q) {
                    const double a0 = o[ct][2 * q], a1 = o[ct][2 * q + 1];
                    const double p0 = __shfl_xor(a0, 1), p1 = __shfl_xor(a1, 1);
                    const double lo = odd ? p1 : a0, hi = odd ? a1 : p0;
                    const int row = r0 + lk + 4 * (2 * q + (odd ? 1 : 0));
                    if (row < ko && 2 * g < ko)
                        *reinterpret_cast<f64x2 *>(blk + (int64_t(g) * ko + row) * 2) =
                            f64x2{lo, 2 * g + 1 < ko ? hi : 0.0};
                }
            }
        }
    };
    prefetch(b0);
    load_ta(b0);
    stage(b0);
    for (int64_t b = b0; b + 1 < b1; ++b) block(b, std::true_type{});
    block(b1 - 1, std::false_type{});
}

}  // namespace

// One tree up: leaves, then levels q .. lmin+1.
// (IN_T: the tree is stored transposed, V_j^T and F_c^T: the column tree.)
template <bool IN_T>
static hipError_t orthogonalize_tree(const OrthLaunch &L, const int64_t *leaf_in, const int64_t *leaf_n,
                                     const int64_t *leaf_tr, const int64_t *xfer_in, const int64_t *xfer_n,
                                     const int64_t *xfer_tr, double *T, hipStream_t st) {
    hipLaunchKernelGGL(orth_leaf_kernel<IN_T>, dim3(unsigned(L.nleaves)), dim3(256), 0, st, L.basis, leaf_in, leaf_n,
                       leaf_tr, L.leaf_begin, L.leaf_end, L.level_rank[L.q], T, L.kmax, L.first_leaf);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    for (int l = L.q; l > L.lmin; --l) {
        const int64_t nparents = int64_t(1) << (l - 1);
        hipLaunchKernelGGL(orth_level_kernel<IN_T>, dim3(unsigned(nparents)), dim3(256), 0, st, L.basis, xfer_in,
                           xfer_n, xfer_tr, L.level_rank[l], L.level_rank[l - 1], T, L.kmax, nparents - 1);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_orthogonalize(const OrthLaunch &L, hipStream_t st) {
    if (L.nleaves <= 0) return hipSuccess;
    if (L.kmax < 1 || L.kmax > QR_MAXN) return hipErrorInvalidValue;
    hipError_t e;
    if (!L.T_col) {   // one tree: U_j and V_j^T, E_c and F_c^T written together
        e = orthogonalize_tree<false>(L, L.off_U, L.off_U, L.off_VT, L.off_E, L.off_E, L.off_FT, L.T, st);
        if (e != hipSuccess) return e;
        return launch_project(L.blocks, L.blocks, L.proj, L.nproj, L.T, L.T, L.kmax, st, true);
    }
    e = orthogonalize_tree<false>(L, L.off_U, L.off_U, nullptr, L.off_E, L.off_E, nullptr, L.T, st);
    if (e != hipSuccess) return e;
    e = orthogonalize_tree<true>(L, L.off_VT, nullptr, L.off_VT, L.off_FT, nullptr, L.off_FT, L.T_col, st);
    if (e != hipSuccess) return e;
    return launch_project(L.blocks, L.blocks, L.proj, L.nproj, L.T, L.T_col, L.kmax, st, true);
}

hipError_t launch_project(const double *in, double *out, const ProjDesc *desc, int64_t n, const double *T,
                          const double *T_col, int kmax, hipStream_t st, bool triangular) {
    if (n <= 0) return hipSuccess;
    if (kmax < 1 || kmax > QR_MAXN) return hipErrorInvalidValue;
    const int64_t grid = n < 65536 ? n : 65536;
    if (triangular)
        hipLaunchKernelGGL(project_kernel<true>, dim3(unsigned(grid)), dim3(256), 0, st, in, out, desc, n, T, T_col,
                           kmax);
    else
        hipLaunchKernelGGL(project_kernel<false>, dim3(unsigned(grid)), dim3(256), 0, st, in, out, desc, n, T, T_col,
                           kmax);
    return hipGetLastError();
}

}  // namespace h2
