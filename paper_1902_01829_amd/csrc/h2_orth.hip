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
    __shared__ double A[(64 + QR_PAD) * QR_MAXN], tau[QR_MAXN], sgn[QR_MAXN], scal[2];
    const int64_t j = blockIdx.x;
    const int M = int(leaf_end[j] - leaf_begin[j]), N = kq;
    const double *B = basis + in[j];
    const int ld = M + QR_PAD;
    for (int i = threadIdx.x; i < M * N; i += blockDim.x) {
        const int c = i / M, r = i - c * M;
        A[c * ld + r] = IN_T ? B[at2(N, c, r)] : B[at2(M, r, c)];
    }
    __syncthreads();
    householder_qr(A, tau, scal, sgn, M, N, T + (first_leaf + j) * kmax * kmax, kmax);
    for (int i = threadIdx.x; i < M * N; i += blockDim.x) {
        const int c = i / M, r = i - c * M;
        if (out_n) basis[out_n[j] + at2(M, r, c)] = A[c * ld + r];   // M x N
        if (out_t) basis[out_t[j] + at2(N, c, r)] = A[c * ld + r];   // N x M
    }
}

// Parents of level l - 1 (2^(l-1) workgroups): Z = [T_c1 E_c1; T_c2 E_c2].
// Transfers are read from `in` (kc x kp as stored, or its transpose when
// IN_T) and the new ones written to out_n (kc x kp) and/or out_t (kp x kc).
template <bool IN_T>
__global__ __launch_bounds__(256) void orth_level_kernel(double *basis, const int64_t *in,
                                                         const int64_t *out_n, const int64_t *out_t, int kc, int kp,
                                                         double *T, int kmax, int64_t first_parent) {
    __shared__ double A[(QR_MAXM + QR_PAD) * QR_MAXN], tau[QR_MAXN], sgn[QR_MAXN], scal[2];
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
    householder_qr(A, tau, scal, sgn, M, N, T + p * kmax * kmax, kmax);
    for (int h = 0; h < 2; ++h) {
        const int64_t ch = 2 * p + 1 + h;
        for (int i = threadIdx.x; i < kc * kp; i += blockDim.x) {
            const int c = i / kc, r = i - c * kc;
            const double v = A[c * ld + h * kc + r];
            if (out_n) basis[out_n[ch] + at2(kc, r, c)] = v;   // kc x kp
            if (out_t) basis[out_t[ch] + at2(kp, c, r)] = v;   // kp x kc
        }
    }
}

// Coupling block b: S' = T_i S T_j^T with T_i, T_j cut to their first kout
// rows (kout = k in the orthogonalization), on the FP64 matrix cores
// (v_mfma_f64_16x16x4_f64: lane l supplies A(l % 16, l / 16) and B(l / 16,
// l % 16) and holds D(l / 16 + 4 e, l % 16), e = 0..3 -- the rows of a lane's
// four results are 4 apart, unlike the FP32 16 x 16 forms).  Wavefront w
// owns output rows 16 w .. 16 w + 15: first W_w = T_i(rows, :) S, staged in
// the wave's own LDS slice, then S'(rows, :) = W_w T_j^T, staged back in the
// S buffer and stored as whole 16-byte items.  S is loaded as 16-byte items
// (two columns of a row), the next block's while this one's products run,
// and zero-padded to a multiple of 16; T_i and T_j are read as operands from
// memory (column-major, leading dimension kmax).  Each workgroup takes one
// contiguous run of the list: the blocks of a block row share T_i, which
// then stays in the caches.  TRI: T_i and T_j are upper triangular (the
// orthogonalization's R factors), so the K steps that meet only their zeros
// are skipped: below a wavefront's first row in T_i S, before an output
// column tile's first column in W T_j^T (3/8 of the matrix-core work of a
// rank-64 block).
constexpr int PS_LD = 68;   // LDS leading dimension of S (spread over the banks)

__device__ inline void proj_load(const double *blocks, const ProjDesc &d, f64x2 (&v)[8]) {
    const int k = d.k, kp = (k + 15) & ~15, rows = kp, ng = kp >> 1;
    const double *blk = blocks + d.off;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const int i = threadIdx.x + 256 * j, g = i / rows, r = i - g * rows;
        v[j] = (g < ng && r < k && 2 * g < k) ? __builtin_nontemporal_load(reinterpret_cast<const f64x2 *>(
                                                     blk + (int64_t(g) * k + r) * 2))
                                               : f64x2{0.0, 0.0};
    }
}

template <bool TRI>
__global__ __launch_bounds__(256) void project_kernel(const double *in, double *outp, const ProjDesc *desc,
                                                      int64_t nblocks, const double *T, const double *Tcol, int kmax) {
    __shared__ double S[64 * PS_LD];     // column-major
    __shared__ double Wl[4][16 * 64];    // per wave: 16 x 64, column-major, ld 16
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63, lr = lane & 15, lk = lane >> 4;
    const int64_t per = (nblocks + gridDim.x - 1) / gridDim.x;
    const int64_t b0 = int64_t(blockIdx.x) * per, b1 = b0 + per < nblocks ? b0 + per : nblocks;
    f64x2 nxt[8];
    if (b0 < b1) proj_load(in, desc[b0], nxt);
    for (int64_t b = b0; b < b1; ++b) {
        const ProjDesc d = desc[b];
        const int k = d.k, kp = (k + 15) & ~15, nt = kp >> 4;   // input: k x k, nt column tiles
        const int ko = d.kout, nto = (ko + 15) >> 4;             // output: ko x ko, nto row tiles
#pragma unroll
        for (int j = 0; j < 8; ++j) {   // this block's items into LDS
            const int i = threadIdx.x + 256 * j, g = i / kp, r = i - g * kp;
            if (g < (kp >> 1)) {
                S[(2 * g) * PS_LD + r] = nxt[j].x;
                S[(2 * g + 1) * PS_LD + r] = nxt[j].y;
            }
        }
        __syncthreads();
        if (b + 1 < b1) proj_load(in, desc[b + 1], nxt);   // in flight during the products
        const double *Ti = T + d.row * kmax * kmax, *Tj = Tcol + d.col * kmax * kmax;
        const int r0 = 16 * wv;
        if (wv < nto) {
            const int s0 = TRI ? 4 * wv : 0;   // T_i(rows r0 .., kk) = 0 for kk < r0
            double ta[16];   // T_i(r0 + lr, 4 s + lk)
#pragma unroll
            for (int s4 = 0; s4 < 16; ++s4) {
                const int kk = 4 * s4 + lk, row = r0 + lr;
                ta[s4] = (s4 >= s0 && row < ko && kk < k) ? Ti[int64_t(kk) * kmax + row] : 0.0;
            }
#pragma unroll
            for (int ct = 0; ct < 4; ++ct) {
                if (ct >= nt) break;   // wave-uniform
                f64x4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int s4 = 0; s4 < 16; ++s4) {
                    if (4 * s4 >= kp) break;
                    if (s4 < s0) continue;   // wave-uniform
                    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(ta[s4], S[(16 * ct + lr) * PS_LD + 4 * s4 + lk], acc, 0,
                                                               0, 0);
                }
#pragma unroll
                for (int e = 0; e < 4; ++e) Wl[wv][(16 * ct + lr) * 16 + lk + 4 * e] = acc[e];
            }
        }
        __syncthreads();   // S is free from here on: S' goes into it
        if (wv < nto) {
            double tb[2][16];   // T_j(16 ct + lr, 4 s + lk), one column tile ahead
            auto load_tb = [&](int ct, double (&o)[16]) {
                const int col = 16 * ct + lr;
#pragma unroll
                for (int s4 = 0; s4 < 16; ++s4) {
                    const int kk = 4 * s4 + lk;
                    o[s4] = (col < ko && kk < k) ? Tj[int64_t(kk) * kmax + col] : 0.0;
                }
            };
            load_tb(0, tb[0]);
#pragma unroll
            for (int ct = 0; ct < 4; ++ct) {
                if (ct >= nto) break;   // unrolled, so the buffer indices are static
                if (ct + 1 < nto) load_tb(ct + 1, tb[(ct + 1) & 1]);
                const double(&cur)[16] = tb[ct & 1];
                f64x4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int s4 = 0; s4 < 16; ++s4) {
                    if (4 * s4 >= kp) break;
                    if (TRI && s4 < 4 * ct) continue;   // T_j(cols 16 ct .., kk) = 0 for kk < 16 ct
                    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(Wl[wv][(4 * s4 + lk) * 16 + lr], cur[s4], acc, 0, 0, 0);
                }
#pragma unroll
                for (int e = 0; e < 4; ++e) S[(16 * ct + lr) * PS_LD + r0 + lk + 4 * e] = acc[e];
            }
        }
        __syncthreads();
        double *blk = outp + d.out;
        for (int i = threadIdx.x; i < ko * ((ko + 1) >> 1); i += 256) {   // S' as 16-byte items
            const int g = i / ko, r = i - g * ko;
            const double hi = 2 * g + 1 < ko ? S[(2 * g + 1) * PS_LD + r] : 0.0;
            *reinterpret_cast<f64x2 *>(blk + (int64_t(g) * ko + r) * 2) = f64x2{S[(2 * g) * PS_LD + r], hi};
        }
        __syncthreads();   // S is rewritten by the next block
    }
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
