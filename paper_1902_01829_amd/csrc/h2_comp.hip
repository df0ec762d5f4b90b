// Algebraic compression of a symmetric H^2 matrix with orthonormal nested
// bases (Sec. 5.2 and 5.3), FP64.
//
// Basis generation, top-down: node i of level l stacks
//     Sbar_i = [R_i+ E_i^T; S_ij1^T; ...; S_ijb^T]
// (i+ its parent, S_ij the coupling blocks of its block row; when the blocks
// are not symmetric, the blocks S_ji of its block column follow, since the
// one basis tree serves the columns too) and keeps the triangular factor R_i
// of its QR factorization.  The stack is not formed
// whole: a workgroup holds 128 x 64 in registers, so blocks are appended
// under the current factor and folded into it with a QR of the stack
// whenever the next block would not fit (the same R up to row signs, which
// the truncation does not see: it uses R only through R^T R).
//
// A matrix with a row and a column tree of their own runs basis generation
// and truncation once per tree (the column tree from the block columns,
// through V_j^T and F_c^T read transposed), a level taking the larger rank.
//
// Truncation, bottom-up: leaves decompose W_i = U_i R_i^T; as U_i has
// orthonormal columns, the left singular vectors of W_i are U_i times those
// of R_i^T, so the SVD runs on the k x k matrix R_i^T.  Parents decompose
// W_p = Z_p R_p^T with Z_p = [T_c1 E_c1; T_c2 E_c2]; a tall W_p is first
// reduced to its triangular factor by a Householder QR (W_p = Q R_w), and
// the left singular vectors are Q times those of R_w.  The SVD is the
// one-sided Jacobi method with accumulated rotations, so the kept vectors
// are orthonormal also past the numerical rank of a node.  A node keeps the
// singular values at least eps times its largest; the host takes the
// largest count of a level as its new rank.
//
// One workgroup per node: 512 threads with the stack in registers for the
// basis generation, 256 threads with every matrix staged column-major in LDS
// for the truncation.

#include <hip/hip_runtime.h>

#include <cstdint>

#include "h2_device.h"
#include "h2_lds_la.h"

namespace h2 {
namespace {

using namespace lds;

typedef double f64x2 __attribute__((ext_vector_type(2)));

constexpr int GEN_LD = QR_MAXM + QR_PAD;   // LDS matrices of up to 128 rows (+ pad) x 64 columns
constexpr int SQ_LD = 64 + QR_PAD;         // LDS square matrices: 64 x 64 (+ pad)
constexpr double JACOBI_TOL = 64 * 2.220446049250313e-16;
constexpr int JACOBI_SWEEPS = 30;

__device__ inline int64_t level_first(int l) { return (int64_t(1) << l) - 1; }

// Basis generation of one node, a 256 x k stack held in registers of a
// 1024-thread workgroup: wave w owns columns 4 w .. 4 w + 3, lanes
// 16 h .. 16 h + 15 of it column 4 w + h, and lane j = l % 16 of those rows
// j, j + 16, ..., j + 240 (a[i] = row j + 16 i; consecutive lanes touch
// consecutive LDS words).  Rows 0 .. 63 (i < 4) hold the current triangular
// factor (first: the parent term), rows 64 .. 255 the coupling blocks
// appended since (as many k-row blocks as fit).  A fold is a Householder QR
// without Q over all 256 rows: per column c the sixteen lanes of column c
// form the reflector and publish it in LDS (double buffered, so one barrier
// per column), and every lane of a later column applies it to its 16 rows;
// entries below the diagonal are set to zero as they are eliminated, so
// after a fold rows k .. 255 are zero.  The lanes of a column are one DPP
// row, so their sums are four DPP moves.  Register arrays are indexed
// statically only (the diagonal row is selected by comparison).
constexpr int BG_THREADS = 1024, BG_ROWS = 16, BG_STACK = 256, BG_TLD = 65;

__device__ inline void fold_r(double (&a)[BG_ROWS], int k, int col, int j, double (*vbuf)[BG_STACK],
                              double *tbuf) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int c = 0; c < k; ++c) {
        double *v = vbuf[c & 1];
        if (wv == (c >> 2) && (lane >> 4) == (c & 3)) {   // the sixteen lanes of column c
            double sq = 0.0, al = 0.0;
#pragma unroll
            for (int i = 0; i < BG_ROWS; ++i) {
                const int r = j + 16 * i;
                sq += r > c ? a[i] * a[i] : 0.0;
                al += r == c ? a[i] : 0.0;
            }
            sq = dpp_sum16(sq);
            al = dpp_sum16(al);
            const double nrm = sqrt(sq + al * al);
            double beta = al, tc = 0.0, sc = 0.0;
            if (sq > 0.0) {
                beta = al >= 0.0 ? -nrm : nrm;
                tc = (beta - al) / beta;
                sc = 1.0 / (al - beta);
            }
#pragma unroll
            for (int i = 0; i < BG_ROWS; ++i) {
                const int r = j + 16 * i;
                v[r] = r > c ? a[i] * sc : (r == c ? 1.0 : 0.0);
                a[i] = r > c ? 0.0 : (r == c ? beta : a[i]);
            }
            if (j == 0) tbuf[c & 1] = tc;
        }
        __syncthreads();
        const double tc = tbuf[c & 1];
        if (col > c && col < k && tc != 0.0) {   // uniform over the sixteen lanes of a column
            double d = 0.0;
#pragma unroll
            for (int i = 0; i < BG_ROWS; ++i) d += v[j + 16 * i] * a[i];
            d = dpp_sum16(d) * tc;
#pragma unroll
            for (int i = 0; i < BG_ROWS; ++i) a[i] -= d * v[j + 16 * i];
        }
    }
    __syncthreads();   // the last reflector's readers are done before vbuf is reused
}

__global__ __launch_bounds__(BG_THREADS) void basis_generation_kernel(CompLaunch L, int level, int k, int kp,
                                                                      int parent_term) {
    __shared__ double vbuf[2][BG_STACK], tbuf[2];
    __shared__ double tile[64 * BG_TLD];   // staging of R_parent (column-major) and of each coupling block (row-major)
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int col = 4 * wv + (lane >> 4), j = lane & 15;
    const int64_t node = level_first(level) + blockIdx.x;
    double a[BG_ROWS];
#pragma unroll
    for (int i = 0; i < BG_ROWS; ++i) a[i] = 0.0;
    bool dirty = false;   // rows hold entries not yet folded into a triangular factor
    if (parent_term) {    // rows 0 .. kp-1: P = R_parent E_i^T (kp x k), R_parent upper triangular
        const double *Rp = L.R + ((node - 1) >> 1) * L.kmax * L.kmax;   // zero below its diagonal
        for (int i = t; i < 64 * kp; i += BG_THREADS) {
            const int c = i >> 6, r = i & 63;
            tile[c * BG_TLD + r] = r < kp ? Rp[int64_t(c) * L.kmax + r] : 0.0;
        }
        __syncthreads();
        const double *E = L.basis + L.off_E[node];   // k x kp (or its transpose)
        if (col < k)
            for (int u = 0; u < kp; ++u) {
                const double e = L.x_t ? E[at2(kp, u, col)] : E[at2(k, col, u)];
#pragma unroll
                for (int i = 0; i < 4; ++i) a[i] += tile[u * BG_TLD + j + 16 * i] * e;
            }
        dirty = true;
    }
    // the stack's blocks: those of block row i, transposed, then (when the
    // coupling blocks are not symmetric) those of block column i as they are
    const int64_t nrow = L.use_rows ? L.row_start[node + 1] - L.row_start[node] : 0;
    const int64_t nb = nrow + (L.columns ? L.col_start[node + 1] - L.col_start[node] : 0);
    const int ng = (k + 1) >> 1;
    int64_t b = 0;
    for (;;) {   // append as many blocks as fit under the factor, then fold (one call site)
        for (int bot = 0; b < nb && bot + k <= BG_STACK - 64; ++b, bot += k) {
            __syncthreads();   // the tile's previous contents are consumed
            const bool from_row = b < nrow;
            const double *S = L.blocks + (from_row ? L.blk[L.row_start[node] + b].off
                                                   : L.col_blk[L.col_start[node] + (b - nrow)]);
            for (int i = t; i < ng * k; i += BG_THREADS) {   // S(r, 2g .. 2g+1) is one 16-byte item
                const int g = i / k, r = i - g * k;
                const f64x2 v = *reinterpret_cast<const f64x2 *>(S + (int64_t(g) * k + r) * 2);
                tile[r * BG_TLD + 2 * g] = v.x;
                tile[r * BG_TLD + 2 * g + 1] = v.y;   // column k when k is odd: padding, never read
            }
            __syncthreads();
            // rows 64 + bot .. 64 + bot + k - 1: row rr, column col is S(col, rr) for a row block
            // (S^T) and S(rr, col) for a column block
            if (col < k) {
#pragma unroll
                for (int i = 4; i < BG_ROWS; ++i) {
                    const int rr = j + 16 * i - 64 - bot;
                    if (rr >= 0 && rr < k) a[i] = from_row ? tile[col * BG_TLD + rr] : tile[rr * BG_TLD + col];
                }
            }
            dirty = true;
        }
        if (!dirty) break;
        fold_r(a, k, col, j, vbuf, tbuf);
        dirty = false;
        if (b >= nb) break;
    }
    double *R = L.R + node * L.kmax * L.kmax;   // rows 0 .. k-1 (zero below the diagonal)
    if (col < k) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int r = j + 16 * i;
            if (r < k) R[int64_t(col) * L.kmax + r] = a[i];
        }
    }
}

// After jacobi_svd: the singular values s (column norms of G, n columns of
// length Lrows), rank[j] = position of column j in descending order (ties by
// index), sigma (n values, descending) and the count kept for eps.
__device__ inline void sort_and_count(const double *G, int ldg, int Lrows, int n, double eps, double *s, int *rank,
                                      double *sigma, int32_t *count) {
    const int t = threadIdx.x;
    if (t < n) {
        double a = 0.0;
        for (int r = 0; r < Lrows; ++r) a += G[t * ldg + r] * G[t * ldg + r];
        s[t] = sqrt(a);
    }
    __syncthreads();
    if (t < n) {
        const double v = s[t];
        int rk = 0;
        for (int i = 0; i < n; ++i) rk += (s[i] > v) || (s[i] == v && i < t);
        rank[t] = rk;
        sigma[rk] = v;
    }
    if (t == 0) {
        double smax = 0.0;
        for (int i = 0; i < n; ++i) smax = s[i] > smax ? s[i] : smax;
        int cnt = 0;
        if (smax > 0.0)
            for (int i = 0; i < n; ++i) cnt += s[i] >= eps * smax;
        *count = cnt;
    }
    __syncthreads();
}

__global__ __launch_bounds__(256) void truncate_leaves_kernel(CompLaunch L, int k, double eps) {
    __shared__ double G[64 * SQ_LD], Y[64 * SQ_LD], s[64];
    __shared__ int rank[64], flag;
    const int t = threadIdx.x;
    const int64_t j = blockIdx.x, node = L.first_leaf + j;
    // the rows of R_j^T are the columns of R_j
    const double *R = L.R + node * L.kmax * L.kmax;
    for (int i = t; i < k * k; i += 256) {
        const int c = i / k, r = i - c * k;
        G[c * SQ_LD + r] = R[int64_t(c) * L.kmax + r];
        Y[c * SQ_LD + r] = r == c ? 1.0 : 0.0;
    }
    __syncthreads();
    jacobi_svd(G, SQ_LD, k, Y, SQ_LD, k, JACOBI_TOL, JACOBI_SWEEPS, &flag, s);
    sort_and_count(G, SQ_LD, k, k, eps, s, rank, L.sigma + j * 64, L.count + j);
    double *X = L.X + j * COMP_XSLOT;
    for (int i = t; i < k * k; i += 256) {
        const int c = i / k, r = i - c * k;
        X[int64_t(rank[c]) * COMP_XLD + r] = Y[c * SQ_LD + r];
    }
}

__global__ __launch_bounds__(256) void truncate_leaves_apply_kernel(CompLaunch L, int k, int kt) {
    __shared__ double Uo[64 * SQ_LD], Xs[64 * SQ_LD];
    const int t = threadIdx.x;
    const int64_t j = blockIdx.x, node = L.first_leaf + j;
    const int m = int(L.leaf_end[j] - L.leaf_begin[j]);
    const double *U = L.basis + L.off_U[j];   // m x k (or its transpose)
    const double *X = L.X + j * COMP_XSLOT;
    for (int i = t; i < m * k; i += 256) {
        const int c = i / m, r = i - c * m;
        Uo[c * SQ_LD + r] = L.b_t ? U[at2(k, c, r)] : U[at2(m, r, c)];
    }
    for (int i = t; i < k * kt; i += 256) {
        const int c = i / k, r = i - c * k;
        Xs[c * SQ_LD + r] = X[int64_t(c) * COMP_XLD + r];
    }
    __syncthreads();
    double *Un = L.Unew + j * COMP_USLOT;
    for (int i = t; i < m * kt; i += 256) {   // U_new = U X(:, 0:kt)
        const int c = i / m, r = i - c * m;
        double acc = 0.0;
        for (int u = 0; u < k; ++u) acc += Uo[u * SQ_LD + r] * Xs[c * SQ_LD + u];
        Un[c * 64 + r] = acc;
    }
    double *T = L.T + node * L.kmax * L.kmax;   // T_j = X(:, 0:kt)^T (kt x k)
    for (int i = t; i < kt * k; i += 256) {
        const int c = i / kt, r = i - c * kt;
        T[int64_t(c) * L.kmax + r] = Xs[r * SQ_LD + c];
    }
}

// Z_p = [T_c1 E_c1; T_c2 E_c2] (2 kt x kp) into Z (leading dimension ldz);
// Ts and Es are 64 x 64 LDS staging buffers.
__device__ inline void form_z(const CompLaunch &L, int64_t p, int kc, int kt, int kp, double *Z, int ldz, double *Ts,
                              double *Es) {
    const int t = threadIdx.x;
    for (int h = 0; h < 2; ++h) {
        const int64_t ch = 2 * p + 1 + h;
        const double *Tc = L.T + ch * L.kmax * L.kmax;   // kt x kc
        const double *E = L.basis + L.off_E[ch];        // kc x kp (or its transpose)
        for (int i = t; i < kt * kc; i += 256) {
            const int c = i / kt, r = i - c * kt;
            Ts[c * SQ_LD + r] = Tc[int64_t(c) * L.kmax + r];
        }
        for (int i = t; i < kc * kp; i += 256) {
            const int c = i / kc, r = i - c * kc;
            Es[c * SQ_LD + r] = L.x_t ? E[at2(kp, c, r)] : E[at2(kc, r, c)];
        }
        __syncthreads();
        for (int i = t; i < kt * kp; i += 256) {
            const int c = i / kt, r = i - c * kt;
            double acc = 0.0;
            for (int u = 0; u < kc; ++u) acc += Ts[u * SQ_LD + r] * Es[c * SQ_LD + u];
            Z[c * ldz + h * kt + r] = acc;
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void truncate_level_kernel(CompLaunch L, int l, int kc, int kt, int kp, double eps) {
    __shared__ double A[GEN_LD * QR_MAXN], G[64 * SQ_LD], Y[64 * SQ_LD];
    __shared__ double tau[QR_MAXN], sgn[QR_MAXN], s[64];
    __shared__ int rank[64], flag;
    const int t = threadIdx.x;
    const int64_t i0 = blockIdx.x, p = level_first(l - 1) + i0;
    const int M = 2 * kt, ldz = M + QR_PAD;   // the leading dimension householder_qr uses
    form_z(L, p, kc, kt, kp, A, ldz, G, Y);
    // W = Z R_p^T (M x kp): R_p staged in G, the products held in registers
    const double *Rp = L.R + p * L.kmax * L.kmax;
    for (int i = t; i < kp * kp; i += 256) {
        const int c = i / kp, r = i - c * kp;
        G[c * SQ_LD + r] = Rp[int64_t(c) * L.kmax + r];
    }
    __syncthreads();
    double w[32];
#pragma unroll
    for (int q = 0; q < 32; ++q) {
        const int i = t + 256 * q, c = i / M, r = i - c * M;
        double acc = 0.0;
        if (c < kp)
            for (int u = c; u < kp; ++u) acc += A[u * ldz + r] * G[u * SQ_LD + c];   // Z(r, u) R_p(c, u)
        w[q] = acc;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 32; ++q) {
        const int i = t + 256 * q, c = i / M, r = i - c * M;
        if (c < kp) A[c * ldz + r] = w[q];
    }
    __syncthreads();
    const bool tall = M > kp;
    int n, Lrows;
    if (tall) {   // W = Q R_w: Q in A, R_w in Y, then G = R_w^T (its rows as columns)
        householder_qr(A, tau, sgn, M, kp, Y, SQ_LD);
        n = kp;
        Lrows = kp;
        for (int i = t; i < kp * kp; i += 256) {
            const int c = i / kp, r = i - c * kp;
            G[c * SQ_LD + r] = Y[r * SQ_LD + c];
        }
        __syncthreads();
        for (int i = t; i < kp * kp; i += 256) {
            const int c = i / kp, r = i - c * kp;
            Y[c * SQ_LD + r] = r == c ? 1.0 : 0.0;
        }
    } else {      // G = W^T: the M rows of W as columns of length kp
        n = M;
        Lrows = kp;
        for (int i = t; i < kp * M; i += 256) {
            const int c = i / kp, r = i - c * kp;
            G[c * SQ_LD + r] = A[r * ldz + c];
        }
        for (int i = t; i < M * M; i += 256) {
            const int c = i / M, r = i - c * M;
            Y[c * SQ_LD + r] = r == c ? 1.0 : 0.0;
        }
    }
    __syncthreads();
    jacobi_svd(G, SQ_LD, Lrows, Y, SQ_LD, n, JACOBI_TOL, JACOBI_SWEEPS, &flag, s);
    sort_and_count(G, SQ_LD, Lrows, n, eps, s, rank, L.sigma + i0 * 64, L.count + i0);
    double *X = L.X + i0 * COMP_XSLOT;   // left singular vectors of W: M x n
    if (tall) {
        for (int i = t; i < M * n; i += 256) {
            const int c = i / M, r = i - c * M;
            double acc = 0.0;
            for (int u = 0; u < kp; ++u) acc += A[u * ldz + r] * Y[c * SQ_LD + u];
            X[int64_t(rank[c]) * COMP_XLD + r] = acc;
        }
    } else {
        for (int i = t; i < M * n; i += 256) {
            const int c = i / M, r = i - c * M;
            X[int64_t(rank[c]) * COMP_XLD + r] = Y[c * SQ_LD + r];
        }
    }
}

__global__ __launch_bounds__(256) void truncate_level_apply_kernel(CompLaunch L, int l, int kc, int kt, int kp,
                                                                   int ktp) {
    __shared__ double A[GEN_LD * QR_MAXN], G[64 * SQ_LD], Y[64 * SQ_LD];
    const int t = threadIdx.x;
    const int64_t i0 = blockIdx.x, p = level_first(l - 1) + i0;
    const int M = 2 * kt, ldz = M + QR_PAD;
    const double *X = L.X + i0 * COMP_XSLOT;   // M x ktp used
    for (int h = 0; h < 2; ++h) {              // new transfers: the two kt x ktp blocks of X
        double *En = L.Enew + (2 * p + 1 + h) * L.kmax * L.kmax;
        for (int i = t; i < kt * ktp; i += 256) {
            const int c = i / kt, r = i - c * kt;
            En[int64_t(c) * L.kmax + r] = X[int64_t(c) * COMP_XLD + h * kt + r];
        }
    }
    form_z(L, p, kc, kt, kp, A, ldz, G, Y);
    double *T = L.T + p * L.kmax * L.kmax;     // T_p = X(:, 0:ktp)^T Z_p (ktp x kp)
    for (int i = t; i < ktp * kp; i += 256) {
        const int c = i / ktp, r = i - c * ktp;
        double acc = 0.0;
        for (int u = 0; u < M; ++u) acc += X[int64_t(r) * COMP_XLD + u] * A[c * ldz + u];
        T[int64_t(c) * L.kmax + r] = acc;
    }
}

__global__ __launch_bounds__(256) void symmetry_check_kernel(const double *blocks, const MirrorDesc *desc, int64_t n,
                                                             int32_t *flag) {
    for (int64_t p = blockIdx.x; p < n; p += gridDim.x) {
        const MirrorDesc d = desc[p];
        int diff = 0;
        for (int e = threadIdx.x; e < d.k * d.k; e += 256) {
            const int c = e / d.k, r = e - c * d.k;
            diff |= blocks[d.a + at2(d.k, r, c)] != blocks[d.b + at2(d.k, c, r)];
        }
        if (__syncthreads_or(diff) && threadIdx.x == 0) *flag = 1;
    }
}

__global__ __launch_bounds__(256) void place_kernel(const double *src, double *dst, const PlaceDesc *desc, int64_t n) {
    for (int64_t b = blockIdx.x; b < n; b += gridDim.x) {
        const PlaceDesc d = desc[b];
        const int64_t ne = int64_t((d.C + 1) >> 1) * d.R * 2;
        for (int64_t e = threadIdx.x; e < ne; e += 256) {
            const int w = int(e & 1);
            const int64_t g = e >> 1;
            const int r = int(g % d.R), c = int(g / d.R) * 2 + w;
            double v = 0.0;
            if (c < d.C) v = d.transpose ? src[d.src + int64_t(r) * d.ld + c] : src[d.src + int64_t(c) * d.ld + r];
            dst[d.dst + e] = v;
        }
    }
}

}  // namespace

hipError_t launch_basis_generation(const CompLaunch &L, int level, int k, int kp, bool parent_term, hipStream_t st) {
    if (k < 1 || k > QR_MAXN || kp > QR_MAXN || (parent_term && kp < 1)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(basis_generation_kernel, dim3(unsigned(int64_t(1) << level)), dim3(BG_THREADS), 0, st, L,
                       level, k, kp, parent_term ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_truncate_leaves(const CompLaunch &L, int k, double eps, hipStream_t st) {
    if (k < 1 || k > QR_MAXN) return hipErrorInvalidValue;
    hipLaunchKernelGGL(truncate_leaves_kernel, dim3(unsigned(L.nleaves)), dim3(256), 0, st, L, k, eps);
    return hipGetLastError();
}

hipError_t launch_truncate_leaves_apply(const CompLaunch &L, int k, int kt, hipStream_t st) {
    if (k < 1 || k > QR_MAXN || kt < 1 || kt > k) return hipErrorInvalidValue;
    hipLaunchKernelGGL(truncate_leaves_apply_kernel, dim3(unsigned(L.nleaves)), dim3(256), 0, st, L, k, kt);
    return hipGetLastError();
}

hipError_t launch_truncate_level(const CompLaunch &L, int l, int kc, int kt, int kp, double eps, hipStream_t st) {
    if (l < 1 || kc < 1 || kc > QR_MAXN || kt < 1 || kt > kc || 2 * kt > QR_MAXM || kp < 1 || kp > QR_MAXN)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(truncate_level_kernel, dim3(unsigned(int64_t(1) << (l - 1))), dim3(256), 0, st, L, l, kc, kt,
                       kp, eps);
    return hipGetLastError();
}

hipError_t launch_truncate_level_apply(const CompLaunch &L, int l, int kc, int kt, int kp, int ktp, hipStream_t st) {
    if (l < 1 || kc < 1 || kc > QR_MAXN || kt < 1 || kt > kc || 2 * kt > QR_MAXM || kp < 1 || kp > QR_MAXN ||
        ktp < 1 || ktp > kp || ktp > 2 * kt)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(truncate_level_apply_kernel, dim3(unsigned(int64_t(1) << (l - 1))), dim3(256), 0, st, L, l, kc,
                       kt, kp, ktp);
    return hipGetLastError();
}

hipError_t launch_symmetry_check(const double *blocks, const MirrorDesc *desc, int64_t n, int32_t *flag,
                                 hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const int64_t grid = n < 65536 ? n : 65536;
    hipLaunchKernelGGL(symmetry_check_kernel, dim3(unsigned(grid)), dim3(256), 0, st, blocks, desc, n, flag);
    return hipGetLastError();
}

hipError_t launch_place(const double *src, double *dst, const PlaceDesc *desc, int64_t n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const int64_t grid = n < 65536 ? n : 65536;
    hipLaunchKernelGGL(place_kernel, dim3(unsigned(grid)), dim3(256), 0, st, src, dst, desc, n);
    return hipGetLastError();
}

}  // namespace h2
