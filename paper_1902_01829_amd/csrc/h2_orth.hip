// Basis orthogonalization and projection of the coupling blocks (Sec. 5.1,
// Alg. 6 and Alg. 7), FP64, for the symmetric case U = V, E = F.
//
// Leaves: U_j = Q_j T_j (thin Householder QR), Q_j the new leaf basis.  Up the
// tree, parent p with children c1, c2: Z = [T_c1 E_c1; T_c2 E_c2] = Q T_p, the
// two blocks of Q the new transfers.  Then every coupling block S_ij becomes
// T_i S_ij T_j^T.  The diagonal of every T is made non-negative, which makes
// the factorization unique for full-column-rank inputs.
//
// One workgroup (256 threads) per factorization or per coupling block; the
// matrices are staged column-major in LDS (up to 128 x 64 FP64 for Z).  In a
// factorization four threads share a column: thread t owns column t / 4 and
// rows (t % 4) + 4 i, and the four combine their partial dot products with
// lane shuffles.

#include <hip/hip_runtime.h>

#include <cstdint>

#include "h2_device.h"

namespace h2 {
namespace {

constexpr int QR_MAXM = 128, QR_MAXN = 64;

// Element (r, c) of an R-row FP64 block in 16-byte column groups (2 columns).
__device__ inline int64_t at2(int R, int r, int c) { return (int64_t(c >> 1) * R + r) * 2 + (c & 1); }

__device__ inline double sum4(double v) {   // over the 4 threads of a column (consecutive lanes)
    v += __shfl_xor(v, 1);
    v += __shfl_xor(v, 2);
    return v;
}

// In-place Householder QR of the M x N matrix A (column-major, ld M, LDS),
// M >= N: R in the upper triangle, v_c below the diagonal (v_c[c] = 1
// implicit), tau[c].  Then Q (M x N, ld M) formed explicitly, and the signs of
// R's rows and Q's columns flipped so that diag(R) >= 0.
__device__ void householder_qr(double *A, double *Q, double *tau, double *scal, int M, int N) {
    const int t = threadIdx.x, col = t >> 2, sub = t & 3;
    for (int c = 0; c < N; ++c) {
        // norm of A[c:M, c] (column c's four threads), then the reflector
        if (col == c) {
            double s = 0.0;
            for (int r = c + sub; r < M; r += 4) s += A[c * M + r] * A[c * M + r];
            s = sum4(s);
            if (sub == 0) {
                const double alpha = A[c * M + c], nrm = sqrt(s);
                double tc = 0.0, beta = alpha, sc = 0.0;
                if (nrm > 0.0) {
                    beta = alpha >= 0.0 ? -nrm : nrm;
                    tc = (beta - alpha) / beta;
                    sc = 1.0 / (alpha - beta);
                }
                tau[c] = tc;
                scal[0] = sc;
                scal[1] = beta;
            }
        }
        __syncthreads();
        const double sc = scal[0], tc = tau[c];
        if (col == c) {
            for (int r = c + 1 + sub; r < M; r += 4) A[c * M + r] *= sc;
        }
        __syncthreads();
        if (col == c && sub == 0) A[c * M + c] = scal[1];
        // apply H_c = I - tau v v^T to the columns to the right
        if (col > c && col < N && tc != 0.0) {
            double w = sub == 0 ? A[col * M + c] : 0.0;
            for (int r = c + 1 + sub; r < M; r += 4) w += A[c * M + r] * A[col * M + r];
            w = sum4(w) * tc;
            if (sub == 0) A[col * M + c] -= w;
            for (int r = c + 1 + sub; r < M; r += 4) A[col * M + r] -= w * A[c * M + r];
        }
        __syncthreads();
    }
    // Q = H_0 ... H_(N-1) [I; 0], applied from the last reflector back
    for (int i = t; i < M * N; i += blockDim.x) {
        const int c = i / M, r = i - c * M;
        Q[i] = r == c ? 1.0 : 0.0;
    }
    __syncthreads();
    for (int c = N - 1; c >= 0; --c) {
        const double tc = tau[c];
        if (col >= c && col < N && tc != 0.0) {
            double w = sub == 0 ? Q[col * M + c] : 0.0;
            for (int r = c + 1 + sub; r < M; r += 4) w += A[c * M + r] * Q[col * M + r];
            w = sum4(w) * tc;
            if (sub == 0) Q[col * M + c] -= w;
            for (int r = c + 1 + sub; r < M; r += 4) Q[col * M + r] -= w * A[c * M + r];
        }
        __syncthreads();
    }
    // signs: diag(R) >= 0
    for (int i = t; i < M * N; i += blockDim.x) {
        const int c = i / M;
        if (A[c * M + c] < 0.0) Q[i] = -Q[i];
    }
    __syncthreads();
}

// Writes R (N x N, upper triangle of A with the signs fixed) into T (ld ldt).
__device__ void store_r(const double *A, int M, int N, double *T, int ldt) {
    for (int i = threadIdx.x; i < N * N; i += blockDim.x) {
        const int c = i / N, r = i - c * N;
        const double sgn = A[r * M + r] < 0.0 ? -1.0 : 1.0;
        T[int64_t(c) * ldt + r] = r <= c ? sgn * A[c * M + r] : 0.0;
    }
}

__global__ __launch_bounds__(256) void orth_leaf_kernel(double *basis, const int64_t *off_U, const int64_t *off_VT,
                                                        const int64_t *leaf_begin, const int64_t *leaf_end, int kq,
                                                        double *T, int kmax, int64_t first_leaf) {
    __shared__ double A[QR_MAXM * QR_MAXN], Q[QR_MAXM * QR_MAXN], tau[QR_MAXN], scal[2];
    const int64_t j = blockIdx.x;
    const int M = int(leaf_end[j] - leaf_begin[j]), N = kq;
    const double *U = basis + off_U[j];
    for (int i = threadIdx.x; i < M * N; i += blockDim.x) {
        const int c = i / M, r = i - c * M;
        A[i] = U[at2(M, r, c)];
    }
    __syncthreads();
    householder_qr(A, Q, tau, scal, M, N);
    double *Uo = basis + off_U[j], *VT = basis + off_VT[j];
    for (int i = threadIdx.x; i < M * N; i += blockDim.x) {
        const int c = i / M, r = i - c * M;
        Uo[at2(M, r, c)] = Q[i];      // U_j: M x N
        VT[at2(N, c, r)] = Q[i];      // V_j^T: N x M
    }
    store_r(A, M, N, T + (first_leaf + j) * kmax * kmax, kmax);
}

// Parents of level l - 1 (2^(l-1) workgroups): Z = [T_c1 E_c1; T_c2 E_c2].
__global__ __launch_bounds__(256) void orth_level_kernel(double *basis, const int64_t *off_E, const int64_t *off_FT,
                                                         int kc, int kp, double *T, int kmax, int64_t first_parent) {
    __shared__ double A[QR_MAXM * QR_MAXN], Q[QR_MAXM * QR_MAXN], tau[QR_MAXN], scal[2];
    const int64_t p = first_parent + blockIdx.x;
    const int M = 2 * kc, N = kp;
    for (int h = 0; h < 2; ++h) {
        const int64_t ch = 2 * p + 1 + h;
        const double *E = basis + off_E[ch];                    // kc x kp
        const double *Tc = T + ch * kmax * kmax;                // kc x kc, upper triangular
        for (int i = threadIdx.x; i < kc * kp; i += blockDim.x) {
            const int c = i / kc, r = i - c * kc;
            double s = 0.0;
            for (int u = r; u < kc; ++u) s += Tc[int64_t(u) * kmax + r] * E[at2(kc, u, c)];
            A[c * M + h * kc + r] = s;
        }
    }
    __syncthreads();
    householder_qr(A, Q, tau, scal, M, N);
    for (int h = 0; h < 2; ++h) {
        const int64_t ch = 2 * p + 1 + h;
        double *E = basis + off_E[ch], *FT = basis + off_FT[ch];
        for (int i = threadIdx.x; i < kc * kp; i += blockDim.x) {
            const int c = i / kc, r = i - c * kc;
            const double v = Q[c * M + h * kc + r];
            E[at2(kc, r, c)] = v;       // E_c: kc x kp
            FT[at2(kp, c, r)] = v;      // F_c^T: kp x kc
        }
    }
    store_r(A, M, N, T + p * kmax * kmax, kmax);
}

// Coupling block b: S <- T_i S T_j^T (k x k, in place).
__global__ __launch_bounds__(256) void orth_project_kernel(double *blocks, const ProjDesc *desc, int64_t nblocks,
                                                           const double *T, int kmax) {
    __shared__ double S[64 * 64], W[64 * 64], Ti[64 * 64], Tj[64 * 64];
    for (int64_t b = blockIdx.x; b < nblocks; b += gridDim.x) {
        const ProjDesc d = desc[b];
        const int k = d.k;
        double *blk = blocks + d.off;
        const double *Ta = T + d.row * kmax * kmax, *Tb = T + d.col * kmax * kmax;
        for (int i = threadIdx.x; i < k * k; i += blockDim.x) {
            const int c = i / k, r = i - c * k;
            S[i] = blk[at2(k, r, c)];
            Ti[i] = Ta[int64_t(c) * kmax + r];
            Tj[i] = Tb[int64_t(c) * kmax + r];
        }
        __syncthreads();
        for (int i = threadIdx.x; i < k * k; i += blockDim.x) {   // W = T_i S (T_i upper triangular)
            const int c = i / k, r = i - c * k;
            double s = 0.0;
            for (int u = r; u < k; ++u) s += Ti[u * k + r] * S[c * k + u];
            W[i] = s;
        }
        __syncthreads();
        for (int i = threadIdx.x; i < k * k; i += blockDim.x) {   // S' = W T_j^T: (W T_j^T)(r,c) = sum_u W(r,u) T_j(c,u)
            const int c = i / k, r = i - c * k;
            double s = 0.0;
            for (int u = c; u < k; ++u) s += W[u * k + r] * Tj[u * k + c];
            blk[at2(k, r, c)] = s;
        }
        __syncthreads();
    }
}

}  // namespace

hipError_t launch_orthogonalize(const OrthLaunch &L, hipStream_t st) {
    if (L.nleaves <= 0) return hipSuccess;
    if (L.kmax < 1 || L.kmax > QR_MAXN) return hipErrorInvalidValue;
    hipLaunchKernelGGL(orth_leaf_kernel, dim3(unsigned(L.nleaves)), dim3(256), 0, st, L.basis, L.off_U, L.off_VT,
                       L.leaf_begin, L.leaf_end, L.level_rank[L.q], L.T, L.kmax, L.first_leaf);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    for (int l = L.q; l > L.lmin; --l) {
        const int64_t nparents = int64_t(1) << (l - 1);
        hipLaunchKernelGGL(orth_level_kernel, dim3(unsigned(nparents)), dim3(256), 0, st, L.basis, L.off_E, L.off_FT,
                           L.level_rank[l], L.level_rank[l - 1], L.T, L.kmax, nparents - 1);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (L.nproj > 0) {
        const int64_t grid = L.nproj < 65536 ? L.nproj : 65536;
        hipLaunchKernelGGL(orth_project_kernel, dim3(unsigned(grid)), dim3(256), 0, st, L.blocks, L.proj, L.nproj, L.T,
                           L.kmax);
        e = hipGetLastError();
    }
    return e;
}

}  // namespace h2
