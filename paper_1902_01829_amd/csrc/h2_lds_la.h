// Small dense FP64 factorizations of one workgroup (256 threads) on matrices
// staged column-major in LDS: the Householder QR of the orthogonalization
// (Sec. 5.1) and the one-sided Jacobi SVD of the truncation (Sec. 5.3).
// Internal to libh2mv; included by its HIP sources only.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace h2 {
namespace lds {

constexpr int QR_MAXM = 128, QR_MAXN = 64;
// Columns of the LDS matrices are QR_PAD doubles longer than their rows: the
// threads of a wavefront read 16 columns at once, and a column stride of a
// multiple of 64 doubles would put them all on the same LDS banks.
constexpr int QR_PAD = 4;

// Element (r, c) of an R-row FP64 block in 16-byte column groups (2 columns).
__device__ inline int64_t at2(int R, int r, int c) { return (int64_t(c >> 1) * R + r) * 2 + (c & 1); }

__device__ inline double sum4(double v) {   // over the 4 threads of a column (consecutive lanes)
    v += __shfl_xor(v, 1);
    v += __shfl_xor(v, 2);
    return v;
}

// In-place Householder QR of the M x N matrix A (column-major, ld M + QR_PAD, LDS),
// M >= N.  R, with its rows' signs flipped so that diag(R) >= 0, goes to T
// (ld ldt); then A is overwritten by the thin Q (M x N) with the matching
// columns flipped.  Q is formed in place from the stored reflectors, the last
// one first (column c of Q is final once reflectors c .. N-1 are applied).
// Four threads share a column: thread t owns column t / 4 and rows
// (t % 4) + 4 i, combining partial dot products with lane shuffles.
__device__ inline void householder_qr(double *A, double *tau, double *scal, double *sgn, int M, int N, double *T,
                                      int ldt) {
    const int t = threadIdx.x, col = t >> 2, sub = t & 3, ld = M + QR_PAD;
    for (int c = 0; c < N; ++c) {
        if (col == c) {   // norm of A[c:M, c] over the column's four threads, then the reflector
            double s = 0.0;
            for (int r = c + sub; r < M; r += 4) s += A[c * ld + r] * A[c * ld + r];
            s = sum4(s);
            if (sub == 0) {
                const double alpha = A[c * ld + c], nrm = sqrt(s);
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
        if (col == c) {   // v below the diagonal (v_c = 1 implicit), beta on it
            for (int r = c + 1 + sub; r < M; r += 4) A[c * ld + r] *= sc;
            if (sub == 0) A[c * ld + c] = scal[1];
        }
        __syncthreads();
        if (col > c && col < N && tc != 0.0) {   // H_c = I - tau v v^T on the columns to the right
            double w = sub == 0 ? A[col * ld + c] : 0.0;
            for (int r = c + 1 + sub; r < M; r += 4) w += A[c * ld + r] * A[col * ld + r];
            w = sum4(w) * tc;
            if (sub == 0) A[col * ld + c] -= w;
            for (int r = c + 1 + sub; r < M; r += 4) A[col * ld + r] -= w * A[c * ld + r];
        }
        __syncthreads();
    }
    for (int i = t; i < N * N; i += blockDim.x) {   // R with diag(R) >= 0
        const int c = i / N, r = i - c * N;
        const double sr = A[r * ld + r] < 0.0 ? -1.0 : 1.0;
        T[int64_t(c) * ldt + r] = r <= c ? sr * A[c * ld + r] : 0.0;
    }
    for (int c = t; c < N; c += blockDim.x) sgn[c] = A[c * ld + c] < 0.0 ? -1.0 : 1.0;
    __syncthreads();
    for (int c = N - 1; c >= 0; --c) {
        const double tc = tau[c];
        if (col > c && col < N) {   // apply H_c to the finished columns (their rows < col are zero)
            double w = sub == 0 ? A[col * ld + c] : 0.0;
            for (int r = c + 1 + sub; r < M; r += 4) w += A[c * ld + r] * A[col * ld + r];
            w = sum4(w) * tc;
            if (sub == 0) A[col * ld + c] -= w;
            for (int r = c + 1 + sub; r < M; r += 4) A[col * ld + r] -= w * A[c * ld + r];
        }
        __syncthreads();
        if (col == c) {   // column c of Q: H_c e_c
            for (int r = c + 1 + sub; r < M; r += 4) A[c * ld + r] *= -tc;
            for (int r = sub; r < c; r += 4) A[c * ld + r] = 0.0;
            if (sub == 0) A[c * ld + c] = 1.0 - tc;
        }
        __syncthreads();
    }
    for (int i = t; i < M * N; i += blockDim.x) {
        const int c = i / M, r = i - c * M;
        A[c * ld + r] *= sgn[c];
    }
    __syncthreads();
}

template <int CTRL>
__device__ inline double dpp_f64(double x) {   // a DPP move of a double (two 32-bit halves)
    const int64_t b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_update_dpp(0, int(b), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, int(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double((int64_t(hi) << 32) | uint32_t(lo));
}

__device__ inline double dpp_sum8(double v) {   // over lanes 8 j .. 8 j + 7 (all active)
    v += dpp_f64<0xB1>(v);    // quad_perm [1,0,3,2]: lane ^ 1
    v += dpp_f64<0x4E>(v);    // quad_perm [2,3,0,1]: lane ^ 2
    v += dpp_f64<0x141>(v);   // row_half_mirror: i <-> 7 - i within 8, the other quad
    return v;
}

__device__ inline double dpp_sum16(double v) {   // over the 16 lanes of a DPP row (all active)
    v = dpp_sum8(v);
    v += dpp_f64<0x140>(v);   // row_mirror: i <-> 15 - i, the other half
    return v;
}

// One-sided (Hestenes) Jacobi SVD.  G is the L x n matrix (column-major,
// leading dimension ldg, LDS) whose columns are the rows of the matrix B to
// decompose (G = B^T); Y (n x n, leading dimension ldy, LDS) starts as the
// identity.  Plane rotations applied to pairs of columns of G and Y make the
// columns of G mutually orthogonal, so that G_0 Y = G and B = Y diag(s) V^T
// with s_j = |column j of G|: the columns of Y are left singular vectors of
// B, orthonormal to rounding also where s_j = 0.  Pairs are visited in the
// round-robin order of the cyclic parallel Jacobi method (n/2 disjoint pairs
// per step, 8 adjacent threads per pair, 8 rows each held in registers, sums
// by DPP); a pair is rotated when |g_p . g_q| exceeds tol |g_p| |g_q| and
// neither column is negligible, i.e. of norm at most 1e-15 |G|_F (rotations
// are norm preserving, so |G|_F is fixed): such columns are rounding noise,
// and turning them changes a column of norm s by at most 1e-15 |G|_F / s in
// direction.  Sweeps stop after one
// without a rotation, or after max_sweeps.  n <= 64, L <= 64.  red is 64
// doubles of LDS scratch.  Returns the number of sweeps done.
__device__ inline int jacobi_svd(double *G, int ldg, int L, double *Y, int ldy, int n, double tol, int max_sweeps,
                                 int *flag, double *red) {
    const int t = threadIdx.x, pr = t >> 3, sub = t & 7;
    const int m = (n + 1) & ~1;   // even number of positions; an odd n pairs one column with nothing each step
    if (t < n) {
        double a = 0.0;
        for (int r = 0; r < L; ++r) a += G[t * ldg + r] * G[t * ldg + r];
        red[t] = a;
    }
    __syncthreads();
    double f2 = 0.0;
    for (int i = 0; i < n; ++i) f2 += red[i];
    const double negligible = 1e-30 * f2;
    int sweeps = 0;
    for (; sweeps < max_sweeps; ++sweeps) {
        if (t == 0) *flag = 0;
        __syncthreads();
        for (int step = 0; step + 1 < m; ++step) {
            if (pr < (m >> 1)) {
                // circle method: position 0 fixed, positions 1 .. m-1 rotate by one each step
                const int a = pr, b = m - 1 - pr;
                int p = a == 0 ? 0 : 1 + (a - 1 + step) % (m - 1);
                int q = 1 + (b - 1 + step) % (m - 1);
                if (p > q) {
                    const int x = p;
                    p = q;
                    q = x;
                }
                if (q < n) {
                    // this thread's rows sub, sub + 8, ... of both columns, all loads issued at once
                    double gp[8], gq[8], al = 0.0, be = 0.0, ga = 0.0;
#pragma unroll
                    for (int i = 0; i < 8; ++i) {
                        const int r = sub + 8 * i;
                        gp[i] = r < L ? G[p * ldg + r] : 0.0;
                        gq[i] = r < L ? G[q * ldg + r] : 0.0;
                    }
#pragma unroll
                    for (int i = 0; i < 8; ++i) {
                        al += gp[i] * gp[i];
                        be += gq[i] * gq[i];
                        ga += gp[i] * gq[i];
                    }
                    al = dpp_sum8(al);
                    be = dpp_sum8(be);
                    ga = dpp_sum8(ga);
                    if (ga != 0.0 && al > negligible && be > negligible && ga * ga > tol * tol * al * be) {
                        const double zeta = (be - al) / (2.0 * ga);
                        const double tt = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                        const double cs = 1.0 / sqrt(1.0 + tt * tt), sn = cs * tt;
                        double yp[8], yq[8];
#pragma unroll
                        for (int i = 0; i < 8; ++i) {
                            const int r = sub + 8 * i;
                            yp[i] = r < n ? Y[p * ldy + r] : 0.0;
                            yq[i] = r < n ? Y[q * ldy + r] : 0.0;
                        }
#pragma unroll
                        for (int i = 0; i < 8; ++i) {
                            const int r = sub + 8 * i;
                            if (r < L) {
                                G[p * ldg + r] = cs * gp[i] - sn * gq[i];
                                G[q * ldg + r] = sn * gp[i] + cs * gq[i];
                            }
                            if (r < n) {
                                Y[p * ldy + r] = cs * yp[i] - sn * yq[i];
                                Y[q * ldy + r] = sn * yp[i] + cs * yq[i];
                            }
                        }
                        if (sub == 0) *flag = 1;
                    }
                }
            }
            __syncthreads();
        }
        const int rotated = *flag;
        __syncthreads();
        if (!rotated) break;
    }
    return sweeps;
}

}  // namespace lds
}  // namespace h2
