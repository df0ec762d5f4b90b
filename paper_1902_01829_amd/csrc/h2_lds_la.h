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

template <int CTRL>
__device__ inline double dpp_f64(double x) {   // a DPP move of a double (two 32-bit halves)
    const int64_t b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_update_dpp(0, int(b), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, int(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double((int64_t(hi) << 32) | uint32_t(lo));
}

__device__ inline double quad_sum(double v) {   // over lanes 4 j .. 4 j + 3 (all active), by DPP
    v += dpp_f64<0xB1>(v);   // quad_perm [1, 0, 3, 2]
    return v + dpp_f64<0x4E>(v);   // quad_perm [2, 3, 0, 1]
}

// v(rows of this thread) of the reflector stored in column j of the
// reflector array (zeros above row j and past row M - 1 are stored, so the
// reads need no masks); all LDS reads are issued before any use.
template <int MR, int LDV>
__device__ __forceinline__ void qr_load_v(const double *V, int j, int sub, double (&v)[MR]) {
#pragma unroll
    for (int i = 0; i < MR; ++i) v[i] = V[j * LDV + sub + 4 * i];
    __builtin_amdgcn_sched_barrier(0);
}
// a -= tau (v . a) v over the column's four threads (four partial sums)
template <int MR>
__device__ __forceinline__ void qr_reflect(const double (&v)[MR], double tau, double (&a)[MR]) {
    double p[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int i = 0; i < MR; ++i) p[i & 3] += v[i] * a[i];
    const double w = quad_sum((p[0] + p[1]) + (p[2] + p[3])) * tau;
#pragma unroll
    for (int i = 0; i < MR; ++i) a[i] -= w * v[i];
}

// In-place Householder QR of the M x N matrix A (column-major, ld M + QR_PAD,
// LDS), N <= M <= MAXM, N <= 64, with the whole workgroup (256 threads).  R,
// with its rows' signs flipped so that diag(R) >= 0, goes to T (ld ldt); then
// A is overwritten by the thin Q (M x N) with the matching columns flipped.
//
// Thread t keeps column t / 4 of the matrix in registers, rows (t % 4) + 4 i
// (the four threads of a column are consecutive lanes and combine partial
// sums by DPP), so the only LDS traffic is the reflectors: step c, column
// c's threads form v_c (v_c(c) = 1) and tau_c and store v_c whole (zeros
// above row c and past row M - 1) in the array's space, now laid out with
// leading dimension MAXM + QR_PAD; one barrier; every column to the right
// reads v_c and applies H_c = I - tau_c v_c v_c^T to itself.  Each stored
// column is written once, so one barrier per step suffices.  Q = H_0 ..
// H_(N-1) [I; 0] is then formed column by column in registers from the
// stored reflectors, without barriers (H_j leaves e_c unchanged for c < j).
// The caller's array holds (MAXM + QR_PAD) x 64 doubles or more.  The step
// of column c is serial (one wavefront's four lanes), so it is kept short:
// no masks on rows past M, R(c, c) in a register of its own.
template <int MAXM = QR_MAXM>
__device__ __forceinline__ void householder_qr(double *A, double *tau, double *sgn, int M, int N, double *T, int ldt) {
    static_assert(MAXM % 4 == 0 && MAXM <= QR_MAXM, "rows per thread");
    constexpr int MR = MAXM / 4, LDV = MAXM + QR_PAD;
    const int t = threadIdx.x, col = t >> 2, sub = t & 3, ld = M + QR_PAD;
    const bool mine = col < N;
    double a[MR];
#pragma unroll
    for (int i = 0; i < MR; ++i) {
        const int r = sub + 4 * i;
        a[i] = (mine && r < M) ? A[col * ld + r] : 0.0;   // rows past M stay zero throughout
    }
    __syncthreads();   // A's space holds reflectors (leading dimension LDV) from here on
    double rcc = 0.0;  // R(col, col)
    for (int c = 0; c < N; ++c) {
        if (col == c) {   // the reflector of column c (the four threads of the column)
            // (cu: c as a value the compiler cannot equate with col, or it
            // hoists every row's mask out of the loop and spills them)
            const int cu = __builtin_amdgcn_readfirstlane(c);
            double p[4] = {0.0, 0.0, 0.0, 0.0}, al = 0.0;
#pragma unroll
            for (int i = 0; i < MR; ++i) {
                const int r = sub + 4 * i;
                const double x = r >= cu ? a[i] : 0.0;
                p[i & 3] += x * x;
                al = r == cu ? a[i] : al;
            }
            const double s = quad_sum((p[0] + p[1]) + (p[2] + p[3]));
            const double alpha = quad_sum(al), nrm = sqrt(s);
            double tc = 0.0, beta = alpha, sc = 0.0;
            if (nrm > 0.0) {
                beta = alpha >= 0.0 ? -nrm : nrm;
                tc = (beta - alpha) / beta;
                sc = 1.0 / (alpha - beta);
            }
#pragma unroll
            for (int i = 0; i < MR; ++i) {
                const int r = sub + 4 * i;
                A[cu * LDV + r] = r > cu ? a[i] * sc : (r == cu ? 1.0 : 0.0);
            }
            rcc = beta;
            if (sub == 0) {
                tau[c] = tc;
                sgn[c] = beta < 0.0 ? -1.0 : 1.0;
            }
        }
        __syncthreads();
        if (mine && col > c) {   // H_c applied to this column
            double v[MR];
            qr_load_v<MR, LDV>(A, c, sub, v);
            qr_reflect<MR>(v, tau[c], a);
        }
    }
    // R with diag(R) >= 0: rows above the diagonal of this column (final
    // since their steps) and R(col, col)
    if (mine) {
#pragma unroll
        for (int i = 0; i < MR; ++i) {
            const int r = sub + 4 * i;
            if (r < N) T[int64_t(col) * ldt + r] = r < col ? sgn[r] * a[i] : (r == col ? sgn[col] * rcc : 0.0);
        }
    }
    // column col of Q: H_col .. H_0 applied in reverse order to e_col
    if (mine) {
#pragma unroll
        for (int i = 0; i < MR; ++i) a[i] = sub + 4 * i == col ? 1.0 : 0.0;
        for (int j = col; j >= 0; --j) {
            double v[MR];
            qr_load_v<MR, LDV>(A, j, sub, v);
            qr_reflect<MR>(v, tau[j], a);
        }
    }
    __syncthreads();   // every reflector read
    if (mine) {
        const double sc = sgn[col];
#pragma unroll
        for (int i = 0; i < MR; ++i) {
            const int r = sub + 4 * i;
            if (r < M) A[col * ld + r] = sc * a[i];
        }
    }
    __syncthreads();
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
