/*
 * h2oracle.h -- plain, slow, FP64 CPU oracle for the H^2 matrix-vector product
 * of Boukaram, Turkiyyah and Keyes, "Hierarchical Matrix Operations on GPUs:
 * Matrix-Vector Multiplication and Compression" (arXiv:1902.01829).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this code; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or helper with
 * the HIP library: the two meet only through the seeded inputs (points, x).
 *
 * What it computes (paper section given per function in h2oracle.c):
 *   - construction of an H^2 matrix from points (Sec. 4.6 "ab initio"):
 *     KD-tree bisection, tight boxes, tensor Chebyshev interpolation bases
 *     (leaf bases U = V, transfers E = F, Eq. (1) of Sec. 2.2), a dual
 *     traversal with the admissibility max(diam s, diam t) <= eta*dist(s,t),
 *     coupling blocks S = K at interpolation nodes, dense blocks D = K at the
 *     points, every level stored as a block-sparse-row matrix (Sec. 4.3,
 *     Fig. 5);
 *   - the O(n) product y = A x of Sec. 4 (upsweep Sec. 4.2, tree multiply
 *     Sec. 4.3, downsweep Sec. 4.4, dense part Sec. 4.1), in stored mode
 *     (blocks kept) or matrix-free mode (blocks regenerated when used);
 *   - the explicit dense expansion of the representation, the brute-force
 *     kernel product, and emulation of reduced storage (FP32, or BF16 with a
 *     per-block FP32 scale) as exact dequantized FP64 values.
 *
 * Conventions: 0-based heap numbering of the cluster tree (level l holds nodes
 * [2^l - 1, 2^(l+1) - 1), children of v are 2v+1 and 2v+2); vectors are in
 * tree order (x_tree[i] = x_input[perm[i]]); blocks are column-major.
 * Functions returning int give 0 on success and a negative value on invalid
 * arguments.
 */
#ifndef H2ORACLE_H
#define H2ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct or_h2 or_h2;

enum { OR_KERNEL_EXP = 0, OR_KERNEL_POLY2 = 1 };
enum { OR_STORE_FP64 = 0, OR_STORE_FP32 = 1, OR_STORE_BF16 = 2 };

/* Chebyshev nodes of the first kind on [-1,1]: t_a = cos((2a+1) pi / (2p)). */
void or_cheb_nodes(int p, double *t);
/* 1-D Lagrange polynomial of node a over the nodes t[0..p-1], at s. */
double or_lagrange_1d(int p, const double *t, int a, double s);

/* Kernel entry between two d-dimensional points. */
double or_kernel(int kernel, int d, double ell, const double *a, const double *b);

/* Reduced-storage emulation of one block of len values, in place. */
void or_quantize_block(int storage, int64_t len, double *vals);
/* Round one value to FP32, and one FP32 value to BF16 (round to nearest even). */
double or_round_fp32(double v);
double or_round_bf16(double v);

/* Build from points (n x d, row-major, input order).  keep_blocks != 0 stores
 * every S and D block (stored mode); 0 regenerates them (matrix-free mode). */
int or_build(const double *pts, int64_t n, int d, int m, int p, double eta,
             double ell, int kernel, int storage, int keep_blocks, or_h2 **out);
void or_free(or_h2 *h);

/* sizes[0..8] = n, d, m, p, k, q, lmin, nnodes, total coupling blocks;
 * lmin = q + 1 when there is no coupling block. */
void or_sizes(const or_h2 *h, int64_t *sizes);
void or_perm(const or_h2 *h, int64_t *perm);
void or_ranges(const or_h2 *h, int64_t *begin, int64_t *end);
void or_boxes(const or_h2 *h, double *lo, double *hi);
int64_t or_coupling_count(const or_h2 *h, int level);
void or_coupling_bsr(const or_h2 *h, int level, int32_t *rowptr, int32_t *colidx);
int64_t or_dense_count(const or_h2 *h);
void or_dense_bsr(const or_h2 *h, int32_t *rowptr, int32_t *colidx);
int64_t or_near_ties(const or_h2 *h);
/* Flattened tree of Sec. 3.1 (Fig. 3), 0-based, -1 = empty:
 * levelptr[q+2], parent/head/next[nnodes]. */
void or_flat_tree(const or_h2 *h, int64_t *levelptr, int64_t *parent, int64_t *head,
                  int64_t *next);
/* Block-sparse-row assembly of nb blocks given as (row, col): rowptr[nrows+1],
 * colidx[nb], order[nb] (position of each output block in the input list). */
void or_bsr_assemble(int32_t nrows, int64_t nb, const int32_t *row, const int32_t *col,
                     int32_t *rowptr, int32_t *colidx, int64_t *order);

/* Representation data (all column-major, FP64, after storage emulation). */
void or_leaf_basis(const or_h2 *h, int64_t node, double *U);        /* m_i x k */
void or_transfer(const or_h2 *h, int64_t node, double *E);          /* k x k   */
void or_coupling_block(const or_h2 *h, int level, int64_t idx, double *S);
void or_dense_block(const or_h2 *h, int64_t idx, double *D);
/* Explicit basis of a node (|node| x k): method 0 through the transfers down to
 * the leaves, method 1 by evaluating the node's own Lagrange polynomials. */
void or_explicit_basis(const or_h2 *h, int64_t node, int method, double *Uhat);

/* y = A x in tree order (O(n) sweeps). */
void or_matvec(const or_h2 *h, const double *x, double *y);

/* y = A x for an H^2 matrix given by its arrays, with a rank per level
 * (layout in h2oracle.c).  Returns 0, or -1 on invalid sizes. */
int or_arrays_matvec(int64_t n, int q, const int32_t *lrank, const int64_t *begin, const int64_t *end,
                     const double *U, const double *V, const double *E, const double *F,
                     const int32_t *const *S_rowptr, const int32_t *const *S_colidx,
                     const double *const *S, const int32_t *D_rowptr, const int32_t *D_colidx,
                     const double *D, const double *x, double *y);
/* Rows of y = A x for the listed leaves only: y holds the leaves' rows in the
 * order given (sum of leaf sizes values). */
void or_matvec_leaves(const or_h2 *h, const double *x, int64_t nleaves,
                      const int64_t *leaves, double *y);
/* Intermediate vector trees of the sweep: xh and yh (nnodes x k, zero above
 * lmin), y_near and y_far (n). Any pointer may be NULL. */
void or_matvec_parts(const or_h2 *h, const double *x, double *xh, double *yh,
                     double *y_near, double *y_far);
/* Explicit A_H (n x n, row-major, tree order). */
void or_dense_expand(const or_h2 *h, double *A);
/* Brute-force kernel product for the listed rows: y[r] = sum_j K(P_rows[r], P_j) x_j
 * over points given in any fixed order (x in that order). */
void or_kernel_matvec(const double *pts, int64_t n, int d, double ell, int kernel,
                      const double *x, int64_t nrows, const int64_t *rows, double *y);

#ifdef __cplusplus
}
#endif
#endif
