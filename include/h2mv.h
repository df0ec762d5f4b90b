/*
 * h2mv.h -- C ABI of an MI355X (gfx950) library for the H^2 hierarchical
 * matrix-vector product of Boukaram, Turkiyyah and Keyes, "Hierarchical Matrix
 * Operations on GPUs: Matrix-Vector Multiplication and Compression"
 * (arXiv:1902.01829).
 *
 * The matrix A ~ K(P, P) is the covariance of n points P under the isotropic
 * exponential kernel K(a, b) = exp(-|a - b| / corr_len) (Sec. 4.6).  It is held
 * as an H^2 matrix (Sec. 2.2): a binary cluster tree, explicit leaf bases U = V
 * and transfer matrices E = F (Eq. (1)), a matrix tree of k x k coupling blocks
 * S stored per level as block-sparse rows (Sec. 4.3, Fig. 5), and dense m x m
 * near-field blocks D at the finest level.  The product y = A x is computed as
 * leaf projection and upsweep (Sec. 4.2), tree multiplication (Sec. 4.3),
 * downsweep and leaf expansion (Sec. 4.4), plus the dense part, all added in
 * FP64 at the end (Sec. 4.1, Sec. 4.5).
 *
 * Conventions
 *  - Ordering.  Vectors are in cluster-tree order: x_tree[i] = x_input[perm[i]],
 *    with perm from h2_get_perm.
 *  - Pointers.  "host" pointers are read or written before the call returns;
 *    "device" pointers are HIP device memory owned by the caller.  Input host
 *    arrays are copied; the handle owns all device memory it allocates (the
 *    representation and its workspace) until h2_free.
 *  - Streams.  Every device operation is enqueued on the given hipStream_t
 *    (NULL = default stream) and is asynchronous.  A handle's workspace is shared
 *    by its calls: do not run two calls on one handle concurrently.
 *  - Graphs.  h2_matvec, and h2_matmat after the first call on a handle (which
 *    times its block loops and synchronizes), only enqueue kernels: they may
 *    be captured into a HIP graph while profiling is off (h2_profile records
 *    events).  A captured product reads x / X and writes y / Y at the
 *    addresses given at capture.
 *  - Errors.  Every call returns an h2_status; no C++ exception crosses the ABI.
 *    On error *out is set to NULL, nothing is leaked, outputs are untouched,
 *    and h2_last_error() describes the failure (thread-local text).
 *  - Limits.  rank k = cheb_p^dim <= 64 and leaf_size <= 64, else
 *    H2_ERR_UNSUPPORTED; n < 2^31.
 */
#ifndef H2MV_H
#define H2MV_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct h2_matrix_ *h2_handle;
typedef struct h2_batch_ *h2_batch;

typedef enum {
    H2_OK = 0,
    H2_ERR_INVALID_ARG = 1,   /* a bad size, pointer, parameter or NaN input          */
    H2_ERR_OOM = 2,           /* device allocation failed (or exceeded a set cap)     */
    H2_ERR_DEVICE = 3,        /* a HIP runtime error; text in h2_last_error()         */
    H2_ERR_UNSUPPORTED = 4,   /* rank or leaf size beyond the compiled limit (64)     */
    H2_ERR_INTERNAL = 5       /* any other failure                                    */
} h2_status;

/* Storage of the coupling blocks S and dense blocks D (an extension of the
 * paper, which stores all blocks in the working precision).  H2_FP64: all in
 * FP64, FP64 arithmetic.  H2_FP32: S, D and the bases in FP32, FP32 products.
 * H2_BF16_SCALED: S and D in BF16 with one FP32 scale per block (the block's
 * max-abs), bases in FP32, FP32 products.  In the reduced modes, partial sums
 * of one block are FP32, sums over blocks are FP64, and the near and far
 * fields are added in FP64. */
typedef enum { H2_FP64 = 0, H2_FP32 = 1, H2_BF16_SCALED = 2 } h2_storage;

/* Storage modifier, OR-ed into an h2_storage value: blocks stored by halves
 * (a use of the format that the symmetric case allows, Sec. 2.2: S_ji =
 * S_ij^T and D_ji = D_ij^T with V = U and F = E).  Only the coupling and dense
 * blocks with column >= row are held (diagonal dense blocks in full), which
 * about halves the bytes a product streams; the product reads each stored
 * block once for both S_ij x_j and S_ij^T x_i, and adds the transposed
 * contributions of every segment (partial slots of 64 FP64 values, or FP32 in
 * the reduced modes, one per column segment and group of up to 4 consecutive
 * block rows, summed in FP64; partial_slots in h2_info counts them) in a
 * second launch.  Products match the full storage up
 * to rounding order.  h2_get_info reports the modifier in storage and the
 * stored bytes in bytes_coupling and bytes_dense.  Handles stored by halves
 * are rejected with UNSUPPORTED by h2_orthogonalize, h2_compress,
 * h2_transpose (such a matrix is its own transpose) and h2_batch_create;
 * h2_matmat runs one single-vector product per column. */
#define H2_HALF_STORAGE 16

/* flags */
#define H2_FLAG_STRUCTURE_ONLY 1u   /* build the host-side structure only: no device
                                       memory, matvec/matmat then return INVALID_ARG */

/* Construction parameters (Sec. 4.6): dim in {2,3}; leaf_size m >= 2 (the tree
 * is bisected until every leaf holds at most m points); cheb_p >= 1 Chebyshev
 * points per axis (rank k = cheb_p^dim); eta > 0, a pair of clusters (s, t) is
 * admissible when max(diam s, diam t) <= eta * dist(s, t) over their tight
 * boxes; corr_len > 0. */
typedef struct {
    int dim;
    int leaf_size;
    int cheb_p;
    double eta;
    double corr_len;
    int storage;          /* h2_storage */
    unsigned flags;
} h2_params;

/* Sizes of a built matrix.  bytes_* are the bytes one product streams from
 * HBM for that part of the representation (for bandwidth figures). */
typedef struct {
    int64_t n;
    int dim, leaf_size, cheb_p, rank, levels_q, lmin, storage;
    int64_t nnodes;            /* 2^(q+1) - 1                                      */
    int64_t coupling_blocks;   /* all levels                                       */
    int64_t dense_blocks;
    int64_t bytes_coupling, bytes_dense, bytes_leaf_bases, bytes_transfers;
    int64_t bytes_device_total; /* all device memory held by the handle           */
    int64_t near_ties;         /* admissibility tests within 1e-12 of equality     */
    int64_t partial_slots;     /* stored by halves: partial slots of 64 values the
                                  product writes and reads once (else 0)           */
} h2_info;

/* Build an H^2 matrix from points (Sec. 4.6).
 *  points  host, n x dim, row-major, input order; finite values.
 *  n       1 <= n < 2^31.
 *  prm     host; see h2_params.
 *  stream  hipStream_t for the uploads and the fill kernels.
 *  out     host; receives the handle (NULL on error).
 * The call returns after the device representation is complete.
 * Errors: INVALID_ARG for n < 1, dim not in {2,3}, leaf_size < 2, cheb_p < 1,
 * eta <= 0 or NaN, corr_len <= 0 or NaN, storage out of range (an h2_storage,
 * optionally | H2_HALF_STORAGE), non-finite coordinates or NULL pointers, and
 * with H2_HALF_STORAGE a block pattern that is not symmetric; UNSUPPORTED for
 * rank or leaf_size > 64; OOM; DEVICE. */
h2_status h2_build_from_points(const double *points, int64_t n, const h2_params *prm,
                               void *stream, h2_handle *out);

/* An H^2 matrix given by its arrays (Sec. 2.2; the flattened per-level
 * storage of Sec. 3 and Fig. 3; the matrix tree as per-level block-sparse
 * rows, Fig. 5), 0-based, all host memory, read during the call only.
 *  n           rows (= columns) of A, 1 <= n < 2^31; vectors are in the tree
 *              order these arrays define (h2_get_perm then gives the identity).
 *  q           leaf level, 0 <= q <= 29.  Nodes 0 .. 2^(q+1)-2 in heap order:
 *              level l holds nodes 2^l-1 .. 2^(l+1)-2, children of v are
 *              2v+1 and 2v+2.
 *  level_rank  q+1 ranks k_0 .. k_q of the levels' bases, 1 <= k_l <= 64.
 *  node_begin, node_end  2^(q+1)-1 values each: node v holds rows
 *              [begin, end); the root holds [0, n), children split their
 *              parent into two non-empty consecutive ranges, leaves hold at
 *              most 64 rows.
 *  U, V        leaf bases: leaf j (node 2^q-1+j) has U_j and V_j, m_j x k_q
 *              column-major, concatenated in leaf order (V may equal U).
 *  E, F        transfers (Eq. (1)): every node c >= 1 of level l has E_c and
 *              F_c, k_l x k_(l-1) column-major, concatenated in node order
 *              (F may equal E); U_parent = [U_c1 E_c1; U_c2 E_c2].  May be NULL
 *              when q = 0.
 *  S_rowptr, S_colidx, S   q+1 pointers each: for level l, 2^l+1 row offsets,
 *              the level-local column node of every block, and the k_l x k_l
 *              column-major coupling blocks S_ij in that order (a level
 *              without blocks may have NULL colidx and S).
 *  D_rowptr, D_colidx, D   dense blocks over the leaves: 2^q+1 row offsets,
 *              leaf-local columns, m_i x m_j column-major blocks in that order.
 * A = sum of D_ij over dense blocks + sum over levels and coupling blocks of
 * U^l_i S_ij (V^l_j)^T, with the nested bases of Eq. (1).  U and V may be
 * NULL when no level has a coupling block.  Values are not checked (NaN in,
 * NaN out); the partition of A into blocks is the caller's (a pair listed
 * twice is added twice). */
typedef struct {
    int64_t n;
    int q;
    const int32_t *level_rank;
    const int64_t *node_begin, *node_end;
    const double *U, *V, *E, *F;
    const int32_t *const *S_rowptr;
    const int32_t *const *S_colidx;
    const double *const *S;
    const int32_t *D_rowptr, *D_colidx;
    const double *D;
} h2_arrays;

/* Build a handle from arrays (values converted to the storage's layout and
 * element type on the host and uploaded in pieces of at most 64 MiB).
 *  storage  h2_storage, optionally | H2_HALF_STORAGE; H2_FP32 /
 *           H2_BF16_SCALED round as described above.  With H2_HALF_STORAGE the
 *           arrays must be symmetric bit for bit: V = U, F = E, every pair
 *           (i, j) listed once per BSR list, its mirror (j, i) listed too, and
 *           S_ji = S_ij^T, D_ji = D_ij^T (INVALID_ARG otherwise); the export
 *           gives the full arrays back.
 *  stream   stream of the uploads; the call returns when they are done.
 * h2_get_info reports dim 0, cheb_p 0, leaf_size = the largest leaf and rank
 * = the largest level rank.  Errors: INVALID_ARG for NULL required pointers,
 * inconsistent node ranges, BSR offsets that are not non-decreasing from 0,
 * or block columns out of range; UNSUPPORTED for ranks or leaves above 64 or
 * q > 29; OOM; DEVICE. */
h2_status h2_build_from_arrays(const h2_arrays *arrays, int storage, void *stream, h2_handle *out);

/* The representation of A read back, in the layout h2_build_from_arrays
 * takes (host buffers owned by the caller, column-major FP64 values; reduced storage is
 * returned as stored: FP32 values, or BF16 code x block scale in FP32).  Any
 * pointer may be NULL to skip that array, so a first call with level_rank,
 * node_begin and node_end only gives the sizes: U and V hold sum_j m_j k_q
 * values, E and F sum over levels l >= 1 of 2^l k_l k_(l-1), S[l] 2^l + 1
 * offsets' last value times k_l^2, D the sum of m_i m_j over dense blocks.
 * Transfers at or above the first level with a coupling block are not used
 * by the product, not stored, and read back as zero.  For a matrix with no
 * coupling block, U and V read back as zero.  Errors: INVALID_ARG for NULL
 * A / out, or values asked of a structure-only handle; DEVICE. */
typedef struct {
    int32_t *level_rank;
    int64_t *node_begin, *node_end;
    double *U, *V, *E, *F;
    int32_t *const *S_rowptr;
    int32_t *const *S_colidx;
    double *const *S;
    int32_t *D_rowptr, *D_colidx;
    double *D;
} h2_arrays_out;
h2_status h2_export_arrays(h2_handle A, const h2_arrays_out *out, void *stream);

/* Basis orthogonalization (Sec. 5.1, Alg. 6) and projection of the coupling
 * blocks (Alg. 7), in place: every leaf basis becomes Q_j of U_j = Q_j T_j
 * (thin QR), every transfer pair below the first level with a coupling block
 * becomes the two blocks of Q in [T_c1 E_c1; T_c2 E_c2] = Q T_parent, and
 * every coupling block S_ij becomes T_i S_ij T'_j^T, where T' comes from the
 * same steps on the column tree (V, F) when it differs from the row tree
 * (T' = T when V = U and F = E).  The diagonals of the T
 * factors are made non-negative.  A (the product) is unchanged up to
 * rounding; the nested bases of all nodes used by coupling blocks become
 * orthonormal.  The call returns when the device work is done; a matrix
 * without coupling blocks is left as it is.
 * Errors: INVALID_ARG for NULL or structure-only handles; UNSUPPORTED for
 * storage other than H2_FP64, blocks stored by halves, a leaf with fewer rows
 * than the leaf rank, or k_(l-1) > 2 k_l; DEVICE. */
h2_status h2_orthogonalize(h2_handle A, void *stream);

/* The transposed matrix A^T as a new handle (Sec. 2.2: A^T = sum over levels of
 * V S^T U^T plus D^T): the same tree, ranks and permutation; the row and
 * column trees exchange roles (U' = V, V' = U, E' = F, F' = E); block (i, j)
 * of every level's block-sparse rows and of the dense part becomes block
 * (j, i) with the transposed value.  Built on the device from A's stored
 * values (no rounding: BF16 codes and scales are copied), with A's storage;
 * A is unchanged and the two handles are independent (each is freed with
 * h2_free).  For the symmetric matrices of h2_build_from_points, A^T = A.
 *  out  receives the new handle (NULL on error).
 * Errors: INVALID_ARG for NULL arguments or a structure-only handle;
 * UNSUPPORTED for blocks stored by halves; OOM; DEVICE. */
h2_status h2_transpose(h2_handle A, void *stream, h2_handle *out);

/* Algebraic compression (Sec. 5), in place: orthogonalization as
 * h2_orthogonalize; basis generation (Sec. 5.2): for every node i of the
 * levels with coupling blocks, top-down, R_i = the triangular factor of the
 * QR factorization of [R_parent E_i^T; S_ij1^T; ...; S_ijb^T] (its block
 * row's coupling blocks under its parent's factor; when some block has
 * S_ji != S_ij^T bit for bit, the blocks S_ji of block column i are stacked
 * too, as the one basis tree serves both); truncation (Sec. 5.3),
 * bottom-up: the left singular vectors of W_i = U_i R_i^T at the leaves and
 * of W_p = [T_c1 E_c1; T_c2 E_c2] R_p^T above, a node keeping those whose
 * singular value is at least eps times its largest, a level the largest such
 * count over its nodes (at least 1, at most its rank); the kept vectors give
 * the new leaf bases and transfers and T_i = Q_i^T (old basis); then every
 * coupling block S_ij becomes T_i S_ij T'_j^T.  A matrix whose column tree
 * differs from its row tree (V != U or F != E) runs basis generation and
 * truncation per tree (the column tree's R from the blocks S_ij of each block
 * column under R'_parent F^T), a level's rank being the largest count over
 * both trees, and T' from the column tree.  Dense blocks are unchanged.
 * The representation is rebuilt with the new per-level ranks (levels above
 * the first with coupling blocks take that level's rank) and the old one is
 * freed; products after the call use the new one.
 *  eps         relative threshold, finite, >= 0 (0 keeps every rank).
 *  level_rank  NULL, or host, q + 1 ints: the new rank of every level.
 * The call returns when the device work is done; its scratch memory (about
 * 3 nnodes k^2 + 2^q (64^2 + 128 x 64) doubles) is freed on return.
 * Errors: INVALID_ARG for NULL or structure-only handles, eps < 0 or not
 * finite, or a matrix that belongs to a live batch (free the batch first);
 * the UNSUPPORTED cases of h2_orthogonalize; OOM; DEVICE. */
h2_status h2_compress(h2_handle A, double eps, int *level_rank, void *stream);

/* y = A x (Sec. 4, Fig. 4).
 *  x  device, n doubles, tree order.   y  device, n doubles, tree order.
 * x and y must not overlap.  Errors: INVALID_ARG for NULL pointers or a
 * structure-only handle; DEVICE. */
h2_status h2_matvec(h2_handle A, const double *x, double *y, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): y = A x as
 * h2_matvec computes it (same kernels, same order, bitwise the same result),
 * with the product's intermediate vectors -- x^ and y^ (nnodes x rank each),
 * the near field (n) and, for small or half-stored matrices, the partial sums
 * of the stream phase -- in a static device array of H2_NOALLOC_SCRATCH_BYTES
 * per GPU instead of the handle's workspace.  The call allocates nothing,
 * records no profiling events and never synchronizes.  The array belongs to
 * the library, one copy on every GPU the process uses, held until the
 * process ends; all calls on one GPU share it, so two calls that overlap on
 * one GPU (on different streams or host threads) race.  The current device
 * must be the one A was built on.  Errors: INVALID_ARG as h2_matvec;
 * UNSUPPORTED when the product needs more scratch than the array holds (the
 * message gives both sizes: FP64 matrices need 16 bytes per node and rank
 * unit plus 8 per point, e.g. 42 MB for 2^20 points of rank 64); DEVICE. */
#define H2_NOALLOC_SCRATCH_BYTES (64ll << 20)
h2_status h2_matvec_noalloc(h2_handle A, const double *x, double *y, void *stream);

/* Schedule of the single-vector products (h2_matvec, h2_matvec_noalloc, and
 * h2_matmat on FP64 handles) of a handle with full storage.
 *  H2_SCHEDULE_MERGED (default): after the upsweep, one launch multiplies the
 *    coupling blocks of every level and the dense near-field blocks.
 *  H2_SCHEDULE_STREAMED: the near field y_near = D x, which does not need
 *    x^, runs on a second stream owned by the handle, concurrently with the
 *    upsweep, the coupling launch and the downsweep; the leaf phase waits for
 *    it (the overlap of the dense and low-rank parts of Sec. 4.5).  Its rows
 *    (longest first) are cut where their block count reaches the share
 *    near_early of the near field's blocks: the first part starts with the
 *    product, the rest when the coupling launch has finished (so that it
 *    overlaps the downsweep).  near_wg_per_cu = 0 lets the near-field launch
 *    fill the machine; c > 0 makes it request enough LDS that at most c of
 *    its workgroups share a compute unit, so the other stream's launches
 *    always find room (the paper gives the low-rank stream a higher priority
 *    instead; stream priorities are not used here).
 * The result is bitwise the same under both schedules (same rows, same
 * summation order).  The product's phase events (h2_profile) are recorded on
 * the caller's stream: under the streamed schedule the stream phase covers
 * the coupling rows and the leaf phase includes the wait for the near field.
 * A product under the streamed schedule may be captured into a HIP graph: the
 * second stream joins the capture through events.  Errors: INVALID_ARG for a
 * NULL or structure-only handle, an unknown schedule, near_wg_per_cu < 0, or
 * near_early outside [0, 1]; UNSUPPORTED for H2_SCHEDULE_STREAMED on blocks
 * stored by halves, or a cap the device's LDS sizes cannot express (the
 * message gives them; 2 and 3 work on gfx950); DEVICE. */
#define H2_SCHEDULE_MERGED 0
#define H2_SCHEDULE_STREAMED 1
h2_status h2_set_schedule(h2_handle A, int schedule, int near_wg_per_cu, double near_early);

/* Y = A X for nrhs right-hand sides at once: the same phases with every
 * per-node vector replaced by a k x nrhs tile, so each block product becomes a
 * dense contraction.
 *  X  device, column-major n x nrhs, leading dimension ldx >= n, tree order.
 *  Y  device, column-major n x nrhs, leading dimension ldy >= n.
 * H2_FP64 handles, and handles stored by halves, run nrhs single-vector
 * products; other H2_FP32 and H2_BF16_SCALED handles
 * run on the matrix cores (FP32 MFMA), 32 right-hand sides per pass.  The first
 * such call on a handle times the candidate launch shapes (the block loop's
 * prefetch depth 0..7 as listed at h2_batch_tuning, one workgroup per item
 * group or a persistent grid of 1 or 2 workgroups per compute unit, and the
 * MFMA tile width 16 or 32 for passes of at most 16 right-hand sides) on its
 * first pass and keeps the
 * fastest (cached like a batch's choice, below; h2_matmat_tuning reports it).
 * Errors: INVALID_ARG for nrhs < 1, ldx < n, ldy < n, NULL pointers or a
 * structure-only handle; DEVICE. */
h2_status h2_matmat(h2_handle A, const double *X, int64_t ldx, double *Y, int64_t ldy,
                    int nrhs, void *stream);

/* Launch shape h2_matmat chose on A for passes of more than 16 right-hand
 * sides (narrow = 0) or of at most 16 (narrow = 1): pipelined, grid and
 * tile_width as for batches (h2_batch_tuning), and the timed pass in ms (-1
 * before the first such pass; 0 when the choice came from the cache). */
h2_status h2_matmat_tuning(h2_handle A, int narrow, int *pipelined, int64_t *grid, int *tile_width,
                           double *tuned_ms);
/* Fixes that shape instead of timing the candidates (pipelined 0..7, 4 and 5
 * with tile_width 32 only, 6 and 7 with tile_width 16 only; grid >= 0; tile_width 32, or 16 for narrow passes).  Every shape gives the same
 * products to rounding.  Errors: INVALID_ARG. */
h2_status h2_matmat_set_tuning(h2_handle A, int narrow, int pipelined, int64_t grid, int tile_width);

/* Release every device and host resource of A.  NULL is a no-op.  The caller
 * must make sure no enqueued work on A is still running. */
void h2_free(h2_handle A);

/* Sizes and byte counts of A (host struct). */
h2_status h2_get_info(h2_handle A, h2_info *info);

/* perm: host, n int64 (tree position -> input index). */
h2_status h2_get_perm(h2_handle A, int64_t *perm);

/* Block-sparse-row structure of one level of the matrix tree (Sec. 4.3,
 * Fig. 5), 0-based: rowptr host (2^level + 1 values), colidx host (count
 * values); level = -1 gives the dense near-field blocks (rows = leaves).
 * count (host) receives the number of blocks; rowptr/colidx may be NULL to
 * query the count only. */
h2_status h2_get_level_bsr(h2_handle A, int level, int64_t *count, int32_t *rowptr,
                           int32_t *colidx);

/* Per-phase device times of the products on A, measured with HIP events on
 * the call's stream while enabled (enable != 0 starts recording and clears the
 * totals).  ms: host, 8 doubles: leaf projection + upsweep, coupling and dense
 * streaming, downsweep, leaf expansion and sum, whole call; then calls: host
 * int64 number of calls recorded.  Reading the totals synchronizes the device. */
h2_status h2_profile(h2_handle A, int enable);
h2_status h2_profile_read(h2_handle A, double *ms, int64_t *calls);

/* ---- Batches: many independent H^2 matrices per launch.
 * The paper fixes one rank per level because its batched kernels need equal
 * sizes, and names variable-size batches as future work (Sec. 3); here the
 * members' per-level work lists are concatenated, so matrices of different n,
 * rank and leaf size run together, one launch per level slot (upsweep slots
 * aligned at the leaves, downsweep slots aligned at the leaves, one streaming
 * and one leaf slot), the whole sequence captured once in a HIP graph and
 * replayed.  The launch configuration (the block loop's prefetch depth, the
 * persistent grid size and the MFMA tile width) is chosen by timing the
 * candidates at the first product; the choice is cached per process and, when
 * the environment variable H2MV_AUTOTUNE_CACHE names a file, in that file.
 *
 * h2_batch_create
 *  mats    host, count handles, all built with the same storage, H2_FP32 or
 *          H2_BF16_SCALED (H2_FP64 or blocks stored by halves give
 *          UNSUPPORTED); the handles must outlive
 *          the batch and must not be used by other calls while a batch product
 *          runs (the batch reads their representation).
 *  nrhs    1 <= nrhs <= 32 right-hand sides per member (UNSUPPORTED above).
 *  stream  stream for the set-up copies; the call returns when they are done.
 *  out     host; receives the batch (NULL on error).
 * The batch owns its tile workspace, a private stream and the graph.
 *
 * h2_batch_matmat: Y_b = A_b X_b for every member b.
 *  X, Y    host arrays of count device pointers: member b's column-major
 *          n_b x nrhs matrices (tree order), leading dimensions ldx[b], ldy[b]
 *          (host arrays, >= n_b).
 *  stream  the product is ordered after prior work on stream, and later work
 *          on stream is ordered after it (it runs on the batch's stream).
 * The first call also times the candidate configurations (runs the product
 * several times).  Errors: INVALID_ARG for NULL pointers or ld < n; DEVICE. */
h2_status h2_batch_create(const h2_handle *mats, int count, int nrhs, void *stream, h2_batch *out);
h2_status h2_batch_matmat(h2_batch B, const double *const *X, const int64_t *ldx, double *const *Y,
                          const int64_t *ldy, void *stream);
/* Chosen configuration: pipelined (the block loop's prefetch depth: 0 none,
 * 1 the next block, 2 or 3 a ring of that many blocks refilled chunk by
 * chunk; with 32-wide tiles also 4 or 5, a ring of 1 or 2 blocks with the
 * two 32-row halves of a row in one workgroup sharing each input tile
 * through LDS; with 16-wide tiles also 6 or 7, a ring of 6 or 8 column
 * chunks of 16 (FP32) or 32 (BF16) block columns, so that rows of narrow
 * blocks keep more blocks in flight), grid
 * (workgroups; 0 = one per item group), tile_width (16: 16x16
 * MFMAs; 32: 32x32 MFMAs) and the tuned time in ms of one product (-1 before
 * the first product; 0 when the choice came from the cache or
 * h2_batch_set_tuning). */
h2_status h2_batch_tuning(h2_batch B, int *pipelined, int64_t *grid, int *tile_width, double *tuned_ms);
/* Fixes the configuration instead of timing the candidates: pipelined 0..7
 * (4 and 5 with tile_width 32 only, 6 and 7 with tile_width 16 only), grid >= 0, tile_width 16 (at most 16
 * right-hand sides) or 32; every choice
 * gives the members' products to rounding (the tile width changes the order
 * of a block's FP32 sums).  Waits for the batch's running products and drops
 * its captured graph (the next product captures again).  Errors:
 * INVALID_ARG; DEVICE. */
h2_status h2_batch_set_tuning(h2_batch B, int pipelined, int64_t grid, int tile_width);
void h2_batch_free(h2_batch B);   /* NULL is a no-op; wait for running products first */

/* Measurement aid: a plain streaming read of bytes (a positive multiple of
 * 16) at buf (device) by grid (1 .. 65536) workgroups of 256 threads, with
 * the 16-byte non-temporal loads of the product kernels (each wavefront load
 * one contiguous kilobyte); the measured rate is the HBM read ceiling the
 * products are compared with.  sink: device, grid 8-byte values written (an
 * XOR of the data, so the loads cannot be dropped).  Asynchronous on stream.
 * Errors: INVALID_ARG; DEVICE. */
h2_status h2_read_probe(const void *buf, int64_t bytes, int grid, void *sink, void *stream);

/* Text of the last failure on this thread ("" if none). */
const char *h2_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
