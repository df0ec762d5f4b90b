/*
 * h2oracle.c -- FP64 CPU oracle for the H^2 matrix-vector product
 * (Boukaram, Turkiyyah, Keyes, arXiv:1902.01829).  TEST INFRASTRUCTURE ONLY:
 * only tests, the smoke check and the benchmark's CPU baseline call it.
 *
 * Written for a reader holding the paper: plain loops, no blocking, no fusion.
 * Each function names the passage it follows.  Readings taken where the paper
 * is silent (split rule, boxes, admissibility, node kind, kernel scale,
 * reduced-storage rounding) are stated where they are used.
 */
#include "h2oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

struct or_h2 {
    int64_t n;
    int d, m, p, k, q, lmin;
    double eta, ell;
    int kernel, storage, keep;
    int64_t nnodes;
    double *pts;        /* n x d, tree order */
    int64_t *perm;      /* tree position -> input index */
    int64_t *begin, *end;
    double *lo, *hi;    /* widened tight boxes, nnodes x d */
    double *cheb;       /* p 1-D nodes */
    double *U;          /* leaf bases, concatenated m_i x k column-major blocks */
    int64_t *U_off;     /* per leaf (local leaf index) */
    double *E;          /* transfers, nnodes x (k x k); root entry unused */
    /* coupling matrix tree: per level BSR (rows = nodes of the level) */
    int32_t **S_rowptr, **S_colidx;
    int64_t *S_count;
    double **S;         /* stored mode: S_count[l] blocks of k x k */
    /* dense near field: BSR over the leaves */
    int32_t *D_rowptr, *D_colidx;
    int64_t D_count;
    int64_t *D_off;     /* offset of each dense block in D (stored mode) */
    double *D;
    int64_t near_ties;
};

static int level_of(int64_t v) {
    int l = 0;
    while (((int64_t)2 << l) - 1 <= v) l++;
    return l;
}
static int64_t first_of(int l) { return ((int64_t)1 << l) - 1; }

/* ---- Chebyshev interpolation (Sec. 4.6: "Chebyshev interpolation", rank
 * p^d from 8x8 and 4x4x4 grids).  Reading: first-kind nodes; tensor index
 * nu = a_0 + p*a_1 + p^2*a_2 (axis 0 fastest). */
void or_cheb_nodes(int p, double *t) {
    for (int a = 0; a < p; a++) t[a] = cos((2.0 * a + 1.0) * M_PI / (2.0 * p));
}

double or_lagrange_1d(int p, const double *t, int a, double s) {
    double v = 1.0;
    for (int b = 0; b < p; b++)
        if (b != a) v *= (s - t[b]) / (t[a] - t[b]);
    return v;
}

/* Interpolation node nu of a node's box: xi = c + h * (t_a0, t_a1, ...). */
static void cheb_point(const or_h2 *h, int64_t v, int nu, double *xi) {
    for (int ax = 0; ax < h->d; ax++) {
        int a = nu % h->p;
        nu /= h->p;
        double c = 0.5 * (h->lo[v * h->d + ax] + h->hi[v * h->d + ax]);
        double hw = 0.5 * (h->hi[v * h->d + ax] - h->lo[v * h->d + ax]);
        xi[ax] = c + hw * h->cheb[a];
    }
}

/* Lagrange polynomial nu of node v's box at the point x (product over axes
 * of 1-D Lagrange polynomials in the box-local coordinate). */
static double lagrange(const or_h2 *h, int64_t v, int nu, const double *x) {
    double val = 1.0;
    for (int ax = 0; ax < h->d; ax++) {
        int a = nu % h->p;
        nu /= h->p;
        double c = 0.5 * (h->lo[v * h->d + ax] + h->hi[v * h->d + ax]);
        double hw = 0.5 * (h->hi[v * h->d + ax] - h->lo[v * h->d + ax]);
        val *= or_lagrange_1d(h->p, h->cheb, a, (x[ax] - c) / hw);
    }
    return val;
}

/* ---- Kernel (Sec. 4.6: isotropic exponential covariance with correlation
 * length ell).  Reading: unit variance, no nugget: K = exp(-|a-b|/ell).
 * OR_KERNEL_POLY2 = (1 + a.b)^2 is a test-only kernel that tensor Chebyshev
 * interpolation with p >= 3 reproduces exactly. */
double or_kernel(int kernel, int d, double ell, const double *a, const double *b) {
    if (kernel == OR_KERNEL_POLY2) {
        double dot = 0.0;
        for (int i = 0; i < d; i++) dot += a[i] * b[i];
        return (1.0 + dot) * (1.0 + dot);
    }
    double r2 = 0.0;
    for (int i = 0; i < d; i++) r2 += (a[i] - b[i]) * (a[i] - b[i]);
    return exp(-sqrt(r2) / ell);
}

/* ---- Reduced storage emulation (an extension, not in the paper).
 * FP32: round to nearest even.  BF16: per-block scale s = max |fp32(a)|
 * (an FP32 value), code = bf16_rne(fp32(a) / s) with the quotient rounded to
 * FP32 first, value = fp32(float(code) * s). */
double or_round_fp32(double v) { return (double)(float)v; }

double or_round_bf16(double v) {
    float f = (float)v;
    uint32_t u;
    memcpy(&u, &f, 4);
    uint32_t lsb = (u >> 16) & 1u;
    u = (u + 0x7fffu + lsb) & 0xffff0000u;
    memcpy(&f, &u, 4);
    return (double)f;
}

void or_quantize_block(int storage, int64_t len, double *vals) {
    if (storage == OR_STORE_FP32) {
        for (int64_t i = 0; i < len; i++) vals[i] = or_round_fp32(vals[i]);
    } else if (storage == OR_STORE_BF16) {
        float s = 0.0f;
        for (int64_t i = 0; i < len; i++) {
            float a = fabsf((float)vals[i]);
            if (a > s) s = a;
        }
        for (int64_t i = 0; i < len; i++) {
            if (s == 0.0f) { vals[i] = 0.0; continue; }
            float qf = (float)vals[i] / s;
            float code = (float)or_round_bf16((double)qf);
            float deq = code * s;
            vals[i] = (double)deq;
        }
    }
}

/* ---- Cluster tree (Sec. 2.2: binary basis tree; Sec. 4.6: KD-tree; Alg. 2
 * and 4 imply a complete tree with n/m leaves).  Reading: q is the smallest
 * level with n <= m 2^q; every node above q is split at the median of the
 * widest axis of its tight box (ties: lowest axis); its points are sorted by
 * (coordinate on that axis, input index) and the left child gets the first
 * floor(c/2). */
typedef struct { double key; int64_t idx; } sort_item;

static int cmp_item(const void *a, const void *b) {
    const sort_item *x = a, *y = b;
    if (x->key < y->key) return -1;
    if (x->key > y->key) return 1;
    return (x->idx > y->idx) - (x->idx < y->idx);
}

static void tight_box(const double *in_pts, int d, const int64_t *perm, int64_t b,
                      int64_t e, double *lo, double *hi) {
    for (int ax = 0; ax < d; ax++) { lo[ax] = INFINITY; hi[ax] = -INFINITY; }
    for (int64_t i = b; i < e; i++)
        for (int ax = 0; ax < d; ax++) {
            double c = in_pts[perm[i] * d + ax];
            if (c < lo[ax]) lo[ax] = c;
            if (c > hi[ax]) hi[ax] = c;
        }
}

static void build_tree(or_h2 *h, const double *in_pts) {
    int d = h->d;
    for (int64_t i = 0; i < h->n; i++) h->perm[i] = i;
    h->begin[0] = 0;
    h->end[0] = h->n;
    for (int l = 0; l < h->q; l++) {
        int64_t f = first_of(l), cnt = (int64_t)1 << l;
#pragma omp parallel for schedule(dynamic, 1)
        for (int64_t j = 0; j < cnt; j++) {
            int64_t v = f + j, b = h->begin[v], e = h->end[v], c = e - b;
            double lo[3], hi[3];
            tight_box(in_pts, d, h->perm, b, e, lo, hi);
            int axis = 0;
            for (int ax = 1; ax < d; ax++)
                if (hi[ax] - lo[ax] > hi[axis] - lo[axis]) axis = ax;
            sort_item *it = malloc((size_t)(c > 0 ? c : 1) * sizeof(sort_item));
            for (int64_t i = 0; i < c; i++) {
                it[i].idx = h->perm[b + i];
                it[i].key = in_pts[it[i].idx * d + axis];
            }
            qsort(it, (size_t)c, sizeof(sort_item), cmp_item);
            for (int64_t i = 0; i < c; i++) h->perm[b + i] = it[i].idx;
            free(it);
            h->begin[2 * v + 1] = b;
            h->end[2 * v + 1] = b + c / 2;
            h->begin[2 * v + 2] = b + c / 2;
            h->end[2 * v + 2] = e;
        }
    }
    for (int64_t i = 0; i < h->n; i++)
        for (int ax = 0; ax < d; ax++) h->pts[i * d + ax] = in_pts[h->perm[i] * d + ax];
}

/* Boxes.  Reading: the tight axis-aligned box of the node's points; an axis of
 * zero extent is widened symmetrically to delta = 1e-12 * max(1, widest root
 * extent), so that every box has a positive half-width on every axis. */
static void build_boxes(or_h2 *h) {
    int d = h->d;
    for (int64_t v = 0; v < h->nnodes; v++) {
        for (int ax = 0; ax < d; ax++) { h->lo[v * d + ax] = INFINITY; h->hi[v * d + ax] = -INFINITY; }
        for (int64_t i = h->begin[v]; i < h->end[v]; i++)
            for (int ax = 0; ax < d; ax++) {
                double c = h->pts[i * d + ax];
                if (c < h->lo[v * d + ax]) h->lo[v * d + ax] = c;
                if (c > h->hi[v * d + ax]) h->hi[v * d + ax] = c;
            }
    }
    double ext = 0.0;
    for (int ax = 0; ax < d; ax++)
        if (h->hi[ax] - h->lo[ax] > ext) ext = h->hi[ax] - h->lo[ax];
    double delta = 1e-12 * (ext > 1.0 ? ext : 1.0);
    for (int64_t v = 0; v < h->nnodes; v++)
        for (int ax = 0; ax < d; ax++)
            if (h->hi[v * d + ax] - h->lo[v * d + ax] == 0.0) {
                h->lo[v * d + ax] -= 0.5 * delta;
                h->hi[v * d + ax] += 0.5 * delta;
            }
}

/* ---- Leaf bases and transfers (Sec. 2.2, Eq. (1); Sec. 4.6).
 * U_i[r, nu] = L^(i)_nu(point r of leaf i); V = U (same row/column tree, the
 * symmetric case of Sec. 2.2).  E_c[mu, nu] = L^(parent c)_nu(xi^(c)_mu), a
 * k_c x k_p block, so that U_parent = [U_c1 E_c1; U_c2 E_c2]; F = E. */
static void build_bases(or_h2 *h) {
    int k = h->k;
    int64_t nleaves = (int64_t)1 << h->q, f = first_of(h->q);
    int64_t off = 0;
    for (int64_t j = 0; j < nleaves; j++) {
        h->U_off[j] = off;
        off += (h->end[f + j] - h->begin[f + j]) * k;
    }
    h->U = malloc((size_t)(off > 0 ? off : 1) * sizeof(double));
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < nleaves; j++) {
        int64_t v = f + j, mi = h->end[v] - h->begin[v];
        double *Ui = h->U + h->U_off[j];
        for (int nu = 0; nu < k; nu++)
            for (int64_t r = 0; r < mi; r++)
                Ui[nu * mi + r] = lagrange(h, v, nu, h->pts + (h->begin[v] + r) * h->d);
    }
    h->E = calloc((size_t)h->nnodes * k * k, sizeof(double));
#pragma omp parallel for schedule(static)
    for (int64_t c = 1; c < h->nnodes; c++) {
        int64_t par = (c - 1) / 2;
        double *Ec = h->E + c * k * k, xi[3];
        for (int mu = 0; mu < k; mu++) {
            cheb_point(h, c, mu, xi);
            for (int nu = 0; nu < k; nu++) Ec[nu * k + mu] = lagrange(h, par, nu, xi);
        }
    }
    if (h->storage != OR_STORE_FP64) {
        or_quantize_block(OR_STORE_FP32, off, h->U);
        or_quantize_block(OR_STORE_FP32, h->nnodes * k * k, h->E);
    }
}

/* ---- Block-sparse-row assembly (Sec. 4.3, Fig. 5): blocks sorted by
 * (row, column); rowptr[i]..rowptr[i+1] index the blocks of row i. */
typedef struct { int32_t row, col; int64_t pos; } pair_item;

static int cmp_pair(const void *a, const void *b) {
    const pair_item *x = a, *y = b;
    if (x->row != y->row) return (x->row > y->row) - (x->row < y->row);
    return (x->col > y->col) - (x->col < y->col);
}

void or_bsr_assemble(int32_t nrows, int64_t nb, const int32_t *row, const int32_t *col,
                     int32_t *rowptr, int32_t *colidx, int64_t *order) {
    pair_item *it = malloc((size_t)(nb > 0 ? nb : 1) * sizeof(pair_item));
    for (int64_t i = 0; i < nb; i++) { it[i].row = row[i]; it[i].col = col[i]; it[i].pos = i; }
    qsort(it, (size_t)nb, sizeof(pair_item), cmp_pair);
    for (int32_t r = 0; r <= nrows; r++) rowptr[r] = 0;
    for (int64_t i = 0; i < nb; i++) rowptr[it[i].row + 1]++;
    for (int32_t r = 0; r < nrows; r++) rowptr[r + 1] += rowptr[r];
    for (int64_t i = 0; i < nb; i++) {
        colidx[i] = it[i].col;
        if (order) order[i] = it[i].pos;
    }
    free(it);
}

/* ---- Partition by dual traversal (Sec. 4.6, Sec. 2.2: admissible blocks are
 * coupling blocks at the level where they occur, dense m x m blocks only at
 * the finest level).  Reading: adm(s,t) = max(diam s, diam t) <= eta dist(s,t)
 * with Euclidean box diameters and box gap; start at (root, root); an
 * inadmissible pair recurses into its four child pairs, or is dense at level q. */
static double box_diam(const or_h2 *h, int64_t v) {
    double s = 0.0;
    for (int ax = 0; ax < h->d; ax++) {
        double e = h->hi[v * h->d + ax] - h->lo[v * h->d + ax];
        s += e * e;
    }
    return sqrt(s);
}

static double box_dist(const or_h2 *h, int64_t s, int64_t t) {
    double acc = 0.0;
    for (int ax = 0; ax < h->d; ax++) {
        double g = 0.0;
        double g1 = h->lo[s * h->d + ax] - h->hi[t * h->d + ax];
        double g2 = h->lo[t * h->d + ax] - h->hi[s * h->d + ax];
        if (g1 > g) g = g1;
        if (g2 > g) g = g2;
        acc += g * g;
    }
    return sqrt(acc);
}

typedef struct { int32_t *row, *col; int64_t n, cap; } pair_list;

static void push_pair(pair_list *pl, int32_t r, int32_t c) {
    if (pl->n == pl->cap) {
        pl->cap = pl->cap ? 2 * pl->cap : 64;
        pl->row = realloc(pl->row, (size_t)pl->cap * sizeof(int32_t));
        pl->col = realloc(pl->col, (size_t)pl->cap * sizeof(int32_t));
    }
    pl->row[pl->n] = r;
    pl->col[pl->n] = c;
    pl->n++;
}

static void build_partition(or_h2 *h) {
    int q = h->q;
    pair_list *lev = calloc((size_t)q + 1, sizeof(pair_list));
    pair_list dense = {0};
    int64_t cap = 1024, top = 0;
    int64_t *stack = malloc((size_t)cap * 2 * sizeof(int64_t));
    stack[0] = 0; stack[1] = 0; top = 1;
    while (top > 0) {
        top--;
        int64_t s = stack[2 * top], t = stack[2 * top + 1];
        int l = level_of(s);
        double ds = box_diam(h, s), dt = box_diam(h, t);
        double lhs = ds > dt ? ds : dt, rhs = h->eta * box_dist(h, s, t);
        if (rhs > 0.0 && fabs(lhs - rhs) < 1e-12 * rhs) h->near_ties++;
        if (lhs <= rhs && rhs > 0.0) {
            push_pair(&lev[l], (int32_t)(s - first_of(l)), (int32_t)(t - first_of(l)));
        } else if (l == q) {
            push_pair(&dense, (int32_t)(s - first_of(l)), (int32_t)(t - first_of(l)));
        } else {
            if (top + 4 > cap) { cap *= 2; stack = realloc(stack, (size_t)cap * 2 * sizeof(int64_t)); }
            int64_t ch[4][2] = {{2 * s + 1, 2 * t + 1}, {2 * s + 1, 2 * t + 2},
                                {2 * s + 2, 2 * t + 1}, {2 * s + 2, 2 * t + 2}};
            for (int i = 0; i < 4; i++) {
                stack[2 * top] = ch[i][0];
                stack[2 * top + 1] = ch[i][1];
                top++;
            }
        }
    }
    free(stack);
    h->S_rowptr = calloc((size_t)q + 1, sizeof(int32_t *));
    h->S_colidx = calloc((size_t)q + 1, sizeof(int32_t *));
    h->S_count = calloc((size_t)q + 1, sizeof(int64_t));
    h->S = calloc((size_t)q + 1, sizeof(double *));
    h->lmin = q + 1;
    for (int l = q; l >= 0; l--) {
        int32_t nrows = (int32_t)((int64_t)1 << l);
        h->S_count[l] = lev[l].n;
        h->S_rowptr[l] = malloc((size_t)(nrows + 1) * sizeof(int32_t));
        h->S_colidx[l] = malloc((size_t)(lev[l].n > 0 ? lev[l].n : 1) * sizeof(int32_t));
        or_bsr_assemble(nrows, lev[l].n, lev[l].row, lev[l].col, h->S_rowptr[l], h->S_colidx[l], NULL);
        if (lev[l].n > 0) h->lmin = l;
        free(lev[l].row);
        free(lev[l].col);
    }
    free(lev);
    int32_t nleaves = (int32_t)((int64_t)1 << q);
    h->D_count = dense.n;
    h->D_rowptr = malloc((size_t)(nleaves + 1) * sizeof(int32_t));
    h->D_colidx = malloc((size_t)(dense.n > 0 ? dense.n : 1) * sizeof(int32_t));
    or_bsr_assemble(nleaves, dense.n, dense.row, dense.col, h->D_rowptr, h->D_colidx, NULL);
    free(dense.row);
    free(dense.col);
}

/* ---- Block entries (Sec. 4.6: couplings are the kernel at interpolation
 * nodes; Sec. 2.2: dense blocks are the matrix entries themselves). */
static void gen_coupling(const or_h2 *h, int l, int64_t sl, int64_t tl, double *S) {
    int k = h->k;
    int64_t s = first_of(l) + sl, t = first_of(l) + tl;
    double xs[3], xt[3];
    for (int nu = 0; nu < k; nu++) {
        cheb_point(h, t, nu, xt);
        for (int mu = 0; mu < k; mu++) {
            cheb_point(h, s, mu, xs);
            S[nu * k + mu] = or_kernel(h->kernel, h->d, h->ell, xs, xt);
        }
    }
    or_quantize_block(h->storage, (int64_t)k * k, S);
}

static void gen_dense(const or_h2 *h, int64_t sl, int64_t tl, double *D) {
    int64_t s = first_of(h->q) + sl, t = first_of(h->q) + tl;
    int64_t ms = h->end[s] - h->begin[s], mt = h->end[t] - h->begin[t];
    for (int64_t b = 0; b < mt; b++)
        for (int64_t a = 0; a < ms; a++)
            D[b * ms + a] = or_kernel(h->kernel, h->d, h->ell, h->pts + (h->begin[s] + a) * h->d,
                                      h->pts + (h->begin[t] + b) * h->d);
    or_quantize_block(h->storage, ms * mt, D);
}

static void store_blocks(or_h2 *h) {
    int k = h->k;
    for (int l = 0; l <= h->q; l++) {
        if (h->S_count[l] == 0) continue;
        h->S[l] = malloc((size_t)h->S_count[l] * k * k * sizeof(double));
        int64_t nrows = (int64_t)1 << l;
#pragma omp parallel for schedule(dynamic, 4)
        for (int64_t i = 0; i < nrows; i++)
            for (int32_t b = h->S_rowptr[l][i]; b < h->S_rowptr[l][i + 1]; b++)
                gen_coupling(h, l, i, h->S_colidx[l][b], h->S[l] + (int64_t)b * k * k);
    }
    int64_t nleaves = (int64_t)1 << h->q, f = first_of(h->q), off = 0;
    h->D_off = malloc((size_t)(h->D_count + 1) * sizeof(int64_t));
    for (int64_t i = 0; i < nleaves; i++)
        for (int32_t b = h->D_rowptr[i]; b < h->D_rowptr[i + 1]; b++) {
            int64_t j = h->D_colidx[b];
            h->D_off[b] = off;
            off += (h->end[f + i] - h->begin[f + i]) * (h->end[f + j] - h->begin[f + j]);
        }
    h->D_off[h->D_count] = off;
    h->D = malloc((size_t)(off > 0 ? off : 1) * sizeof(double));
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t i = 0; i < nleaves; i++)
        for (int32_t b = h->D_rowptr[i]; b < h->D_rowptr[i + 1]; b++)
            gen_dense(h, i, h->D_colidx[b], h->D + h->D_off[b]);
}

int or_build(const double *pts, int64_t n, int d, int m, int p, double eta,
             double ell, int kernel, int storage, int keep_blocks, or_h2 **out) {
    *out = NULL;
    if (n < 1 || (d != 2 && d != 3) || m < 2 || p < 1 || !(eta > 0.0) || !(ell > 0.0))
        return -1;
    for (int64_t i = 0; i < n * d; i++)
        if (!isfinite(pts[i])) return -1;
    or_h2 *h = calloc(1, sizeof(or_h2));
    h->n = n; h->d = d; h->m = m; h->p = p; h->eta = eta; h->ell = ell;
    h->kernel = kernel; h->storage = storage; h->keep = keep_blocks;
    h->k = 1;
    for (int i = 0; i < d; i++) h->k *= p;
    h->q = 0;
    while ((((int64_t)m) << h->q) < n) h->q++;
    h->nnodes = ((int64_t)2 << h->q) - 1;
    h->pts = malloc((size_t)n * d * sizeof(double));
    h->perm = malloc((size_t)n * sizeof(int64_t));
    h->begin = malloc((size_t)h->nnodes * sizeof(int64_t));
    h->end = malloc((size_t)h->nnodes * sizeof(int64_t));
    h->lo = malloc((size_t)h->nnodes * d * sizeof(double));
    h->hi = malloc((size_t)h->nnodes * d * sizeof(double));
    h->cheb = malloc((size_t)p * sizeof(double));
    h->U_off = malloc(((size_t)1 << h->q) * sizeof(int64_t));
    or_cheb_nodes(p, h->cheb);
    build_tree(h, pts);
    build_boxes(h);
    build_bases(h);
    build_partition(h);
    if (keep_blocks) store_blocks(h);
    *out = h;
    return 0;
}

void or_free(or_h2 *h) {
    if (!h) return;
    for (int l = 0; l <= h->q; l++) {
        free(h->S_rowptr[l]);
        free(h->S_colidx[l]);
        free(h->S[l]);
    }
    free(h->S_rowptr); free(h->S_colidx); free(h->S_count); free(h->S);
    free(h->D_rowptr); free(h->D_colidx); free(h->D_off); free(h->D);
    free(h->pts); free(h->perm); free(h->begin); free(h->end); free(h->lo); free(h->hi);
    free(h->cheb); free(h->U); free(h->U_off); free(h->E);
    free(h);
}

/* ---- Accessors. */
void or_sizes(const or_h2 *h, int64_t *s) {
    int64_t tot = 0;
    for (int l = 0; l <= h->q; l++) tot += h->S_count[l];
    s[0] = h->n; s[1] = h->d; s[2] = h->m; s[3] = h->p; s[4] = h->k;
    s[5] = h->q; s[6] = h->lmin; s[7] = h->nnodes; s[8] = tot;
}
void or_perm(const or_h2 *h, int64_t *perm) { memcpy(perm, h->perm, (size_t)h->n * sizeof(int64_t)); }
void or_ranges(const or_h2 *h, int64_t *b, int64_t *e) {
    memcpy(b, h->begin, (size_t)h->nnodes * sizeof(int64_t));
    memcpy(e, h->end, (size_t)h->nnodes * sizeof(int64_t));
}
void or_boxes(const or_h2 *h, double *lo, double *hi) {
    memcpy(lo, h->lo, (size_t)h->nnodes * h->d * sizeof(double));
    memcpy(hi, h->hi, (size_t)h->nnodes * h->d * sizeof(double));
}
int64_t or_coupling_count(const or_h2 *h, int l) { return (l < 0 || l > h->q) ? 0 : h->S_count[l]; }
void or_coupling_bsr(const or_h2 *h, int l, int32_t *rowptr, int32_t *colidx) {
    memcpy(rowptr, h->S_rowptr[l], (((size_t)1 << l) + 1) * sizeof(int32_t));
    memcpy(colidx, h->S_colidx[l], (size_t)h->S_count[l] * sizeof(int32_t));
}
int64_t or_dense_count(const or_h2 *h) { return h->D_count; }
void or_dense_bsr(const or_h2 *h, int32_t *rowptr, int32_t *colidx) {
    memcpy(rowptr, h->D_rowptr, (((size_t)1 << h->q) + 1) * sizeof(int32_t));
    memcpy(colidx, h->D_colidx, (size_t)h->D_count * sizeof(int32_t));
}
int64_t or_near_ties(const or_h2 *h) { return h->near_ties; }

/* Flattened tree (Sec. 3.1): parent, first child (head) and next sibling of
 * every node of the heap-numbered binary tree, and the first node of every
 * level. */
void or_flat_tree(const or_h2 *h, int64_t *levelptr, int64_t *parent, int64_t *head,
                  int64_t *next) {
    for (int l = 0; l <= h->q + 1; l++) levelptr[l] = first_of(l);
    for (int64_t v = 0; v < h->nnodes; v++) {
        parent[v] = v == 0 ? -1 : (v - 1) / 2;
        head[v] = level_of(v) < h->q ? 2 * v + 1 : -1;
        next[v] = (v % 2 == 1) ? v + 1 : -1;
    }
}

void or_leaf_basis(const or_h2 *h, int64_t node, double *U) {
    int64_t j = node - first_of(h->q), mi = h->end[node] - h->begin[node];
    memcpy(U, h->U + h->U_off[j], (size_t)(mi * h->k) * sizeof(double));
}
void or_transfer(const or_h2 *h, int64_t node, double *E) {
    memcpy(E, h->E + node * h->k * h->k, (size_t)h->k * h->k * sizeof(double));
}

static int64_t coupling_row_of(const or_h2 *h, int l, int64_t idx) {
    int64_t lo = 0, hi = ((int64_t)1 << l);
    while (hi - lo > 1) {              /* last row whose rowptr <= idx */
        int64_t mid = (lo + hi) / 2;
        if (h->S_rowptr[l][mid] <= idx) lo = mid; else hi = mid;
    }
    return lo;
}

void or_coupling_block(const or_h2 *h, int l, int64_t idx, double *S) {
    if (h->keep) {
        memcpy(S, h->S[l] + idx * h->k * h->k, (size_t)h->k * h->k * sizeof(double));
        return;
    }
    gen_coupling(h, l, coupling_row_of(h, l, idx), h->S_colidx[l][idx], S);
}

void or_dense_block(const or_h2 *h, int64_t idx, double *D) {
    int64_t lo = 0, hi = ((int64_t)1 << h->q);
    while (hi - lo > 1) {
        int64_t mid = (lo + hi) / 2;
        if (h->D_rowptr[mid] <= idx) lo = mid; else hi = mid;
    }
    if (h->keep) {
        memcpy(D, h->D + h->D_off[idx], (size_t)(h->D_off[idx + 1] - h->D_off[idx]) * sizeof(double));
        return;
    }
    gen_dense(h, lo, h->D_colidx[idx], D);
}

/* Explicit basis of a node (Eq. (1) of Sec. 2.2). */
void or_explicit_basis(const or_h2 *h, int64_t v, int method, double *Uh) {
    int k = h->k;
    int64_t mv = h->end[v] - h->begin[v];
    if (method == 1) {
        for (int nu = 0; nu < k; nu++)
            for (int64_t r = 0; r < mv; r++)
                Uh[nu * mv + r] = lagrange(h, v, nu, h->pts + (h->begin[v] + r) * h->d);
        return;
    }
    if (level_of(v) == h->q) { or_leaf_basis(h, v, Uh); return; }
    for (int c = 0; c < 2; c++) {
        int64_t ch = 2 * v + 1 + c, mc = h->end[ch] - h->begin[ch], roff = h->begin[ch] - h->begin[v];
        double *Uc = malloc((size_t)(mc * k > 0 ? mc * k : 1) * sizeof(double));
        or_explicit_basis(h, ch, 0, Uc);
        const double *Ec = h->E + ch * k * k;
        for (int nu = 0; nu < k; nu++)
            for (int64_t r = 0; r < mc; r++) {
                double s = 0.0;
                for (int mu = 0; mu < k; mu++) s += Uc[mu * mc + r] * Ec[nu * k + mu];
                Uh[nu * mv + roff + r] = s;
            }
        free(Uc);
    }
}

/* ---- The O(n) product (Sec. 4.1: A = A_D + A_LR).
 * Upsweep (Sec. 4.2): xh^q_j = V_j^T x(j); for l = q..lmin+1:
 *   xh^{l-1}_{j+} = F_{j1}^T xh^l_{j1} + F_{j2}^T xh^l_{j2}  (from zero, j1 then j2). */
static void upsweep(const or_h2 *h, const double *x, double *xh) {
    int k = h->k, q = h->q;
    if (h->lmin > q) return;
    int64_t f = first_of(q), nleaves = (int64_t)1 << q;
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < nleaves; j++) {
        int64_t v = f + j, mj = h->end[v] - h->begin[v];
        const double *Vj = h->U + h->U_off[j];
        for (int nu = 0; nu < k; nu++) {
            double s = 0.0;
            for (int64_t r = 0; r < mj; r++) s += Vj[nu * mj + r] * x[h->begin[v] + r];
            xh[v * k + nu] = s;
        }
    }
    for (int l = q; l > h->lmin; l--) {
        int64_t fp = first_of(l - 1), np = (int64_t)1 << (l - 1);
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < np; i++) {
            int64_t par = fp + i;
            for (int nu = 0; nu < k; nu++) xh[par * k + nu] = 0.0;
            for (int c = 0; c < 2; c++) {
                int64_t ch = 2 * par + 1 + c;
                const double *Fc = h->E + ch * k * k;
                for (int nu = 0; nu < k; nu++) {
                    double s = 0.0;
                    for (int mu = 0; mu < k; mu++) s += Fc[nu * k + mu] * xh[ch * k + mu];
                    xh[par * k + nu] += s;
                }
            }
        }
    }
}

/* Tree multiply of one block row (Sec. 4.3): yh^l_i = sum_{j in b_i} S^l_ij xh^l_j,
 * j ascending. */
static void tree_multiply_row(const or_h2 *h, int l, int64_t i, const double *xh,
                              double *yrow, double *Sbuf) {
    int k = h->k;
    int64_t f = first_of(l);
    for (int mu = 0; mu < k; mu++) yrow[mu] = 0.0;
    for (int32_t b = h->S_rowptr[l][i]; b < h->S_rowptr[l][i + 1]; b++) {
        int64_t j = h->S_colidx[l][b];
        const double *S;
        if (h->keep) S = h->S[l] + (int64_t)b * k * k;
        else { gen_coupling(h, l, i, j, Sbuf); S = Sbuf; }
        const double *xj = xh + (f + j) * k;
        for (int mu = 0; mu < k; mu++) {
            double s = 0.0;
            for (int nu = 0; nu < k; nu++) s += S[nu * k + mu] * xj[nu];
            yrow[mu] += s;
        }
    }
}

/* Dense near field of one leaf row (Sec. 4.1): y_near(i) = sum_j D_ij x(j). */
static void dense_row(const or_h2 *h, int64_t i, const double *x, double *yrow, double *Dbuf) {
    int64_t f = first_of(h->q), s = f + i, ms = h->end[s] - h->begin[s];
    for (int64_t a = 0; a < ms; a++) yrow[a] = 0.0;
    for (int32_t b = h->D_rowptr[i]; b < h->D_rowptr[i + 1]; b++) {
        int64_t t = f + h->D_colidx[b], mt = h->end[t] - h->begin[t];
        const double *D;
        if (h->keep) D = h->D + h->D_off[b];
        else { gen_dense(h, i, h->D_colidx[b], Dbuf); D = Dbuf; }
        for (int64_t a = 0; a < ms; a++) {
            double sacc = 0.0;
            for (int64_t c = 0; c < mt; c++) sacc += D[c * ms + a] * x[h->begin[t] + c];
            yrow[a] += sacc;
        }
    }
}

/* Downsweep step (Sec. 4.4): yh^l_c = yh^l_c + E_c yh^{l-1}_{c+}. */
static void downsweep_node(const or_h2 *h, int64_t c, double *yh) {
    int k = h->k;
    int64_t par = (c - 1) / 2;
    const double *Ec = h->E + c * k * k;
    for (int mu = 0; mu < k; mu++) {
        double s = 0.0;
        for (int nu = 0; nu < k; nu++) s += Ec[nu * k + mu] * yh[par * k + nu];
        yh[c * k + mu] += s;
    }
}

/* Leaf expansion (Sec. 4.4, last step of the downsweep): y(i) = U_i yh^q_i. */
static void leaf_expand(const or_h2 *h, int64_t j, const double *yh, double *yrow) {
    int k = h->k;
    int64_t v = first_of(h->q) + j, mj = h->end[v] - h->begin[v];
    const double *Uj = h->U + h->U_off[j];
    for (int64_t r = 0; r < mj; r++) {
        double s = 0.0;
        for (int nu = 0; nu < k; nu++) s += Uj[nu * mj + r] * yh[v * k + nu];
        yrow[r] = s;
    }
}

void or_matvec_parts(const or_h2 *h, const double *x, double *xh_out, double *yh_out,
                     double *y_near, double *y_far) {
    int k = h->k, q = h->q;
    int64_t nn = h->nnodes, nleaves = (int64_t)1 << q, f = first_of(q);
    double *xh = calloc((size_t)nn * k, sizeof(double));
    double *yh = calloc((size_t)nn * k, sizeof(double));
    double *yn = calloc((size_t)h->n, sizeof(double));
    double *yf = calloc((size_t)h->n, sizeof(double));
    int64_t mmax = 0;
    for (int64_t j = 0; j < nleaves; j++)
        if (h->end[f + j] - h->begin[f + j] > mmax) mmax = h->end[f + j] - h->begin[f + j];
    upsweep(h, x, xh);
    if (h->lmin <= q) {
        for (int l = h->lmin; l <= q; l++) {
            int64_t nrows = (int64_t)1 << l, fl = first_of(l);
#pragma omp parallel
            {
                double *Sbuf = malloc((size_t)k * k * sizeof(double));
#pragma omp for schedule(dynamic, 4)
                for (int64_t i = 0; i < nrows; i++) tree_multiply_row(h, l, i, xh, yh + (fl + i) * k, Sbuf);
                free(Sbuf);
            }
        }
        for (int l = h->lmin + 1; l <= q; l++) {
            int64_t nrows = (int64_t)1 << l, fl = first_of(l);
#pragma omp parallel for schedule(static)
            for (int64_t i = 0; i < nrows; i++) downsweep_node(h, fl + i, yh);
        }
#pragma omp parallel for schedule(static)
        for (int64_t j = 0; j < nleaves; j++) leaf_expand(h, j, yh, yf + h->begin[f + j]);
    }
#pragma omp parallel
    {
        double *Dbuf = malloc((size_t)(mmax * mmax > 0 ? mmax * mmax : 1) * sizeof(double));
#pragma omp for schedule(dynamic, 4)
        for (int64_t i = 0; i < nleaves; i++) dense_row(h, i, x, yn + h->begin[f + i], Dbuf);
        free(Dbuf);
    }
    if (xh_out) memcpy(xh_out, xh, (size_t)nn * k * sizeof(double));
    if (yh_out) memcpy(yh_out, yh, (size_t)nn * k * sizeof(double));
    if (y_near) memcpy(y_near, yn, (size_t)h->n * sizeof(double));
    if (y_far) memcpy(y_far, yf, (size_t)h->n * sizeof(double));
    free(xh); free(yh); free(yn); free(yf);
}

/* y = y_near + y_far (Sec. 4.1, Fig. 4: the two parts are added at the end). */
void or_matvec(const or_h2 *h, const double *x, double *y) {
    double *yn = malloc((size_t)h->n * sizeof(double));
    double *yf = malloc((size_t)h->n * sizeof(double));
    or_matvec_parts(h, x, NULL, NULL, yn, yf);
    for (int64_t i = 0; i < h->n; i++) y[i] = yn[i] + yf[i];
    free(yn); free(yf);
}

/* ---- Product of an H^2 matrix given by its arrays (Sec. 2.2 with Eq. (1);
 * the flattened per-level storage of Sec. 3 and Fig. 3; every level of the
 * matrix tree as block-sparse rows, Fig. 5), 0-based, with a rank k_l per
 * level.  Layout: leaf j's U_j, V_j are m_j x k_q column-major, concatenated
 * in leaf order; node c >= 1 of level l has E_c, F_c, k_l x k_(l-1)
 * column-major, concatenated in node order; level l's coupling blocks are
 * k_l x k_l column-major in BSR order; dense blocks m_i x m_j column-major in
 * BSR order.  The sweeps of Sec. 4 in the paper's order: leaf projection and
 * upsweep to the root (x^ from zero, children c1 then c2; Sec. 4.2), tree
 * multiplication of every level (blocks in row order; Sec. 4.3), downsweep
 * from the root (Sec. 4.4), leaf expansion, and y = y_near + y_far (Sec. 4.1).
 * Returns 0, or -1 on invalid sizes. */
int or_arrays_matvec(int64_t n, int q, const int32_t *lrank, const int64_t *begin, const int64_t *end,
                     const double *U, const double *V, const double *E, const double *F,
                     const int32_t *const *S_rowptr, const int32_t *const *S_colidx,
                     const double *const *S, const int32_t *D_rowptr, const int32_t *D_colidx,
                     const double *D, const double *x, double *y) {
    if (n < 1 || q < 0 || q > 29) return -1;
    int64_t nn = ((int64_t)2 << q) - 1, nleaves = (int64_t)1 << q, lf = first_of(q);
    int kmax = 0;
    for (int l = 0; l <= q; l++) {
        if (lrank[l] < 1) return -1;
        if (lrank[l] > kmax) kmax = lrank[l];
    }
    double *xh = calloc((size_t)nn * kmax, sizeof(double));
    double *yh = calloc((size_t)nn * kmax, sizeof(double));
    int64_t *eoff = calloc((size_t)nn, sizeof(int64_t));   /* start of E_c / F_c */
    int64_t *uoff = calloc((size_t)nleaves, sizeof(int64_t));
    int64_t acc = 0;
    for (int l = 1; l <= q; l++)
        for (int64_t c = first_of(l); c < first_of(l + 1); c++) {
            eoff[c] = acc;
            acc += (int64_t)lrank[l] * lrank[l - 1];
        }
    acc = 0;
    for (int64_t j = 0; j < nleaves; j++) {
        uoff[j] = acc;
        acc += (end[lf + j] - begin[lf + j]) * lrank[q];
    }
    int kq = lrank[q];
    int has_low_rank = 0;
    for (int l = 0; l <= q; l++)
        if (S_rowptr[l][(int64_t)1 << l] > 0) has_low_rank = 1;
    if (has_low_rank) {
        /* leaf projection x^_j = V_j^T x(j) */
        for (int64_t j = 0; j < nleaves; j++) {
            int64_t v = lf + j, mj = end[v] - begin[v];
            const double *Vj = V + uoff[j];
            for (int nu = 0; nu < kq; nu++) {
                double s = 0.0;
                for (int64_t r = 0; r < mj; r++) s += Vj[nu * mj + r] * x[begin[v] + r];
                xh[v * kmax + nu] = s;
            }
        }
        /* upsweep x^_p = F_c1^T x^_c1 + F_c2^T x^_c2, levels q .. 1 */
        for (int l = q; l >= 1; l--) {
            int kc = lrank[l], kp = lrank[l - 1];
            for (int64_t p = first_of(l - 1); p < first_of(l); p++) {
                for (int nu = 0; nu < kp; nu++) xh[p * kmax + nu] = 0.0;
                for (int c = 0; c < 2; c++) {
                    int64_t ch = 2 * p + 1 + c;
                    const double *Fc = F + eoff[ch];   /* kc x kp column-major */
                    for (int nu = 0; nu < kp; nu++) {
                        double s = 0.0;
                        for (int mu = 0; mu < kc; mu++) s += Fc[nu * kc + mu] * xh[ch * kmax + mu];
                        xh[p * kmax + nu] += s;
                    }
                }
            }
        }
        /* tree multiplication y^_i = sum_j S_ij x^_j on every level */
        for (int l = 0; l <= q; l++) {
            int k = lrank[l];
            int64_t fl = first_of(l);
            for (int64_t i = 0; i < ((int64_t)1 << l); i++)
                for (int32_t b = S_rowptr[l][i]; b < S_rowptr[l][i + 1]; b++) {
                    const double *Sb = S[l] + (int64_t)b * k * k;
                    int64_t jn = fl + S_colidx[l][b];
                    for (int mu = 0; mu < k; mu++) {
                        double s = 0.0;
                        for (int nu = 0; nu < k; nu++) s += Sb[nu * k + mu] * xh[jn * kmax + nu];
                        yh[(fl + i) * kmax + mu] += s;
                    }
                }
        }
        /* downsweep y^_c += E_c y^_parent, levels 1 .. q */
        for (int l = 1; l <= q; l++) {
            int kc = lrank[l], kp = lrank[l - 1];
            for (int64_t c = first_of(l); c < first_of(l + 1); c++) {
                const double *Ec = E + eoff[c];   /* kc x kp column-major */
                int64_t par = (c - 1) / 2;
                for (int mu = 0; mu < kc; mu++) {
                    double s = 0.0;
                    for (int nu = 0; nu < kp; nu++) s += Ec[nu * kc + mu] * yh[par * kmax + nu];
                    yh[c * kmax + mu] += s;
                }
            }
        }
    }
    /* leaf expansion and dense near field: y(i) = y_near(i) + U_i y^_i */
    int64_t doff = 0;
    for (int64_t i = 0; i < nleaves; i++) {
        int64_t s = lf + i, ms = end[s] - begin[s];
        for (int64_t a = 0; a < ms; a++) {
            double yf = 0.0;
            if (has_low_rank) {
                const double *Ui = U + uoff[i];
                for (int nu = 0; nu < kq; nu++) yf += Ui[nu * ms + a] * yh[s * kmax + nu];
            }
            y[begin[s] + a] = yf;
        }
        for (int64_t a = 0; a < ms; a++) {
            double yn = 0.0;
            int64_t o = doff;
            for (int32_t b = D_rowptr[i]; b < D_rowptr[i + 1]; b++) {
                int64_t t = lf + D_colidx[b], mt = end[t] - begin[t];
                double sacc = 0.0;
                for (int64_t c = 0; c < mt; c++) sacc += D[o + c * ms + a] * x[begin[t] + c];
                yn += sacc;
                o += ms * mt;
            }
            y[begin[s] + a] = yn + y[begin[s] + a];
        }
        for (int32_t b = D_rowptr[i]; b < D_rowptr[i + 1]; b++) {
            int64_t t = lf + D_colidx[b];
            doff += ms * (end[t] - begin[t]);
        }
    }
    free(xh); free(yh); free(eoff); free(uoff);
    return 0;
}

/* Same operations as or_matvec, restricted to the rows of the listed leaves:
 * the full upsweep, then the tree multiply and downsweep along each leaf's
 * chain of ancestors only. */
void or_matvec_leaves(const or_h2 *h, const double *x, int64_t nleaves_s,
                      const int64_t *leaves, double *y) {
    int k = h->k, q = h->q;
    int64_t nn = h->nnodes, f = first_of(q);
    double *xh = calloc((size_t)nn * k, sizeof(double));
    upsweep(h, x, xh);
    int64_t *outoff = malloc((size_t)(nleaves_s + 1) * sizeof(int64_t));
    outoff[0] = 0;
    int64_t mmax = 0;
    for (int64_t s = 0; s < nleaves_s; s++) {
        int64_t v = leaves[s], mv = h->end[v] - h->begin[v];
        outoff[s + 1] = outoff[s] + mv;
    }
    for (int64_t j = 0; j < ((int64_t)1 << q); j++)
        if (h->end[f + j] - h->begin[f + j] > mmax) mmax = h->end[f + j] - h->begin[f + j];
#pragma omp parallel
    {
        double *yh = calloc((size_t)nn * k, sizeof(double));
        double *Sbuf = malloc((size_t)k * k * sizeof(double));
        double *Dbuf = malloc((size_t)(mmax * mmax > 0 ? mmax * mmax : 1) * sizeof(double));
        double *yn = malloc((size_t)(mmax > 0 ? mmax : 1) * sizeof(double));
        double *yf = calloc((size_t)(mmax > 0 ? mmax : 1), sizeof(double));
#pragma omp for schedule(dynamic, 1)
        for (int64_t s = 0; s < nleaves_s; s++) {
            int64_t v = leaves[s], j = v - f, mv = h->end[v] - h->begin[v];
            for (int64_t r = 0; r < mv; r++) yf[r] = 0.0;
            if (h->lmin <= q) {
                for (int l = h->lmin; l <= q; l++) {
                    int64_t a = v;
                    for (int up = q; up > l; up--) a = (a - 1) / 2;
                    tree_multiply_row(h, l, a - first_of(l), xh, yh + a * k, Sbuf);
                    if (l > h->lmin) downsweep_node(h, a, yh);
                }
                leaf_expand(h, j, yh, yf);
            }
            dense_row(h, j, x, yn, Dbuf);
            for (int64_t r = 0; r < mv; r++) y[outoff[s] + r] = yn[r] + yf[r];
        }
        free(yh); free(Sbuf); free(Dbuf); free(yn); free(yf);
    }
    free(outoff);
    free(xh);
}

/* Explicit A_H (row-major n x n, tree order): each coupling block is
 * Uhat_s S Uhat_t^T (bases through the transfers), each dense block copied. */
void or_dense_expand(const or_h2 *h, double *A) {
    int k = h->k, q = h->q;
    int64_t n = h->n;
    memset(A, 0, (size_t)n * n * sizeof(double));
    for (int l = 0; l <= q; l++) {
        int64_t nrows = (int64_t)1 << l, fl = first_of(l);
        for (int64_t i = 0; i < nrows; i++)
            for (int32_t b = h->S_rowptr[l][i]; b < h->S_rowptr[l][i + 1]; b++) {
                int64_t s = fl + i, t = fl + h->S_colidx[l][b];
                int64_t ms = h->end[s] - h->begin[s], mt = h->end[t] - h->begin[t];
                double *Us = malloc((size_t)ms * k * sizeof(double));
                double *Ut = malloc((size_t)mt * k * sizeof(double));
                double *S = malloc((size_t)k * k * sizeof(double));
                double *US = malloc((size_t)ms * k * sizeof(double));
                or_explicit_basis(h, s, 0, Us);
                or_explicit_basis(h, t, 0, Ut);
                or_coupling_block(h, l, b, S);
                for (int nu = 0; nu < k; nu++)
                    for (int64_t a = 0; a < ms; a++) {
                        double acc = 0.0;
                        for (int mu = 0; mu < k; mu++) acc += Us[mu * ms + a] * S[nu * k + mu];
                        US[nu * ms + a] = acc;
                    }
                for (int64_t a = 0; a < ms; a++)
                    for (int64_t c = 0; c < mt; c++) {
                        double acc = 0.0;
                        for (int nu = 0; nu < k; nu++) acc += US[nu * ms + a] * Ut[nu * mt + c];
                        A[(h->begin[s] + a) * n + h->begin[t] + c] += acc;
                    }
                free(Us); free(Ut); free(S); free(US);
            }
    }
    int64_t f = first_of(q), nleaves = (int64_t)1 << q;
    for (int64_t i = 0; i < nleaves; i++)
        for (int32_t b = h->D_rowptr[i]; b < h->D_rowptr[i + 1]; b++) {
            int64_t s = f + i, t = f + h->D_colidx[b];
            int64_t ms = h->end[s] - h->begin[s], mt = h->end[t] - h->begin[t];
            double *D = malloc((size_t)ms * mt * sizeof(double));
            or_dense_block(h, b, D);
            for (int64_t a = 0; a < ms; a++)
                for (int64_t c = 0; c < mt; c++)
                    A[(h->begin[s] + a) * n + h->begin[t] + c] += D[c * ms + a];
            free(D);
        }
}

/* Brute-force kernel product over the listed rows (Sec. 4.6: error measured
 * against the exact covariance, on a sample of rows for large n). */
void or_kernel_matvec(const double *pts, int64_t n, int d, double ell, int kernel,
                      const double *x, int64_t nrows, const int64_t *rows, double *y) {
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t r = 0; r < nrows; r++) {
        double s = 0.0;
        for (int64_t j = 0; j < n; j++) s += or_kernel(kernel, d, ell, pts + rows[r] * d, pts + j * d) * x[j];
        y[r] = s;
    }
}
