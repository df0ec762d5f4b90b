// Host-side construction of the H^2 structure (Sec. 4.6 "ab initio"
// generation): KD-tree bisection of the points, tight boxes, and the dual
// traversal that splits the matrix into admissible (coupling) blocks at every
// level and dense blocks at the leaf level (Sec. 2.2), each level kept as
// block-sparse rows (Sec. 4.3, Fig. 5).
//
// Rules taken where the paper leaves the choice open:
//  - leaf level q is the smallest with n <= leaf * 2^q, and every node above
//    it is bisected (a complete tree, as the per-level batch sizes of the
//    upsweep and downsweep algorithms imply);
//  - a node is split along the widest axis of its tight box (lowest axis on
//    ties), its points ordered by (coordinate, input index), the first half
//    (rounded down) going to the first child;
//  - boxes are tight; an axis of zero extent is widened symmetrically to
//    1e-12 * max(1, widest extent of the root box);
//  - (s, t) is admissible when max(diam s, diam t) <= eta * dist(s, t) > 0,
//    with Euclidean box diameters and box gap.
#include "h2_structure.h"

#include <algorithm>
#include <cmath>
#include <future>
#include <numeric>
#include <thread>

namespace h2 {
namespace {

// Splits every node of one level; nodes are independent, so they are spread
// over a few host threads.
void split_level(const double *points, int dim, int level, Structure &s) {
    const int64_t first = Structure::first(level), count = int64_t(1) << level;
    auto work = [&](int64_t j0, int64_t j1) {
        std::vector<int64_t> idx;
        for (int64_t j = j0; j < j1; ++j) {
            const int64_t v = first + j, b = s.begin[v], e = s.end[v];
            double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
            for (int64_t i = b; i < e; ++i)
                for (int a = 0; a < dim; ++a) {
                    const double c = points[s.perm[i] * dim + a];
                    lo[a] = std::min(lo[a], c);
                    hi[a] = std::max(hi[a], c);
                }
            int axis = 0;
            for (int a = 1; a < dim; ++a)
                if (hi[a] - lo[a] > hi[axis] - lo[axis]) axis = a;
            idx.assign(s.perm.begin() + b, s.perm.begin() + e);
            std::sort(idx.begin(), idx.end(), [&](int64_t x, int64_t y) {
                const double cx = points[x * dim + axis], cy = points[y * dim + axis];
                return cx < cy || (cx == cy && x < y);
            });
            std::copy(idx.begin(), idx.end(), s.perm.begin() + b);
            const int64_t mid = b + (e - b) / 2;
            s.begin[2 * v + 1] = b;
            s.end[2 * v + 1] = mid;
            s.begin[2 * v + 2] = mid;
            s.end[2 * v + 2] = e;
        }
    };
    if (s.n < 50000) {
        work(0, count);
        return;
    }
    parallel_ranges(count, 1, work);
}

void compute_boxes(Structure &s) {
    const int dim = s.dim;
    s.lo.assign(s.nnodes * dim, INFINITY);
    s.hi.assign(s.nnodes * dim, -INFINITY);
    // leaves from their points, inner nodes as the union of their children
    const int64_t lf = Structure::first(s.q);
    for (int64_t v = lf; v < s.nnodes; ++v)
        for (int64_t i = s.begin[v]; i < s.end[v]; ++i)
            for (int a = 0; a < dim; ++a) {
                s.lo[v * dim + a] = std::min(s.lo[v * dim + a], s.pts[i * dim + a]);
                s.hi[v * dim + a] = std::max(s.hi[v * dim + a], s.pts[i * dim + a]);
            }
    for (int64_t v = lf - 1; v >= 0; --v)
        for (int a = 0; a < dim; ++a) {
            s.lo[v * dim + a] = std::min(s.lo[(2 * v + 1) * dim + a], s.lo[(2 * v + 2) * dim + a]);
            s.hi[v * dim + a] = std::max(s.hi[(2 * v + 1) * dim + a], s.hi[(2 * v + 2) * dim + a]);
        }
    double widest = 0.0;
    for (int a = 0; a < dim; ++a) widest = std::max(widest, s.hi[a] - s.lo[a]);
    const double delta = 1e-12 * std::max(1.0, widest);
    for (int64_t v = 0; v < s.nnodes; ++v)
        for (int a = 0; a < dim; ++a)
            if (s.hi[v * dim + a] - s.lo[v * dim + a] == 0.0) {
                s.lo[v * dim + a] -= 0.5 * delta;
                s.hi[v * dim + a] += 0.5 * delta;
            }
}

struct Traversal {
    Structure &s;
    std::vector<double> diam;
    std::vector<std::vector<std::pair<int32_t, int32_t>>> lists;   // per level
    std::vector<std::pair<int32_t, int32_t>> dense;

    explicit Traversal(Structure &st) : s(st), diam(st.nnodes), lists(st.q + 1) {
        for (int64_t v = 0; v < s.nnodes; ++v) {
            double acc = 0.0;
            for (int a = 0; a < s.dim; ++a) {
                const double e = s.hi[v * s.dim + a] - s.lo[v * s.dim + a];
                acc += e * e;
            }
            diam[v] = std::sqrt(acc);
        }
    }

    double gap(int64_t a, int64_t b) const {
        double acc = 0.0;
        for (int x = 0; x < s.dim; ++x) {
            double g = 0.0;
            g = std::max(g, s.lo[a * s.dim + x] - s.hi[b * s.dim + x]);
            g = std::max(g, s.lo[b * s.dim + x] - s.hi[a * s.dim + x]);
            acc += g * g;
        }
        return std::sqrt(acc);
    }

    void visit(int64_t a, int64_t b, int level) {
        const double size = std::max(diam[a], diam[b]);
        const double far = s.eta * gap(a, b);
        if (far > 0.0 && std::fabs(size - far) < 1e-12 * far) ++s.near_ties;
        const int64_t f = Structure::first(level);
        if (far > 0.0 && size <= far) {
            lists[level].emplace_back(int32_t(a - f), int32_t(b - f));
        } else if (level == s.q) {
            dense.emplace_back(int32_t(a - f), int32_t(b - f));
        } else {
            for (int i = 1; i <= 2; ++i)
                for (int j = 1; j <= 2; ++j) visit(2 * a + i, 2 * b + j, level + 1);
        }
    }
};

Bsr to_bsr(int64_t rows, std::vector<std::pair<int32_t, int32_t>> &pairs) {
    std::sort(pairs.begin(), pairs.end());
    Bsr m;
    m.rowptr.assign(rows + 1, 0);
    m.colidx.resize(pairs.size());
    for (size_t i = 0; i < pairs.size(); ++i) {
        ++m.rowptr[pairs[i].first + 1];
        m.colidx[i] = pairs[i].second;
    }
    std::partial_sum(m.rowptr.begin(), m.rowptr.end(), m.rowptr.begin());
    return m;
}

}  // namespace

std::string build_structure(const double *points, int64_t n, int dim, int leaf, int cheb_p,
                            double eta, double corr_len, Structure &s) {
    s = Structure();
    s.n = n;
    s.dim = dim;
    s.leaf = leaf;
    s.cheb_p = cheb_p;
    s.eta = eta;
    s.corr_len = corr_len;
    s.rank = 1;
    for (int a = 0; a < dim; ++a) s.rank *= cheb_p;
    while ((int64_t(leaf) << s.q) < n) ++s.q;
    if (s.q > 29) return "tree deeper than 29 levels";
    s.nnodes = (int64_t(2) << s.q) - 1;
    s.lrank.assign(s.q + 1, s.rank);
    s.perm.resize(n);
    std::iota(s.perm.begin(), s.perm.end(), int64_t(0));
    s.begin.assign(s.nnodes, 0);
    s.end.assign(s.nnodes, 0);
    s.end[0] = n;
    for (int l = 0; l < s.q; ++l) split_level(points, dim, l, s);
    s.pts.resize(n * dim);
    for (int64_t i = 0; i < n; ++i)
        for (int a = 0; a < dim; ++a) s.pts[i * dim + a] = points[s.perm[i] * dim + a];
    compute_boxes(s);

    Traversal t(s);
    t.visit(0, 0, 0);
    s.coupling.resize(s.q + 1);
    s.lmin = s.q + 1;
    for (int l = s.q; l >= 0; --l) {
        s.coupling[l] = to_bsr(int64_t(1) << l, t.lists[l]);
        if (s.coupling[l].blocks() > 0) s.lmin = l;
    }
    s.dense = to_bsr(int64_t(1) << s.q, t.dense);
    return std::string();
}

}  // namespace h2
