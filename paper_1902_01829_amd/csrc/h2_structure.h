// Host-side structure of an H^2 matrix: cluster tree, boxes and the
// block-sparse-row partition.  Internal to libh2mv.
#pragma once

#include <algorithm>
#include <cstdint>
#include <future>
#include <string>
#include <thread>
#include <vector>

namespace h2 {

// Host threads of the library's set-up loops: the machine's, at most 16.
inline int64_t host_threads() {
    return std::max<int64_t>(1, std::min<int64_t>(16, int64_t(std::thread::hardware_concurrency())));
}

// Runs f(i0, i1) on contiguous pieces of [0, n), one per host thread, with
// at least min_piece items per piece (all on the calling thread when n is
// small; a piece whose thread cannot be started runs on the calling thread
// when its result is collected).  An exception thrown by a piece reaches the
// caller.
template <typename F>
void parallel_ranges(int64_t n, int64_t min_piece, const F &f) {
    const int64_t t = std::min(host_threads(), std::max<int64_t>(1, n / std::max<int64_t>(1, min_piece)));
    if (t <= 1) {
        f(int64_t(0), n);
        return;
    }
    std::vector<std::future<void>> jobs;
    for (int64_t i = 1; i < t; ++i)
        jobs.push_back(std::async(std::launch::async | std::launch::deferred, f, n * i / t, n * (i + 1) / t));
    f(int64_t(0), n / t);
    for (auto &j : jobs) j.get();
}

struct Bsr {
    std::vector<int32_t> rowptr;   // rows + 1
    std::vector<int32_t> colidx;   // blocks, sorted by (row, col)
    int64_t blocks() const { return static_cast<int64_t>(colidx.size()); }
};

struct Structure {
    int64_t n = 0;
    int dim = 0, leaf = 0, cheb_p = 0, rank = 0, q = 0, lmin = 0;
    double eta = 0, corr_len = 0;
    int64_t nnodes = 0;
    std::vector<int64_t> perm;           // tree position -> input index
    std::vector<int64_t> begin, end;     // node ranges in tree order
    std::vector<double> pts;             // n x dim, tree order
    std::vector<double> lo, hi;          // nnodes x dim, widened tight boxes
    std::vector<Bsr> coupling;           // per level 0..q, rows = nodes of the level
    Bsr dense;                           // rows = leaves
    std::vector<int> lrank;              // rank of every level 0..q (rank = their maximum)
    int64_t near_ties = 0;

    static int64_t first(int level) { return (int64_t(1) << level) - 1; }
    int64_t size(int64_t v) const { return end[v] - begin[v]; }
};

// Builds the structure; returns an empty string on success, else the reason.
std::string build_structure(const double *points, int64_t n, int dim, int leaf, int cheb_p,
                            double eta, double corr_len, Structure &s);

}  // namespace h2
