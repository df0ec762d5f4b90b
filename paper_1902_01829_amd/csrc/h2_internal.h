// Internals shared by the host sources of libh2mv: the handle structures
// behind h2_handle and h2_batch, the device arena, the work lists of a
// product, and the steps each source file provides to the others.
#pragma once

#include "h2mv.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <memory>
#include <new>
#include <mutex>
#include <string>
#include <vector>

#include "h2_device.h"
#include "h2_structure.h"

namespace h2i {

using h2::BlkDesc;
using h2::RowDesc;
using h2::Structure;

// Message of the last failed call on this thread (h2_last_error).
extern thread_local std::string g_last_error;

struct Failure {
    h2_status code;
    std::string what;
};

[[noreturn]] inline void fail(h2_status code, const std::string &what) { throw Failure{code, what}; }

inline void check_hip(hipError_t e, const char *where) {
    if (e != hipSuccess) fail(H2_ERR_DEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

// Device allocations of one owner; a test-only cap (environment variable
// H2MV_DEVICE_BYTE_CAP, bytes) turns any allocation past it into H2_ERR_OOM.
struct DeviceArena {
    std::vector<void *> ptrs;
    int64_t bytes = 0;
    int64_t cap = -1;

    DeviceArena() {
        if (const char *c = std::getenv("H2MV_DEVICE_BYTE_CAP")) cap = std::atoll(c);
    }
    DeviceArena(const DeviceArena &) = delete;
    DeviceArena &operator=(const DeviceArena &) = delete;
    ~DeviceArena() {
        for (void *p : ptrs) (void)hipFree(p);
    }
    void swap(DeviceArena &o) {
        std::swap(ptrs, o.ptrs);
        std::swap(bytes, o.bytes);
        std::swap(cap, o.cap);
    }
    void *alloc(int64_t nbytes) {
        if (nbytes <= 0) nbytes = 16;
        nbytes = (nbytes + 255) / 256 * 256;
        if (cap >= 0 && bytes + nbytes > cap) fail(H2_ERR_OOM, "device byte cap exceeded");
        void *p = nullptr;
        hipError_t e = hipMalloc(&p, size_t(nbytes));
        if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) {
            (void)hipGetLastError();
            fail(H2_ERR_OOM, "hipMalloc of " + std::to_string(nbytes) + " bytes failed");
        }
        check_hip(e, "hipMalloc");
        ptrs.push_back(p);
        bytes += nbytes;
        return p;
    }
    template <typename T>
    // Copies v to new device memory; returns once v may be released (set-up
    // only, never inside a product).
    T *upload(const std::vector<T> &v, hipStream_t st) {
        T *d = static_cast<T *>(alloc(int64_t(v.size() * sizeof(T))));
        if (!v.empty()) {
            check_hip(hipMemcpyAsync(d, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, st),
                      "hipMemcpyAsync");
            check_hip(hipStreamSynchronize(st), "upload");
        }
        return d;
    }
};

enum Phase { PH_UP = 0, PH_STREAM = 1, PH_DOWN = 2, PH_LEAF = 3, PH_COUNT = 4 };

struct WorkList {
    Phase phase;
    int kind;   // element kind of its data
    const void *data;
    const h2::RowDesc *rows;
    int64_t nrows;
    const h2::BlkDesc *blks;
    const int32_t *items = nullptr;   // tile lists: wavefront items in dispatch order
    int64_t nitems = 0;
    const int32_t *pitems = nullptr;  // tile lists: pair items (two per workgroup) in dispatch order
    int64_t npitems = 0;
    // split stream list (single vector, small matrices): the rows are chunks
    // writing FP64 partial sums, added up by a second launch
    const h2::ReduceDesc *red = nullptr;
    int64_t nred = 0;
    void *partials = nullptr;   // FP64 (FP32 for the half-storage list of a reduced-storage matrix)
    int64_t partials_bytes = 0;
    // stream list of a matrix stored by halves: the wavefronts' row groups,
    // every block's slot code and the groups' merged partial slots (see
    // h2::HalfGroup); red then adds the slots to the row sums
    const int32_t *slot = nullptr;
    const h2::HalfGroup *groups = nullptr;
    int64_t ngroups = 0;
    const int32_t *gslot = nullptr;
    // single-vector stream list, full storage: the same rows (chunks, for a
    // split list) with the coupling rows first and the near-field rows after,
    // each part in the list's own order, and (split list) the row sums
    // ordered the same way -- the near field can then run as a launch of its
    // own (H2_SCHEDULE_STREAMED)
    const h2::RowDesc *srows = nullptr;
    int64_t nsrows_coupling = 0;
    const h2::ReduceDesc *sred = nullptr;
    int64_t nsred_coupling = 0;
    std::vector<int64_t> near_cum;   // blocks of the near-field rows of srows, cumulative (size rows + 1)
};

// A single-vector stream list with fewer block rows than this is split into
// chunks: one wavefront per row would leave most of the machine idle.
constexpr int64_t kSplitRows = 4096;
constexpr int64_t kSplitWaves = 4096;   // target number of chunks (about 16 per CU)

// ---------------------------------------------------------------- batches
// Many H^2 matrices of uneven size and rank per launch: the members' tile
// lists are concatenated per "level slot" -- upsweep lists aligned by their
// distance from the leaves, downsweep lists aligned at their end (the leaf
// level), one streaming slot and one leaf slot -- so every slot is one
// grid-strided launch over all members.  Tiles of all members live in one
// pool; block operands are absolute addresses into the members' storage.
struct BatchSlot {
    Phase phase;
    int kind;
    h2::RowDesc *rows;
    int64_t nrows;
    h2::BlkDesc *blks;
    int32_t *items;
    int64_t nitems;
    int32_t *pitems;
    int64_t npitems;
};

}  // namespace h2i

// The matrix behind an h2_handle: its structure, device storage and work lists.
struct h2_matrix_ {
    h2::Structure st;
    int storage = H2_FP64;
    bool structure_only = false;
    int basis_kind = h2::ELEM_F64, block_kind = h2::ELEM_F64;
    bool vec_f64 = true;
    h2i::DeviceArena mem;
    void *basis = nullptr, *blocks = nullptr;
    float *scales = nullptr;
    void *xh = nullptr, *yh = nullptr, *ynear = nullptr;
    std::vector<h2i::WorkList> lists;      // single right-hand side (vector offsets)
    std::vector<h2i::WorkList> mm_lists;   // tiles of MM_TILE right-hand sides (tile offsets)
    std::vector<std::vector<h2::RowDesc>> mm_host_rows;   // host copies of mm_lists (for batches)
    std::vector<std::vector<h2::BlkDesc>> mm_host_blks;
    int64_t nscales = 0;
    int64_t tile_slot = 0;            // elements per leaf in point tiles
    int64_t *d_leaf_begin = nullptr, *d_leaf_end = nullptr;
    float *t_xh = nullptr, *t_yh = nullptr, *t_x = nullptr, *t_ynear = nullptr;   // tile workspace (lazy)
    // block loop chosen at the first pass of each tile width (32, or 16 for
    // passes of at most 16 right-hand sides)
    h2::MmConfig mm_cfg[2] = {{1, 0, 0}, {1, 0, 0}};
    bool mm_tuned[2] = {false, false};
    double mm_tuned_ms[2] = {0.0, 0.0};   // timed choice's pass time (0: from the cache)
    int64_t bytes_coupling = 0, bytes_dense = 0, bytes_leaf = 0, bytes_transfer = 0;
    // layout: element offsets of U_j, V_j^T (per leaf), E_c, F_c^T (per node,
    // -1 where not stored) in basis, and of every block in blocks (coupling
    // blocks level by level in BSR order, then dense blocks)
    std::vector<int64_t> off_U, off_VT, off_E, off_FT, off_blk;
    int64_t basis_elems = 0, block_elems = 0;   // lengths of the two regions
    bool symmetric = true;                      // V = U and F = E
    // stored by halves (H2_HALF_STORAGE): only blocks with column >= row; for
    // every block of the full BSR lists (coupling levels, then dense) its
    // index in off_blk, or -(index + 1) of the stored block it mirrors
    bool half = false;
    std::vector<int64_t> blk_store;
    int batch_refs = 0;                         // batches holding addresses into this matrix
    // schedule of the single-vector product (h2_set_schedule): the near field
    // on the handle's second stream, its launch's LDS request (caps its
    // workgroups per compute unit; 0: no cap) and the share of its rows
    // launched at the start of the product (the rest follows the coupling launch)
    int schedule = H2_SCHEDULE_MERGED;
    int near_wg_per_cu = 0;
    int near_lds_bytes = 0;
    double near_early = 1.0;
    hipStream_t aux = nullptr;
    hipEvent_t ev_fork = nullptr, ev_mid = nullptr, ev_join = nullptr;
    // profiling: PH_COUNT + 1 events per recorded call
    bool prof = false;
    std::vector<hipEvent_t> pending, spare;
    double prof_ms[8] = {0};
    int64_t prof_calls = 0;

    ~h2_matrix_() {
        for (hipEvent_t e : pending) (void)hipEventDestroy(e);
        for (hipEvent_t e : spare) (void)hipEventDestroy(e);
        for (hipEvent_t e : {ev_fork, ev_mid, ev_join})
            if (e) (void)hipEventDestroy(e);
        if (aux) (void)hipStreamDestroy(aux);
    }
};

// A batch of matrices behind an h2_batch: one launch per level slot.
struct h2_batch_ {
    std::vector<h2_matrix_ *> mats;
    int nrhs = 0;
    h2i::DeviceArena mem;
    float *pool = nullptr;
    float *scales = nullptr;
    std::vector<h2i::BatchSlot> slots;
    h2::PackEntry *pack = nullptr;
    int64_t npack = 0;
    double **d_Xtab = nullptr, **d_Ytab = nullptr;
    int64_t *d_ldx = nullptr, *d_ldy = nullptr;
    hipStream_t own = nullptr;
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    // pinned host copy of the per-call tables (X, Y pointers, ldx, ldy), and
    // the event after their upload: the next call waits for it before rewriting
    int64_t *h_tables = nullptr;
    hipEvent_t ev_tables = nullptr;
    bool tables_pending = false;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    h2::MmConfig cfg{1, 0, 0};
    bool tuned = false;
    double tuned_ms = 0.0;
    std::string signature;
    int64_t cu_count = 256;
    bool counted = false;   // the members' batch_refs include this batch

    ~h2_batch_() {
        if (counted)
            for (h2_matrix_ *m : mats) --m->batch_refs;
        if (ev_tables) {
            if (tables_pending) (void)hipEventSynchronize(ev_tables);
            (void)hipEventDestroy(ev_tables);
        }
        if (h_tables) (void)hipHostFree(h_tables);
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (ev_in) (void)hipEventDestroy(ev_in);
        if (ev_out) (void)hipEventDestroy(ev_out);
        if (own) (void)hipStreamDestroy(own);
    }
};

namespace h2i {

// h2_build.cpp
std::vector<int32_t> wave_items(const std::vector<h2::RowDesc> &rows, const std::vector<h2::BlkDesc> &blks);
std::vector<int32_t> pair_items(const std::vector<h2::RowDesc> &rows, const std::vector<h2::BlkDesc> &blks);
void convert_block(const double *src, int R, int C, bool transpose, int kind, void *dst, float *scale);
std::vector<h2::FillDesc> make_layout(h2_matrix_ &A, int64_t &ncoupling);
void build_device(h2_matrix_ &A, const h2_arrays *src, hipStream_t stream);
void build_lists(h2_matrix_ &A, const std::vector<h2::FillDesc> &fill, int64_t ncoupling, hipStream_t stream);
void validate_params(const double *points, int64_t n, const h2_params *prm);
void structure_from_arrays(const h2_arrays *a, h2::Structure &s);
void export_arrays(h2_matrix_ &A, const h2_arrays_out *o, hipStream_t st);

// h2_run.cpp
// Intermediate vectors of one single-vector product: the trees x^ and y^, the
// near field, and the partial sums of a split or half-storage stream list.
struct Workspace {
    void *xh, *yh, *ynear, *partials;
};
// Bytes of each part (rounded up to 256), in the order above; the sum is the
// whole.
void workspace_bytes(const h2_matrix_ &A, int64_t part[4]);
// Enqueues the whole single-vector product on st, in the handle's own
// workspace, or in ws (then without profiling events).
void run_product(h2_matrix_ &A, const double *x, double *y, hipStream_t st, const Workspace *ws = nullptr);
void run_tile_pass(h2_matrix_ &A, const double *X, int64_t ldx, double *Y, int64_t ldy, int nrhs, int j0,
                   const h2::MmConfig &cfg, hipStream_t st);
void run_tiles(h2_matrix_ &A, const double *X, int64_t ldx, double *Y, int64_t ldy, int nrhs, hipStream_t st);

// h2_batch.cpp
// Chooses the block loop (pipelined or not) for this matrix and the tile
// width of pass j0 by timing both on that pass, unless cached.
void tune_tiles(h2_matrix_ &A, const double *X, int64_t ldx, double *Y, int64_t ldy, int nrhs, int j0,
                hipStream_t st);

// h2_transform.cpp
void orthogonalize(h2_matrix_ &A, hipStream_t st);
h2_matrix_ *transpose_matrix(h2_matrix_ &A, hipStream_t st);
void compress(h2_matrix_ &A, double eps, hipStream_t st, int *ranks_out);

}  // namespace h2i
