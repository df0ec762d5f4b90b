// C ABI of libh2mv (include/h2mv.h): the error message, the handle's
// release and its queries.  Construction, products, batches and
// transformations sit in h2_build.cpp, h2_run.cpp, h2_batch.cpp and
// h2_transform.cpp.
#include "h2_internal.h"

namespace h2i {

thread_local std::string g_last_error;

}  // namespace h2i

using namespace h2i;

extern "C" {

const char *h2_last_error(void) { return g_last_error.c_str(); }

void h2_free(h2_handle A) { delete A; }

h2_status h2_get_info(h2_handle A, h2_info *info) {
    if (!A || !info) {
        g_last_error = "NULL argument";
        return H2_ERR_INVALID_ARG;
    }
    const h2::Structure &s = A->st;
    h2_info r;
    std::memset(&r, 0, sizeof(r));
    r.n = s.n;
    r.dim = s.dim;
    r.leaf_size = s.leaf;
    r.cheb_p = s.cheb_p;
    r.rank = s.rank;
    r.levels_q = s.q;
    r.lmin = s.lmin;
    r.storage = A->storage | (A->half ? H2_HALF_STORAGE : 0);
    r.nnodes = s.nnodes;
    for (const auto &B : s.coupling) r.coupling_blocks += B.blocks();
    r.dense_blocks = s.dense.blocks();
    r.bytes_coupling = A->bytes_coupling;
    r.bytes_dense = A->bytes_dense;
    r.bytes_leaf_bases = A->bytes_leaf;
    r.bytes_transfers = A->bytes_transfer;
    r.bytes_device_total = A->mem.bytes;
    r.near_ties = s.near_ties;
    if (A->half)
        for (const WorkList &w : A->lists)
            if (w.slot) r.partial_slots += w.partials_bytes / (64 * (A->vec_f64 ? 8 : 4));
    *info = r;
    return H2_OK;
}

h2_status h2_get_perm(h2_handle A, int64_t *perm) {
    if (!A || !perm) {
        g_last_error = "NULL argument";
        return H2_ERR_INVALID_ARG;
    }
    if (!A->st.perm.empty()) std::memcpy(perm, A->st.perm.data(), A->st.perm.size() * sizeof(int64_t));
    return H2_OK;
}

h2_status h2_get_level_bsr(h2_handle A, int level, int64_t *count, int32_t *rowptr, int32_t *colidx) {
    if (!A || !count || level < -1 || level > A->st.q) {
        g_last_error = "bad argument";
        return H2_ERR_INVALID_ARG;
    }
    const h2::Bsr &B = level < 0 ? A->st.dense : A->st.coupling[level];
    *count = B.blocks();
    // (empty vectors may hand out a null data(), which memcpy must not get)
    if (rowptr && !B.rowptr.empty()) std::memcpy(rowptr, B.rowptr.data(), B.rowptr.size() * sizeof(int32_t));
    if (colidx && !B.colidx.empty()) std::memcpy(colidx, B.colidx.data(), B.colidx.size() * sizeof(int32_t));
    return H2_OK;
}

h2_status h2_read_probe(const void *buf, int64_t bytes, int grid, void *sink, void *stream) {
    try {
        if (!buf || !sink) fail(H2_ERR_INVALID_ARG, "NULL argument");
        if (bytes < 16 || bytes % 16 != 0) fail(H2_ERR_INVALID_ARG, "bytes must be a positive multiple of 16");
        if (grid < 1 || grid > 65536) fail(H2_ERR_INVALID_ARG, "grid must be in [1, 65536]");
        check_hip(h2::launch_read_probe(buf, bytes, grid, sink, static_cast<hipStream_t>(stream)), "read probe");
        return H2_OK;
    } catch (const Failure &f) {
        g_last_error = f.what;
        return f.code;
    }
}

}  // extern "C"
