// Batches of H^2 matrices of uneven size and rank, one launch per level
// slot, and the timing that picks the block loop of the tile products.
#include "h2_internal.h"

namespace h2i {

namespace {

struct BatchConfigCache {
    std::mutex mu;   // handles may be tuned from several host threads
    std::vector<std::pair<std::string, h2::MmConfig>> entries;
};
BatchConfigCache &config_cache() {
    static BatchConfigCache c;
    return c;
}

// Enqueues one batched product (tables already set) with configuration cfg.
void batch_enqueue(h2_batch_ &B, const h2::MmConfig &cfg, hipStream_t st) {
    check_hip(h2::launch_batch_pack(B.pack, B.npack, B.d_Xtab, B.d_ldx, B.nrhs, B.pool,
                                    cfg.grid > 0 ? cfg.grid : 0, st),
              "batch pack");
    for (const BatchSlot &sl : B.slots) {
        h2::MmBatchLaunch L{sl.rows, sl.items, sl.nitems, sl.pitems, sl.npitems, sl.blks, B.scales, B.pool,
                            B.d_Ytab, B.d_ldy, B.nrhs};
        check_hip(h2::launch_mm_batch(L, sl.kind, int(sl.phase), cfg, st), "batch launch");
    }
}

std::string config_file() {
    const char *p = std::getenv("H2MV_AUTOTUNE_CACHE");
    return p ? std::string(p) : std::string();
}

// The cache file holds one "signature pipelined grid tile_width" line per
// entry (a line without the tile width means 0: chosen by the pass width).
bool cached_config(const std::string &sig, h2::MmConfig &cfg) {
    std::lock_guard<std::mutex> lock(config_cache().mu);
    for (auto &e : config_cache().entries)
        if (e.first == sig) {
            cfg = e.second;
            return true;
        }
    const std::string f = config_file();
    if (f.empty()) return false;
    FILE *fp = std::fopen(f.c_str(), "r");
    if (!fp) return false;
    char line[512];
    bool found = false;
    while (std::fgets(line, sizeof line, fp)) {
        char key[400];
        int pipe = 0, nt = 0;
        long long grid = 0;
        const int got = std::sscanf(line, "%399s %d %lld %d", key, &pipe, &grid, &nt);
        if (got >= 3 && sig == key && pipe >= 0 && pipe <= h2::MM_MAX_PIPE && grid >= 0 &&
            (nt == 0 ? pipe < h2::MM_FIRST_PAIR : (nt == 16 || nt == 32) && h2::mm_pipe_fits(pipe, nt))) {
            cfg = {pipe, grid, got == 4 ? nt : 0};
            found = true;
        }
    }
    std::fclose(fp);
    if (found) config_cache().entries.push_back({sig, cfg});
    return found;
}

void store_config(const std::string &sig, const h2::MmConfig &cfg) {
    std::lock_guard<std::mutex> lock(config_cache().mu);
    config_cache().entries.push_back({sig, cfg});
    const std::string f = config_file();
    if (f.empty()) return;
    if (FILE *fp = std::fopen(f.c_str(), "a")) {
        std::fprintf(fp, "%s %d %lld %d\n", sig.c_str(), cfg.pipelined, static_cast<long long>(cfg.grid), cfg.nt);
        std::fclose(fp);
    }
}

// Launch shapes the tuners try: the block loop's prefetch depth (0 plain, 1
// the next block, 2 and 3 rings of block slots in registers, 4 and 5 rings
// with a row's halves sharing the input tile (32-wide tiles), 6 and 7 rings
// of 6 or 8 column chunks (16-wide tiles)), and for passes of at most 16
// right-hand sides the MFMA tile width (16: 16x16 MFMAs, half the matrix-core
// work and registers of 32, but every tile pads 8 right-hand sides to 16;
// 32: 32x32 MFMAs).  Depth 3 with 32-wide tiles runs one wavefront per SIMD.
constexpr int kDepths = h2::MM_MAX_PIPE + 1;   // each with the tile widths h2::mm_pipe_fits allows

std::vector<int> tile_widths(int ncols) {
    return ncols <= 16 ? std::vector<int>{16, 32} : std::vector<int>{32};
}

// Times every candidate configuration on the batch (tables set) and keeps the
// fastest: prefetch depth x tile width x grid (persistent grids of 1, 2 and 4
// workgroups per compute unit, or one workgroup per two rows).
void batch_autotune(h2_batch_ &B) {
    h2::MmConfig best{1, 0, 0};
    if (cached_config(B.signature, best)) {
        B.cfg = best;
        B.tuned = true;
        return;
    }
    hipEvent_t t0, t1;
    check_hip(hipEventCreate(&t0), "hipEventCreate");
    check_hip(hipEventCreate(&t1), "hipEventCreate");
    double best_ms = 1e30;
    const int64_t cu = (B.cu_count + h2::MM_XCDS - 1) / h2::MM_XCDS * h2::MM_XCDS;
    const int64_t grids[4] = {0, cu, 2 * cu, 4 * cu};
    for (int nt : tile_widths(B.nrhs))
        for (int pipe = 0; pipe < kDepths; ++pipe)
            for (int64_t grid : grids) {
                if (!h2::mm_pipe_fits(pipe, nt)) continue;
                const h2::MmConfig c{pipe, grid, nt};
                batch_enqueue(B, c, B.own);   // warm-up
                float ms_best = 1e30f;
                for (int rep = 0; rep < 2; ++rep) {
                    check_hip(hipEventRecord(t0, B.own), "hipEventRecord");
                    batch_enqueue(B, c, B.own);
                    check_hip(hipEventRecord(t1, B.own), "hipEventRecord");
                    check_hip(hipEventSynchronize(t1), "hipEventSynchronize");
                    float ms = 0.0f;
                    check_hip(hipEventElapsedTime(&ms, t0, t1), "hipEventElapsedTime");
                    ms_best = std::min(ms_best, ms);
                }
                if (ms_best < best_ms) {
                    best_ms = ms_best;
                    best = c;
                }
            }
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    B.cfg = best;
    B.tuned = true;
    B.tuned_ms = best_ms;
    store_config(B.signature, best);
}

void build_batch(h2_batch_ &B, hipStream_t stream) {
    const int nm = int(B.mats.size());
    const int kind_basis = B.mats[0]->basis_kind, kind_block = B.mats[0]->block_kind;
    for (h2_matrix_ *M : B.mats) {
        if (M->structure_only) fail(H2_ERR_INVALID_ARG, "structure-only member");
        if (M->storage == H2_FP64) fail(H2_ERR_UNSUPPORTED, "batches need FP32 or BF16 storage");
        if (M->half) fail(H2_ERR_UNSUPPORTED, "batch member stored by halves");
        if (M->basis_kind != kind_basis || M->block_kind != kind_block)
            fail(H2_ERR_UNSUPPORTED, "all batch members need the same storage");
    }
    // pool layout and scale concatenation
    std::vector<int64_t> xh(nm), yh(nm), xp(nm), yn(nm), sb(nm);
    int64_t pool = 0, nsc = 0;
    for (int b = 0; b < nm; ++b) {
        const h2_matrix_ &M = *B.mats[b];
        const int64_t kp = (M.st.rank + 15) / 16 * 16;
        const int64_t tree = M.st.nnodes * kp * h2::MM_TILE, pts = (int64_t(1) << M.st.q) * M.tile_slot;
        xh[b] = pool; pool += tree;
        yh[b] = pool; pool += tree;
        xp[b] = pool; pool += pts;
        yn[b] = pool; pool += pts;
        sb[b] = nsc; nsc += M.nscales;
    }
    B.pool = static_cast<float *>(B.mem.alloc(pool * 4));
    B.scales = static_cast<float *>(B.mem.alloc(std::max<int64_t>(1, nsc) * 4));
    for (int b = 0; b < nm; ++b)
        if (B.mats[b]->nscales > 0)
            check_hip(hipMemcpyAsync(B.scales + sb[b], B.mats[b]->scales, B.mats[b]->nscales * 4,
                                     hipMemcpyDeviceToDevice, stream),
                      "copy scales");
    // per-member list indices by phase
    std::vector<std::vector<int>> up(nm), down(nm);
    std::vector<int> strm(nm, -1), leaf(nm, -1);
    size_t nu = 0, nd = 0;
    for (int b = 0; b < nm; ++b) {
        const auto &L = B.mats[b]->mm_lists;
        for (int li = 0; li < int(L.size()); ++li) {
            if (L[li].phase == PH_UP) up[b].push_back(li);
            if (L[li].phase == PH_DOWN) down[b].push_back(li);
            if (L[li].phase == PH_STREAM) strm[b] = li;
            if (L[li].phase == PH_LEAF) leaf[b] = li;
        }
        nu = std::max(nu, up[b].size());
        nd = std::max(nd, down[b].size());
    }
    // translates member b's list li into the slot's rows/blocks
    auto append = [&](int b, int li, std::vector<h2::RowDesc> &rows, std::vector<h2::BlkDesc> &blks) {
        const h2_matrix_ &M = *B.mats[b];
        const WorkList &w = M.mm_lists[li];
        const int64_t es = h2::elem_bytes(w.kind);
        const int64_t base = int64_t(reinterpret_cast<uintptr_t>(w.data));
        const auto &hr = M.mm_host_rows[li];
        const auto &hb = M.mm_host_blks[li];
        for (const h2::RowDesc &r0 : hr) {
            h2::RowDesc r = r0;
            const bool in_x = (r.sel & h2::ROW_IN_X) != 0, out_p = (r.sel & h2::ROW_OUT_P) != 0;
            int64_t in_base = 0;
            switch (w.phase) {
                case PH_UP:
                    r.out += xh[b];
                    in_base = in_x ? xp[b] : xh[b];
                    break;
                case PH_STREAM:
                    r.out += out_p ? yn[b] : yh[b];
                    in_base = in_x ? xp[b] : xh[b];
                    break;
                case PH_DOWN:
                    r.out += yh[b];
                    if (r.init >= 0) r.init += yh[b];
                    in_base = yh[b];
                    break;
                default:
                    r.init += yn[b];
                    r.sel |= b << 8;
                    in_base = yh[b];
                    break;
            }
            const int32_t b0 = int32_t(blks.size());
            for (int32_t k = r0.b0; k < r0.b1; ++k) {
                h2::BlkDesc d = hb[k];
                d.a = base + d.a * es;
                d.in += in_base;
                d.sidx += int32_t(sb[b]);
                blks.push_back(d);
            }
            r.b0 = b0;
            r.b1 = int32_t(blks.size());
            rows.push_back(r);
        }
    };
    auto add_slot = [&](Phase ph, int kind, std::vector<h2::RowDesc> &rows, std::vector<h2::BlkDesc> &blks) {
        if (rows.empty()) return;
        const std::vector<int32_t> it = wave_items(rows, blks), pit = pair_items(rows, blks);
        BatchSlot sl{ph, kind, B.mem.upload(rows, stream), int64_t(rows.size()), B.mem.upload(blks, stream),
                     B.mem.upload(it, stream), int64_t(it.size()), B.mem.upload(pit, stream),
                     int64_t(pit.size())};
        B.slots.push_back(sl);
    };
    std::vector<h2::RowDesc> rows;
    std::vector<h2::BlkDesc> blks;
    for (size_t j = 0; j < nu; ++j) {
        rows.clear(); blks.clear();
        for (int b = 0; b < nm; ++b)
            if (j < up[b].size()) append(b, up[b][j], rows, blks);
        add_slot(PH_UP, kind_basis, rows, blks);
    }
    rows.clear(); blks.clear();
    for (int b = 0; b < nm; ++b) append(b, strm[b], rows, blks);
    add_slot(PH_STREAM, kind_block, rows, blks);
    for (size_t j = 0; j < nd; ++j) {
        rows.clear(); blks.clear();
        for (int b = 0; b < nm; ++b) {
            const int64_t k = int64_t(j) - int64_t(nd - down[b].size());
            if (k >= 0) append(b, down[b][k], rows, blks);
        }
        add_slot(PH_DOWN, kind_basis, rows, blks);
    }
    rows.clear(); blks.clear();
    for (int b = 0; b < nm; ++b) append(b, leaf[b], rows, blks);
    add_slot(PH_LEAF, kind_basis, rows, blks);
    // point-tile pack entries
    std::vector<h2::PackEntry> pe;
    int64_t total_rows = 0, total_blocks = 0;
    for (int b = 0; b < nm; ++b) {
        const h2_matrix_ &M = *B.mats[b];
        const int64_t nl = int64_t(1) << M.st.q, lf = Structure::first(M.st.q);
        for (int64_t j = 0; j < nl; ++j)
            pe.push_back({xp[b] + j * M.tile_slot, M.st.begin[lf + j], int32_t(M.st.size(lf + j)), b});
    }
    for (const BatchSlot &sl : B.slots) total_rows += sl.nrows;
    for (h2_matrix_ *M : B.mats)
        for (const auto &hb : M->mm_host_blks) total_blocks += int64_t(hb.size());
    B.pack = B.mem.upload(pe, stream);
    B.npack = int64_t(pe.size());
    B.d_Xtab = static_cast<double **>(B.mem.alloc(nm * 8));
    B.d_Ytab = static_cast<double **>(B.mem.alloc(nm * 8));
    B.d_ldx = static_cast<int64_t *>(B.mem.alloc(nm * 8));
    B.d_ldy = static_cast<int64_t *>(B.mem.alloc(nm * 8));
    int dev = 0, cus = 256;
    check_hip(hipGetDevice(&dev), "hipGetDevice");
    check_hip(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev), "device attribute");
    B.cu_count = cus;
    B.signature = "batch-k" + std::to_string(kind_block) + "-r" + std::to_string(B.nrhs) + "-m" + std::to_string(nm) +
                  "-rows" + std::to_string(total_rows) + "-blocks" + std::to_string(total_blocks) + "-cu" +
                  std::to_string(cus);
    check_hip(hipStreamCreateWithFlags(&B.own, hipStreamNonBlocking), "hipStreamCreate");
    check_hip(hipEventCreateWithFlags(&B.ev_in, hipEventDisableTiming), "hipEventCreate");
    check_hip(hipEventCreateWithFlags(&B.ev_out, hipEventDisableTiming), "hipEventCreate");
    check_hip(hipEventCreateWithFlags(&B.ev_tables, hipEventDisableTiming), "hipEventCreate");
    check_hip(hipHostMalloc(reinterpret_cast<void **>(&B.h_tables), size_t(4 * nm) * 8, hipHostMallocDefault),
              "hipHostMalloc");
    check_hip(hipStreamSynchronize(stream), "batch build");
}

}  // namespace

void tune_tiles(h2_matrix_ &A, const double *X, int64_t ldx, double *Y, int64_t ldy, int nrhs, int j0,
                hipStream_t st) {
    const int ncols = std::min(h2::MM_TILE, nrhs - j0);
    const int w = ncols <= 16 ? 1 : 0;
    int64_t nblocks = 0;
    for (const auto &hb : A.mm_host_blks) nblocks += int64_t(hb.size());
    const std::string sig = "single-k" + std::to_string(A.block_kind) + "-n" + std::to_string(A.st.n) + "-r" +
                            std::to_string(A.st.rank) + "-blocks" + std::to_string(nblocks) + "-nt" +
                            std::to_string(w ? 16 : 32);
    h2::MmConfig best{1, 0, 0};
    double best_ms = 0.0;
    if (!cached_config(sig, best)) {
        const bool prof = A.prof;   // tuning runs stay out of the profile
        A.prof = false;
        hipEvent_t t0, t1;
        check_hip(hipEventCreate(&t0), "hipEventCreate");
        check_hip(hipEventCreate(&t1), "hipEventCreate");
        float bms = 1e30f;
        int dev = 0, cus = 256;
        check_hip(hipGetDevice(&dev), "hipGetDevice");
        check_hip(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev), "device attribute");
        const int64_t cu = (cus + h2::MM_XCDS - 1) / h2::MM_XCDS * h2::MM_XCDS;
        for (int nt : tile_widths(ncols))
            for (int pipe = 0; pipe < kDepths; ++pipe)
                for (int64_t grid : {int64_t(0), cu, 2 * cu}) {
                    if (!h2::mm_pipe_fits(pipe, nt)) continue;
                    const h2::MmConfig c{pipe, grid, nt};
                    run_tile_pass(A, X, ldx, Y, ldy, nrhs, j0, c, st);   // warm-up
                    check_hip(hipEventRecord(t0, st), "hipEventRecord");
                    run_tile_pass(A, X, ldx, Y, ldy, nrhs, j0, c, st);
                    check_hip(hipEventRecord(t1, st), "hipEventRecord");
                    check_hip(hipEventSynchronize(t1), "hipEventSynchronize");
                    float ms = 0.0f;
                    check_hip(hipEventElapsedTime(&ms, t0, t1), "hipEventElapsedTime");
                    if (ms < bms) {
                        bms = ms;
                        best = c;
                    }
                }
        (void)hipEventDestroy(t0);
        (void)hipEventDestroy(t1);
        A.prof = prof;
        best_ms = bms;
        store_config(sig, best);
    }
    A.mm_cfg[w] = best;
    A.mm_tuned[w] = true;
    A.mm_tuned_ms[w] = best_ms;
}

}  // namespace h2i

using namespace h2i;

extern "C" {

h2_status h2_batch_create(const h2_handle *mats, int count, int nrhs, void *stream, h2_batch *out) {
    if (out) *out = nullptr;
    h2_batch_ *B = nullptr;
    try {
        if (!out || !mats || count < 1) fail(H2_ERR_INVALID_ARG, "NULL argument or count < 1");
        if (nrhs < 1) fail(H2_ERR_INVALID_ARG, "nrhs must be >= 1");
        if (nrhs > h2::MM_TILE) fail(H2_ERR_UNSUPPORTED, "batches take at most 32 right-hand sides");
        B = new h2_batch_();
        for (int b = 0; b < count; ++b) {
            if (!mats[b]) fail(H2_ERR_INVALID_ARG, "NULL member");
            B->mats.push_back(mats[b]);
        }
        B->nrhs = nrhs;
        build_batch(*B, static_cast<hipStream_t>(stream));
        for (h2_matrix_ *m : B->mats) ++m->batch_refs;
        B->counted = true;
        *out = B;
        return H2_OK;
    } catch (const Failure &f) {
        delete B;
        g_last_error = f.what;
        return f.code;
    } catch (const std::bad_alloc &) {
        delete B;
        g_last_error = "host allocation failed";
        return H2_ERR_OOM;
    } catch (...) {
        delete B;
        g_last_error = "internal error";
        return H2_ERR_INTERNAL;
    }
}

h2_status h2_batch_matmat(h2_batch B, const double *const *X, const int64_t *ldx, double *const *Y,
                          const int64_t *ldy, void *stream) {
    try {
        if (!B || !X || !ldx || !Y || !ldy) fail(H2_ERR_INVALID_ARG, "NULL argument");
        const int nm = int(B->mats.size());
        for (int b = 0; b < nm; ++b) {
            if (!X[b] || !Y[b]) fail(H2_ERR_INVALID_ARG, "NULL member matrix");
            if (ldx[b] < B->mats[b]->st.n || ldy[b] < B->mats[b]->st.n)
                fail(H2_ERR_INVALID_ARG, "leading dimension below n");
        }
        // pointer tables: written to pinned memory (after the previous call's upload
        // of them has run) and uploaded outside the graph
        if (B->tables_pending) check_hip(hipEventSynchronize(B->ev_tables), "hipEventSynchronize");
        int64_t *tab = B->h_tables;
        for (int b = 0; b < nm; ++b) {
            tab[b] = int64_t(reinterpret_cast<uintptr_t>(X[b]));
            tab[nm + b] = int64_t(reinterpret_cast<uintptr_t>(Y[b]));
            tab[2 * nm + b] = ldx[b];
            tab[3 * nm + b] = ldy[b];
        }
        const hipStream_t user = static_cast<hipStream_t>(stream);
        check_hip(hipEventRecord(B->ev_in, user), "hipEventRecord");
        check_hip(hipStreamWaitEvent(B->own, B->ev_in, 0), "hipStreamWaitEvent");
        check_hip(hipMemcpyAsync(B->d_Xtab, tab, nm * 8, hipMemcpyHostToDevice, B->own), "copy tables");
        check_hip(hipMemcpyAsync(B->d_Ytab, tab + nm, nm * 8, hipMemcpyHostToDevice, B->own), "copy tables");
        check_hip(hipMemcpyAsync(B->d_ldx, tab + 2 * nm, nm * 8, hipMemcpyHostToDevice, B->own), "copy tables");
        check_hip(hipMemcpyAsync(B->d_ldy, tab + 3 * nm, nm * 8, hipMemcpyHostToDevice, B->own), "copy tables");
        check_hip(hipEventRecord(B->ev_tables, B->own), "hipEventRecord");
        B->tables_pending = true;
        if (!B->tuned) batch_autotune(*B);
        if (!B->exec) {
            check_hip(hipStreamBeginCapture(B->own, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
            try {
                batch_enqueue(*B, B->cfg, B->own);
            } catch (...) {
                hipGraph_t aborted = nullptr;   // leave the stream out of capture mode
                (void)hipStreamEndCapture(B->own, &aborted);
                if (aborted) (void)hipGraphDestroy(aborted);
                throw;
            }
            check_hip(hipStreamEndCapture(B->own, &B->graph), "hipStreamEndCapture");
            check_hip(hipGraphInstantiate(&B->exec, B->graph, nullptr, nullptr, 0), "hipGraphInstantiate");
        }
        check_hip(hipGraphLaunch(B->exec, B->own), "hipGraphLaunch");
        check_hip(hipEventRecord(B->ev_out, B->own), "hipEventRecord");
        check_hip(hipStreamWaitEvent(user, B->ev_out, 0), "hipStreamWaitEvent");
        return H2_OK;
    } catch (const Failure &f) {
        g_last_error = f.what;
        return f.code;
    } catch (...) {
        g_last_error = "internal error";
        return H2_ERR_INTERNAL;
    }
}

h2_status h2_batch_tuning(h2_batch B, int *pipelined, int64_t *grid, int *tile_width, double *tuned_ms) {
    if (!B || !pipelined || !grid || !tile_width || !tuned_ms) {
        g_last_error = "NULL argument";
        return H2_ERR_INVALID_ARG;
    }
    *pipelined = B->cfg.pipelined;
    *grid = B->cfg.grid;
    *tile_width = B->cfg.nt ? B->cfg.nt : (B->nrhs <= 16 ? 16 : 32);
    *tuned_ms = B->tuned ? B->tuned_ms : -1.0;
    return H2_OK;
}

h2_status h2_batch_set_tuning(h2_batch B, int pipelined, int64_t grid, int tile_width) {
    try {
        if (!B) fail(H2_ERR_INVALID_ARG, "NULL batch");
        if (pipelined < 0 || pipelined > h2::MM_MAX_PIPE) fail(H2_ERR_INVALID_ARG, "pipelined must be 0 .. 7");
        if (!h2::mm_pipe_fits(pipelined, tile_width))
            fail(H2_ERR_INVALID_ARG, "pipelined 4, 5 need 32-wide tiles, 6, 7 16-wide tiles");
        if (grid < 0) fail(H2_ERR_INVALID_ARG, "grid must be >= 0");
        if (tile_width != 16 && tile_width != 32) fail(H2_ERR_INVALID_ARG, "tile_width must be 16 or 32");
        if (tile_width == 16 && B->nrhs > 16) fail(H2_ERR_INVALID_ARG, "16-wide tiles take at most 16 right-hand sides");
        // the captured graph holds the old launches: drop it (the next
        // product captures again); wait for products that may still replay it
        check_hip(hipStreamSynchronize(B->own), "hipStreamSynchronize");
        if (B->exec) (void)hipGraphExecDestroy(B->exec);
        if (B->graph) (void)hipGraphDestroy(B->graph);
        B->exec = nullptr;
        B->graph = nullptr;
        B->cfg = {pipelined, grid, tile_width};
        B->tuned = true;
        B->tuned_ms = 0.0;
        return H2_OK;
    } catch (const Failure &f) {
        g_last_error = f.what;
        return f.code;
    } catch (...) {
        g_last_error = "internal error";
        return H2_ERR_INTERNAL;
    }
}

h2_status h2_matmat_tuning(h2_handle A, int narrow, int *pipelined, int64_t *grid, int *tile_width,
                           double *tuned_ms) {
    if (!A || !pipelined || !grid || !tile_width || !tuned_ms || (narrow != 0 && narrow != 1)) {
        g_last_error = "NULL argument or narrow not 0 / 1";
        return H2_ERR_INVALID_ARG;
    }
    const h2::MmConfig &c = A->mm_cfg[narrow];
    *pipelined = c.pipelined;
    *grid = c.grid;
    *tile_width = c.nt ? c.nt : (narrow ? 16 : 32);
    *tuned_ms = A->mm_tuned[narrow] ? A->mm_tuned_ms[narrow] : -1.0;
    return H2_OK;
}

h2_status h2_matmat_set_tuning(h2_handle A, int narrow, int pipelined, int64_t grid, int tile_width) {
    if (!A || (narrow != 0 && narrow != 1) || pipelined < 0 || pipelined > h2::MM_MAX_PIPE || grid < 0 ||
        (tile_width != 16 && tile_width != 32) || (tile_width == 16 && narrow == 0) ||
        !h2::mm_pipe_fits(pipelined, tile_width)) {
        g_last_error = "bad argument (narrow 0/1, pipelined 0..7 (4, 5 with 32-wide tiles, 6, 7 with 16-wide), "
                       "grid >= 0, tile_width 16 or 32, 16 only for narrow passes)";
        return H2_ERR_INVALID_ARG;
    }
    A->mm_cfg[narrow] = {pipelined, grid, tile_width};
    A->mm_tuned[narrow] = true;
    A->mm_tuned_ms[narrow] = 0.0;
    return H2_OK;
}

void h2_batch_free(h2_batch B) { delete B; }

}  // extern "C"
