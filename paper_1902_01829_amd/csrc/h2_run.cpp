// The product: y = A x as a fixed sequence of block-row launches over the
// work lists built at construction (the per-call marshaling of pointer
// batches of Sec. 3.2 becomes static lists), and Y = A X in tiles of
// right-hand sides on the matrix cores.
#include "h2_internal.h"

namespace h2i {

namespace {

hipEvent_t take_event(h2_matrix_ &A) {
    if (!A.spare.empty()) {
        hipEvent_t e = A.spare.back();
        A.spare.pop_back();
        return e;
    }
    hipEvent_t e;
    check_hip(hipEventCreate(&e), "hipEventCreate");
    return e;
}

// Enqueues the lists in order, with profiling events at phase boundaries
// when enabled; launch(w) enqueues one list.
template <class Launch>
void run_lists(h2_matrix_ &A, const std::vector<WorkList> &lists, hipStream_t st, Launch launch,
               bool allow_prof = true) {
    const bool prof = A.prof && allow_prof;
    hipEvent_t ev[PH_COUNT + 1] = {};
    if (prof)
        for (auto &e : ev) e = take_event(A);
    int next_phase = 0;   // lists are in phase order; each phase's event precedes its lists
    for (const WorkList &w : lists) {
        while (prof && next_phase <= int(w.phase))
            check_hip(hipEventRecord(ev[next_phase++], st), "hipEventRecord");
        launch(w);
    }
    if (prof) {
        while (next_phase <= PH_COUNT) check_hip(hipEventRecord(ev[next_phase++], st), "hipEventRecord");
        A.pending.insert(A.pending.end(), ev, ev + PH_COUNT + 1);
    }
}

// Tile workspace of the many-right-hand-side product, allocated at first use.
void ensure_tiles(h2_matrix_ &A) {
    if (A.t_xh) return;
    const int64_t kp = (A.st.rank + 15) / 16 * 16;
    const int64_t tree = A.st.nnodes * kp * h2::MM_TILE, pts = (int64_t(1) << A.st.q) * A.tile_slot;
    A.t_xh = static_cast<float *>(A.mem.alloc(tree * 4));
    A.t_yh = static_cast<float *>(A.mem.alloc(tree * 4));
    A.t_x = static_cast<float *>(A.mem.alloc(pts * 4));
    A.t_ynear = static_cast<float *>(A.mem.alloc(pts * 4));
}

}  // namespace

void workspace_bytes(const h2_matrix_ &A, int64_t part[4]) {
    auto r256 = [](int64_t b) { return (b + 255) / 256 * 256; };
    const int64_t vb = A.vec_f64 ? 8 : 4;
    part[0] = part[1] = r256(A.st.nnodes * A.st.rank * vb);
    part[2] = r256(A.st.n * vb);
    part[3] = 0;
    for (const WorkList &w : A.lists) part[3] = std::max(part[3], r256(w.partials_bytes));
}

void run_product(h2_matrix_ &A, const double *x, double *y, hipStream_t st, const Workspace *ws) {
    const Workspace own{A.xh, A.yh, A.ynear, nullptr};
    const Workspace &W = ws ? *ws : own;
    auto row_launch = [&](const WorkList &w) {
        h2::RowLaunch L;
        L.rows = w.rows;
        L.nrows = w.nrows;
        L.blks = w.blks;
        L.data = w.data;
        L.scales = A.scales;
        L.in1 = x;
        L.init = nullptr;
        L.out1 = nullptr;
        return L;
    };
    // Streamed schedule: the near-field rows of the stream list run on the
    // handle's second stream, a share from the start of the product and the
    // rest after the coupling rows; the leaf phase waits for them.
    const WorkList *sl = nullptr;
    if (A.schedule == H2_SCHEDULE_STREAMED)
        for (const WorkList &w : A.lists)
            if (w.phase == PH_STREAM && w.srows) sl = &w;
    int64_t nnear = 0, near_split = 0;
    auto near_launch = [&](int64_t r0, int64_t r1) {
        if (r1 <= r0) return;
        h2::RowLaunch L = row_launch(*sl);
        L.rows = sl->srows + sl->nsrows_coupling + r0;
        L.nrows = r1 - r0;
        L.in0 = W.xh;
        L.out0 = W.yh;
        L.out1 = W.ynear;
        L.lds_bytes = A.near_lds_bytes;
        if (sl->red) {
            L.out0 = L.out1 = ws ? ws->partials : sl->partials;
            check_hip(h2::launch_blockrow(L, sl->kind, A.vec_f64, PH_STREAM, A.aux, 1), "near-field launch");
        } else {
            check_hip(h2::launch_blockrow(L, sl->kind, A.vec_f64, PH_STREAM, A.aux), "near-field launch");
        }
    };
    if (sl) {
        nnear = int64_t(sl->near_cum.size()) - 1;
        const int64_t target = std::llround(A.near_early * double(sl->near_cum.back()));
        near_split = std::lower_bound(sl->near_cum.begin(), sl->near_cum.end(), target) - sl->near_cum.begin();
        near_split = std::min(near_split, nnear);
        check_hip(hipEventRecord(A.ev_fork, st), "hipEventRecord");
        check_hip(hipStreamWaitEvent(A.aux, A.ev_fork, 0), "hipStreamWaitEvent");
        near_launch(0, near_split);
    }
    run_lists(A, A.lists, st, [&](const WorkList &w) {
        void *partials = ws ? ws->partials : w.partials;
        h2::RowLaunch L = row_launch(w);
        if (&w == sl) {
            // coupling rows here; the rest of the near field on the second stream
            L.rows = sl->srows;
            L.nrows = sl->nsrows_coupling;
            L.in0 = W.xh;
            L.out0 = W.yh;
            L.out1 = W.ynear;
            if (w.red) {
                L.out0 = L.out1 = partials;
                check_hip(h2::launch_blockrow(L, w.kind, A.vec_f64, int(w.phase), st, 1), "blockrow launch");
                check_hip(h2::launch_reduce_chunks(w.sred, w.nsred_coupling, partials, false, W.yh, W.ynear,
                                                   A.vec_f64, st),
                          "chunk sum launch");
            } else {
                check_hip(h2::launch_blockrow(L, w.kind, A.vec_f64, int(w.phase), st), "blockrow launch");
            }
            check_hip(hipEventRecord(A.ev_mid, st), "hipEventRecord");
            check_hip(hipStreamWaitEvent(A.aux, A.ev_mid, 0), "hipStreamWaitEvent");
            near_launch(near_split, nnear);
            if (w.red)
                check_hip(h2::launch_reduce_chunks(w.sred + w.nsred_coupling, w.nred - w.nsred_coupling, partials,
                                                   false, W.yh, W.ynear, A.vec_f64, A.aux),
                          "chunk sum launch");
            check_hip(hipEventRecord(A.ev_join, A.aux), "hipEventRecord");
            return;
        }
        if (sl && w.phase == PH_LEAF) check_hip(hipStreamWaitEvent(st, A.ev_join, 0), "hipStreamWaitEvent");
        switch (w.phase) {
            case PH_UP:
                L.in0 = W.xh;
                L.out0 = W.xh;
                break;
            case PH_STREAM:
                L.in0 = W.xh;
                L.out0 = W.yh;
                L.out1 = W.ynear;
                if (w.slot) {   // stored by halves: row sums and transposed partials, then their sums
                    check_hip(h2::launch_stream_half(L, w.groups, w.ngroups, w.slot, w.gslot, partials, w.kind,
                                                     A.vec_f64, st),
                              "half-storage stream launch");
                    check_hip(h2::launch_reduce_chunks(w.red, w.nred, partials, !A.vec_f64, W.yh, W.ynear, A.vec_f64,
                                                       st, true),
                              "partial sum launch");
                    return;
                }
                if (w.red) {   // chunks of a split list: partial sums, then their sums per row
                    L.out0 = L.out1 = partials;
                    check_hip(h2::launch_blockrow(L, w.kind, A.vec_f64, int(w.phase), st, 1), "blockrow launch");
                    check_hip(h2::launch_reduce_chunks(w.red, w.nred, partials, false, W.yh, W.ynear, A.vec_f64, st),
                              "chunk sum launch");
                    return;
                }
                break;
            case PH_DOWN:
                L.in0 = W.yh;
                L.init = W.yh;
                L.out0 = W.yh;
                break;
            default:
                L.in0 = W.yh;
                L.init = W.ynear;
                L.out0 = W.yh;
                L.out1 = y;
                break;
        }
        check_hip(h2::launch_blockrow(L, w.kind, A.vec_f64, int(w.phase), st), "blockrow launch");
    }, ws == nullptr);
}

// One pass of up to MM_TILE right-hand sides on the matrix cores.
void run_tile_pass(h2_matrix_ &A, const double *X, int64_t ldx, double *Y, int64_t ldy, int nrhs, int j0,
                   const h2::MmConfig &cfg, hipStream_t st) {
    const int64_t nleaves = int64_t(1) << A.st.q;
    {
        check_hip(h2::launch_pack(X, ldx, j0, nrhs, A.d_leaf_begin, A.d_leaf_end, nleaves, A.tile_slot, A.t_x, st),
                  "pack launch");
        run_lists(A, A.mm_lists, st, [&](const WorkList &w) {
            h2::MmLaunch L;
            L.rows = w.rows;
            L.items = w.items;
            L.nitems = w.nitems;
            L.pitems = w.pitems;
            L.npitems = w.npitems;
            L.blks = w.blks;
            L.data = w.data;
            L.scales = A.scales;
            L.in_tree = nullptr;
            L.in_pts = A.t_x;
            L.init = nullptr;
            L.out_tree = nullptr;
            L.out_pts = nullptr;
            L.Y = Y + int64_t(j0) * ldy;
            L.ldy = ldy;
            L.ncols = std::min(h2::MM_TILE, nrhs - j0);
            switch (w.phase) {
                case PH_UP:
                    L.in_tree = A.t_xh;
                    L.out_tree = A.t_xh;
                    break;
                case PH_STREAM:
                    L.in_tree = A.t_xh;
                    L.out_tree = A.t_yh;
                    L.out_pts = A.t_ynear;
                    break;
                case PH_DOWN:
                    L.in_tree = A.t_yh;
                    L.init = A.t_yh;
                    L.out_tree = A.t_yh;
                    break;
                default:
                    L.in_tree = A.t_yh;
                    L.init = A.t_ynear;
                    break;
            }
            check_hip(h2::launch_mm(L, w.kind, int(w.phase), cfg, st), "mfma launch");
        });
    }
}

// Y = A X on the matrix cores, MM_TILE right-hand sides per pass.
void run_tiles(h2_matrix_ &A, const double *X, int64_t ldx, double *Y, int64_t ldy, int nrhs, hipStream_t st) {
    ensure_tiles(A);
    for (int j0 = 0; j0 < nrhs; j0 += h2::MM_TILE) {
        const int w = std::min(h2::MM_TILE, nrhs - j0) <= 16 ? 1 : 0;
        if (!A.mm_tuned[w]) tune_tiles(A, X, ldx, Y, ldy, nrhs, j0, st);
        run_tile_pass(A, X, ldx, Y, ldy, nrhs, j0, A.mm_cfg[w], st);
    }
}

}  // namespace h2i

using namespace h2i;

extern "C" {

h2_status h2_matvec(h2_handle A, const double *x, double *y, void *stream) {
    try {
        if (!A || !x || !y) fail(H2_ERR_INVALID_ARG, "NULL argument");
        if (A->structure_only) fail(H2_ERR_INVALID_ARG, "structure-only handle");
        run_product(*A, x, y, static_cast<hipStream_t>(stream));
        return H2_OK;
    } catch (const Failure &f) {
        g_last_error = f.what;
        return f.code;
    } catch (...) {
        g_last_error = "internal error";
        return H2_ERR_INTERNAL;
    }
}

h2_status h2_matmat(h2_handle A, const double *X, int64_t ldx, double *Y, int64_t ldy, int nrhs,
                    void *stream) {
    try {
        if (!A || !X || !Y) fail(H2_ERR_INVALID_ARG, "NULL argument");
        if (A->structure_only) fail(H2_ERR_INVALID_ARG, "structure-only handle");
        if (nrhs < 1) fail(H2_ERR_INVALID_ARG, "nrhs must be >= 1");
        if (ldx < A->st.n || ldy < A->st.n) fail(H2_ERR_INVALID_ARG, "leading dimension below n");
        const hipStream_t st = static_cast<hipStream_t>(stream);
        if (A->storage == H2_FP64 || A->half) {
            // FP64 storage, or blocks stored by halves: one single-vector
            // product per column
            for (int j = 0; j < nrhs; ++j) run_product(*A, X + int64_t(j) * ldx, Y + int64_t(j) * ldy, st);
        } else {
            run_tiles(*A, X, ldx, Y, ldy, nrhs, st);
        }
        return H2_OK;
    } catch (const Failure &f) {
        g_last_error = f.what;
        return f.code;
    } catch (...) {
        g_last_error = "internal error";
        return H2_ERR_INTERNAL;
    }
}

h2_status h2_set_schedule(h2_handle A, int schedule, int near_wg_per_cu, double near_early) {
    try {
        if (!A) fail(H2_ERR_INVALID_ARG, "NULL handle");
        if (A->structure_only) fail(H2_ERR_INVALID_ARG, "structure-only handle");
        if (schedule != H2_SCHEDULE_MERGED && schedule != H2_SCHEDULE_STREAMED)
            fail(H2_ERR_INVALID_ARG, "unknown schedule");
        if (near_wg_per_cu < 0) fail(H2_ERR_INVALID_ARG, "near_wg_per_cu must be >= 0");
        if (!(near_early >= 0.0 && near_early <= 1.0)) fail(H2_ERR_INVALID_ARG, "near_early must be in [0, 1]");
        if (schedule == H2_SCHEDULE_MERGED) {
            A->schedule = schedule;
            return H2_OK;
        }
        if (A->half) fail(H2_ERR_UNSUPPORTED, "the streamed schedule needs full storage");
        int lds_bytes = 0;
        if (near_wg_per_cu > 0) {
            // LDS request above 1 / (cap + 1) of a compute unit's LDS: at most
            // cap of the launch's workgroups fit on one compute unit (the
            // block-row kernels' own LDS is at most 4 KiB; 1 KiB of slack per
            // workgroup for the allocation granularity)
            int dev = 0, lds_cu = 0, lds_wg = 0;
            check_hip(hipGetDevice(&dev), "hipGetDevice");
            check_hip(hipDeviceGetAttribute(&lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev),
                      "hipDeviceGetAttribute");
            check_hip(hipDeviceGetAttribute(&lds_wg, hipDeviceAttributeMaxSharedMemoryPerBlock, dev),
                      "hipDeviceGetAttribute");
            const int64_t own = 4096, pad = int64_t(lds_cu) / (near_wg_per_cu + 1) + 1;
            if (lds_cu <= 0 || pad + own > lds_wg || int64_t(near_wg_per_cu) * (pad + own + 1024) > lds_cu)
                fail(H2_ERR_UNSUPPORTED, "near_wg_per_cu = " + std::to_string(near_wg_per_cu) +
                                             " cannot be set through the LDS request on this device (" +
                                             std::to_string(lds_cu) + " bytes per compute unit, " +
                                             std::to_string(lds_wg) + " per workgroup)");
            lds_bytes = int(pad);
        }
        if (!A->aux) {
            hipStream_t s = nullptr;
            check_hip(hipStreamCreateWithFlags(&s, hipStreamNonBlocking), "hipStreamCreateWithFlags");
            A->aux = s;
        }
        for (hipEvent_t *e : {&A->ev_fork, &A->ev_mid, &A->ev_join})
            if (!*e) check_hip(hipEventCreateWithFlags(e, hipEventDisableTiming), "hipEventCreateWithFlags");
        A->schedule = schedule;
        A->near_wg_per_cu = near_wg_per_cu;
        A->near_lds_bytes = lds_bytes;
        A->near_early = near_early;
        return H2_OK;
    } catch (const Failure &f) {
        g_last_error = f.what;
        return f.code;
    } catch (...) {
        g_last_error = "internal error";
        return H2_ERR_INTERNAL;
    }
}

h2_status h2_profile(h2_handle A, int enable) {
    if (!A) {
        g_last_error = "NULL handle";
        return H2_ERR_INVALID_ARG;
    }
    A->prof = enable != 0;
    if (A->prof) {
        std::fill(A->prof_ms, A->prof_ms + 8, 0.0);
        A->prof_calls = 0;
    }
    return H2_OK;
}

h2_status h2_profile_read(h2_handle A, double *ms, int64_t *calls) {
    try {
        if (!A || !ms || !calls) fail(H2_ERR_INVALID_ARG, "NULL argument");
        for (size_t i = 0; i + PH_COUNT < A->pending.size(); i += PH_COUNT + 1) {
            hipEvent_t *ev = &A->pending[i];
            check_hip(hipEventSynchronize(ev[PH_COUNT]), "hipEventSynchronize");
            for (int p = 0; p < PH_COUNT; ++p) {
                float t = 0.0f;
                // end of phase p = start of the next recorded phase
                check_hip(hipEventElapsedTime(&t, ev[p], ev[p + 1]), "hipEventElapsedTime");
                A->prof_ms[p] += t;
            }
            float tot = 0.0f;
            check_hip(hipEventElapsedTime(&tot, ev[0], ev[PH_COUNT]), "hipEventElapsedTime");
            A->prof_ms[PH_COUNT] += tot;
            ++A->prof_calls;
        }
        A->spare.insert(A->spare.end(), A->pending.begin(), A->pending.end());
        A->pending.clear();
        std::copy(A->prof_ms, A->prof_ms + 8, ms);
        *calls = A->prof_calls;
        return H2_OK;
    } catch (const Failure &f) {
        g_last_error = f.what;
        return f.code;
    }
}

}  // extern "C"
