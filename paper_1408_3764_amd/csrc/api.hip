// C ABI entry points for the moves, the energies and the batches.  Argument
// checking and launch configuration only; all arithmetic is in the kernels.
#include <string.h>

#include <algorithm>
#include <numeric>
#include <vector>

#include "gcmc_internal.h"

using namespace gcmc;

static int poisoned_check(gcmc_box* box, hipStream_t s, BoxState* h) {
    int rc = read_box_state(box, h, s);
    if (rc) return rc;
    if (h->error) return set_error(GCMC_ERR_POISONED, "box holds a latched device error");
    return GCMC_OK;
}

extern "C" {

int gcmc_box_set_launch(gcmc_box* box, int32_t waves, int32_t rows) {
    if (!box) return set_error(GCMC_ERR_INVALID_ARG, "box is NULL");
    if (rows == 0) {
        if (!spec_cfg_exists(waves)) return set_error(GCMC_ERR_INVALID_ARG, "unsupported speculative width");
        if (!spec_supported(box->d))
            return set_error(GCMC_ERR_UNSUPPORTED, "speculative rounds need one species and <= 512 stencil cells");
    } else if (rows == -1) {
        if (!async_cfg_exists(waves)) return set_error(GCMC_ERR_INVALID_ARG, "unsupported pipeline width");
        if (!async_supported(box->d))
            return set_error(GCMC_ERR_UNSUPPORTED, "the pipelined chain needs one species, <= 32 stencil cells, "
                                                   "2 x stencil x cell_cap <= 8192 and <= 1024 cells per axis");
    } else if (rows == -2) {
        if (!paper_cfg_exists(waves)) return set_error(GCMC_ERR_INVALID_ARG, "unsupported cell-per-thread width");
    } else if (rows == -3) {
        if (!resident_cfg_exists(waves)) return set_error(GCMC_ERR_INVALID_ARG, "unsupported resident width");
    } else if (!chain_cfg_exists(waves, rows)) {
        return set_error(GCMC_ERR_INVALID_ARG, "unsupported waves x rows");
    }
    box->waves = waves;
    box->rows = rows;
    return GCMC_OK;
}

int gcmc_delta_energy(gcmc_box* box, const gcmc_move* d_moves, int64_t n_moves, double* d_dU_pair,
                      double* d_dU_tail, double* d_dW_pair, void* stream) {
    if (!box || (n_moves > 0 && (!d_moves || !d_dU_pair)) || n_moves < 0)
        return set_error(GCMC_ERR_INVALID_ARG, "bad arguments");
    if (n_moves == 0) return GCMC_OK;
    hipStream_t s = (hipStream_t)stream;
    launch_delta(box->d_desc, box->d.ns > 1, n_moves, d_moves, d_dU_pair, d_dU_tail, d_dW_pair, s);
    GCMC_HIP(hipGetLastError());
    return GCMC_OK;
}

int gcmc_delta_energy_allpairs(gcmc_box* box, const gcmc_move* d_moves, int64_t n_moves, double* d_dU_pair,
                               double* d_dU_tail, double* d_dW_pair, void* stream) {
    if (!box || (n_moves > 0 && (!d_moves || !d_dU_pair)) || n_moves < 0)
        return set_error(GCMC_ERR_INVALID_ARG, "bad arguments");
    if (n_moves == 0) return GCMC_OK;
    hipStream_t s = (hipStream_t)stream;
    BoxState h;
    int rc = read_box_state(box, &h, s);
    if (rc) return rc;
    const int64_t chunk = ap_chunk_len();
    const int64_t nch = std::max<int64_t>(1, (h.n + chunk - 1) / chunk);
    for (int64_t m0 = 0; m0 < n_moves; m0 += 65535) {
        const int64_t nm = std::min<int64_t>(65535, n_moves - m0);
        if ((rc = ensure_scratch(box, nm * nch * 4))) return rc;
        if (launch_delta_allpairs(box->d_desc, h.n, d_moves + m0, nm, box->scratch, d_dU_pair + m0,
                                  d_dU_tail ? d_dU_tail + m0 : nullptr, d_dW_pair ? d_dW_pair + m0 : nullptr, s))
            return set_error(GCMC_ERR_INVALID_ARG, "too many moves");
        GCMC_HIP(hipGetLastError());
    }
    return GCMC_OK;
}

int gcmc_commit(gcmc_box* box, const gcmc_move* d_move, const double* d_dU_pair, const double* d_dW_pair,
                void* stream) {
    if (!box || !d_move || !d_dU_pair) return set_error(GCMC_ERR_INVALID_ARG, "NULL argument");
    launch_commit(box->d_desc, d_move, d_dU_pair, d_dW_pair, (hipStream_t)stream);
    GCMC_HIP(hipGetLastError());
    return GCMC_OK;
}

int gcmc_step(gcmc_box* box, int64_t n_moves, uint64_t counter0, gcmc_stats* d_stats, gcmc_log* d_log,
              void* stream) {
    if (!box || n_moves < 0) return set_error(GCMC_ERR_INVALID_ARG, "bad arguments");
    if (box->d.ns != 1) return set_error(GCMC_ERR_UNSUPPORTED, "the chain supports one species");
    int r;
    if (box->rows == -3)
        r = launch_chain_resident(box->d_desc, nullptr, 1, box->waves, n_moves, counter0, d_stats, d_log,
                                  (hipStream_t)stream);
    else if (box->rows == -2)
        r = launch_chain_paper(box->d_desc, nullptr, 1, box->waves, n_moves, counter0, d_stats, d_log,
                               (hipStream_t)stream);
    else if (box->rows == -1 && async_supported(box->d))
        r = launch_chain_async(box->d_desc, nullptr, 1, box->waves, n_moves, counter0, d_stats, d_log,
                               (hipStream_t)stream);
    else if (box->rows == 0 && spec_supported(box->d))
        r = launch_chain_spec(box->d_desc, nullptr, 1, box->waves, n_moves, counter0, d_stats, d_log,
                              (hipStream_t)stream, spec_needs_groups(box->d));
    else {
        // a shape the box's kernel cannot take falls back to the per-move 4x4
        const int rows = box->rows > 0 ? box->rows : 4;
        const bool ok = chain_cfg_exists(box->waves, rows);
        r = launch_chain(box->d_desc, nullptr, 1, ok ? box->waves : 4, ok ? rows : 4, n_moves, counter0, d_stats,
                         d_log, (hipStream_t)stream);
    }
    if (r) return set_error(GCMC_ERR_INVALID_ARG, "unsupported launch shape");
    GCMC_HIP(hipGetLastError());
    return GCMC_OK;
}

int gcmc_step_allpairs(gcmc_box* box, int64_t n_moves, uint64_t counter0, gcmc_stats* d_stats, gcmc_log* d_log,
                       void* stream) {
    if (!box || n_moves < 0) return set_error(GCMC_ERR_INVALID_ARG, "bad arguments");
    if (box->d.ns != 1) return set_error(GCMC_ERR_UNSUPPORTED, "the chain supports one species");
    hipStream_t s = (hipStream_t)stream;
    if (!box->ap_chain) {
        if (hipMalloc(&box->ap_chain, ap_chain_state_bytes()) != hipSuccess) {
            box->ap_chain = nullptr;
            return set_error(GCMC_ERR_OOM, "chain state allocation failed");
        }
    }
    const int64_t chunk = ap_chunk_len();
    const int64_t nch = std::max<int64_t>(1, (box->d.max_n + chunk - 1) / chunk);
    int rc = ensure_scratch(box, nch * 4);
    if (rc) return rc;
    launch_ap_chain_begin(box->d_desc, box->ap_chain, counter0, s);
    for (int64_t m = 0; m < n_moves; ++m) launch_ap_chain_move(box->d_desc, box->ap_chain, nch, box->scratch, d_log, s);
    // the end also folds the launch into the box's cumulative statistics and counter
    launch_ap_chain_end(box->d_desc, box->ap_chain, d_stats, s);
    GCMC_HIP(hipGetLastError());
    return GCMC_OK;
}

int gcmc_total_energy(gcmc_box* box, int32_t all_pairs, double* d_U, double* d_e, void* stream) {
    if (!box || !d_U) return set_error(GCMC_ERR_INVALID_ARG, "NULL argument");
    hipStream_t s = (hipStream_t)stream;
    BoxState h;
    int rc = poisoned_check(box, s, &h);
    if (rc) return rc;
    const int64_t need = total_partials_needed(box->d, h.maxcount, all_pairs != 0, h.n);
    if ((rc = ensure_scratch(box, need))) return rc;
    const int r = launch_total(box->d, box->d_desc, h.maxcount, all_pairs != 0, d_e, box->scratch, box->scratch_len,
                               d_U, s, h.n);
    if (r) return set_error(GCMC_ERR_INVALID_ARG, "scratch too small");
    GCMC_HIP(hipGetLastError());
    return GCMC_OK;
}

int gcmc_virial(gcmc_box* box, double* d_out, void* stream) {
    if (!box || !d_out) return set_error(GCMC_ERR_INVALID_ARG, "NULL argument");
    hipStream_t s = (hipStream_t)stream;
    BoxState h;
    int rc = poisoned_check(box, s, &h);
    if (rc) return rc;
    if ((rc = ensure_scratch(box, total_partials_needed(box->d, h.maxcount, false, h.n)))) return rc;
    const int r = launch_virial(box->d, box->d_desc, h.maxcount, box->scratch, box->scratch_len, d_out, s, h.n);
    if (r) return set_error(GCMC_ERR_INVALID_ARG, "scratch too small");
    GCMC_HIP(hipGetLastError());
    return GCMC_OK;
}

int gcmc_backward(gcmc_box* box, double* d_grad, double* d_deps, double* d_dsig, void* stream) {
    if (!box) return set_error(GCMC_ERR_INVALID_ARG, "box is NULL");
    hipStream_t s = (hipStream_t)stream;
    BoxState h;
    int rc = poisoned_check(box, s, &h);
    if (rc) return rc;
    if ((rc = ensure_scratch(box, grad_partials_needed(box->d, h.maxcount, h.n)))) return rc;
    const int r = launch_grad(box->d, box->d_desc, h.maxcount, d_grad, box->scratch, d_deps, d_dsig, s, h.n);
    if (r) return set_error(GCMC_ERR_INVALID_ARG, "scratch too small");
    GCMC_HIP(hipGetLastError());
    return GCMC_OK;
}

int gcmc_neighbor_ids(gcmc_box* box, const double* d_points, const int32_t* d_exclude, int64_t n, int32_t max_ids,
                      int32_t* d_ids, int32_t* d_counts, void* stream) {
    if (!box || n < 0 || max_ids < 0 || (n > 0 && (!d_points || !d_ids || !d_counts)))
        return set_error(GCMC_ERR_INVALID_ARG, "bad arguments");
    if (n == 0) return GCMC_OK;
    launch_neighbors(box->d_desc, d_points, d_exclude, n, max_ids, d_ids, d_counts, (hipStream_t)stream);
    GCMC_HIP(hipGetLastError());
    return GCMC_OK;
}

// ---------------------------------------------------------------- batches
int gcmc_batch_create(gcmc_box* const* boxes, int32_t n_boxes, gcmc_batch** out) {
    if (!boxes || n_boxes < 1 || !out) return set_error(GCMC_ERR_INVALID_ARG, "bad arguments");
    *out = nullptr;
    std::vector<int64_t> ns(n_boxes);
    for (int32_t b = 0; b < n_boxes; ++b) {
        if (!boxes[b]) return set_error(GCMC_ERR_INVALID_ARG, "NULL box");
        if (boxes[b]->d.ns != 1) return set_error(GCMC_ERR_UNSUPPORTED, "the chain supports one species");
        BoxState h;
        int rc = read_box_state(boxes[b], &h, nullptr);
        if (rc) return rc;
        ns[b] = h.n;
    }
    gcmc_batch* bt = new gcmc_batch();
    memset(bt, 0, sizeof(*bt));
    bt->n = n_boxes;
    bt->boxes = new gcmc_box*[n_boxes];
    for (int32_t b = 0; b < n_boxes; ++b) bt->boxes[b] = boxes[b];
    std::vector<int32_t> order(n_boxes);
    std::iota(order.begin(), order.end(), 0);
    // largest boxes first, so the longest-running workgroups start first
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t c) { return ns[a] > ns[c]; });
    if (hipMalloc(&bt->d_descs, sizeof(DevBox) * n_boxes) != hipSuccess ||
        hipMalloc(&bt->d_order, sizeof(int32_t) * n_boxes) != hipSuccess) {
        gcmc_batch_destroy(bt);
        return set_error(GCMC_ERR_OOM, "batch allocation failed");
    }
    bt->by_n = new int32_t[n_boxes];
    bt->h_order = new int32_t[n_boxes];
    bt->h_descs = new DevBox[n_boxes];
    for (int32_t b = 0; b < n_boxes; ++b) bt->by_n[b] = bt->h_order[b] = order[b];
    // the descriptors and order are uploaded by the first step (launch groups from the boxes' shapes)
    memset(bt->h_descs, 0xFF, sizeof(DevBox) * n_boxes);
    *out = bt;
    return GCMC_OK;
}

int gcmc_batch_destroy(gcmc_batch* bt) {
    if (!bt) return set_error(GCMC_ERR_INVALID_ARG, "batch is NULL");
    (void)hipDeviceSynchronize();
    if (bt->d_descs) (void)hipFree(bt->d_descs);
    if (bt->d_order) (void)hipFree(bt->d_order);
    for (int g = 0; g < kMaxBatchGroups; ++g) {
        if (bt->side[g]) (void)hipStreamDestroy(bt->side[g]);
        if (bt->ev_join[g]) (void)hipEventDestroy(bt->ev_join[g]);
    }
    if (bt->ev_fork) (void)hipEventDestroy(bt->ev_fork);
    delete[] bt->boxes;
    delete[] bt->by_n;
    delete[] bt->h_order;
    delete[] bt->h_descs;
    delete bt;
    return GCMC_OK;
}

// Launch path and shape of a box as gcmc_step would run it.
static void launch_key(const gcmc_box* b, int32_t* key) {
    if (b->rows == -3) {
        key[0] = 4; key[1] = b->waves; key[2] = -3;
    } else if (b->rows == -2) {
        key[0] = 3; key[1] = b->waves; key[2] = -2;
    } else if (b->rows == -1 && async_supported(b->d)) {
        key[0] = 1; key[1] = b->waves; key[2] = -1;
    } else if (b->rows == 0 && spec_supported(b->d)) {
        key[0] = 0; key[1] = b->waves; key[2] = 0;
    } else {
        // a shape the box's kernel cannot take falls back to the per-move 4x4
        const int rows = b->rows > 0 ? b->rows : 4;
        const bool ok = chain_cfg_exists(b->waves, rows);
        key[0] = 2; key[1] = ok ? b->waves : 4; key[2] = ok ? rows : 4;
    }
}

int gcmc_batch_step(gcmc_batch* bt, int64_t moves_per_box, uint64_t counter0, gcmc_stats* d_stats, void* stream) {
    if (!bt || moves_per_box < 0) return set_error(GCMC_ERR_INVALID_ARG, "bad arguments");
    hipStream_t s = (hipStream_t)stream;
    // boxes grouped by launch path and shape (groups in the order of their largest box, decreasing
    // N within a group): one launch per group
    int32_t ng = 0, gkey[kMaxBatchGroups][3], gcount[kMaxBatchGroups] = {0};
    std::vector<int32_t> grp(bt->n);
    for (int32_t q = 0; q < bt->n; ++q) {
        int32_t key[3];
        launch_key(bt->boxes[bt->by_n[q]], key);
        int g = 0;
        while (g < ng && memcmp(gkey[g], key, sizeof key) != 0) ++g;
        if (g == ng) {
            if (ng == kMaxBatchGroups) return set_error(GCMC_ERR_INVALID_ARG, "more than 8 launch shapes in a batch");
            memcpy(gkey[ng++], key, sizeof key);
        }
        grp[q] = g;
        gcount[g] += 1;
    }
    std::vector<int32_t> order;
    order.reserve(bt->n);
    int32_t gstart[kMaxBatchGroups];
    for (int g = 0; g < ng; ++g) {
        gstart[g] = (int32_t)order.size();
        for (int32_t q = 0; q < bt->n; ++q)
            if (grp[q] == g) order.push_back(bt->by_n[q]);
    }
    // descriptors and order in launch order: re-uploaded only when a box was rebuilt or the grouping
    // changed; the groups' launch paths and shapes are taken afresh on every call (a new shape for
    // a group of the same boxes changes neither the order nor the descriptors)
    bool changed = ng != bt->ngroups;
    for (int32_t q = 0; q < bt->n && !changed; ++q)
        changed = order[q] != bt->h_order[q] ||
                  memcmp(&bt->h_descs[q], &bt->boxes[order[q]]->d, sizeof(DevBox)) != 0;
    if (changed) {
        for (int32_t q = 0; q < bt->n; ++q) {
            bt->h_order[q] = order[q];
            bt->h_descs[q] = bt->boxes[order[q]]->d;
        }
        GCMC_HIP(hipMemcpyAsync(bt->d_descs, bt->h_descs, sizeof(DevBox) * bt->n, hipMemcpyHostToDevice, s));
        GCMC_HIP(hipMemcpyAsync(bt->d_order, bt->h_order, sizeof(int32_t) * bt->n, hipMemcpyHostToDevice, s));
        GCMC_HIP(hipStreamSynchronize(s));
        bt->ngroups = ng;
    }
    for (int g = 0; g < ng; ++g) {
        bt->gstart[g] = gstart[g];
        bt->gcount[g] = gcount[g];
        memcpy(bt->gkey[g], gkey[g], sizeof gkey[g]);
    }
    // groups after the first run on side streams (default priority) forked from and joined to `s`
    if (ng > 1) {
        if (!bt->ev_fork) GCMC_HIP(hipEventCreateWithFlags(&bt->ev_fork, hipEventDisableTiming));
        for (int g = 1; g < ng; ++g) {
            if (!bt->side[g]) GCMC_HIP(hipStreamCreateWithFlags(&bt->side[g], hipStreamNonBlocking));
            if (!bt->ev_join[g]) GCMC_HIP(hipEventCreateWithFlags(&bt->ev_join[g], hipEventDisableTiming));
        }
        GCMC_HIP(hipEventRecord(bt->ev_fork, s));
        for (int g = 1; g < ng; ++g) GCMC_HIP(hipStreamWaitEvent(bt->side[g], bt->ev_fork, 0));
    }
    for (int g = 0; g < ng; ++g) {
        const hipStream_t sg = g == 0 ? s : bt->side[g];
        const DevBox* dd = bt->d_descs + bt->gstart[g];
        const int32_t* od = bt->d_order + bt->gstart[g];
        const int cnt = bt->gcount[g];
        const int32_t* key = bt->gkey[g];
        int r;
        if (key[0] == 4) {
            r = launch_chain_resident(dd, od, cnt, key[1], moves_per_box, counter0, d_stats, nullptr, sg);
        } else if (key[0] == 3) {
            r = launch_chain_paper(dd, od, cnt, key[1], moves_per_box, counter0, d_stats, nullptr, sg);
        } else if (key[0] == 1) {
            r = launch_chain_async(dd, od, cnt, key[1], moves_per_box, counter0, d_stats, nullptr, sg);
        } else if (key[0] == 0) {
            int ngr = 0;
            for (int32_t q = 0; q < cnt; ++q)
                ngr = std::max(ngr, spec_needs_groups(bt->boxes[bt->h_order[bt->gstart[g] + q]]->d));
            r = launch_chain_spec(dd, od, cnt, key[1], moves_per_box, counter0, d_stats, nullptr, sg, ngr);
        } else {
            r = launch_chain(dd, od, cnt, key[1], key[2], moves_per_box, counter0, d_stats, nullptr, sg);
        }
        if (r) return set_error(GCMC_ERR_INVALID_ARG, "unsupported launch shape");
        GCMC_HIP(hipGetLastError());
    }
    if (ng > 1) {
        for (int g = 1; g < ng; ++g) {
            GCMC_HIP(hipEventRecord(bt->ev_join[g], bt->side[g]));
            GCMC_HIP(hipStreamWaitEvent(s, bt->ev_join[g], 0));
        }
    }
    return GCMC_OK;
}

}  // extern "C"

static_assert(sizeof(gcmc_box_desc) == 128, "gcmc_box_desc layout");
static_assert(sizeof(gcmc_move) == 40, "gcmc_move layout");
static_assert(sizeof(gcmc_stats) == 192, "gcmc_stats layout");
static_assert(sizeof(gcmc_log) == 72, "gcmc_log layout");
static_assert(sizeof(gcmc_checkpoint) == 136, "gcmc_checkpoint layout");
