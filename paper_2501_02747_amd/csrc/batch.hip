// batch.hip -- many scenes of uneven size in one run (host side of ivm_batch_*).
//
// Per scene the orientation cull and the candidate scan are small launches;
// the any-hit work of every scene then goes through ONE persistent pair launch
// whose atomic queue runs over the concatenated candidate pairs of all scenes,
// and ONE persistent Tx/Rx launch over the concatenated (scene, snapshot, side,
// sample chunk) items, so large and small scenes share the whole GPU.  The
// sequence is captured into a hipGraph on the first run and replayed after.
// Counters are cleared by fill kernels inside the graph.
#include <cstring>
#include <new>
#include <vector>

#include "ivm_internal.h"

using namespace ivm;

struct ivm_batch {
    int n;
    std::vector<ivm_batch_item> items;
    PairJob *d_pjobs;
    PointJob *d_qjobs;
    uint32_t *d_base;
    uint32_t *d_queue;
    long long total_units;
    TraverseOpts o;
    ivm_stats *stats;
    hipGraph_t graph;
    hipGraphExec_t exec;
};

namespace {

inline size_t al(size_t x) { return (x + 255) & ~size_t(255); }

size_t batch_bytes(int n) {
    return al(sizeof(PairJob) * (size_t)n) + al(sizeof(PointJob) * (size_t)n) + al(sizeof(uint32_t) * (size_t)(2 * n + 2)) +
           256;
}

hipError_t record(ivm_batch *b, hipStream_t s) {
    hipError_t e;
    for (int k = 0; k < b->n; ++k) {
        const ivm_batch_item &it = b->items[k];
        Scene &sc = it.scene->s;
        if (sc.dev.F >= 2) {
            if ((e = launch_cull_scan(sc, it.d_M, b->stats, s)) != hipSuccess) return e;
        } else if ((e = launch_fill_u64(it.d_M, 0ull, (size_t)sc.dev.F * sc.dev.W, s)) != hipSuccess) {
            return e;
        }
    }
    if ((e = launch_fill_u32(b->d_queue, 0u, 64, s)) != hipSuccess) return e;
    // probe rounds over all scenes at once, each followed by every scene's
    // compaction of its undecided pairs; then the pair kernel over those
    auto undecided_all = [&]() -> hipError_t {
        for (int k = 0; k < b->n; ++k) {
            const ivm_batch_item &it = b->items[k];
            Scene &sc = it.scene->s;
            hipError_t r;
            if (sc.dev.F >= 2 && (r = launch_undecided(sc, it.d_M, s)) != hipSuccess) return r;
        }
        return hipSuccess;
    };
    const int rounds = b->o.exhaustive ? 0 : kProbeRounds;
    for (int round = 0; round < rounds; ++round) {
        if ((e = launch_job_base(b->d_pjobs, b->n, b->d_base, round > 0, s)) != hipSuccess) return e;
        if ((e = launch_probe_jobs(b->d_pjobs, b->d_base, b->n, b->d_queue, round, b->o, b->stats, s)) != hipSuccess)
            return e;
        if ((e = undecided_all()) != hipSuccess) return e;
    }
    if (rounds == 0 && (e = undecided_all()) != hipSuccess) return e;
    for (int k = 0; k < b->n; ++k) {  // the learned treelet order of each scene's undecided pairs
        Scene &sc = b->items[k].scene->s;
        if (sc.dev.F >= 2 && b->o.order_mode == IVM_ORDER_LEARNED && sc.model && sc.lay.learned_bytes &&
            (e = launch_learned_order(sc, *sc.model, s)) != hipSuccess)
            return e;
    }
    if ((e = launch_job_base(b->d_pjobs, b->n, b->d_base, true, s)) != hipSuccess) return e;
    if ((e = launch_pair_jobs(b->d_pjobs, b->d_base, b->n, b->d_queue, b->o, b->stats, s)) != hipSuccess) return e;
    for (int k = 0; k < b->n; ++k) {
        const ivm_batch_item &it = b->items[k];
        if ((e = launch_points_prep(it.scene->s, it.n_snap, it.d_tx, it.d_rx, it.d_tx_vis, it.d_rx_vis, s)) !=
            hipSuccess)
            return e;
    }
    if ((e = launch_point_jobs(b->d_qjobs, b->n, b->total_units, b->d_queue, b->o, b->stats, s)) != hipSuccess) return e;
    for (int k = 0; k < b->n; ++k) {
        const ivm_batch_item &it = b->items[k];
        if ((e = launch_los(it.scene->s, b->o, it.n_snap, it.d_tx, it.d_rx, it.d_los, s)) != hipSuccess) return e;
        if (it.d_counts && it.n_snap > 0 &&
            (e = launch_candidates_count(it.scene->s.dev, it.d_M, it.n_snap, it.d_tx_vis, it.d_rx_vis, it.d_los, 2,
                                         it.d_counts, s)) != hipSuccess)
            return e;
    }
    return hipSuccess;
}

TraverseOpts batch_opts(const ivm_matrix_opts *o) {
    TraverseOpts t = make_opts(o);
    t.events = nullptr;  // a captured graph records no caller events
    return t;
}

}  // namespace

extern "C" {

ivm_status ivm_batch_workspace_size(int32_t n_items, size_t *bytes) {
    if (n_items <= 0 || !bytes) return IVM_ERR_INVALID_ARGUMENT;
    *bytes = batch_bytes(n_items);
    return IVM_OK;
}

ivm_status ivm_batch_create(int32_t n_items, const ivm_batch_item *items, const ivm_matrix_opts *opts,
                            ivm_stats *d_stats, void *d_workspace, size_t workspace_bytes, ivm_batch **out) {
    if (!out) return IVM_ERR_INVALID_ARGUMENT;
    *out = nullptr;
    if (n_items <= 0 || !items || !d_workspace || ((uintptr_t)d_workspace & 255u)) return IVM_ERR_INVALID_ARGUMENT;
    if (opts && (opts->order_mode < IVM_ORDER_PLAIN || opts->order_mode > IVM_ORDER_REVERSED))
        return IVM_ERR_INVALID_ARGUMENT;
    if (workspace_bytes < batch_bytes(n_items)) return IVM_ERR_WORKSPACE;
    for (int k = 0; k < n_items; ++k) {
        const ivm_batch_item &it = items[k];
        if (!it.scene || !it.d_M || it.n_snap < 0 || it.n_snap > IVM_MAX_SNAPSHOTS) return IVM_ERR_INVALID_ARGUMENT;
        if (it.n_snap > 0 && (!it.d_tx || !it.d_rx || !it.d_tx_vis || !it.d_rx_vis || !it.d_los))
            return IVM_ERR_INVALID_ARGUMENT;
    }
    ivm_batch *b = new (std::nothrow) ivm_batch();
    if (!b) return IVM_ERR_INVALID_ARGUMENT;
    b->n = n_items;
    b->items.assign(items, items + n_items);
    char *ws = (char *)d_workspace;
    b->d_pjobs = (PairJob *)ws;
    ws += al(sizeof(PairJob) * (size_t)n_items);
    b->d_qjobs = (PointJob *)ws;
    ws += al(sizeof(PointJob) * (size_t)n_items);
    b->d_base = (uint32_t *)ws;
    ws += al(sizeof(uint32_t) * (size_t)(2 * n_items + 2));
    b->d_queue = (uint32_t *)ws;
    b->o = batch_opts(opts);
    b->stats = d_stats;
    b->graph = nullptr;
    b->exec = nullptr;
    std::vector<PairJob> pj(n_items);
    std::vector<PointJob> qj(n_items);
    std::vector<int> jS(n_items), jN(n_items);
    for (int k = 0; k < n_items; ++k) {
        jS[k] = items[k].scene->s.dev.S;
        jN[k] = items[k].n_snap;
    }
    const int U = point_unit_len(jS.data(), jN.data(), n_items, b->o.grid_blocks);
    long long base = 0;
    const bool learned = b->o.order_mode == IVM_ORDER_LEARNED;
    for (int k = 0; k < n_items; ++k) {
        const ivm_batch_item &it = items[k];
        Scene &sc = it.scene->s;
        pj[k] = make_pair_job(sc, it.d_M, learned && sc.model != nullptr);
        qj[k] = make_point_job(sc, it.n_snap, it.d_tx, it.d_rx, it.d_tx_vis, it.d_rx_vis, base, U);
        base += point_units(sc, it.n_snap, U);
    }
    b->total_units = base;
    if (hipMemcpy(b->d_pjobs, pj.data(), sizeof(PairJob) * n_items, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(b->d_qjobs, qj.data(), sizeof(PointJob) * n_items, hipMemcpyHostToDevice) != hipSuccess) {
        delete b;
        return IVM_ERR_HIP;
    }
    *out = b;
    return IVM_OK;
}

ivm_status ivm_batch_run(ivm_batch *b, hipStream_t stream) {
    if (!b) return IVM_ERR_INVALID_ARGUMENT;
    if (!b->exec) {
        if (hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal) != hipSuccess) return IVM_ERR_HIP;
        hipError_t e = record(b, stream);
        hipGraph_t g = nullptr;
        hipError_t e2 = hipStreamEndCapture(stream, &g);
        if (e != hipSuccess || e2 != hipSuccess || !g) {
            if (g) hipGraphDestroy(g);
            return IVM_ERR_HIP;
        }
        b->graph = g;
        if (hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0) != hipSuccess) {
            b->exec = nullptr;
            return IVM_ERR_HIP;
        }
    }
    if (hipGraphLaunch(b->exec, stream) != hipSuccess) return IVM_ERR_HIP;
    return IVM_OK;
}

ivm_status ivm_batch_destroy(ivm_batch *b) {
    if (!b) return IVM_ERR_INVALID_ARGUMENT;
    if (b->exec) hipGraphExecDestroy(b->exec);
    if (b->graph) hipGraphDestroy(b->graph);
    delete b;
    return IVM_OK;
}

}  // extern "C"
