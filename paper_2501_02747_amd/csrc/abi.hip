// abi.hip -- the extern "C" entry points of libivm (declared in include/ivm.h).
// Host code only: argument checks, workspace layout, option defaults, launches.
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>

#include "ivm_internal.h"

using namespace ivm;

struct ivm_model {
    Model m;
    void *ws;
    size_t bytes;
};

namespace {

ivm_status status_from_bits(int bits) {
    if (bits & kStInvalid) return IVM_ERR_INVALID_ARGUMENT;
    if (bits & (kStGrid | kStAngleRange | kStPathRange)) return IVM_ERR_GRID;
    if (bits & kStDegenerate) return IVM_ERR_DEGENERATE;
    return IVM_OK;
}

bool desc_sizes_ok(const ivm_scene_desc *d) {
    if (!d) return false;
    if (d->n_vertices < 0 || d->n_triangles < 0 || d->n_facets < 0 || d->n_samples < 0) return false;
    if (d->n_facets > 65535 || d->n_triangles > (1 << 27)) return false;
    if (d->grid_vertex_log2 < -30 || d->grid_vertex_log2 > 30) return false;
    if (d->grid_sample_log2 < d->grid_vertex_log2 || d->grid_sample_log2 > 30) return false;
    if (d->n_facets > 0 && !d->sample_offsets) return false;
    if (d->n_triangles > 0 && (!d->tri_vertices || !d->tri_facet || !d->vertices || d->n_vertices == 0)) return false;
    if (d->n_samples > 0 && !d->samples) return false;
    if (d->n_solids < 0 || d->n_solids > 65535) return false;
    return true;
}


}  // namespace

namespace ivm {

TraverseOpts make_opts(const ivm_matrix_opts *o) {
    TraverseOpts t{};
    t.order_mode = o ? o->order_mode : IVM_ORDER_PLAIN;
    t.fp64_only = o ? o->fp64_only : 0;
    int depth = (o && o->stack_depth > 0) ? o->stack_depth : kDefaultStack;
    if (depth < 2) depth = 2;
    if (depth > IVM_MAX_STACK) depth = IVM_MAX_STACK;
    t.stack_depth = depth;
    float eps = (o && o->eps > 0.f) ? o->eps : kDefaultEps;
    if (!(eps >= kDefaultEps)) eps = kDefaultEps;  // never below the sound margin (NaN -> default)
    t.eps6 = std::isinf(eps) ? INFINITY : 6.0f * eps;
    int wpc = (o && o->waves_per_cu > 0) ? o->waves_per_cu : kDefaultWavesPerCu;
    if (wpc > 64) wpc = 64;
    long long blocks = (long long)device_cu_count() * wpc / 4;
    if (blocks < 1) blocks = 1;
    t.grid_blocks = (int)blocks;
    t.events = o ? o->timing_events : nullptr;
    t.exhaustive = o ? o->exhaustive : 0;
    t.no_tile = (o ? o->no_tile : 0) || t.exhaustive;
    const int cap = (o && o->tile_cap > 0) ? o->tile_cap : 64;
    t.tile_cap = cap > 64 ? 64 : cap;
    const int tt = (o && o->tile_treelets > 0) ? o->tile_treelets : kDefaultTileTreelets;
    t.tile_treelets = tt > kTreelets ? kTreelets : tt;
    const int pc = o ? o->pair_chunk : 0;
    t.pair_chunk = pc <= 0 ? 0 : (pc > 256 ? 256 : pc);
    const int xp = (o && o->xcd_parts > 0) ? o->xcd_parts : 1;
    t.xcd_parts = xp > kXcdParts ? kXcdParts : xp;
    return t;
}

}  // namespace ivm

extern "C" {

const char *ivm_status_string(ivm_status s) {
    switch (s) {
        case IVM_OK: return "IVM_OK";
        case IVM_ERR_INVALID_ARGUMENT: return "IVM_ERR_INVALID_ARGUMENT";
        case IVM_ERR_WORKSPACE: return "IVM_ERR_WORKSPACE";
        case IVM_ERR_GRID: return "IVM_ERR_GRID";
        case IVM_ERR_DEGENERATE: return "IVM_ERR_DEGENERATE";
        case IVM_ERR_HIP: return "IVM_ERR_HIP";
        case IVM_ERR_CAPACITY: return "IVM_ERR_CAPACITY";
        case IVM_ERR_MODEL: return "IVM_ERR_MODEL";
        default: return "IVM_ERR_UNKNOWN";
    }
}

ivm_status ivm_scene_workspace_size(const ivm_scene_desc *desc, size_t *bytes) {
    if (!desc || !bytes || !desc_sizes_ok(desc)) return IVM_ERR_INVALID_ARGUMENT;
    *bytes = make_layout(desc->n_facets, desc->n_triangles, desc->n_samples,
                         (desc->flags & IVM_SCENE_LEARNED) != 0, desc->n_solids)
                 .total;
    return IVM_OK;
}

ivm_status ivm_build_scene(const ivm_scene_desc *desc, void *d_workspace, size_t workspace_bytes, hipStream_t stream,
                           ivm_scene **out) {
    if (!out) return IVM_ERR_INVALID_ARGUMENT;
    *out = nullptr;
    if (!desc || !desc_sizes_ok(desc) || !d_workspace) return IVM_ERR_INVALID_ARGUMENT;
    if (((uintptr_t)d_workspace & 255u) != 0) return IVM_ERR_INVALID_ARGUMENT;
    Layout L = make_layout(desc->n_facets, desc->n_triangles, desc->n_samples, (desc->flags & IVM_SCENE_LEARNED) != 0,
                           desc->n_solids);
    if (workspace_bytes < L.total) return IVM_ERR_WORKSPACE;
    ivm_scene *h = new (std::nothrow) ivm_scene();
    if (!h) return IVM_ERR_INVALID_ARGUMENT;
    Scene &sc = h->s;
    sc.desc = *desc;
    sc.ws = d_workspace;
    sc.ws_bytes = workspace_bytes;
    sc.lay = L;
    sc.build_stream = stream;
    sc.model = nullptr;
    const int F = desc->n_facets;
    SceneDev &d = sc.dev;
    char *ws = (char *)d_workspace;
    d.F = F;
    d.T = desc->n_triangles;
    d.S = desc->n_samples;
    d.W = (F + 63) / 64;
    d.n_treelets = desc->n_triangles < kTreelets ? desc->n_triangles : kTreelets;
    d.max_spf = kMaxSamplesPerFacet;
    d.g = desc->grid_vertex_log2;
    d.gs = desc->grid_sample_log2;
    d.tri = (const IVM_GLOBAL float4 *)(ws + L.tri);
    d.tri_orig = (const IVM_GLOBAL int *)(ws + L.tri_orig);
    d.tri_group = (const IVM_GLOBAL int *)(ws + L.tri_group);
    d.nodes = (const IVM_GLOBAL Node *)(ws + L.nodes);
    d.nodes4 = (const IVM_GLOBAL Node4 *)(ws + L.nodes4);
    d.tl_box = (const IVM_GLOBAL float *)(ws + L.tl_box);
    d.tl_root = (const IVM_GLOBAL int *)(ws + L.tl_root);
    d.fplane = (const IVM_GLOBAL double *)(ws + L.fplane);
    d.fbox = (const IVM_GLOBAL float *)(ws + L.fbox);
    d.soff = (const IVM_GLOBAL int *)(ws + L.soff);
    d.smp = (const IVM_GLOBAL float4 *)(ws + L.smp);
    d.sfacet = (const IVM_GLOBAL int *)(ws + L.sfacet);
    d.tri_caller = (const IVM_GLOBAL float4 *)(ws + L.tri_caller);
    d.ftri = (const IVM_GLOBAL int *)(ws + L.ffirst);
    d.fhull = (const IVM_GLOBAL int *)(ws + L.fhull);
    d.fhull_n = (const IVM_GLOBAL int *)(ws + L.fhull_n);
    d.scluster = (const IVM_GLOBAL int *)(ws + L.scluster);
    d.fchull = (const IVM_GLOBAL int *)(ws + L.fchull);
    d.fchull_n = (const IVM_GLOBAL int *)(ws + L.fchull_n);
    d.ffeat = (const IVM_GLOBAL float *)(ws + L.ffeat);
    d.fnorm = (const IVM_GLOBAL float *)(ws + L.fnorm);
    d.status = (IVM_GLOBAL int *)(ws + L.status);
    d.extent = (const IVM_GLOBAL double *)(ws + L.extent);
    d.fflags = (const IVM_GLOBAL int *)(ws + L.fflags);
    d.fsolid = (const IVM_GLOBAL int *)(ws + L.fsolid);
    d.solid = (const IVM_GLOBAL int4 *)(ws + L.sol_rec);
    d.splane = (const IVM_GLOBAL int4 *)(ws + L.sol_plane);
    d.sbox = (const IVM_GLOBAL float4 *)(ws + L.sol_box);
    d.gridp = (const IVM_GLOBAL float4 *)(ws + L.grid_p);
    d.gridi = (const IVM_GLOBAL int *)(ws + L.grid_p + sizeof(float4));
    d.gcell_off = (const IVM_GLOBAL int *)(ws + L.grid_off);
    d.gcell_list = (const IVM_GLOBAL int *)(ws + L.grid_list);
    d.gcell_ent = (const IVM_GLOBAL float4 *)(ws + L.grid_ent);
    d.n_solids = desc->facet_solid ? desc->n_solids : 0;
    sc.n_items = F * d.W;
    if (launch_build(sc, stream) != hipSuccess) {
        delete h;
        return IVM_ERR_HIP;
    }
    *out = h;
    return IVM_OK;
}

ivm_status ivm_scene_status(ivm_scene *scene) {
    if (!scene) return IVM_ERR_INVALID_ARGUMENT;
    int bits = 0;
    if (hipStreamSynchronize(scene->s.build_stream) != hipSuccess) return IVM_ERR_HIP;
    if (hipMemcpy(&bits, scene->s.dev.status, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess) return IVM_ERR_HIP;
    return status_from_bits(bits);
}

ivm_status ivm_scene_solids(ivm_scene *scene, int32_t *n_verified) {
    if (!scene || !n_verified) return IVM_ERR_INVALID_ARGUMENT;
    if (hipStreamSynchronize(scene->s.build_stream) != hipSuccess) return IVM_ERR_HIP;
    int n = 0;
    if (hipMemcpy(&n, (const char *)scene->s.ws + scene->s.lay.sol_nver, sizeof(int), hipMemcpyDeviceToHost) !=
        hipSuccess)
        return IVM_ERR_HIP;
    *n_verified = n;
    return IVM_OK;
}

ivm_status ivm_scene_info(const ivm_scene *scene, ivm_scene_info_t *info) {
    if (!scene || !info) return IVM_ERR_INVALID_ARGUMENT;
    const SceneDev &d = scene->s.dev;
    info->n_facets = d.F;
    info->n_triangles = d.T;
    info->n_samples = d.S;
    info->words_per_row = d.W;
    info->n_treelets = d.n_treelets;
    info->max_samples_per_facet = d.max_spf;
    info->n_nodes = d.T;
    info->workspace_bytes = scene->s.lay.total;
    return IVM_OK;
}

ivm_status ivm_destroy_scene(ivm_scene *scene) {
    if (!scene) return IVM_ERR_INVALID_ARGUMENT;
    delete scene;
    return IVM_OK;
}

ivm_status ivm_intervisibility_matrix(ivm_scene *scene, const ivm_matrix_opts *opts, uint64_t *d_M,
                                      ivm_stats *d_stats, hipStream_t stream) {
    if (!scene || !d_M) return IVM_ERR_INVALID_ARGUMENT;
    if (opts && (opts->order_mode < IVM_ORDER_PLAIN || opts->order_mode > IVM_ORDER_REVERSED))
        return IVM_ERR_INVALID_ARGUMENT;
    TraverseOpts o = make_opts(opts);
    ivm_status ret = IVM_OK;
    if (o.order_mode == IVM_ORDER_LEARNED && (!scene->s.model || scene->s.lay.learned_bytes == 0)) {
        o.order_mode = IVM_ORDER_PLAIN;
        ret = IVM_ERR_MODEL;
        // stats flag bit 0: learned order requested but unavailable
        if (d_stats && launch_fill_u64(&d_stats->flags, 1ull, 1, stream) != hipSuccess) return IVM_ERR_HIP;
    }
    if (launch_matrix(scene->s, o, d_M, d_stats, nullptr, stream) != hipSuccess) return IVM_ERR_HIP;
    return ret;
}

ivm_status ivm_txrx_visibility_table(ivm_scene *scene, const ivm_matrix_opts *opts, int32_t n_snap,
                                     const float *d_tx, const float *d_rx, uint64_t *d_tx_vis, uint64_t *d_rx_vis,
                                     uint8_t *d_los, ivm_stats *d_stats, hipStream_t stream) {
    if (!scene || n_snap < 0 || n_snap > IVM_MAX_SNAPSHOTS) return IVM_ERR_INVALID_ARGUMENT;
    if (n_snap > 0 && (!d_tx || !d_rx || !d_tx_vis || !d_rx_vis || !d_los)) return IVM_ERR_INVALID_ARGUMENT;
    if (opts && (opts->order_mode < IVM_ORDER_PLAIN || opts->order_mode > IVM_ORDER_REVERSED))
        return IVM_ERR_INVALID_ARGUMENT;
    TraverseOpts o = make_opts(opts);
    if (n_snap == 0) return IVM_OK;
    if (launch_points(scene->s, o, n_snap, d_tx, d_rx, d_tx_vis, d_rx_vis, d_los, d_stats, stream) != hipSuccess)
        return IVM_ERR_HIP;
    return IVM_OK;
}

ivm_status ivm_image_tree_candidates(ivm_scene *scene, const uint64_t *d_M, int32_t n_snap,
                                     const uint64_t *d_tx_vis, const uint64_t *d_rx_vis, const uint8_t *d_los,
                                     int32_t max_order, int64_t *d_counts, int64_t *d_offsets, int32_t *d_paths,
                                     size_t paths_cap, hipStream_t stream) {
    if (!scene || n_snap < 0 || max_order < 1 || max_order > 4) return IVM_ERR_INVALID_ARGUMENT;
    if (n_snap > 0 && (!d_M || !d_tx_vis || !d_rx_vis || !d_los || !d_counts)) return IVM_ERR_INVALID_ARGUMENT;
    if (d_paths && !d_offsets) return IVM_ERR_INVALID_ARGUMENT;
    const SceneDev &d = scene->s.dev;
    if (n_snap == 0) return IVM_OK;
    if (max_order >= 3 && !candidates_high_fits(d.F)) return IVM_ERR_INVALID_ARGUMENT;
    const hipError_t ce =
        max_order >= 3
            ? launch_candidates_high(scene->s, d_M, n_snap, d_tx_vis, d_rx_vis, d_los, max_order, d_counts, stream)
            : launch_candidates_count(d, d_M, n_snap, d_tx_vis, d_rx_vis, d_los, max_order, d_counts, stream);
    if (ce != hipSuccess) return IVM_ERR_HIP;
    if (!d_paths) {
        if (d_offsets && launch_candidates_offsets(n_snap, max_order, d_counts, d_offsets, stream) != hipSuccess)
            return IVM_ERR_HIP;
        return IVM_OK;
    }
    if (launch_candidates_offsets(n_snap, max_order, d_counts, d_offsets, stream) != hipSuccess) return IVM_ERR_HIP;
    int64_t total = 0;
    if (hipMemcpyAsync(&total, d_offsets + (size_t)n_snap * max_order, sizeof(total), hipMemcpyDeviceToHost,
                       stream) != hipSuccess)
        return IVM_ERR_HIP;
    if (hipStreamSynchronize(stream) != hipSuccess) return IVM_ERR_HIP;
    if ((size_t)total > paths_cap) return IVM_ERR_CAPACITY;
    if (launch_candidates_fill(d, d_M, n_snap, d_tx_vis, d_rx_vis, max_order, d_offsets, d_paths, stream) !=
        hipSuccess)
        return IVM_ERR_HIP;
    return IVM_OK;
}

ivm_status ivm_interface_relations(const ivm_scene *scene, const uint64_t *d_M, uint64_t *d_par, uint64_t *d_per,
                                   int8_t *d_facet_class, hipStream_t stream) {
    if (!scene || !d_M || !d_par || !d_per || !d_facet_class) return IVM_ERR_INVALID_ARGUMENT;
    if (launch_relations(scene->s.dev, d_M, d_par, d_per, d_facet_class, stream) != hipSuccess) return IVM_ERR_HIP;
    return IVM_OK;
}

ivm_status ivm_edge_visibility(ivm_scene *scene, const ivm_matrix_opts *opts, int32_t n_edges,
                               int32_t samples_per_edge, const int32_t *d_edge_facets, const float *d_edge_samples,
                               int32_t n_snap, const float *d_tx, const float *d_rx, uint64_t *d_tx_edges,
                               uint64_t *d_rx_edges, int64_t *d_diffraction, hipStream_t stream) {
    if (!scene || n_edges < 0 || n_snap < 0 || samples_per_edge < 1 || samples_per_edge > 64)
        return IVM_ERR_INVALID_ARGUMENT;
    if ((long long)n_edges * samples_per_edge > 0x7fffffffLL) return IVM_ERR_INVALID_ARGUMENT;
    if (opts && (opts->order_mode < IVM_ORDER_PLAIN || opts->order_mode > IVM_ORDER_REVERSED))
        return IVM_ERR_INVALID_ARGUMENT;
    if (n_snap > 0 && (!d_tx || !d_rx)) return IVM_ERR_INVALID_ARGUMENT;
    if (n_snap > 0 && n_edges > 0 && (!d_edge_facets || !d_edge_samples || !d_tx_edges || !d_rx_edges))
        return IVM_ERR_INVALID_ARGUMENT;
    if (n_snap == 0) return IVM_OK;
    const TraverseOpts o = make_opts(opts);
    if (launch_edges(scene->s, o, n_snap, n_edges, samples_per_edge, d_edge_facets, d_edge_samples, d_tx, d_rx,
                     d_tx_edges, d_rx_edges, d_diffraction, stream) != hipSuccess)
        return IVM_ERR_HIP;
    return IVM_OK;
}

ivm_status ivm_visibility_ranges_workspace_size(int32_t n_snap, size_t *bytes) {
    if (!bytes || n_snap < 1) return IVM_ERR_INVALID_ARGUMENT;
    *bytes = ranges_workspace_bytes(n_snap);
    return IVM_OK;
}

ivm_status ivm_visibility_ranges(const ivm_scene *scene, int32_t n_snap, const uint64_t *d_tx_vis,
                                 const uint64_t *d_rx_vis, const uint8_t *d_los, const float *d_tx, const float *d_rx,
                                 double dt, void *d_workspace, size_t workspace_bytes, int32_t *d_events,
                                 int32_t *d_range_start, double *d_range_tc, double *d_range_dist, int32_t *d_n_ranges,
                                 double *d_tc_mean, hipStream_t stream) {
    if (!scene || n_snap < 1 || !(dt > 0.0) || !std::isfinite(dt)) return IVM_ERR_INVALID_ARGUMENT;
    if (!d_tx_vis || !d_rx_vis || !d_los || !d_tx || !d_rx || !d_events || !d_range_start || !d_range_tc ||
        !d_range_dist || !d_n_ranges || !d_tc_mean || !d_workspace || ((uintptr_t)d_workspace & 255u))
        return IVM_ERR_INVALID_ARGUMENT;
    if (workspace_bytes < ranges_workspace_bytes(n_snap)) return IVM_ERR_WORKSPACE;
    if (launch_ranges(scene->s.dev, n_snap, d_tx_vis, d_rx_vis, d_los, d_tx, d_rx, dt, d_workspace, d_events,
                      d_range_start, d_range_tc, d_range_dist, d_n_ranges, d_tc_mean, stream) != hipSuccess)
        return IVM_ERR_HIP;
    return IVM_OK;
}

ivm_status ivm_visibility_ranges_noalloc(const ivm_scene *scene, int32_t n_snap, const uint64_t *d_tx_vis,
                                         const uint64_t *d_rx_vis, const uint8_t *d_los, const float *d_tx,
                                         const float *d_rx, double dt, int32_t *d_events, int32_t *d_range_start,
                                         double *d_range_tc, double *d_range_dist, int32_t *d_n_ranges,
                                         double *d_tc_mean, hipStream_t stream) {
    if (!scene || n_snap < 1 || !(dt > 0.0) || !std::isfinite(dt)) return IVM_ERR_INVALID_ARGUMENT;
    if (!d_tx_vis || !d_rx_vis || !d_los || !d_tx || !d_rx || !d_events || !d_range_start || !d_range_tc ||
        !d_range_dist || !d_n_ranges || !d_tc_mean)
        return IVM_ERR_INVALID_ARGUMENT;
    if (n_snap > kRangesNoAllocMaxSnap) return IVM_ERR_WORKSPACE;
    void *ws = nullptr;
    if (ranges_scratch(&ws) != hipSuccess || !ws) return IVM_ERR_HIP;
    if (launch_ranges(scene->s.dev, n_snap, d_tx_vis, d_rx_vis, d_los, d_tx, d_rx, dt, ws, d_events, d_range_start,
                      d_range_tc, d_range_dist, d_n_ranges, d_tc_mean, stream) != hipSuccess)
        return IVM_ERR_HIP;
    return IVM_OK;
}

ivm_status ivm_angular_ranges(ivm_scene *scene, const uint64_t *d_M, int64_t *d_offsets, int32_t *d_cols,
                              double *d_ranges, size_t cap, hipStream_t stream) {
    if (!scene || !d_M || !d_offsets || (!d_cols) != (!d_ranges)) return IVM_ERR_INVALID_ARGUMENT;
    const SceneDev &d = scene->s.dev;
    if (d.F == 0) return launch_fill_u64((uint64_t *)d_offsets, 0ull, 1, stream) == hipSuccess ? IVM_OK : IVM_ERR_HIP;
    if (launch_angle_offsets(d, d_M, d_offsets, stream) != hipSuccess) return IVM_ERR_HIP;
    if (!d_cols) return IVM_OK;
    int64_t total = 0;
    if (hipMemcpyAsync(&total, d_offsets + d.F, sizeof(total), hipMemcpyDeviceToHost, stream) != hipSuccess)
        return IVM_ERR_HIP;
    if (hipStreamSynchronize(stream) != hipSuccess) return IVM_ERR_HIP;
    if ((size_t)total > cap) return IVM_ERR_CAPACITY;
    if (total > 0 && launch_angles(d, d_M, d_offsets, d_cols, d_ranges, stream) != hipSuccess) return IVM_ERR_HIP;
    int bits = 0;
    if (hipMemcpyAsync(&bits, d.status, sizeof(int), hipMemcpyDeviceToHost, stream) != hipSuccess) return IVM_ERR_HIP;
    if (hipStreamSynchronize(stream) != hipSuccess) return IVM_ERR_HIP;
    return (bits & kStAngleRange) ? IVM_ERR_GRID : IVM_OK;
}

ivm_status ivm_edge_rows(ivm_scene *scene, const ivm_matrix_opts *opts, int32_t n_edges, int32_t samples_per_edge,
                         const int32_t *d_edge_facets, const float *d_edge_samples, int32_t n_rows,
                         const int32_t *d_rows, uint64_t *d_edge_facet, uint64_t *d_edge_edge, hipStream_t stream) {
    if (!scene || n_edges < 0 || n_rows < 0 || samples_per_edge < 1 || samples_per_edge > 64)
        return IVM_ERR_INVALID_ARGUMENT;
    if ((long long)n_edges * samples_per_edge > 0x7fffffffLL) return IVM_ERR_INVALID_ARGUMENT;
    if (opts && (opts->order_mode < IVM_ORDER_PLAIN || opts->order_mode > IVM_ORDER_REVERSED))
        return IVM_ERR_INVALID_ARGUMENT;
    if (n_rows > 0 && (!d_rows || !d_edge_facet || (n_edges > 0 && (!d_edge_edge || !d_edge_facets ||
                                                                     !d_edge_samples))))
        return IVM_ERR_INVALID_ARGUMENT;
    if (n_rows == 0) return IVM_OK;
    const TraverseOpts o = make_opts(opts);
    if (launch_edge_rows(scene->s, o, n_edges, samples_per_edge, d_edge_facets, d_edge_samples, n_rows, d_rows,
                         d_edge_facet, d_edge_edge, stream) != hipSuccess)
        return IVM_ERR_HIP;
    return IVM_OK;
}

ivm_status ivm_validate_paths(ivm_scene *scene, int32_t n_snap, const float *d_tx, const float *d_rx,
                              int32_t max_order, const int64_t *d_offsets, const int32_t *d_paths, int64_t n_elems,
                              uint8_t *d_valid, int64_t *d_valid_counts, ivm_stats *d_stats, hipStream_t stream) {
    if (!scene || n_snap < 0 || max_order < 1 || max_order > 4 || n_elems < 0) return IVM_ERR_INVALID_ARGUMENT;
    if ((long long)n_snap * max_order > 0x7fffffffLL) return IVM_ERR_INVALID_ARGUMENT;
    if (n_snap > 0 && (!d_tx || !d_rx || !d_offsets)) return IVM_ERR_INVALID_ARGUMENT;
    if (n_elems > 0 && (!d_paths || !d_valid || n_snap == 0)) return IVM_ERR_INVALID_ARGUMENT;
    if (n_snap == 0) return IVM_OK;
    const SceneDev &d = scene->s.dev;
    if (launch_validate_paths(d, n_snap, max_order, d_tx, d_rx, d_offsets, d_paths, n_elems, d_valid, d_valid_counts,
                              d_stats ? (unsigned long long *)&d_stats->tri_tests : nullptr, stream) != hipSuccess)
        return IVM_ERR_HIP;
    int bits = 0;
    if (hipMemcpyAsync(&bits, d.status, sizeof(int), hipMemcpyDeviceToHost, stream) != hipSuccess) return IVM_ERR_HIP;
    if (hipStreamSynchronize(stream) != hipSuccess) return IVM_ERR_HIP;
    if (bits & kStInvalid) return IVM_ERR_INVALID_ARGUMENT;
    return (bits & (kStPathRange | kStGrid)) ? IVM_ERR_GRID : IVM_OK;
}

ivm_status ivm_model_workspace_size(int32_t max_batch, size_t *bytes) {
    if (!bytes || max_batch <= 0 || max_batch > (1 << 24)) return IVM_ERR_INVALID_ARGUMENT;
    *bytes = model_workspace_bytes(max_batch);
    return IVM_OK;
}

ivm_status ivm_model_create(void *d_workspace, size_t workspace_bytes, int32_t max_batch, int32_t precision,
                            ivm_model **out) {
    if (!out) return IVM_ERR_INVALID_ARGUMENT;
    *out = nullptr;
    if (!d_workspace || max_batch <= 0 || max_batch > (1 << 24)) return IVM_ERR_INVALID_ARGUMENT;
    if (precision != IVM_MODEL_BF16 && precision != IVM_MODEL_FP32) return IVM_ERR_INVALID_ARGUMENT;
    if (((uintptr_t)d_workspace & 255u) != 0) return IVM_ERR_INVALID_ARGUMENT;
    if (workspace_bytes < model_workspace_bytes(max_batch)) return IVM_ERR_WORKSPACE;
    ivm_model *h = new (std::nothrow) ivm_model();
    if (!h) return IVM_ERR_INVALID_ARGUMENT;
    h->ws = d_workspace;
    h->bytes = workspace_bytes;
    model_bind(h->m, d_workspace, max_batch, precision);
    if (launch_fill_u32((uint32_t *)h->m.params, 0u, 4 * (size_t)kParams, nullptr) != hipSuccess ||
        hipStreamSynchronize(nullptr) != hipSuccess) {
        delete h;
        return IVM_ERR_HIP;
    }
    *out = h;
    return IVM_OK;
}

ivm_status ivm_model_destroy(ivm_model *model) {
    if (!model) return IVM_ERR_INVALID_ARGUMENT;
    delete model;
    return IVM_OK;
}

ivm_status ivm_model_set_params(ivm_model *model, const float *d_params, hipStream_t stream) {
    if (!model || !d_params) return IVM_ERR_INVALID_ARGUMENT;
    Model &m = model->m;
    if (hipMemcpyAsync(m.params, d_params, sizeof(float) * kParams, hipMemcpyDeviceToDevice, stream) != hipSuccess)
        return IVM_ERR_HIP;
    if (launch_fill_u32((uint32_t *)m.m, 0u, 2 * (size_t)kParams, stream) != hipSuccess) return IVM_ERR_HIP;
    m.step = 0;
    return IVM_OK;
}

ivm_status ivm_model_get_params(const ivm_model *model, float *d_params, hipStream_t stream) {
    if (!model || !d_params) return IVM_ERR_INVALID_ARGUMENT;
    if (hipMemcpyAsync(d_params, model->m.params, sizeof(float) * kParams, hipMemcpyDeviceToDevice, stream) !=
        hipSuccess)
        return IVM_ERR_HIP;
    return IVM_OK;
}

ivm_status ivm_model_forward(ivm_model *model, int32_t n, const float *d_x, float *d_logits, hipStream_t stream) {
    if (!model || n < 0 || n > model->m.max_batch || (n > 0 && (!d_x || !d_logits))) return IVM_ERR_INVALID_ARGUMENT;
    if (n == 0) return IVM_OK;
    if (model_forward(model->m, n, d_x, stream) != hipSuccess) return IVM_ERR_HIP;
    if (hipMemcpyAsync(d_logits, model->m.logits, sizeof(float) * (size_t)n * kOut, hipMemcpyDeviceToDevice,
                       stream) != hipSuccess)
        return IVM_ERR_HIP;
    return IVM_OK;
}

ivm_status ivm_model_loss_grad(ivm_model *model, int32_t n, const float *d_x, const float *d_y, float *d_loss,
                               float *d_grad, hipStream_t stream) {
    if (!model || n <= 0 || n > model->m.max_batch || !d_x || !d_y || !d_loss || !d_grad)
        return IVM_ERR_INVALID_ARGUMENT;
    Model &m = model->m;
    if (launch_fill_u32((uint32_t *)m.loss, 0u, 1, stream) != hipSuccess) return IVM_ERR_HIP;
    if (model_backward(m, n, d_x, d_y, d_grad, stream) != hipSuccess) return IVM_ERR_HIP;
    if (hipMemcpyAsync(d_loss, m.loss, sizeof(float), hipMemcpyDeviceToDevice, stream) != hipSuccess)
        return IVM_ERR_HIP;
    return IVM_OK;
}

ivm_status ivm_model_train_step(ivm_model *model, int32_t n, const float *d_x, const float *d_y, float lr,
                                float *d_loss, hipStream_t stream) {
    if (!model || n <= 0 || n > model->m.max_batch || !d_x || !d_y || !(lr >= 0.f)) return IVM_ERR_INVALID_ARGUMENT;
    Model &m = model->m;
    if (launch_fill_u32((uint32_t *)m.loss, 0u, 1, stream) != hipSuccess) return IVM_ERR_HIP;
    if (model_backward(m, n, d_x, d_y, m.grad, stream) != hipSuccess) return IVM_ERR_HIP;
    if (model_adam(m, lr, stream) != hipSuccess) return IVM_ERR_HIP;
    if (d_loss && hipMemcpyAsync(d_loss, m.loss, sizeof(float), hipMemcpyDeviceToDevice, stream) != hipSuccess)
        return IVM_ERR_HIP;
    return IVM_OK;
}

ivm_status ivm_pair_features(const ivm_scene *scene, int32_t n, const int32_t *d_i, const int32_t *d_j, float *d_x,
                             hipStream_t stream) {
    if (!scene || n < 0 || (n > 0 && (!d_i || !d_j || !d_x))) return IVM_ERR_INVALID_ARGUMENT;
    if (launch_pair_features(scene->s.dev, n, d_i, d_j, d_x, stream) != hipSuccess) return IVM_ERR_HIP;
    return IVM_OK;
}

ivm_status ivm_pair_occluder_labels(ivm_scene *scene, int32_t n, const int32_t *d_i, const int32_t *d_j,
                                    uint32_t *d_labels, hipStream_t stream) {
    if (!scene || n < 0 || (n > 0 && (!d_i || !d_j || !d_labels))) return IVM_ERR_INVALID_ARGUMENT;
    TraverseOpts o = make_opts(nullptr);
    if (launch_pair_labels(scene->s, o, n, d_i, d_j, d_labels, stream) != hipSuccess) return IVM_ERR_HIP;
    return IVM_OK;
}

ivm_status ivm_scene_set_model(ivm_scene *scene, const ivm_model *model) {
    if (!scene) return IVM_ERR_INVALID_ARGUMENT;
    if (model && scene->s.lay.learned_bytes == 0) return IVM_ERR_MODEL;
    scene->s.model = model ? const_cast<Model *>(&model->m) : nullptr;
    return IVM_OK;
}

ivm_status ivm_triangle_groups(const ivm_scene *scene, int32_t *d_group, hipStream_t stream) {
    if (!scene || (!d_group && scene->s.dev.T > 0)) return IVM_ERR_INVALID_ARGUMENT;
    if (launch_triangle_groups(scene->s.dev, d_group, stream) != hipSuccess) return IVM_ERR_HIP;
    return IVM_OK;
}

}  // extern "C"
