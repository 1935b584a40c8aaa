// ivm_internal.h -- device data layout and launchers shared by the libivm
// translation units.  Not part of the public interface (see include/ivm.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/ivm.h"

namespace ivm {

constexpr int kWave = 64;
constexpr int kTreelets = 32;      // top-level subtrees: contiguous equal-count Morton ranges
constexpr int kLeafMax = 4;        // subtrees of <= kLeafMax triangles become leaves
constexpr int kDefaultStack = 24;
constexpr int kDefaultWavesPerCu = 24;    // persistent grid: waves per compute unit
constexpr int kDefaultTileTreelets = 2;   // near-field tile only for bundles meeting <= this many treelets
constexpr int kMaxSamplesPerFacet = IVM_MAX_SAMPLES_PER_FACET;
constexpr float kDefaultEps = 1e-5f;
constexpr int kHullMax = 8;       // sample convex hull points kept per facet (0 = none kept)
constexpr int kSolidMaxFacets = 64;   // facets per solid group considered by the prism check
constexpr int kSolidMaxTris = 128;    // triangles per solid group
constexpr int kSolidMaxPlanes = 16;   // wall planes per solid
constexpr int kConvexMaxTris = 16;    // triangles per facet considered by the convexity check

// 2-D grid over the footprints of the verified solids (to find the solids a
// segment passes over): G x G cells with G = clamp(ceil(sqrt(2 n_solids)), 1, 256);
// a solid is listed in every cell its footprint box overlaps (up to
// kGridMaxCellsPerSolid cells; larger solids are left out, which only costs
// speed); at most kGridEntriesPerSolid * n_solids + 1024 entries, else the grid
// is marked unusable and scans go over all solids.
constexpr int kGridMaxCellsPerSolid = 256;
constexpr int kGridEntriesPerSolid = 16;
__host__ __device__ inline int solid_grid_dim(int n_solids) {
    int g = 1;
    while (g < 256 && g * g < 2 * n_solids) ++g;
    return g;
}

// Per-facet flags (fflags).
constexpr int kFacetConvex = 1;       // the facet's triangles tile one convex polygon

// Status bits raised on the device, mapped to ivm_status by the host.
constexpr int kStGrid = 1;
constexpr int kStDegenerate = 2;
constexpr int kStInvalid = 4;
constexpr int kStAngleRange = 8;  // an angular range's integer terms would leave 128 bits
constexpr int kStPathRange = 16;  // a path validation's integers would leave 512 bits

// Node of a binary BVH whose boxes live in the parent (one 64-byte record):
//   a = (lo0.x, lo0.y, lo0.z, hi0.x), b = (hi0.y, hi0.z, lo1.x, lo1.y),
//   c = (lo1.z, hi1.x, hi1.y, hi1.z), d = (ref0, ref1, first, last).
// ref >= 0 is an internal node; ref < 0 is a leaf holding the sorted triangle
// ranks [first, first + count) encoded as ~((first << 3) | (count - 1)).
// first/last is the node's own sorted-rank range (used by the overflow scan).
struct __align__(16) Node {
    float4 a, b, c;
    int4 d;
};

// 4-wide view of the same tree: record x (one per binary internal node x) lists
// the grandchildren of x, a leaf child standing for itself: 2 to 4 children,
// boxes stored across the four lanes of each float4.  Empty slots hold kNoRef.
// Traversal starts at a treelet root's record and only ever reaches records of
// nodes at even depth.
constexpr int kNoRef = 0x7fffffff;
struct __align__(16) Node4 {
    float4 lox, loy, loz, hix, hiy, hiz;
    int4 ref;   // >= 0 binary internal node (and its record); < 0 leaf; kNoRef empty
    int4 pad;   // .x = slots used (2..4), for the box-test counter
};

__host__ __device__ inline int leaf_ref(int first, int count) { return ~((first << 3) | (count - 1)); }
__host__ __device__ inline int leaf_first(int ref) { return (~ref) >> 3; }
__host__ __device__ inline int leaf_count(int ref) { return ((~ref) & 7) + 1; }

// Triangle record in sorted (Morton) order, three float4:
//   [0] = (a.x, a.y, a.z, facet id as int bits)
//   [1] = (e1 = b - a, max |e1_k|)
//   [2] = (e2 = c - a, max |e2_k|)
// All components are exact: vertices sit on a dyadic grid.

// Scene arrays live in global memory.  Device code sees the pointers in the
// global address space, so every access is a global load even when the view is
// read from memory (a batch's job table) or from a private copy; host code sees
// plain pointers (the layout is the same).
#if defined(__HIP_DEVICE_COMPILE__)
#define IVM_GLOBAL __attribute__((address_space(1)))
#else
#define IVM_GLOBAL
#endif

// Device view of a built scene (passed by value to kernels).
struct SceneDev {
    int F, T, S, W, n_treelets, max_spf;
    int g, gs;                 // grid exponents (vertex, sample)
    const IVM_GLOBAL float4 *tri;         // 3 * T
    const IVM_GLOBAL int *tri_orig;       // sorted rank -> caller's triangle index
    const IVM_GLOBAL int *tri_group;      // caller's triangle index -> treelet
    const IVM_GLOBAL Node *nodes;         // T (internal nodes at global slots)
    const IVM_GLOBAL Node4 *nodes4;       // T: 4-wide records, same slots
    const IVM_GLOBAL float *tl_box;       // kTreelets * 6 (lo.xyz, hi.xyz)
    const IVM_GLOBAL int *tl_root;        // kTreelets root refs (0x7fffffff = empty)
    const IVM_GLOBAL double *fplane;      // F * 6: a.xyz, n.xyz
    const IVM_GLOBAL float *fbox;         // F * 6
    const IVM_GLOBAL int *soff;           // F + 1
    const IVM_GLOBAL float4 *smp;         // S
    const IVM_GLOBAL int *sfacet;         // S
    const IVM_GLOBAL float4 *tri_caller;  // 3 * T, same records in the caller's triangle order
    const IVM_GLOBAL int *ftri;           // F * 2: first caller triangle of the facet, triangle count
    const IVM_GLOBAL int *fhull;          // F * kHullMax: sample indices of the convex hull of the facet's samples
    const IVM_GLOBAL int *fhull_n;        // F: hull size (0 = unavailable)
    const IVM_GLOBAL int *scluster;       // S: quadrant cluster (0..3) of each sample within its facet
    const IVM_GLOBAL int *fchull;         // F * 4 * kHullMax: hull sample indices per cluster
    const IVM_GLOBAL int *fchull_n;       // F * 4: cluster hull sizes (0 = unavailable or empty)
    const IVM_GLOBAL float *ffeat;        // F * 8: normalised centroid (3), unit normal (3), area (1), pad
    const IVM_GLOBAL float *fnorm;        // 4: scene-box centre (3) and half-size used to normalise features
    IVM_GLOBAL int *status;    // device status bits
    const IVM_GLOBAL double *extent;      // [0..5] = sample-unit integer box of vertices+samples as doubles; [6] = E
    const IVM_GLOBAL int *fflags;         // F: kFacet* bits
    const IVM_GLOBAL int *fsolid;         // F: verified solid of the facet, or -1
    const IVM_GLOBAL int4 *solid;         // n_solids: (wall planes, top z, base z, 0), sample units; 0 planes = rejected
    const IVM_GLOBAL int4 *splane;        // n_solids * kSolidMaxPlanes: (u.x, u.y, d.x, d.y) sample units; the
                               // outside of wall k is d.y (x - u.x) - d.x (y - u.y) > 0
    int n_solids;
    const IVM_GLOBAL float4 *sbox;        // n_solids * 2: footprint box and (base, top) in .z, metres; empty if rejected
    const IVM_GLOBAL float4 *gridp;       // (x0, y0, cell width, cell height) of the solid grid
    const IVM_GLOBAL int *gridi;          // (G, usable, entries, 0)
    const IVM_GLOBAL int *gcell_off;      // G * G + 1: CSR offsets of the cells' solid lists
    const IVM_GLOBAL int *gcell_list;     // solid ids, sorted within each cell
    const IVM_GLOBAL float4 *gcell_ent;   // the same entries with the solid's footprint box inline: 2 float4 each,
                               // (lo.x, lo.y, lo.z, id as int bits), (hi.x, hi.y, hi.z, 0)
};

// Workspace layout of one scene.
struct Layout {
    size_t tri, tri_orig, tri_group, nodes, tl_box, tl_root, fplane, fbox, soff, smp, sfacet;
    size_t status, extent, ibox, keys, vals, keys2, vals2, node_child, node_range, node_box;
    size_t ffirst, cand, done, und, uprefix, prefix, hi, hi_end, queue, learned, scan_tmp, tri_caller, fhull, fhull_n, scluster, fchull, fchull_n, ffeat, fnorm;
    size_t fflags, fsolid, sol_cnt, sol_off, sol_fac, sol_rec, sol_plane, sol_nver, nodes4, sol_box;
    size_t grid_p, grid_cnt, grid_off, grid_list, grid_ent;
    size_t learned_bytes;
    size_t total;
};
Layout make_layout(int F, int T, int S, bool learned, int n_solids);

// Opaque handle behind ivm_scene.
struct Scene {
    ivm_scene_desc desc;
    void *ws;
    size_t ws_bytes;
    Layout lay;
    SceneDev dev;
    hipStream_t build_stream;
    int n_items;               // F * W pair-cull items
    struct Model *model;       // optional occluder-ordering network
};

// Occluder-ordering network state (device arrays inside the caller's workspace).
struct Model {
    int max_batch, precision;
    float *params, *grad, *m, *v;          // IVM_MLP_PARAMS each
    float *h0, *h1, *h2, *logits, *d0, *d1, *loss;
    long long step;
};

// Offsets of the layers inside the flat parameter array.
constexpr int kIn = IVM_MLP_FEATURES, kHid = IVM_MLP_HIDDEN, kOut = IVM_MLP_OUTPUTS;
constexpr int kOffW0 = 0, kOffB0 = kOffW0 + kHid * kIn, kOffW1 = kOffB0 + kHid, kOffB1 = kOffW1 + kHid * kHid;
constexpr int kOffW2 = kOffB1 + kHid, kOffB2 = kOffW2 + kHid * kHid, kOffW3 = kOffB2 + kHid;
constexpr int kOffB3 = kOffW3 + kOut * kHid, kParams = kOffB3 + kOut;
static_assert(kParams == IVM_MLP_PARAMS, "parameter layout");

struct TraverseOpts {
    int order_mode;
    int fp64_only;
    int stack_depth;
    float eps6;                // 6 * eps: margin factor of the FP32 filter
    int grid_blocks;
    int no_tile;               // 1: skip the near-field tile
    int exhaustive;            // 1: every admissible segment gets its own search
    hipEvent_t *events;        // optional: recorded around the traversal kernel
    int tile_cap;              // near-field tile capacity (1..kTile triangles)
    int tile_treelets;         // gather a tile only for bundles meeting at most this many treelets
    int pair_chunk;            // consecutive undecided pairs a wave takes at a time (0 = by load)
    int xcd_parts;             // ranges the pair queues and table items are split into (1..kXcdParts)
};

// Queue counters of a matrix call (64 zeroed slots): the pair kernel's ranges at
// kQueuePairs, probe round r's at kQueueProbe + kXcdParts r.
constexpr int kXcdParts = 8;
constexpr int kQueuePairs = 8, kQueueProbe = 16;
constexpr int kQueuePoints = 32;  // the Tx/Rx kernel's 64-bit work-unit counter (slots 32 and 33)

// Traversal options from the public ones (defaults and clamping).
TraverseOpts make_opts(const ivm_matrix_opts *o);

// One scene's share of a (possibly multi-scene) persistent pair launch.
struct PairJob {
    SceneDev sc;
    const uint64_t *cand;     // F * W candidate words
    const uint32_t *prefix;   // exclusive prefix of candidate counts (n_items + 1)
    int n_items;
    uint64_t *M;
    const uint64_t *learned;  // per-candidate learned order, or nullptr
    uint64_t *done;           // F * W: pairs the probe kernel proved blocked
    const uint64_t *und;      // F * W: candidates still undecided after the probes
    const uint32_t *uprefix;  // exclusive prefix of their counts (n_items + 1)
};

// One scene's share of a (possibly multi-scene) Tx/Rx point launch.
struct PointJob {
    SceneDev sc;
    int N;
    const float *tx, *rx;
    uint64_t *txv, *rxv;
    long long unit_base;      // first global work unit of this job
    int U;                    // snapshots per work unit (a multiple of kSweptBlock)
};

// Launchers (each returns hipSuccess or the launch error).
hipError_t launch_build(Scene &sc, hipStream_t s);
hipError_t launch_solids(Scene &sc, hipStream_t s);
hipError_t launch_matrix(Scene &sc, const TraverseOpts &o, uint64_t *M, ivm_stats *stats,
                         const uint8_t *learned_order, hipStream_t s);
hipError_t launch_points(Scene &sc, const TraverseOpts &o, int N, const float *tx, const float *rx,
                         uint64_t *txv, uint64_t *rxv, uint8_t *los, ivm_stats *stats, hipStream_t s);
// Orders 3 and 4 of the candidate counts keep two F-entry vectors in LDS: the
// largest F they accept (F^4 < 2^63 keeps the int64 counts exact), and whether
// the device's LDS per block holds them for F facets.
constexpr int kCandHighMaxF = 40960;
constexpr int kHiMinSlab = 1024;  // snapshots of the smallest orders-3/4 slab the layout must hold
bool candidates_high_fits(int F);
// Orders 3 and 4: M^T and a slab of products in the pair scratch [cand, hi_end).
hipError_t launch_candidates_high(const Scene &sc, const uint64_t *M, int N, const uint64_t *txv,
                                  const uint64_t *rxv, const uint8_t *los, int K, int64_t *counts, hipStream_t s);
hipError_t launch_candidates_count(const SceneDev &d, const uint64_t *M, int N, const uint64_t *txv,
                                   const uint64_t *rxv, const uint8_t *los, int K, int64_t *counts,
                                   hipStream_t s);
hipError_t launch_candidates_offsets(int N, int K, const int64_t *counts, int64_t *offsets,
                                     hipStream_t s);
hipError_t launch_candidates_fill(const SceneDev &d, const uint64_t *M, int N, const uint64_t *txv,
                                  const uint64_t *rxv, int K, const int64_t *offsets, int32_t *paths,
                                  hipStream_t s);
hipError_t launch_triangle_groups(const SceneDev &d, int32_t *group, hipStream_t s);
hipError_t launch_facet_features(Scene &sc, hipStream_t s);
hipError_t launch_pair_features(const SceneDev &d, int n, const int32_t *I, const int32_t *J, float *X, hipStream_t s);
hipError_t launch_pair_labels(Scene &sc, const TraverseOpts &o, int n, const int32_t *I, const int32_t *J,
                              uint32_t *labels, hipStream_t s);
hipError_t launch_learned_order(Scene &sc, const Model &m, hipStream_t s);
hipError_t model_forward(Model &m, int n, const float *X, hipStream_t s);
hipError_t model_backward(Model &m, int n, const float *X, const float *Y, float *grad, hipStream_t s);
hipError_t model_adam(Model &m, float lr, hipStream_t s);
size_t model_workspace_bytes(int max_batch);
void model_bind(Model &m, void *ws, int max_batch, int precision);
hipError_t launch_cull_scan(Scene &sc, uint64_t *M, ivm_stats *stats, hipStream_t s);
hipError_t launch_relations(const SceneDev &sc, const uint64_t *M, uint64_t *par, uint64_t *per, int8_t *cls,
                            hipStream_t s);
size_t ranges_workspace_bytes(int N);
// Angular bouncing ranges of the visible pairs: CSR row offsets (int64[F + 1]),
// then the columns and four angles of every set bit of M in row-major order.
hipError_t launch_angle_offsets(const SceneDev &sc, const uint64_t *M, int64_t *offsets, hipStream_t s);
hipError_t launch_angles(const SceneDev &sc, const uint64_t *M, const int64_t *offsets, int32_t *cols,
                         double *ranges, hipStream_t s);
// Largest trajectory of the allocation-free ranges call, and the address of its
// scratch on the current device (looked up once per device).
constexpr int kRangesNoAllocMaxSnap = 32768;
hipError_t ranges_scratch(void **out);
hipError_t launch_ranges(const SceneDev &sc, int N, const uint64_t *tv, const uint64_t *rv, const uint8_t *los,
                         const float *tx, const float *rx, double dt, void *ws, int *events, int *starts, double *tc,
                         double *dist, int *n_ranges, double *mean, hipStream_t s);
constexpr int kSweptBlock = 32;  // points per box of a swept certificate in the Tx/Rx kernel
constexpr int kUnitMax = 512;    // most consecutive snapshots of one sample chunk in a Tx/Rx work unit
constexpr int kProbeRounds = 2;  // probe passes over the candidate pairs before the pair kernel
hipError_t launch_undecided(Scene &scn, uint64_t *M, hipStream_t s);
hipError_t launch_probe_jobs(const PairJob *d_jobs, const uint32_t *d_base, int n_jobs, uint32_t *d_queue, int round,
                             const TraverseOpts &o, ivm_stats *stats, hipStream_t s);
hipError_t launch_pair_jobs(const PairJob *d_jobs, const uint32_t *d_base, int n_jobs, uint32_t *d_queue,
                            const TraverseOpts &o, ivm_stats *stats, hipStream_t s);
hipError_t launch_job_base(const PairJob *d_jobs, int n_jobs, uint32_t *d_base, bool undecided, hipStream_t s);
hipError_t launch_points_prep(Scene &sc, int N, const float *tx, const float *rx, uint64_t *txv, uint64_t *rxv,
                              hipStream_t s);
hipError_t launch_point_jobs(const PointJob *d_jobs, int n_jobs, long long total_units, uint32_t *d_queue,
                             const TraverseOpts &o,
                             ivm_stats *stats, hipStream_t s);
// Edge visibility from Tx/Rx positions (first-order diffraction) and the
// per-snapshot counts of edges seen from both ends (counts may be null).
hipError_t launch_edges(Scene &scn, const TraverseOpts &o, int N, int E, int s, const int *efac, const float *esmp,
                        const float *tx, const float *rx, uint64_t *txe, uint64_t *rxe, int64_t *counts,
                        hipStream_t st);
// Exact image-method validation of candidate lists (CSR of int32 k-tuples, as
// ivm_image_tree_candidates writes them): a verdict byte per element.
hipError_t launch_validate_paths(const SceneDev &sc, int N, int K, const float *tx, const float *rx,
                                 const int64_t *offsets, const int32_t *paths, long long n_elems, uint8_t *valid,
                                 int64_t *valid_counts, unsigned long long *stats, hipStream_t s);
// Edge rows of the matrix (edge to facet and edge to edge) for the listed edges.
hipError_t launch_edge_rows(Scene &scn, const TraverseOpts &o, int E, int s, const int *efac, const float *esmp,
                            int n_rows, const int *rows, uint64_t *ef, uint64_t *ee, hipStream_t st);
hipError_t launch_los(Scene &sc, const TraverseOpts &o, int N, const float *tx, const float *rx, uint8_t *los,
                      hipStream_t s);
PairJob make_pair_job(Scene &sc, uint64_t *M, bool learned);
PointJob make_point_job(Scene &sc, int N, const float *tx, const float *rx, uint64_t *txv, uint64_t *rxv,
                        long long unit_base, int U);
long long point_units(const Scene &sc, int N, int U);
int point_unit_len(const int *S, const int *N, int n_jobs, int grid_blocks);
hipError_t launch_fill_u32(uint32_t *p, uint32_t v, size_t n, hipStream_t s);
hipError_t launch_fill_u64(uint64_t *p, uint64_t v, size_t n, hipStream_t s);

int device_cu_count();

}  // namespace ivm

// The opaque handle of the C interface wraps the scene.
struct ivm_scene {
    ivm::Scene s;
};
