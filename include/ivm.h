/*
 * ivm.h -- C ABI of libivm: facet inter-visibility pre-processing for dynamic
 * ray tracing on AMD Instinct MI355X (gfx950).
 *
 * The calls follow the pre-processing pipeline of Yang et al., "An Efficient
 * Pre-Processing Method for 6G Dynamic Ray-Tracing Channel Modeling" (IEEE TVT
 * 2024): the scenario database (Section III-C, flow chart of Fig. 7) becomes
 * ivm_build_scene; the static inter-visibility matrix (Section II-A/B) becomes
 * ivm_intervisibility_matrix; the inter-visibility table for specific points
 * along a trajectory (Section III-B, Table II; Section III-C) becomes
 * ivm_txrx_visibility_table; the image tree that table prunes (Section II,
 * Section III-B), to the orders of Section IV-C, becomes
 * ivm_image_tree_candidates.  Around them: the interface relations of the
 * visible pairs (Section II-B, Table I), the visibility ranges and coherence
 * times along a trajectory (Section III-C/D, eqs. 8-9) and the edges seen from
 * Tx and Rx for first-order diffraction (Section III-B).
 *
 * Visibility is decided exactly in 3-D over deterministic per-facet sample
 * points:
 *   orient(f, x) = (x - a_f) . ((b_f - a_f) x (c_f - a_f)) with (a_f, b_f, c_f)
 *     the first triangle of facet f; > 0 means x is on f's visible side
 *     (Section II-B, eq. 2: only the side facing away from the building is
 *     visible, and no ray leaves a face through its back side).
 *   Facets i != j see each other iff some sample p of i and q of j have
 *     orient(i, q) > 0, orient(j, p) > 0 and the open segment (p, q) meets no
 *     closed triangle of any other facet transversally (Section II-B: two faces
 *     see each other when no other obstacle lies between them; a third face
 *     blocks).
 *   A point X sees facet f iff orient(f, X) > 0 and some sample p of f has
 *     (X, p) clear of every triangle outside f (Section III-B).
 *   A point X sees the edge where facets fa and fb meet iff orient(fa, X) > 0
 *     or orient(fb, X) > 0 and some sample p of the edge has (X, p) clear of
 *     every triangle outside fa and fb.
 *
 * Conventions
 *   - Every call returns an ivm_status; 0 is success, negative values errors.
 *     No C++ exception crosses this interface.
 *   - Pointers named d_* are device pointers; the caller owns them.  Calls are
 *     asynchronous and ordered on the given stream; results are valid after the
 *     stream has been synchronised.
 *   - Hot calls (matrix, table, candidates in count mode) allocate no device
 *     memory; all device state lives in the caller-provided scene workspace.
 *   - Calls on one scene that only read it (candidates of orders 1-2,
 *     relations, angles, ranges, edges, path validation) may run concurrently
 *     on different streams; ivm_intervisibility_matrix and
 *     ivm_txrx_visibility_table use the scene's scratch area (work queues) and
 *     must not overlap a matrix or table call on the same scene; candidates of
 *     orders 3-4 use the pair scratch and must not overlap a matrix call or
 *     another order-3/4 call on the same scene.
 *   - Bit layout of every facet bit set: bit j of row r is word j >> 6, bit
 *     j & 63, of row r; rows have W = ceil(F / 64) uint64 words; padding bits
 *     are zero.
 */
#ifndef IVM_H
#define IVM_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t ivm_status;

#define IVM_OK 0
#define IVM_ERR_INVALID_ARGUMENT (-1) /* null pointer, bad size, unsorted tri_facet, index out of range */
#define IVM_ERR_WORKSPACE (-2)        /* workspace smaller than ivm_scene_workspace_size */
#define IVM_ERR_GRID (-3)             /* coordinate off its dyadic grid, or FP64 exactness budget exceeded */
#define IVM_ERR_DEGENERATE (-4)       /* zero-area first triangle, non-planar facet, or facet without triangles */
#define IVM_ERR_HIP (-5)              /* a HIP runtime call or kernel launch failed */
#define IVM_ERR_CAPACITY (-6)         /* output list capacity too small (counts are still valid) */
#define IVM_ERR_MODEL (-7)            /* learned order requested without a usable model */

/* Scene description.  Sizes are host values; array pointers are device pointers
 * that must stay valid while the scene handle exists.
 *   vertices        float[n_vertices][3], metres, every coordinate a multiple of
 *                   2^-grid_vertex_log2 and exactly representable in FP32.
 *   tri_vertices    int32[n_triangles][3] vertex indices.
 *   tri_facet       int32[n_triangles], facet id in [0, n_facets), non-decreasing:
 *                   the triangles of one facet are contiguous.  The winding of a
 *                   facet's first triangle defines its visible side.
 *   sample_offsets  int32[n_facets + 1], CSR offsets into samples; at most
 *                   64 samples per facet (IVM_MAX_SAMPLES_PER_FACET): a facet
 *                   with more is reported by ivm_scene_status as
 *                   IVM_ERR_INVALID_ARGUMENT.
 *   samples         float[n_samples][3], every coordinate a multiple of
 *                   2^-grid_sample_log2 (grid_sample_log2 >= grid_vertex_log2).
 * The scene is accepted only if every predicate above is exact in FP64:
 * with D the largest coordinate extent of vertices and samples and E the largest
 * triangle edge component, (6 D E^2 + 12 D^2 E) 2^(3g + 2(gs - g)) < 2^53 and
 * D 2^gs < 2^24, g = grid_vertex_log2, gs = grid_sample_log2. */
typedef struct ivm_scene_desc {
    int32_t n_vertices;
    int32_t n_triangles;
    int32_t n_facets;
    int32_t n_samples;
    const float *vertices;
    const int32_t *tri_vertices;
    const int32_t *tri_facet;
    const int32_t *sample_offsets;
    const float *samples;
    int32_t grid_vertex_log2;
    int32_t grid_sample_log2;
    int32_t flags; /* IVM_SCENE_* */
    /* Optional occluder grouping hint (NULL / 0 = none).  facet_solid is a
     * device int32[n_facets] with values in [0, n_solids) or -1, typically the
     * building each facet belongs to (the scenario database of Section III-C
     * stores faces per building).  The build checks every group exactly and
     * keeps only those that bound a vertical convex prism: wall facets in
     * vertical planes whose traces close into one convex polygon P, roof
     * facets covering P at the top height, walls covering P's edges from the
     * lowest to the top height (covering tested by exact areas plus pairwise
     * interior-disjoint triangles).  A kept group lets the traversal prove a
     * whole bundle of segments blocked at once (every segment entering the
     * prism's interior above its base crosses one of its triangles).  The hint
     * never changes a result bit: a wrong or partial hint only leaves groups
     * unused.  Values outside [-1, n_solids) are treated as -1. */
    const int32_t *facet_solid;
    int32_t n_solids; /* 0..65535 */
} ivm_scene_desc;

/* desc.flags: reserve room for a learned traversal order of every facet pair
 * (8 bytes per unordered pair) so IVM_ORDER_LEARNED can be used on the scene. */
#define IVM_SCENE_LEARNED 1

typedef struct ivm_scene ivm_scene; /* opaque host handle */

/* Scene facts filled by ivm_scene_info (host memory). */
typedef struct ivm_scene_info_t {
    int32_t n_facets;
    int32_t n_triangles;
    int32_t n_samples;
    int32_t words_per_row;     /* W = ceil(F / 64) */
    int32_t n_treelets;        /* top-level BVH subtrees (32, fewer when T < 32) */
    int32_t max_samples_per_facet;
    int64_t n_nodes;
    size_t workspace_bytes;
} ivm_scene_info_t;

/* Device-side counters, accumulated by the hot calls (the caller zeroes them).
 * segments: segments traversed; box_tests: segment/box slab tests (treelet
 * boxes and BVH child boxes); tri_tests: segment/triangle tests; rechecks: tests whose
 * FP32 margin was too small and which were decided in FP64; fallbacks: subtrees
 * scanned linearly because the traversal stack was full; certified: pairs
 * decided blocked by the single-occluder test on sample-hull corners. */
typedef struct ivm_stats {
    uint64_t pairs_total;
    uint64_t pairs_candidate;
    uint64_t pairs_visible;
    uint64_t segments;
    uint64_t box_tests;
    uint64_t tri_tests;
    uint64_t rechecks;
    uint64_t fallbacks;
    uint64_t point_items;
    uint64_t flags; /* bit 0: learned order fell back to the plain order */
    uint64_t certified; /* pairs proven blocked by one convex occluder from hull corners */
    uint64_t subpair_runs; /* pairs whose explicit segments were limited to uncertified sub-pairs or fans */
    uint64_t tiled_pairs;  /* pairs decided from a complete near-field tile, without the BVH */
    uint64_t solid_certified; /* matrix: pairs proven blocked by verified solids on whole or sub-pair
                                 bundles; table: (point, facet) pairs proven blocked by one solid */
    uint64_t traversed;       /* segments sent to a BVH (or near-field tile) any-hit search */
    uint64_t solid_segments;  /* segments decided blocked by a verified solid one at a time */
    uint64_t solid_planes;    /* segment x face-plane steps of solid tests (certificates included) */
    uint64_t reserved[3];
} ivm_stats;

#define IVM_ORDER_PLAIN 0    /* treelets nearest the pair's segment box first */
#define IVM_ORDER_LEARNED 1  /* treelets by the occluder-ordering network's score */
#define IVM_ORDER_INDEX 2    /* treelets in Morton (index) order */
#define IVM_ORDER_REVERSED 3 /* reverse of the plain order (a control) */

/* Traversal options.  None of them changes a result bit. */
typedef struct ivm_matrix_opts {
    int32_t order_mode;     /* IVM_ORDER_* */
    int32_t fp64_only;      /* 1: decide every segment/triangle test in FP64 */
    int32_t stack_depth;    /* 2..IVM_MAX_STACK; 0 = default; overflow scans linearly */
    int32_t waves_per_cu;   /* persistent grid size in waves per compute unit, 1..64; 0 = 24 */
    float eps;              /* FP32 filter margin relative to the magnitude bound;
                               0 = default 1e-5; values < 1e-5 are raised to 1e-5;
                               +inf sends every test to FP64 */
    int32_t no_tile;        /* 1: never decide a pair from its near-field tile alone */
    int32_t exhaustive;     /* 1: give every admissible segment its own BVH search: no
                               probes, no blocker or solid caches, no bundle or point
                               certificates, no near-field tile (a measurement baseline) */
    hipEvent_t *timing_events; /* optional (NULL = none): two caller-created events the
                                  call records on its stream immediately before and
                                  after its traversal kernels (the matrix: both probe
                                  rounds and the pair kernel; the table: the point kernel) */
    int32_t tile_cap;       /* near-field tile capacity in triangles, 1..64; 0 = 64 */
    int32_t tile_treelets;  /* gather a near-field tile only for segment bundles whose box
                               meets at most this many treelets, 1..32; 0 = 2 */
    int32_t pair_chunk;     /* pair-to-wave mapping: consecutive undecided pairs a wave takes
                               from the queue at a time, 1..256; 0 = 4, or 32 when there are
                               more than 2048 pairs per wave */
    int32_t xcd_parts;      /* the pair queues (and the table's item ranges) are split into this
                               many contiguous ranges, 1..8; workgroups start on range (block
                               index mod ranges), one per XCD with 8, so neighbouring rows (or
                               snapshots) share an L2; 0 = 1 (measured: no faster on the
                               configured scenes) */
} ivm_matrix_opts;

#define IVM_MAX_STACK 24
#define IVM_MAX_SAMPLES_PER_FACET 64
#define IVM_MAX_SNAPSHOTS (1 << 24) /* snapshots per Tx/Rx table call or batch item */

const char *ivm_status_string(ivm_status s);

/* Bytes of device workspace ivm_build_scene needs for this description
 * (host-only, synchronous; reads only the size fields). */
ivm_status ivm_scene_workspace_size(const ivm_scene_desc *desc, size_t *bytes);

/* Validate the description, copy and lay out the scene in the workspace, and
 * build the Morton-code LBVH (32 treelets of contiguous Morton ranges).
 * The handle is host memory; d_workspace (>= ivm_scene_workspace_size bytes,
 * 256-byte aligned) is caller-owned and must outlive the handle.
 * Synchronous errors: IVM_ERR_INVALID_ARGUMENT, IVM_ERR_WORKSPACE, IVM_ERR_HIP.
 * Device-side validation (off-grid coordinates, exactness budget, degenerate
 * facets, unsorted tri_facet, indices out of range) is reported by
 * ivm_scene_status. */
ivm_status ivm_build_scene(const ivm_scene_desc *desc, void *d_workspace, size_t workspace_bytes,
                           hipStream_t stream, ivm_scene **out);

/* Synchronises the scene's build stream and returns the first device-reported
 * validation error of the scene (or of a later Tx/Rx position check), else IVM_OK. */
ivm_status ivm_scene_status(ivm_scene *scene);

ivm_status ivm_scene_info(const ivm_scene *scene, ivm_scene_info_t *info);

/* Synchronises the build stream and reports how many groups of the
 * facet_solid hint passed the prism check (host int32). */
ivm_status ivm_scene_solids(ivm_scene *scene, int32_t *n_verified);

ivm_status ivm_destroy_scene(ivm_scene *scene);

/* The static inter-visibility matrix (Section II-A/B): d_M is uint64[F][W],
 * symmetric, zero diagonal.  opts may be NULL (defaults).  d_stats may be NULL.
 * Errors: IVM_ERR_INVALID_ARGUMENT, IVM_ERR_MODEL (learned order without a model
 * attached: the call still runs in plain order and sets stats flag bit 0),
 * IVM_ERR_HIP. */
ivm_status ivm_intervisibility_matrix(ivm_scene *scene, const ivm_matrix_opts *opts, uint64_t *d_M,
                                      ivm_stats *d_stats, hipStream_t stream);

/* Inter-visibility table for specific points (Section III-B, Table II) along a
 * trajectory (Section III-C): for each snapshot n, the facets visible from
 * d_tx[n] and from d_rx[n] (uint64[N][W] each) and line of sight between them
 * (uint8[N]).  Positions are float[N][3] on the sample grid; off-grid positions
 * or positions that break the exactness budget are reported by ivm_scene_status.
 * opts may be NULL.  Errors: IVM_ERR_INVALID_ARGUMENT (also for N above
 * IVM_MAX_SNAPSHOTS), IVM_ERR_HIP. */
ivm_status ivm_txrx_visibility_table(ivm_scene *scene, const ivm_matrix_opts *opts, int32_t n_snap,
                                     const float *d_tx, const float *d_rx, uint64_t *d_tx_vis,
                                     uint64_t *d_rx_vis, uint8_t *d_los, ivm_stats *d_stats,
                                     hipStream_t stream);

/* Image-tree reflection candidates up to max_order (1..4) per snapshot: walks
 * f1 -> ... -> fk with tx_vis(f1), M[f_m][f_m+1] and rx_vis(fk) (Section III-B,
 * Table II: transmitter -> reference face -> aim face; orders 3 and 4 are the
 * iteration of Section II-C to the orders timed in Section IV-C).  d_M need not
 * be symmetric.  d_counts is int64[N][max_order + 1] with column 0 = line of
 * sight; counts are exact (orders 3 and 4 need 1 <= F <= 40960, else
 * IVM_ERR_INVALID_ARGUMENT).  Orders 3 and 4 are integer matrix products over
 * slabs of snapshots held in the scene's pair scratch: such a call must not
 * overlap a matrix call or another order-3/4 call on the same scene.  If d_paths is NULL
 * only counts are produced (asynchronous).  Otherwise d_offsets (int64[N *
 * max_order + 1]) receives CSR offsets of the lists (snapshot-major, order-minor)
 * and d_paths the k-tuples as int32 in lexicographic order; this mode
 * synchronises the stream once to check paths_cap (in int32 elements) and
 * returns IVM_ERR_CAPACITY, with valid counts and offsets, when it is too small.
 * Lists of orders 3 and 4 grow as |tx| d^2 and |tx| d^3 for rows of d set bits:
 * they are meant for small scenes; counts scale to full-size tables. */
ivm_status ivm_image_tree_candidates(ivm_scene *scene, const uint64_t *d_M, int32_t n_snap,
                                     const uint64_t *d_tx_vis, const uint64_t *d_rx_vis,
                                     const uint8_t *d_los, int32_t max_order, int64_t *d_counts,
                                     int64_t *d_offsets, int32_t *d_paths, size_t paths_cap,
                                     hipStream_t stream);

/* Exact image-method validation of image-tree candidates (Section III-A: the
 * image method; Section III-B: the image tree the inter-visibility table
 * prunes; Section IV-B: the pruned tree yields the same valid rays as brute
 * force).  The lists are those of ivm_image_tree_candidates (d_offsets
 * int64[n_snap * max_order + 1] in int32 elements, snapshot-major, order-minor;
 * d_paths int32[n_elems] of k-tuples), any lists of that layout are accepted.
 * Walk f1 -> ... -> fk of snapshot n is valid iff, with T = d_tx[n], R =
 * d_rx[n] and I_1..I_k the images of T mirrored successively in the planes of
 * f1..fk (plane of a facet: its first triangle): tracing back from R (target
 * R, then each reflection point), the target is strictly in front of f_m's
 * plane and I_m strictly behind it, the point where segment (target, I_m)
 * meets the plane lies in the closed facet f_m, and every leg T -> P_1 -> ...
 * -> P_k -> R misses (open segment, closed triangles) every triangle outside
 * the facets at its two ends.  Decisions are exact: rational points are
 * integer homogeneous vectors of 512 bits, segment tests run in FP64 with an
 * error bound and fall back to exact integers within it.
 * d_valid uint8[n_elems]: every element of a walk's k-tuple receives its
 * verdict, 1 valid, 0 not, 2 undecided (an integer left 512 bits: the call then
 * returns IVM_ERR_GRID).  d_valid_counts (int64[n_snap][max_order], may be NULL)
 * receives the valid walks per snapshot and order.  d_stats (may be NULL):
 * tri_tests += segment/triangle tests of the legs, rechecks += those decided in
 * exact integers.  Positions must be on the sample grid (else IVM_ERR_GRID).
 * The call synchronises the stream once at the end to report these errors.
 * Errors: IVM_ERR_INVALID_ARGUMENT (also facet ids out of range or repeated
 * consecutively in a walk), IVM_ERR_GRID, IVM_ERR_HIP. */
ivm_status ivm_validate_paths(ivm_scene *scene, int32_t n_snap, const float *d_tx, const float *d_rx,
                              int32_t max_order, const int64_t *d_offsets, const int32_t *d_paths, int64_t n_elems,
                              uint8_t *d_valid, int64_t *d_valid_counts, ivm_stats *d_stats, hipStream_t stream);

/* Interface relations of the visible facet pairs (Section II-B, Table I: the
 * reference face and the aim face are parallel, PAR, or perpendicular, PER).
 * d_M is a matrix from ivm_intervisibility_matrix; d_par and d_per are
 * uint64[F][W] in its layout, bit (i, j) set when M[i][j] and the planes of
 * facets i and j are parallel / perpendicular (exact integer tests on the
 * normals of the facets' first triangles); d_facet_class is int8[F]: 0 for a
 * vertical facet, 1 horizontal, 2 other (relations between vertical facets
 * belong to the horizontal view, the others to a vertical view).  All
 * caller-owned device memory; asynchronous on `stream`.
 * Errors: IVM_ERR_INVALID_ARGUMENT, IVM_ERR_HIP. */
ivm_status ivm_interface_relations(const ivm_scene *scene, const uint64_t *d_M, uint64_t *d_par, uint64_t *d_per,
                                   int8_t *d_facet_class, hipStream_t stream);

/* Edge visibility for first-order diffraction (Section III-B: the receiver's
 * diffracting edge is found the way a reflecting face is; edges are visibility
 * nodes next to faces).  Edge e is where facets d_edge_facets[e] = (fa, fb) meet
 * (int32[E][2]; fb = -1 for an edge of one facet); it has samples_per_edge
 * (1..64) sample points d_edge_samples[e * s + j] (float[E * s][3], on the
 * sample grid inside the scene's box).  Bit e of d_tx_edges[n] (uint64[N][We],
 * We = ceil(E / 64), padding zero) is set iff d_tx[n] lies strictly on the
 * visible side of fa or of fb and the segment from d_tx[n] to one of the edge's
 * samples meets no triangle of a facet other than fa and fb; the same for
 * d_rx_edges.  d_diffraction (int64[N], may be NULL) receives the number of
 * edges seen from both ends, the first-order diffraction candidates
 * Tx -> edge -> Rx.  Off-grid positions or samples and bad facet ids are
 * reported by ivm_scene_status.  opts may be NULL.  Errors:
 * IVM_ERR_INVALID_ARGUMENT, IVM_ERR_HIP. */
ivm_status ivm_edge_visibility(ivm_scene *scene, const ivm_matrix_opts *opts, int32_t n_edges,
                               int32_t samples_per_edge, const int32_t *d_edge_facets, const float *d_edge_samples,
                               int32_t n_snap, const float *d_tx, const float *d_rx, uint64_t *d_tx_edges,
                               uint64_t *d_rx_edges, int64_t *d_diffraction, hipStream_t stream);

/* Edge rows of the matrix: edges are visibility nodes beside faces (Sections I
 * and II-A), and the face seen for diffraction is the face seen for reflection
 * (Section III-B).  A node is a facet (its samples; side facets {f}) or an edge
 * e (its samples d_edge_samples[e * s + j]; side facets d_edge_facets[e] =
 * (fa, fb), fb = -1 for an edge of one facet; inputs as ivm_edge_visibility).
 * Edge e and node v see each other iff some sample p of e and q of v have q
 * strictly in front of fa or fb, p strictly in front of one of v's side
 * facets, and the open segment (p, q) meets no triangle of a facet outside the
 * side facets of both (exact predicates, as the matrix).  For each k < n_rows
 * and e = d_rows[k] (int32, device): bit f of d_edge_facet[k] (uint64[n_rows][W])
 * is set iff e and facet f see each other, and bit e2 of d_edge_edge[k]
 * (uint64[n_rows][We], We = ceil(E / 64)) iff e and edge e2 != e do; padding
 * bits are zero.  The facet-to-edge columns are the transpose (the relation is
 * symmetric).  Row ids outside [0, E), off-grid samples and bad facet ids are
 * reported by ivm_scene_status.  opts may be NULL; results do not depend on it.
 * Asynchronous on `stream`.  Errors: IVM_ERR_INVALID_ARGUMENT, IVM_ERR_HIP. */
ivm_status ivm_edge_rows(ivm_scene *scene, const ivm_matrix_opts *opts, int32_t n_edges, int32_t samples_per_edge,
                         const int32_t *d_edge_facets, const float *d_edge_samples, int32_t n_rows,
                         const int32_t *d_rows, uint64_t *d_edge_facet, uint64_t *d_edge_edge, hipStream_t stream);

/* Angular bouncing ranges of the visible facet pairs (Section II-A: the scene
 * is read in 2-D views, a horizontal one for vertical faces and a vertical one
 * otherwise, in which each face is a segment; Section II-B, eq. 1: at an end B
 * of the reference face the angle between BA, along the face, and BF, towards
 * an end F of the aim face, is the arccos of their normalised dot product;
 * eq. 2: an angle of 180 degrees or more, measured from the face towards its
 * visible side, is recorded as 0).  For every set bit (i, j) of d_M (row i the
 * reference face, column j the aim face; any matrix, symmetric or not):
 *   - the view looks along d = n_i x n_j (the line where both planes meet),
 *     or for parallel planes along z (vertical facets), x (horizontal facets)
 *     or the horizontal direction (-n_i.y, n_i.x, 0) in facet i's plane; the
 *     first non-zero component of d in the order z, x, y is positive; n_f is
 *     the normal (b - a) x (c - a) of facet f's first triangle;
 *   - facet i's ends are its vertices with the smallest (A) and largest (B)
 *     value of (d x n_i) . v, facet j's ends E and F those of (d x n_j) . v;
 *   - omega = the two angles at B between BA and BE, BF, sorted; mu = the two
 *     angles at A between AB and AE, AF, sorted; each angle is that of the two
 *     vectors projected on the plane normal to d, in degrees in [0, 180], and
 *     0 when the aim vertex is not strictly in front of facet i (eq. 2).
 * The three integer terms of each cosine are exact (128-bit) and rounded once
 * to FP64; the arccos is the device library's (a few ulp).
 * Outputs (caller-owned device memory, row-major over the set bits):
 *   d_offsets int64[F + 1]: CSR row offsets (row i's pairs are
 *     [d_offsets[i], d_offsets[i + 1])); padding bits of d_M are ignored;
 *   d_cols int32[cap]: the aim facet j of each pair, ascending within a row;
 *   d_ranges double[cap][4]: (omega_lo, omega_hi, mu_lo, mu_hi).
 * With d_cols and d_ranges NULL only the offsets are written (asynchronous).
 * Otherwise the call synchronises the stream twice: to check cap (returns
 * IVM_ERR_CAPACITY, with valid offsets, when the pairs do not fit) and at the
 * end to report pairs whose integer terms could leave 128 bits (such a pair
 * gets NaN angles, the call returns IVM_ERR_GRID and so does ivm_scene_status
 * from then on; it needs coordinates and normals far beyond the configured
 * scenes).  Errors: IVM_ERR_INVALID_ARGUMENT, IVM_ERR_CAPACITY, IVM_ERR_GRID,
 * IVM_ERR_HIP. */
ivm_status ivm_angular_ranges(ivm_scene *scene, const uint64_t *d_M, int64_t *d_offsets, int32_t *d_cols,
                              double *d_ranges, size_t cap, hipStream_t stream);

/* Ray creation and suppression points along one trajectory, the visibility
 * ranges between them and their coherence times (Section III-C: the visibility
 * change nodes of the inter-visibility table of a mobile transmitter or
 * receiver; Section III-D, eq. 8: T_c,l = d_l / v_l; eq. 9: their mean).
 * Inputs are the outputs of ivm_txrx_visibility_table for n_snap >= 1
 * snapshots taken dt seconds apart (d_tx_vis, d_rx_vis uint64[N][W], d_los
 * uint8[N]) and the positions float[N][3] in metres; snapshot n's visibility
 * holds until snapshot n + 1 and the last snapshot ends the trajectory.
 * Outputs (caller-owned device memory, capacity N ranges):
 *   d_events int32[N][5]: for n >= 1 the facets that became visible from the
 *     Tx (ray creation), the facets no longer visible from it (suppression),
 *     the same for the Rx, and the LoS change (+1, -1 or 0); row 0 is zero;
 *   d_n_ranges int32[1]: L, the number of visibility ranges; a range starts at
 *     snapshot 0 and at every snapshot where either side's visible set or the
 *     LoS changes; d_range_start int32[L] its first snapshot;
 *   d_range_tc double[L]: the coherence time (seconds) of each range: for each
 *     side, its own range containing it (bounded by that side's changes) has
 *     route distance d (the position steps from its first snapshot to the
 *     next range's, or to N - 1), duration tau = snapshots x dt, velocity
 *     v = d / tau and time d / v; the range takes the smaller of the two, and
 *     a side that does not move (d = 0) sets no limit (+inf when neither moves);
 *   d_range_dist double[L][2]: each side's route distance over the range;
 *   d_tc_mean double[1]: the mean of the finite range times (+inf if none).
 * d_workspace: caller-owned device scratch of at least
 *   ivm_visibility_ranges_workspace_size(n_snap) bytes, 256-byte aligned;
 *   its contents on entry do not matter and calls sharing it must not overlap.
 * The counts and ranges are exact; the FP64 distances and times are summed in
 * snapshot order without contraction.  Asynchronous on `stream`.
 * Errors: IVM_ERR_INVALID_ARGUMENT (NULL pointers, misaligned workspace,
 * n_snap < 1, dt not a positive finite number), IVM_ERR_WORKSPACE (workspace
 * too small), IVM_ERR_HIP. */
ivm_status ivm_visibility_ranges_workspace_size(int32_t n_snap, size_t *bytes);
ivm_status ivm_visibility_ranges(const ivm_scene *scene, int32_t n_snap, const uint64_t *d_tx_vis,
                                 const uint64_t *d_rx_vis, const uint8_t *d_los, const float *d_tx, const float *d_rx,
                                 double dt, void *d_workspace, size_t workspace_bytes, int32_t *d_events,
                                 int32_t *d_range_start, double *d_range_tc, double *d_range_dist, int32_t *d_n_ranges,
                                 double *d_tc_mean, hipStream_t stream);

/* Allocation-free variant of ivm_visibility_ranges, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Arguments, outputs and results are those of
 * ivm_visibility_ranges without the workspace: the scratch is a fixed array of
 * the library, about 1.7 MB on each GPU the library runs on, held until the
 * process ends, sized for at most IVM_RANGES_NOALLOC_MAX_SNAP snapshots.  The
 * call runs on the current device (the stream must belong to it), looks the
 * array's address up on the first call on each device and allocates nothing.
 * Every call on one GPU shares that GPU's array (its contents on entry do not
 * matter): calls that overlap on one GPU, on any streams, race.
 * Errors: IVM_ERR_INVALID_ARGUMENT (as ivm_visibility_ranges), IVM_ERR_WORKSPACE
 * (n_snap > IVM_RANGES_NOALLOC_MAX_SNAP), IVM_ERR_HIP. */
#define IVM_RANGES_NOALLOC_MAX_SNAP 32768
ivm_status ivm_visibility_ranges_noalloc(const ivm_scene *scene, int32_t n_snap, const uint64_t *d_tx_vis,
                                         const uint64_t *d_rx_vis, const uint8_t *d_los, const float *d_tx,
                                         const float *d_rx, double dt, int32_t *d_events, int32_t *d_range_start,
                                         double *d_range_tc, double *d_range_dist, int32_t *d_n_ranges,
                                         double *d_tc_mean, hipStream_t stream);

/* ---- learned occluder ordering ---------------------------------------------
 * A small network scores, for a facet pair, how likely each of the 32 treelets is
 * to hold an occluder; IVM_ORDER_LEARNED visits the treelets in that order.  The
 * exact tests still decide every bit, so the order never changes a result.  The
 * matrix call runs the network on the pairs its visibility probes leave
 * undecided, right before the pair kernel.
 * Network: 24 -> 128 -> 128 -> 128 -> 32, ReLU on hidden layers, linear scores;
 * loss: mean binary cross-entropy with logits; optimiser: Adam (beta1 0.9,
 * beta2 0.999, eps 1e-8, bias-corrected).  Parameters are one FP32 array of
 * IVM_MLP_PARAMS values laid out W0[128][24], b0[128], W1[128][128], b1[128],
 * W2[128][128], b2[128], W3[32][128], b3[32].
 * Features of pair (i, j), with the scene box centre c0 and half-size s (largest
 * axis) of all vertices: centroid of i's samples and of j's, (x - c0) / s (3 + 3);
 * unit normals of i and j (3 + 3); areas / s^2 (1 + 1); distance between the
 * centroids (1); the AABB of both facets, min then max, (x - c0) / s (3 + 3);
 * unit direction from i's centroid to j's (3, zero if they coincide). */
#define IVM_MLP_FEATURES 24
#define IVM_MLP_HIDDEN 128
#define IVM_MLP_OUTPUTS 32
#define IVM_MLP_PARAMS 40352

#define IVM_MODEL_BF16 0 /* GEMMs on BF16 MFMA with FP32 accumulation */
#define IVM_MODEL_FP32 1 /* GEMMs in FP32 on the vector ALUs (reference mode) */

typedef struct ivm_model ivm_model; /* opaque host handle */

/* Device workspace for a model that trains or evaluates batches of up to max_batch rows. */
ivm_status ivm_model_workspace_size(int32_t max_batch, size_t *bytes);
/* d_workspace (caller-owned, 256-byte aligned) holds parameters, gradients, Adam
 * state and activations.  Parameters start at zero: set them before use. */
ivm_status ivm_model_create(void *d_workspace, size_t workspace_bytes, int32_t max_batch, int32_t precision,
                            ivm_model **out);
ivm_status ivm_model_destroy(ivm_model *model);
/* Copy IVM_MLP_PARAMS FP32 values (device) into the model and reset Adam. */
ivm_status ivm_model_set_params(ivm_model *model, const float *d_params, hipStream_t stream);
ivm_status ivm_model_get_params(const ivm_model *model, float *d_params, hipStream_t stream);
/* Scores (logits) float[n][32] for features float[n][24], n <= max_batch. */
ivm_status ivm_model_forward(ivm_model *model, int32_t n, const float *d_x, float *d_logits, hipStream_t stream);
/* Mean BCE-with-logits loss (float[1]) and its gradient (float[IVM_MLP_PARAMS])
 * for labels float[n][32] in {0, 1}; parameters are not changed. */
ivm_status ivm_model_loss_grad(ivm_model *model, int32_t n, const float *d_x, const float *d_y, float *d_loss,
                               float *d_grad, hipStream_t stream);
/* One Adam step with learning rate lr on the batch; d_loss (may be NULL) gets the
 * loss before the step. */
ivm_status ivm_model_train_step(ivm_model *model, int32_t n, const float *d_x, const float *d_y, float lr,
                                float *d_loss, hipStream_t stream);
/* Features float[n][24] of the pairs (d_i[k], d_j[k]) (see above). */
ivm_status ivm_pair_features(const ivm_scene *scene, int32_t n, const int32_t *d_i, const int32_t *d_j, float *d_x,
                             hipStream_t stream);
/* Hit records: for each pair, bit k of d_labels[k] is set iff some triangle of
 * treelet k (see ivm_triangle_groups) meets an admissible segment of the pair
 * (all hits, not the first).  Pairs with no admissible segment get 0. */
ivm_status ivm_pair_occluder_labels(ivm_scene *scene, int32_t n, const int32_t *d_i, const int32_t *d_j,
                                    uint32_t *d_labels, hipStream_t stream);
/* Attach (or, with NULL, detach) the model used by IVM_ORDER_LEARNED.  The scene
 * must have been built with IVM_SCENE_LEARNED. */
ivm_status ivm_scene_set_model(ivm_scene *scene, const ivm_model *model);

/* ---- batched scenes ----------------------------------------------------------
 * Many independent scenes in one run: per-scene orientation culls, then one
 * persistent any-hit launch over the candidate pairs of all scenes, one
 * persistent launch over all Tx/Rx items, then line of sight and candidate
 * counts (orders 0..2) per scene.  The first ivm_batch_run captures the launch
 * sequence in a hipGraph; later runs replay it.  Results per scene are those of
 * ivm_intervisibility_matrix, ivm_txrx_visibility_table and
 * ivm_image_tree_candidates (count mode). */
typedef struct ivm_batch ivm_batch; /* opaque host handle */

typedef struct ivm_batch_item {
    ivm_scene *scene;          /* built scene, kept alive by the caller */
    uint64_t *d_M;             /* uint64[F][W] */
    int32_t n_snap;            /* 0..IVM_MAX_SNAPSHOTS */
    const float *d_tx;         /* float[n_snap][3] */
    const float *d_rx;         /* float[n_snap][3] */
    uint64_t *d_tx_vis;        /* uint64[n_snap][W] */
    uint64_t *d_rx_vis;        /* uint64[n_snap][W] */
    uint8_t *d_los;            /* uint8[n_snap] */
    int64_t *d_counts;         /* int64[n_snap][3], or NULL */
} ivm_batch_item;

/* Device bytes for the batch's job tables and queue. */
ivm_status ivm_batch_workspace_size(int32_t n_items, size_t *bytes);
/* Copies the job tables to d_workspace (synchronous).  Every buffer named by the
 * items, d_stats (may be NULL; counters accumulate over runs) and the workspace
 * must outlive the batch.  opts->timing_events is ignored. */
ivm_status ivm_batch_create(int32_t n_items, const ivm_batch_item *items, const ivm_matrix_opts *opts,
                            ivm_stats *d_stats, void *d_workspace, size_t workspace_bytes, ivm_batch **out);
ivm_status ivm_batch_run(ivm_batch *batch, hipStream_t stream);
ivm_status ivm_batch_destroy(ivm_batch *batch);

/* Treelet (Morton group) index of every triangle in the caller's triangle order:
 * d_group is int32[T].  Treelet k holds sorted ranks [ceil(k T / 32), ceil((k+1) T / 32)). */
ivm_status ivm_triangle_groups(const ivm_scene *scene, int32_t *d_group, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* IVM_H */
