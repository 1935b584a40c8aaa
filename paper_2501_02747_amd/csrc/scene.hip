// scene.hip -- scene validation, layout and the Morton-code LBVH build.
//
// The scenario database of the paper's pre-processing flow (Section III-C,
// Fig. 7: vertex points, face IDs, triangulated faces) arrives as device
// arrays.  This file validates it (dyadic grids, FP64 exactness budget, planar
// facets), lays it out for traversal, and builds a bounding volume hierarchy:
//   1. 30-bit Morton codes of triangle centroids (Z-order, Morton 1966),
//      quantised exactly in integers inside the scene box;
//   2. a stable LSD radix sort of (code, triangle index);
//   3. 32 treelets = contiguous equal-count ranges of the sorted order, each a
//      binary radix tree built with Karras' method (HPG 2012);
//   4. node boxes as exact FP32 min/max over each node's contiguous range;
//   5. 64-byte nodes holding both child boxes, with subtrees of <= 4 triangles
//      collapsed into leaves.
#include <climits>
#include <cmath>

#include "ivm_internal.h"

namespace ivm {

static inline size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

Layout make_layout(int F, int T, int S, bool learned, int n_solids) {
    Layout L{};
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o = align_up(o + (bytes ? bytes : 1));
        return at;
    };
    size_t Tn = T > 0 ? (size_t)T : 1, Fn = F > 0 ? (size_t)F : 1, Sn = S > 0 ? (size_t)S : 1;
    size_t W = ((size_t)Fn + 63) / 64;
    size_t items = Fn * W;
    L.tri = take(Tn * 3 * sizeof(float4));
    L.tri_orig = take(Tn * sizeof(int));
    L.tri_group = take(Tn * sizeof(int));
    L.nodes = take(Tn * sizeof(Node));
    L.tl_box = take(kTreelets * 6 * sizeof(float));
    L.tl_root = take(kTreelets * sizeof(int));
    L.fplane = take(Fn * 6 * sizeof(double));
    L.fbox = take(Fn * 6 * sizeof(float));
    L.soff = take((Fn + 1) * sizeof(int));
    L.smp = take(Sn * sizeof(float4));
    L.sfacet = take(Sn * sizeof(int));
    L.status = take(64);
    L.extent = take(16 * sizeof(double));
    L.ibox = take(32 * sizeof(int));
    L.keys = take(Tn * sizeof(uint32_t));
    L.vals = take(Tn * sizeof(uint32_t));
    L.keys2 = take(Tn * sizeof(uint32_t));
    L.vals2 = take(Tn * sizeof(uint32_t));
    L.node_child = take(Tn * 2 * sizeof(int));
    L.node_range = take(Tn * 2 * sizeof(int));
    L.node_box = take(Tn * 6 * sizeof(float));
    L.ffirst = take(Fn * 2 * sizeof(int));
    L.tri_caller = take(Tn * 3 * sizeof(float4));
    L.fhull = take(Fn * kHullMax * sizeof(int));
    L.fhull_n = take(Fn * sizeof(int));
    L.scluster = take(Sn * sizeof(int));
    L.fchull = take(Fn * 4 * kHullMax * sizeof(int));
    L.fchull_n = take(Fn * 4 * sizeof(int));
    L.ffeat = take(Fn * 8 * sizeof(float));
    L.fnorm = take(8 * sizeof(float));
    const size_t Ns = n_solids > 0 ? (size_t)n_solids : 1;
    L.fflags = take(Fn * sizeof(int));
    L.fsolid = take(Fn * sizeof(int));
    L.sol_cnt = take((Ns + 1) * 2 * sizeof(int));
    L.sol_off = take((Ns + 1) * sizeof(int));
    L.sol_fac = take(Fn * sizeof(int));
    L.sol_rec = take(Ns * sizeof(int4));
    L.sol_plane = take(Ns * kSolidMaxPlanes * sizeof(int4));
    L.sol_nver = take(sizeof(int));
    L.nodes4 = take(Tn * sizeof(Node4));
    L.sol_box = take(Ns * 2 * sizeof(float4));
    {
        const size_t G = (size_t)solid_grid_dim(n_solids > 0 ? n_solids : 1), ncell = G * G;
        L.grid_p = take(2 * sizeof(float4));
        L.grid_cnt = take(2 * ncell * sizeof(int));
        L.grid_off = take((ncell + 1) * sizeof(int));
        L.grid_list = take(((size_t)kGridEntriesPerSolid * Ns + 1024) * sizeof(int));
        L.grid_ent = take(((size_t)kGridEntriesPerSolid * Ns + 1024) * 2 * sizeof(float4));
    }
    L.cand = take(items * sizeof(uint64_t));
    L.done = take(items * sizeof(uint64_t));
    L.und = take(items * sizeof(uint64_t));
    L.uprefix = take((items + 1) * sizeof(uint32_t));
    L.prefix = take((items + 1) * sizeof(uint32_t));
    {
        // orders 3-4 of the candidate counts reuse [cand, hi_end) between matrix
        // calls: M^T (64 W rows of W words), the column sums and a slab of at
        // least kHiMinSlab snapshots (two byte planes and a uint16 row each)
        const size_t Fp = 64 * W, need = Fp * W * 8 + Fp * 4 + (size_t)kHiMinSlab * Fp * 4;
        const size_t have = o - L.cand;
        L.hi = take(need > have ? need - have : 0);
        L.hi_end = o;
    }
    L.scan_tmp = take(((items + 1) / 4096 + 2) * sizeof(uint32_t));
    L.queue = take(256);
    L.learned_bytes = learned ? Fn * (Fn - 1) / 2 * sizeof(uint64_t) : 0;
    L.learned = take(L.learned_bytes);
    L.total = o;
    return L;
}

// ---------------------------------------------------------------------------
// validation and preparation
// ---------------------------------------------------------------------------

// ibox layout (ints): [0..2] vertex lo (vertex units), [3..5] vertex hi,
// [6..8] lo of vertices and samples (sample units), [9..11] hi, [12] E bits,
// [13] max samples per facet.
__global__ void k_init(int *ibox, int *status, int *ffirst, int F) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < 32) {
        const bool is_lo = (i < 3) || (i >= 6 && i < 9);
        const bool is_hi = (i >= 3 && i < 6) || (i >= 9 && i < 12);
        ibox[i] = is_lo ? INT_MAX : (is_hi ? INT_MIN : 0);
    }
    if (i == 0) status[0] = 0;
    for (int f = i; f < F; f += gridDim.x * blockDim.x) {
        ffirst[2 * f] = INT_MAX;
        ffirst[2 * f + 1] = 0;
    }
}

__device__ inline bool on_grid(float x, float scale, int *out) {
    float y = x * scale;  // exact: scale is a power of two
    if (!(fabsf(y) < 16777216.0f) || y != floorf(y)) return false;
    *out = (int)y;
    return true;
}

__global__ void k_tri_prep(ivm_scene_desc d, int *ibox, int *status, int *ffirst) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= d.n_triangles) return;
    const float vs = ldexpf(1.0f, d.grid_vertex_log2);
    const float ss = ldexpf(1.0f, d.grid_sample_log2);
    int f = d.tri_facet[t];
    int bad = 0;
    if (f < 0 || f >= d.n_facets) {
        bad |= kStInvalid;
        f = 0;
    }
    if (t > 0 && d.tri_facet[t - 1] > d.tri_facet[t]) bad |= kStInvalid;
    float v[3][3];
    for (int c = 0; c < 3; ++c) {
        int vi = d.tri_vertices[3 * t + c];
        if (vi < 0 || vi >= d.n_vertices) {
            bad |= kStInvalid;
            vi = 0;
        }
        for (int k = 0; k < 3; ++k) {
            v[c][k] = d.vertices[3 * vi + k];
            int gv, gsv;
            if (!on_grid(v[c][k], vs, &gv) || !on_grid(v[c][k], ss, &gsv)) {
                bad |= kStGrid;
                continue;
            }
            atomicMin(&ibox[k], gv);
            atomicMax(&ibox[3 + k], gv);
            atomicMin(&ibox[6 + k], gsv);
            atomicMax(&ibox[9 + k], gsv);
        }
    }
    float E = 0.0f;
    for (int k = 0; k < 3; ++k) {
        E = fmaxf(E, fabsf(v[1][k] - v[0][k]));
        E = fmaxf(E, fabsf(v[2][k] - v[0][k]));
        E = fmaxf(E, fabsf(v[2][k] - v[1][k]));
    }
    atomicMax(&ibox[12], __float_as_int(E));
    if (!(bad & kStInvalid)) {
        atomicMin(&ffirst[2 * f], t);
        atomicAdd(&ffirst[2 * f + 1], 1);
    }
    if (bad) atomicOr(status, bad);
}

__global__ void k_sample_prep(ivm_scene_desc d, int *ibox, int *status) {
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= d.n_samples) return;
    const float ss = ldexpf(1.0f, d.grid_sample_log2);
    int bad = 0;
    for (int k = 0; k < 3; ++k) {
        int gv;
        if (!on_grid(d.samples[3 * s + k], ss, &gv)) {
            bad |= kStGrid;
            continue;
        }
        atomicMin(&ibox[6 + k], gv);
        atomicMax(&ibox[9 + k], gv);
    }
    if (bad) atomicOr(status, bad);
}


__global__ void k_facet_prep(ivm_scene_desc d, const int *ffirst, double *fplane, float *fbox, int *soff,
                             float4 *smp, int *sfacet, int *ibox, int *status, int *fhull_n, int *scluster) {
    int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= d.n_facets) return;
    int bad = 0;
    int t0 = ffirst[2 * f], nt = ffirst[2 * f + 1];
    // sample range
    int s0 = d.sample_offsets[f], s1 = d.sample_offsets[f + 1];
    if (s0 < 0 || s1 < s0 || s1 > d.n_samples) {
        bad |= kStInvalid;
        s0 = s1 = 0;
    }
    if (f == 0 && s0 != 0) bad |= kStInvalid;
    if (f == d.n_facets - 1 && s1 != d.n_samples) bad |= kStInvalid;
    soff[f] = s0;
    if (f == d.n_facets - 1) soff[f + 1] = s1;
    if (s1 - s0 > kMaxSamplesPerFacet) bad |= kStInvalid;
    atomicMax(&ibox[13], s1 - s0);
    for (int s = s0; s < s1; ++s) {
        smp[s] = make_float4(d.samples[3 * s], d.samples[3 * s + 1], d.samples[3 * s + 2], 0.0f);
        sfacet[s] = f;
    }
    double a[3] = {0, 0, 0}, n[3] = {0, 0, 0};
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    if (nt == 0 || t0 == INT_MAX) {
        bad |= kStDegenerate;
    } else {
        double P[3][3];
        for (int c = 0; c < 3; ++c) {
            int vi = d.tri_vertices[3 * t0 + c];
            vi = (vi < 0 || vi >= d.n_vertices) ? 0 : vi;
            for (int k = 0; k < 3; ++k) P[c][k] = (double)d.vertices[3 * vi + k];
        }
        double e1[3] = {P[1][0] - P[0][0], P[1][1] - P[0][1], P[1][2] - P[0][2]};
        double e2[3] = {P[2][0] - P[0][0], P[2][1] - P[0][1], P[2][2] - P[0][2]};
        n[0] = e1[1] * e2[2] - e1[2] * e2[1];
        n[1] = e1[2] * e2[0] - e1[0] * e2[2];
        n[2] = e1[0] * e2[1] - e1[1] * e2[0];
        for (int k = 0; k < 3; ++k) a[k] = P[0][k];
        if (n[0] == 0.0 && n[1] == 0.0 && n[2] == 0.0) bad |= kStDegenerate;
        for (int t = t0; t < t0 + nt && t < d.n_triangles; ++t) {
            for (int c = 0; c < 3; ++c) {
                int vi = d.tri_vertices[3 * t + c];
                vi = (vi < 0 || vi >= d.n_vertices) ? 0 : vi;
                double x[3];
                for (int k = 0; k < 3; ++k) {
                    x[k] = (double)d.vertices[3 * vi + k];
                    lo[k] = fminf(lo[k], d.vertices[3 * vi + k]);
                    hi[k] = fmaxf(hi[k], d.vertices[3 * vi + k]);
                }
                double o = (x[0] - a[0]) * n[0] + (x[1] - a[1]) * n[1] + (x[2] - a[2]) * n[2];
                if (o != 0.0) bad |= kStDegenerate;  // every triangle of a facet lies in its plane
            }
        }
    }
    for (int k = 0; k < 3; ++k) {
        fplane[6 * f + k] = a[k];
        fplane[6 * f + 3 + k] = n[k];
        fbox[6 * f + k] = lo[k];
        fbox[6 * f + 3 + k] = hi[k];
    }
    const double an0 = fabs(n[0]), an1 = fabs(n[1]), an2 = fabs(n[2]);
    const int drop = (an0 >= an1 && an0 >= an2) ? 0 : (an1 >= an2 ? 1 : 2);
    const int ns = s1 - s0;
    // The sample hulls stand for the facet's sample set in 3-D only when every
    // sample lies in the facet's plane (exact: the orient budget covers samples).
    bool in_plane = true;
    for (int s = s0; s < s1 && in_plane; ++s) {
        const double o = ((double)d.samples[3 * s] - a[0]) * n[0] + ((double)d.samples[3 * s + 1] - a[1]) * n[1] +
                         ((double)d.samples[3 * s + 2] - a[2]) * n[2];
        in_plane = o == 0.0;
    }
    const bool hull_ok = !(bad & kStDegenerate) && in_plane && ns > 0 && ns <= kMaxSamplesPerFacet;
    fhull_n[f] = hull_ok ? 1 : 0;  // a request: k_facet_hulls computes the hulls and their sizes
    // quadrant clusters: split the samples at their centroid along both in-plane axes
    // (exact: u * ns and the sum of u are FP64 integers on the sample grid)
    const int ax = drop == 0 ? 1 : 0, ay = drop == 2 ? 1 : 2;
    double su = 0.0, sv = 0.0;
    for (int s = s0; s < s1; ++s) {
        su += (double)d.samples[3 * s + ax];
        sv += (double)d.samples[3 * s + ay];
    }
    for (int s = s0; s < s1; ++s)
        scluster[s] = ((double)d.samples[3 * s + ax] * ns > su ? 1 : 0) + ((double)d.samples[3 * s + ay] * ns > sv ? 2 : 0);
    if (bad) atomicOr(status, bad);
}

// Convex hulls of each facet's samples and of its four quadrant clusters, in the
// plane that drops the normal's largest axis, one wave per facet (four per
// block): lane m holds sample m's in-plane coordinates and ranks itself in
// (u, v) order (ties by list position), then one lane per hull runs Andrew's
// monotone chain over the ordered points in LDS (strict turns only, so
// collinear and repeated points drop out).  The sample grid makes every cross
// product an exact FP64 integer.  A hull with more than kHullMax points, or a
// facet whose request flag is clear, gets size 0 (unavailable).  Each wave uses
// only its own LDS rows, so waves synchronise on their own.
__global__ __launch_bounds__(256) void k_facet_hulls(ivm_scene_desc d, const double *fplane, const int *soff,
                                                     const int *scluster, int *fhull, int *fhull_n, int *fchull,
                                                     int *fchull_n) {
    __shared__ float sU[4][kMaxSamplesPerFacet], sV[4][kMaxSamplesPerFacet];
    __shared__ unsigned char sOrd[4][5][kMaxSamplesPerFacet];
    __shared__ unsigned char sH[4][5][2 * kMaxSamplesPerFacet + 1];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int f = blockIdx.x * 4 + wv;
    if (f >= d.n_facets) return;  // (wave-uniform)
    const bool want = fhull_n[f] != 0;
    const int s0 = soff[f], ns = want ? soff[f + 1] - s0 : 0;
    const double *nrm = fplane + 6 * f + 3;
    const double an0 = fabs(nrm[0]), an1 = fabs(nrm[1]), an2 = fabs(nrm[2]);
    const int drop = (an0 >= an1 && an0 >= an2) ? 0 : (an1 >= an2 ? 1 : 2);
    const int ax = drop == 0 ? 1 : 0, ay = drop == 2 ? 1 : 2;
    const bool act = lane < ns;
    const float u = act ? d.samples[3 * (s0 + lane) + ax] : 0.f;
    const float v = act ? d.samples[3 * (s0 + lane) + ay] : 0.f;
    const int cl = act ? scluster[s0 + lane] : -1;
    sU[wv][lane] = u;
    sV[wv][lane] = v;
    int r = 0, rc = 0;
    for (int k = 0; k < ns; ++k) {
        const float uk = __shfl(u, k), vk = __shfl(v, k);
        const int ck = __shfl(cl, k);
        const bool before = uk < u || (uk == u && (vk < v || (vk == v && k < lane)));
        r += before;
        rc += before && ck == cl;
    }
    if (act) {
        sOrd[wv][0][r] = (unsigned char)lane;
        sOrd[wv][1 + cl][rc] = (unsigned char)lane;
    }
    int ncl[4];
    for (int c = 0; c < 4; ++c) ncl[c] = __popcll(__ballot(act && cl == c));
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (lane < 5) {
        const int n = lane == 0 ? ns : ncl[lane - 1];
        const unsigned char *o = sOrd[wv][lane];
        unsigned char *h = sH[wv][lane];
        auto U = [&](int m) { return (double)sU[wv][m]; };
        auto V = [&](int m) { return (double)sV[wv][m]; };
        auto turn = [&](int a, int b, int c) { return (U(b) - U(a)) * (V(c) - V(a)) - (V(b) - V(a)) * (U(c) - U(a)); };
        int k = 0;
        for (int m = 0; m < n; ++m) {  // lower hull
            while (k >= 2 && turn(h[k - 2], h[k - 1], o[m]) <= 0.0) --k;
            h[k++] = o[m];
        }
        for (int m = n - 2, lo = k + 1; m >= 0; --m) {  // upper hull
            while (k >= lo && turn(h[k - 2], h[k - 1], o[m]) <= 0.0) --k;
            h[k++] = o[m];
        }
        if (k > 1) --k;  // the last point repeats the first
        if (n <= 0 || k > kHullMax) k = 0;
        int *out = lane == 0 ? fhull + kHullMax * f : fchull + (4 * f + lane - 1) * kHullMax;
        for (int m = 0; m < k; ++m) out[m] = s0 + h[m];
        if (lane == 0) fhull_n[f] = k;
        else fchull_n[4 * f + lane - 1] = k;
    }
}

// Exactness budget (see ivm.h) from the integer boxes.
__global__ void k_budget(ivm_scene_desc d, const int *ibox, double *extent, int *status) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const double inv_s = ldexp(1.0, -d.grid_sample_log2);
    double D = 0.0;
    for (int k = 0; k < 3; ++k) {
        extent[k] = (double)ibox[6 + k];
        extent[3 + k] = (double)ibox[9 + k];
        if (ibox[9 + k] >= ibox[6 + k]) D = fmax(D, ((double)ibox[9 + k] - (double)ibox[6 + k]) * inv_s);
    }
    double E = (double)__int_as_float(ibox[12]);
    extent[6] = E;
    extent[7] = (double)d.grid_vertex_log2;
    extent[8] = (double)d.grid_sample_log2;
    int bad = 0;
    if (d.grid_sample_log2 < d.grid_vertex_log2) bad |= kStGrid;
    const int g = d.grid_vertex_log2, k = d.grid_sample_log2 - d.grid_vertex_log2;
    double bound = (6.0 * D * E * E + 12.0 * D * D * E) * ldexp(1.0, 3 * g + 2 * k);
    if (!(bound < 9007199254740992.0)) bad |= kStGrid;             // 2^53
    if (!(D * ldexp(1.0, d.grid_sample_log2) < 16777216.0)) bad |= kStGrid;  // 2^24
    if (bad) atomicOr(status, bad);
}

// ---------------------------------------------------------------------------
// Morton codes and sort
// ---------------------------------------------------------------------------

__device__ inline uint32_t spread10(uint32_t x) {
    // place bit b of x at bit 3b
    x &= 0x3ffu;
    x = (x | (x << 16)) & 0x030000FFu;
    x = (x | (x << 8)) & 0x0300F00Fu;
    x = (x | (x << 4)) & 0x030C30C3u;
    x = (x | (x << 2)) & 0x09249249u;
    return x;
}

// Centroid quantisation in exact integers: with vertex-unit coordinates,
// c3 = a + b + c and the box [lo, hi] over all vertices of all triangles,
// q = floor((c3 - 3 lo) * 1024 / (3 (hi - lo) + 1)) in [0, 1023] per axis.
// Code bits interleave x (most significant), y, z.
__global__ void k_morton(ivm_scene_desc d, const int *ibox, uint32_t *keys, uint32_t *vals) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= d.n_triangles) return;
    const float vs = ldexpf(1.0f, d.grid_vertex_log2);
    long long c3[3] = {0, 0, 0};
    for (int c = 0; c < 3; ++c) {
        int vi = d.tri_vertices[3 * t + c];
        vi = (vi < 0 || vi >= d.n_vertices) ? 0 : vi;
        for (int k = 0; k < 3; ++k) c3[k] += (long long)(d.vertices[3 * vi + k] * vs);
    }
    uint32_t q[3];
    for (int k = 0; k < 3; ++k) {
        long long lo = ibox[k], hi = ibox[3 + k];
        long long den = 3 * (hi - lo) + 1;
        long long num = (c3[k] - 3 * lo) * 1024;
        long long v = num >= 0 ? num / den : 0;
        q[k] = (uint32_t)(v < 0 ? 0 : (v > 1023 ? 1023 : v));
    }
    keys[t] = (spread10(q[0]) << 2) | (spread10(q[1]) << 1) | spread10(q[2]);
    vals[t] = (uint32_t)t;
}

// Stable LSD radix sort of (key, value) in one workgroup: 4-bit digits, 8
// passes.  Each thread owns a contiguous chunk; per-thread digit counts are
// scanned digit-major so equal digits keep their order.
constexpr int kSortThreads = 512;

__global__ __launch_bounds__(kSortThreads) void k_radix_sort(uint32_t *keys, uint32_t *vals, uint32_t *keys2,
                                                             uint32_t *vals2, int n) {
    __shared__ uint32_t cnt[16 * kSortThreads];
    __shared__ uint32_t part[kSortThreads];
    const int tid = threadIdx.x;
    const int chunk = (n + kSortThreads - 1) / kSortThreads;
    const int beg = min(n, tid * chunk), end = min(n, beg + chunk);
    uint32_t *sk = keys, *sv = vals, *dk = keys2, *dv = vals2;
    for (int pass = 0; pass < 8; ++pass) {
        const int shift = 4 * pass;
        for (int dgt = 0; dgt < 16; ++dgt) cnt[dgt * kSortThreads + tid] = 0;
        for (int i = beg; i < end; ++i) cnt[((sk[i] >> shift) & 15u) * kSortThreads + tid] += 1;
        __syncthreads();
        // exclusive scan over the 16 * kSortThreads counters (16 consecutive per thread)
        uint32_t local = 0;
        for (int m = 0; m < 16; ++m) local += cnt[tid * 16 + m];
        part[tid] = local;
        __syncthreads();
        for (int off = 1; off < kSortThreads; off <<= 1) {
            uint32_t v = tid >= off ? part[tid - off] : 0;
            __syncthreads();
            part[tid] += v;
            __syncthreads();
        }
        uint32_t run = part[tid] - local;
        for (int m = 0; m < 16; ++m) {
            uint32_t c = cnt[tid * 16 + m];
            cnt[tid * 16 + m] = run;
            run += c;
        }
        __syncthreads();
        for (int i = beg; i < end; ++i) {
            uint32_t kk = sk[i];
            uint32_t dgt = (kk >> shift) & 15u;
            uint32_t pos = cnt[dgt * kSortThreads + tid]++;
            dk[pos] = kk;
            dv[pos] = sv[i];
        }
        __syncthreads();
        uint32_t *tk = sk, *tv = sv;
        sk = dk;
        sv = dv;
        dk = tk;
        dv = tv;
    }
}

// ---------------------------------------------------------------------------
// Sorted triangle records and Karras hierarchy per treelet
// ---------------------------------------------------------------------------

__device__ inline void treelet_range(int k, int T, int *s, int *e) {
    *s = (int)(((long long)k * T + kTreelets - 1) / kTreelets);
    *e = (int)(((long long)(k + 1) * T + kTreelets - 1) / kTreelets);
}

__global__ void k_tri_sorted(ivm_scene_desc d, const uint32_t *order, float4 *tri, int *tri_orig, int *tri_group,
                             float4 *tri_caller) {
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= d.n_triangles) return;
    int t = (int)order[r];
    float P[3][3];
    for (int c = 0; c < 3; ++c) {
        int vi = d.tri_vertices[3 * t + c];
        vi = (vi < 0 || vi >= d.n_vertices) ? 0 : vi;
        for (int k = 0; k < 3; ++k) P[c][k] = d.vertices[3 * vi + k];
    }
    int f = d.tri_facet[t];
    float e1[3], e2[3];
    float m1 = 0.f, m2 = 0.f;
    for (int k = 0; k < 3; ++k) {
        e1[k] = P[1][k] - P[0][k];
        e2[k] = P[2][k] - P[0][k];
        m1 = fmaxf(m1, fabsf(e1[k]));
        m2 = fmaxf(m2, fabsf(e2[k]));
    }
    const float4 A = make_float4(P[0][0], P[0][1], P[0][2], __int_as_float(f));
    const float4 B = make_float4(e1[0], e1[1], e1[2], m1);
    const float4 C = make_float4(e2[0], e2[1], e2[2], m2);
    tri[3 * r + 0] = A;
    tri[3 * r + 1] = B;
    tri[3 * r + 2] = C;
    tri_caller[3 * t + 0] = A;
    tri_caller[3 * t + 1] = B;
    tri_caller[3 * t + 2] = C;
    tri_orig[r] = t;
    tri_group[t] = (int)(((long long)r * kTreelets) / d.n_triangles);
}

__device__ inline int delta64(const uint32_t *codes, int base, int n, int a, int b) {
    if (b < 0 || b >= n) return -1;
    unsigned long long ka = ((unsigned long long)codes[base + a] << 32) | (unsigned)(base + a);
    unsigned long long kb = ((unsigned long long)codes[base + b] << 32) | (unsigned)(base + b);
    return __clzll(ka ^ kb);
}

// One thread per global slot x; slot x is internal node li = x - s_k of treelet
// k = floor(32 x / T) when li < n_k - 1.  child[2x+c] = leaf rank | 0x80000000
// or the global slot of an internal child.
__global__ void k_karras(int T, const uint32_t *codes, int *child, int *range) {
    int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= T) return;
    int k = (int)(((long long)x * kTreelets) / T);
    int s, e;
    treelet_range(k, T, &s, &e);
    const int n = e - s;
    const int i = x - s;
    if (i >= n - 1) return;
    const int dir = (delta64(codes, s, n, i, i + 1) - delta64(codes, s, n, i, i - 1)) >= 0 ? 1 : -1;
    const int dmin = delta64(codes, s, n, i, i - dir);
    int lmax = 2;
    while (delta64(codes, s, n, i, i + lmax * dir) > dmin) lmax <<= 1;
    int l = 0;
    for (int t = lmax >> 1; t >= 1; t >>= 1)
        if (delta64(codes, s, n, i, i + (l + t) * dir) > dmin) l += t;
    const int j = i + l * dir;
    const int dnode = delta64(codes, s, n, i, j);
    int sp = 0;
    int t = l;
    do {
        t = (t + 1) >> 1;
        if (delta64(codes, s, n, i, i + (sp + t) * dir) > dnode) sp += t;
    } while (t > 1);
    const int gamma = i + sp * dir + (dir < 0 ? -1 : 0);
    const int lo = min(i, j), hi = max(i, j);
    child[2 * x + 0] = (lo == gamma) ? (int)(0x80000000u | (unsigned)(s + gamma)) : s + gamma;
    child[2 * x + 1] = (hi == gamma + 1) ? (int)(0x80000000u | (unsigned)(s + gamma + 1)) : s + gamma + 1;
    range[2 * x + 0] = s + lo;
    range[2 * x + 1] = s + hi;
}

__device__ inline void tri_box(const float4 *tri, int r, float lo[3], float hi[3]) {
    float4 A = tri[3 * r], B = tri[3 * r + 1], C = tri[3 * r + 2];
    float a[3] = {A.x, A.y, A.z}, b[3] = {A.x + B.x, A.y + B.y, A.z + B.z}, c[3] = {A.x + C.x, A.y + C.y, A.z + C.z};
    for (int k = 0; k < 3; ++k) {
        lo[k] = fminf(a[k], fminf(b[k], c[k]));
        hi[k] = fmaxf(a[k], fmaxf(b[k], c[k]));
    }
}

__device__ inline bool is_internal_slot(int x, int T) {
    int k = (int)(((long long)x * kTreelets) / T);
    int s, e;
    treelet_range(k, T, &s, &e);
    return x - s < e - s - 1;
}

__global__ void k_node_boxes(int T, const float4 *tri, const int *range, float *nbox) {
    int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= T || !is_internal_slot(x, T)) return;
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int r = range[2 * x]; r <= range[2 * x + 1]; ++r) {
        float l2[3], h2[3];
        tri_box(tri, r, l2, h2);
        for (int k = 0; k < 3; ++k) {
            lo[k] = fminf(lo[k], l2[k]);
            hi[k] = fmaxf(hi[k], h2[k]);
        }
    }
    for (int k = 0; k < 3; ++k) {
        nbox[6 * x + k] = lo[k];
        nbox[6 * x + 3 + k] = hi[k];
    }
}

__device__ inline void child_ref_box(int raw, const float4 *tri, const int *range, const float *nbox, int *ref,
                                     float lo[3], float hi[3]) {
    if (raw & 0x80000000) {
        int r = raw & 0x7fffffff;
        *ref = leaf_ref(r, 1);
        tri_box(tri, r, lo, hi);
        return;
    }
    int y = raw;
    int first = range[2 * y], last = range[2 * y + 1];
    *ref = (last - first + 1 <= kLeafMax) ? leaf_ref(first, last - first + 1) : y;
    for (int k = 0; k < 3; ++k) {
        lo[k] = nbox[6 * y + k];
        hi[k] = nbox[6 * y + 3 + k];
    }
}

__global__ void k_finalize(int T, const float4 *tri, const int *child, const int *range, const float *nbox,
                           Node *nodes) {
    int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= T) return;
    Node nd;
    if (!is_internal_slot(x, T)) {
        nd.a = nd.b = nd.c = make_float4(0, 0, 0, 0);
        nd.d = make_int4(0, 0, 0, -1);
        nodes[x] = nd;
        return;
    }
    int r0, r1;
    float l0[3], h0[3], l1[3], h1[3];
    child_ref_box(child[2 * x], tri, range, nbox, &r0, l0, h0);
    child_ref_box(child[2 * x + 1], tri, range, nbox, &r1, l1, h1);
    nd.a = make_float4(l0[0], l0[1], l0[2], h0[0]);
    nd.b = make_float4(h0[1], h0[2], l1[0], l1[1]);
    nd.c = make_float4(l1[2], h1[0], h1[1], h1[2]);
    nd.d = make_int4(r0, r1, range[2 * x], range[2 * x + 1]);
    nodes[x] = nd;
}

// 4-wide records from the finished binary nodes (one thread per slot).
__global__ void k_wide(int T, const Node *nodes, Node4 *nodes4) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= T) return;
    float lo[3][4], hi[3][4];
    int ref[4];
    int n = 0;  // slots used
    for (int q = 0; q < 4; ++q) {
        ref[q] = kNoRef;
        for (int k = 0; k < 3; ++k) {
            lo[k][q] = INFINITY;
            hi[k][q] = -INFINITY;
        }
    }
    if (is_internal_slot(x, T)) {
        const Node nd = nodes[x];
        const int cref[2] = {nd.d.x, nd.d.y};
        const float cb[2][6] = {{nd.a.x, nd.a.y, nd.a.z, nd.a.w, nd.b.x, nd.b.y},
                                {nd.b.z, nd.b.w, nd.c.x, nd.c.y, nd.c.z, nd.c.w}};
        for (int h = 0; h < 2; ++h) {
            if (cref[h] < 0) {  // a leaf child stands for itself
                ref[n] = cref[h];
                for (int k = 0; k < 3; ++k) {
                    lo[k][n] = cb[h][k];
                    hi[k][n] = cb[h][3 + k];
                }
                ++n;
            } else {            // an internal child contributes its two children
                const Node cd = nodes[cref[h]];
                const int gref[2] = {cd.d.x, cd.d.y};
                const float gb[2][6] = {{cd.a.x, cd.a.y, cd.a.z, cd.a.w, cd.b.x, cd.b.y},
                                        {cd.b.z, cd.b.w, cd.c.x, cd.c.y, cd.c.z, cd.c.w}};
                for (int g2 = 0; g2 < 2; ++g2) {
                    ref[n] = gref[g2];
                    for (int k = 0; k < 3; ++k) {
                        lo[k][n] = gb[g2][k];
                        hi[k][n] = gb[g2][3 + k];
                    }
                    ++n;
                }
            }
        }
    }
    Node4 w;
    w.lox = make_float4(lo[0][0], lo[0][1], lo[0][2], lo[0][3]);
    w.loy = make_float4(lo[1][0], lo[1][1], lo[1][2], lo[1][3]);
    w.loz = make_float4(lo[2][0], lo[2][1], lo[2][2], lo[2][3]);
    w.hix = make_float4(hi[0][0], hi[0][1], hi[0][2], hi[0][3]);
    w.hiy = make_float4(hi[1][0], hi[1][1], hi[1][2], hi[1][3]);
    w.hiz = make_float4(hi[2][0], hi[2][1], hi[2][2], hi[2][3]);
    w.ref = make_int4(ref[0], ref[1], ref[2], ref[3]);
    w.pad = make_int4(n, 0, 0, 0);
    nodes4[x] = w;
}

__global__ void k_treelets(int T, const float4 *tri, const float *nbox, float *tl_box, int *tl_root) {
    int k = threadIdx.x;
    if (k >= kTreelets) return;
    int s, e;
    treelet_range(k, T, &s, &e);
    const int n = e - s;
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    int root = 0x7fffffff;
    if (n > 0 && n <= kLeafMax) {
        root = leaf_ref(s, n);
        for (int r = s; r < e; ++r) {
            float l2[3], h2[3];
            tri_box(tri, r, l2, h2);
            for (int c = 0; c < 3; ++c) {
                lo[c] = fminf(lo[c], l2[c]);
                hi[c] = fmaxf(hi[c], h2[c]);
            }
        }
    } else if (n > kLeafMax) {
        root = s;
        for (int c = 0; c < 3; ++c) {
            lo[c] = nbox[6 * s + c];
            hi[c] = nbox[6 * s + 3 + c];
        }
    }
    tl_root[k] = root;
    for (int c = 0; c < 3; ++c) {
        tl_box[6 * k + c] = lo[c];
        tl_box[6 * k + 3 + c] = hi[c];
    }
}

// Per-facet inputs of the pair features: centroid of the samples, unit normal and
// area, normalised by the box of all vertices (centre c0, half-size s of the
// largest axis).
__global__ void k_facet_feat(int F, int g, const int *ibox, const int *soff, const float4 *smp, const double *fplane,
                             const int *ffirst, const float4 *tri_caller, float *ffeat, float *fnorm) {
    const float inv = ldexpf(1.0f, -g);
    float c0[3], hs = 0.f;
    for (int k = 0; k < 3; ++k) {
        const float lo = (float)ibox[k] * inv, hi = (float)ibox[3 + k] * inv;
        c0[k] = 0.5f * (lo + hi);
        hs = fmaxf(hs, 0.5f * (hi - lo));
    }
    if (!(hs > 0.f)) hs = 1.f;
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f == 0) {
        fnorm[0] = c0[0]; fnorm[1] = c0[1]; fnorm[2] = c0[2]; fnorm[3] = hs;
    }
    if (f >= F) return;
    float cx = 0.f, cy = 0.f, cz = 0.f;
    const int s0 = soff[f], s1 = soff[f + 1];
    for (int s = s0; s < s1; ++s) {
        cx += smp[s].x; cy += smp[s].y; cz += smp[s].z;
    }
    const float ns = s1 > s0 ? (float)(s1 - s0) : 1.f;
    const double *pl = fplane + 6 * f;
    const double nl = sqrt(pl[3] * pl[3] + pl[4] * pl[4] + pl[5] * pl[5]);
    float area = 0.f;
    const int t0 = ffirst[2 * f], nt = ffirst[2 * f + 1];
    for (int t = t0; t < t0 + nt; ++t) {
        const float4 B = tri_caller[3 * t + 1], C = tri_caller[3 * t + 2];
        const float x = B.y * C.z - B.z * C.y, y = B.z * C.x - B.x * C.z, z = B.x * C.y - B.y * C.x;
        area += 0.5f * sqrtf(x * x + y * y + z * z);
    }
    float *o = ffeat + 8 * f;
    o[0] = (cx / ns - c0[0]) / hs;
    o[1] = (cy / ns - c0[1]) / hs;
    o[2] = (cz / ns - c0[2]) / hs;
    o[3] = nl > 0.0 ? (float)(pl[3] / nl) : 0.f;
    o[4] = nl > 0.0 ? (float)(pl[4] / nl) : 0.f;
    o[5] = nl > 0.0 ? (float)(pl[5] / nl) : 0.f;
    o[6] = area / (hs * hs);
    o[7] = 0.f;
}

__global__ void k_groups(int T, const int *tri_group, int32_t *out) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < T) out[t] = tri_group[t];
}

static inline unsigned nblk(long long n, int b) { return (unsigned)((n + b - 1) / b); }

hipError_t launch_build(Scene &sc, hipStream_t s) {
    const ivm_scene_desc &d = sc.desc;
    char *ws = (char *)sc.ws;
    const Layout &L = sc.lay;
    int *ibox = (int *)(ws + L.ibox);
    int *status = (int *)(ws + L.status);
    int *ffirst = (int *)(ws + L.ffirst);
    const int F = d.n_facets, T = d.n_triangles, S = d.n_samples;
    hipLaunchKernelGGL(k_init, dim3(nblk(F > 32 ? F : 32, 256)), dim3(256), 0, s, ibox, status, ffirst, F);
    if (T > 0) hipLaunchKernelGGL(k_tri_prep, dim3(nblk(T, 256)), dim3(256), 0, s, d, ibox, status, ffirst);
    if (S > 0) hipLaunchKernelGGL(k_sample_prep, dim3(nblk(S, 256)), dim3(256), 0, s, d, ibox, status);
    if (F > 0)
        hipLaunchKernelGGL(k_facet_prep, dim3(nblk(F, 128)), dim3(128), 0, s, d, ffirst, (double *)(ws + L.fplane),
                           (float *)(ws + L.fbox), (int *)(ws + L.soff), (float4 *)(ws + L.smp),
                           (int *)(ws + L.sfacet), ibox, status, (int *)(ws + L.fhull_n), (int *)(ws + L.scluster));
    if (F > 0)
        hipLaunchKernelGGL(k_facet_hulls, dim3(nblk(F, 4)), dim3(256), 0, s, d, (const double *)(ws + L.fplane),
                           (const int *)(ws + L.soff), (const int *)(ws + L.scluster), (int *)(ws + L.fhull),
                           (int *)(ws + L.fhull_n), (int *)(ws + L.fchull), (int *)(ws + L.fchull_n));
    hipLaunchKernelGGL(k_budget, dim3(1), dim3(64), 0, s, d, ibox, (double *)(ws + L.extent), status);
    if (T > 0) {
        uint32_t *keys = (uint32_t *)(ws + L.keys), *vals = (uint32_t *)(ws + L.vals);
        hipLaunchKernelGGL(k_morton, dim3(nblk(T, 256)), dim3(256), 0, s, d, ibox, keys, vals);
        hipLaunchKernelGGL(k_radix_sort, dim3(1), dim3(kSortThreads), 0, s, keys, vals, (uint32_t *)(ws + L.keys2),
                           (uint32_t *)(ws + L.vals2), T);
        float4 *tri = (float4 *)(ws + L.tri);
        hipLaunchKernelGGL(k_tri_sorted, dim3(nblk(T, 256)), dim3(256), 0, s, d, vals, tri, (int *)(ws + L.tri_orig),
                           (int *)(ws + L.tri_group), (float4 *)(ws + L.tri_caller));
        int *child = (int *)(ws + L.node_child), *range = (int *)(ws + L.node_range);
        float *nbox = (float *)(ws + L.node_box);
        hipLaunchKernelGGL(k_karras, dim3(nblk(T, 256)), dim3(256), 0, s, T, keys, child, range);
        hipLaunchKernelGGL(k_node_boxes, dim3(nblk(T, 128)), dim3(128), 0, s, T, tri, range, nbox);
        hipLaunchKernelGGL(k_finalize, dim3(nblk(T, 256)), dim3(256), 0, s, T, tri, child, range, nbox,
                           (Node *)(ws + L.nodes));
        hipLaunchKernelGGL(k_wide, dim3(nblk(T, 256)), dim3(256), 0, s, T, (const Node *)(ws + L.nodes),
                           (Node4 *)(ws + L.nodes4));
        hipLaunchKernelGGL(k_treelets, dim3(1), dim3(64), 0, s, T, tri, nbox, (float *)(ws + L.tl_box),
                           (int *)(ws + L.tl_root));
    } else {
        hipLaunchKernelGGL(k_treelets, dim3(1), dim3(64), 0, s, 0, (const float4 *)nullptr, (const float *)nullptr,
                           (float *)(ws + L.tl_box), (int *)(ws + L.tl_root));
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if ((e = launch_solids(sc, s)) != hipSuccess) return e;
    return launch_facet_features(sc, s);
}

hipError_t launch_facet_features(Scene &sc, hipStream_t s) {
    char *ws = (char *)sc.ws;
    const Layout &L = sc.lay;
    const int F = sc.desc.n_facets;
    hipLaunchKernelGGL(k_facet_feat, dim3(nblk(F > 0 ? F : 1, 128)), dim3(128), 0, s, F, sc.desc.grid_vertex_log2,
                       (const int *)(ws + L.ibox), (const int *)(ws + L.soff), (const float4 *)(ws + L.smp),
                       (const double *)(ws + L.fplane), (const int *)(ws + L.ffirst),
                       (const float4 *)(ws + L.tri_caller), (float *)(ws + L.ffeat), (float *)(ws + L.fnorm));
    return hipGetLastError();
}

hipError_t launch_triangle_groups(const SceneDev &d, int32_t *group, hipStream_t s) {
    if (d.T > 0) hipLaunchKernelGGL(k_groups, dim3(nblk(d.T, 256)), dim3(256), 0, s, d.T, d.tri_group, group);
    return hipGetLastError();
}

}  // namespace ivm
