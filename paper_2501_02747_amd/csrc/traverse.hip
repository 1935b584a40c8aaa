// traverse.hip -- the inter-visibility hot path on gfx950.
//
//   k_cull     exact orientation cull of every unordered facet pair (Section II-B,
//              eq. 2): a pair is a candidate iff some sample of i lies on j's
//              visible side and some sample of j on i's.  One wave per 64
//              pairs of a row; the ballot is the 64-bit candidate word.
//   scan       exclusive prefix over per-word candidate counts: a dense index
//              for the persistent queue.
//   k_pairs    persistent any-hit kernel: each wave takes one candidate pair
//              from an atomic queue, compacts the admissible samples into LDS,
//              and tests the segments 64 at a time (one per lane) against the
//              LBVH until one is clear (Section II-B: no other obstacle between
//              the faces) or all are blocked.  Per-lane DFS with an LDS stack;
//              leaf tests in FP32 with a semi-static error filter, undecided
//              tests redone in FP64 (exact on the dyadic grid).
//   k_points   the same any-hit core for Tx/Rx -> facet-sample segments
//              (Section III-B, Table II), plus line of sight.
#include <cmath>

#include "ivm_internal.h"

namespace ivm {

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------

__device__ inline void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ inline int lane_id() { return threadIdx.x & (kWave - 1); }

__device__ inline float wave_min(float v) {
    for (int o = 32; o >= 1; o >>= 1) v = fminf(v, __shfl_xor(v, o));
    return v;
}
__device__ inline float wave_max(float v) {
    for (int o = 32; o >= 1; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
    return v;
}
__device__ inline float wave_sum(float v) {
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
    return v;
}
__device__ inline unsigned long long wave_sum_u64(unsigned long long v) {
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// orient(f, x) = (x - a_f) . n_f in FP64 (exact on the grid).
__device__ inline double orient(const double *pl, float x, float y, float z) {
    return ((double)x - pl[0]) * pl[3] + ((double)y - pl[1]) * pl[4] + ((double)z - pl[2]) * pl[5];
}

// ---------------------------------------------------------------------------
// segment, box and triangle predicates
// ---------------------------------------------------------------------------

struct Seg {
    float px, py, pz;   // origin
    float dx, dy, dz;   // q - p (exact on the grid)
    float dm;           // max |d_k|
    float ix, iy, iz;   // 1 / d_k (0 where d_k = 0), set by with_inverse()
};

__device__ inline Seg make_seg(float px, float py, float pz, float qx, float qy, float qz) {
    Seg s;
    s.px = px; s.py = py; s.pz = pz;
    s.dx = qx - px; s.dy = qy - py; s.dz = qz - pz;
    s.dm = fmaxf(fabsf(s.dx), fmaxf(fabsf(s.dy), fabsf(s.dz)));
    s.ix = s.iy = s.iz = 0.f;
    return s;
}

// v_rcp_f32 is within 1 ulp; the slab test below budgets for it.
__device__ inline void with_inverse(Seg &s) {
    s.ix = s.dx != 0.f ? __builtin_amdgcn_rcpf(s.dx) : 0.f;
    s.iy = s.dy != 0.f ? __builtin_amdgcn_rcpf(s.dy) : 0.f;
    s.iz = s.dz != 0.f ? __builtin_amdgcn_rcpf(s.dz) : 0.f;
}

// Conservative slab test of the segment p + t d, t in [0, 1], against a closed
// box.  Box minus origin is exact; each slab parameter carries <= 3 ulp of
// relative error (1 from the reciprocal, 1 from the product, ulp = 2^-23), so
// widening the exit by 2^-20 never rejects a box the exact segment meets.
// Axes with d = 0 are decided exactly by containment.
constexpr float kWiden = 1.00000095367431640625f;  // 1 + 2^-20

__device__ inline bool seg_box(const Seg &s, float lx, float ly, float lz, float hx, float hy, float hz,
                               float &tentry) {
    float t0 = 0.0f, t1 = 1.0f;
    bool out = false;
    if (s.dx != 0.f) {
        float a = (lx - s.px) * s.ix, b = (hx - s.px) * s.ix;
        t0 = fmaxf(t0, fminf(a, b));
        t1 = fminf(t1, fmaxf(a, b));
    } else {
        out |= (s.px < lx) | (s.px > hx);
    }
    if (s.dy != 0.f) {
        float a = (ly - s.py) * s.iy, b = (hy - s.py) * s.iy;
        t0 = fmaxf(t0, fminf(a, b));
        t1 = fminf(t1, fmaxf(a, b));
    } else {
        out |= (s.py < ly) | (s.py > hy);
    }
    if (s.dz != 0.f) {
        float a = (lz - s.pz) * s.iz, b = (hz - s.pz) * s.iz;
        t0 = fmaxf(t0, fminf(a, b));
        t1 = fminf(t1, fmaxf(a, b));
    } else {
        out |= (s.pz < lz) | (s.pz > hz);
    }
    tentry = t0;
    return !out && (t0 <= t1 * kWiden);
}

// Exact test in FP64 (division-free Moller-Trumbore, closed triangle, open
// segment; a segment parallel to the plane never hits).
// The segment comes in registers (a reference would put it in scratch memory
// at every call site of this out-of-line function).
__device__ __noinline__ bool tri_hit_f64(float px, float py, float pz, float sdx, float sdy, float sdz, float4 A,
                                         float4 B, float4 C) {
    const double dx = sdx, dy = sdy, dz = sdz;
    const double ex = B.x, ey = B.y, ez = B.z;   // e1
    const double fx = C.x, fy = C.y, fz = C.z;   // e2
    const double sx = (double)px - (double)A.x, sy = (double)py - (double)A.y, sz = (double)pz - (double)A.z;
    const double hx = dy * fz - dz * fy, hy = dz * fx - dx * fz, hz = dx * fy - dy * fx;
    const double det = ex * hx + ey * hy + ez * hz;
    if (det == 0.0) return false;
    const double u = sx * hx + sy * hy + sz * hz;
    const double gx = sy * ez - sz * ey, gy = sz * ex - sx * ez, gz = sx * ey - sy * ex;
    const double v = dx * gx + dy * gy + dz * gz;
    const double t = fx * gx + fy * gy + fz * gz;
    if (det > 0.0) return u >= 0.0 && v >= 0.0 && u + v <= det && t > 0.0 && t < det;
    return u <= 0.0 && v <= 0.0 && u + v >= det && t < 0.0 && t > det;
}

// FP32 test with a semi-static filter.  With D = max|d_k|, S = max|s_k|,
// E1 = max|e1_k|, E2 = max|e2_k|, the magnitudes of det, u, v, t are bounded
// by 6 D E1 E2, 6 S D E2, 6 D S E1, 6 E2 S E1 and the FP32 rounding error of
// each quantity (and of det-u-v, det-t) stays below 8 * 2^-24 of its bound.
// A comparison is trusted when its value clears eps6/6 (>= 1e-5, i.e. >= 20x
// the error) times that bound; otherwise the whole test is redone in FP64.
// Returns 1 hit, 0 miss; counts rechecks.
__device__ inline bool tri_hit(const Seg &s, float4 A, float4 B, float4 C, float eps6, bool f64only,
                               unsigned &rechecks) {
    if (f64only) return tri_hit_f64(s.px, s.py, s.pz, s.dx, s.dy, s.dz, A, B, C);
    const float sx = s.px - A.x, sy = s.py - A.y, sz = s.pz - A.z;  // exact
    const float hx = s.dy * C.z - s.dz * C.y;
    const float hy = s.dz * C.x - s.dx * C.z;
    const float hz = s.dx * C.y - s.dy * C.x;
    const float det = B.x * hx + B.y * hy + B.z * hz;
    const float mdet = eps6 * s.dm * B.w * C.w;
    if (!(fabsf(det) > mdet)) {
        ++rechecks;
        return tri_hit_f64(s.px, s.py, s.pz, s.dx, s.dy, s.dz, A, B, C);
    }
    const float sg = det > 0.f ? 1.f : -1.f;
    const float S = fmaxf(fabsf(sx), fmaxf(fabsf(sy), fabsf(sz)));
    const float u = (sx * hx + sy * hy + sz * hz) * sg;
    const float mu = eps6 * S * s.dm * C.w;
    if (u < -mu) return false;
    const float gx = sy * B.z - sz * B.y;
    const float gy = sz * B.x - sx * B.z;
    const float gz = sx * B.y - sy * B.x;
    const float v = (s.dx * gx + s.dy * gy + s.dz * gz) * sg;
    const float mv = eps6 * s.dm * S * B.w;
    if (v < -mv) return false;
    const float adet = fabsf(det);
    const float w = adet - u - v;
    const float mw = mdet + mu + mv;
    if (w < -mw) return false;
    const float t = (C.x * gx + C.y * gy + C.z * gz) * sg;
    const float mt = eps6 * C.w * S * B.w;
    if (t < -mt) return false;
    const float x = adet - t;
    const float mx = mdet + mt;
    if (x < -mx) return false;
    if (u > mu && v > mv && w > mw && t > mt && x > mx) return true;
    ++rechecks;
    return tri_hit_f64(s.px, s.py, s.pz, s.dx, s.dy, s.dz, A, B, C);
}

struct Cnt {
    unsigned boxes = 0, tests = 0, rechecks = 0, fallbacks = 0, traversed = 0, solid_segs = 0, solid_planes = 0;
};

// Facets whose triangles a segment test skips: two (a pair's facets, an edge's
// facets) or four (the facets of two edges, or of an edge and a facet).
struct Ex2 {
    int a, b;
    __device__ bool operator()(int f) const { return f == a || f == b; }
};
struct Ex4 {
    int a, b, c, d;
    __device__ bool operator()(int f) const { return f == a || f == b || f == c || f == d; }
};

template <class Ex>
__device__ inline int test_range_ex(const SceneDev &sc, const Seg &s, int first, int count, Ex ex, float eps6,
                                    bool f64, Cnt &c) {
    for (int r = first; r < first + count; ++r) {
        const float4 A = sc.tri[3 * r];
        const int f = __float_as_int(A.w);
        if (ex(f)) continue;
        ++c.tests;
        if (tri_hit(s, A, sc.tri[3 * r + 1], sc.tri[3 * r + 2], eps6, f64, c.rechecks)) return r;
    }
    return -1;
}

__device__ inline int test_range(const SceneDev &sc, const Seg &s, int first, int count, int exA, int exB,
                                 float eps6, bool f64, Cnt &c) {
    return test_range_ex(sc, s, first, count, Ex2{exA, exB}, eps6, f64, c);
}

constexpr int kNone = 0x7fffffff;

// Any-hit traversal of one segment; returns the sorted rank of a triangle that
// the segment hits, or -1 when the segment is clear.  `order` lists treelets to
// visit (LDS or constant memory); `stk` is this lane's LDS stack with a stride of
// one wave.  When the stack is full the far child's whole subtree is scanned
// linearly (its triangles are a contiguous sorted range), so no node is dropped.
template <typename OrderPtr, class Ex>
__device__ int any_hit_ex(const SceneDev &sc, Seg s, Ex ex, OrderPtr order, int n_order, int *stk, int depth,
                          float eps6, bool f64, Cnt &c) {
    with_inverse(s);
    int r = 0, sp = 0;
    int ref = kNone;
    while (true) {
        if (ref == kNone) {
            if (sp > 0) {
                ref = stk[(--sp) * kWave];
            } else {
                while (r < n_order) {
                    const int k = order[r++];
                    const int root = sc.tl_root[k];
                    if (root == kNone) continue;  // empty treelet: its inverted box must never be entered
                    const float *b = sc.tl_box + 6 * k;
                    float te;
                    ++c.boxes;
                    if (seg_box(s, b[0], b[1], b[2], b[3], b[4], b[5], te)) {
                        ref = root;
                        break;
                    }
                }
                if (ref == kNone) return -1;
            }
        }
        if (ref >= 0) {
            c.boxes += 2;
            const Node nd = sc.nodes[ref];
            float t0, t1;
            const bool h0 = seg_box(s, nd.a.x, nd.a.y, nd.a.z, nd.a.w, nd.b.x, nd.b.y, t0);
            const bool h1 = seg_box(s, nd.b.z, nd.b.w, nd.c.x, nd.c.y, nd.c.z, nd.c.w, t1);
            if (h0 && h1) {
                const int nearc = t0 <= t1 ? nd.d.x : nd.d.y;
                const int farc = t0 <= t1 ? nd.d.y : nd.d.x;
                if (sp < depth) {
                    stk[(sp++) * kWave] = farc;
                } else {
                    ++c.fallbacks;
                    int first, count;
                    if (farc < 0) {
                        first = leaf_first(farc);
                        count = leaf_count(farc);
                    } else {
                        const int4 rg = sc.nodes[farc].d;
                        first = rg.z;
                        count = rg.w - rg.z + 1;
                    }
                    const int h = test_range_ex(sc, s, first, count, ex, eps6, f64, c);
                    if (h >= 0) return h;
                }
                ref = nearc;
            } else if (h0) {
                ref = nd.d.x;
            } else if (h1) {
                ref = nd.d.y;
            } else {
                ref = kNone;
            }
        } else {
            const int h = test_range_ex(sc, s, leaf_first(ref), leaf_count(ref), ex, eps6, f64, c);
            if (h >= 0) return h;
            ref = kNone;
        }
    }
}

template <typename OrderPtr>
__device__ int any_hit(const SceneDev &sc, Seg s, int exA, int exB, OrderPtr order, int n_order, int *stk,
                       int depth, float eps6, bool f64, Cnt &c) {
    return any_hit_ex(sc, s, Ex2{exA, exB}, order, n_order, stk, depth, eps6, f64, c);
}

// Wave-synchronous any-hit over one batch: every lane traverses its own
// segment (the same steps as any_hit), and after each step the wave applies an
// abort rule to lanes whose answer no longer matters:
//   kAbortAll      - once any lane is clear, all stop (a pair is visible as soon
//                    as one admissible segment is clear);
//   kAbortSameKey  - once a lane is clear, the lanes with the same key stop (a
//                    facet is visible from a point as soon as one sample is; the
//                    key names the point and the facet).
// Returns the hit rank (>= 0), -1 clear, or -2 for a lane that did not run or
// was stopped.
constexpr int kAbortAll = 1, kAbortSameKey = 2;

template <typename OrderPtr>
__device__ int any_hit_wave(const SceneDev &sc, Seg s, bool active, int exA, int exB, OrderPtr order, int n_order,
                            int *stk, int depth, float eps6, bool f64, Cnt &c, int rule, int key) {
    if (active) with_inverse(s);
    int r = 0, sp = 0;
    int ref = kNone;
    int res = active ? -3 : -2;  // -3 = running
    while (true) {
        const bool run = res == -3;
        if (!__ballot(run)) break;
        if (run) {
            if (ref == kNone) {
                if (sp > 0) {
                    ref = stk[(--sp) * kWave];
                } else {
                    while (r < n_order) {
                        const int k = order[r++];
                        const int root = sc.tl_root[k];
                        if (root == kNone) continue;  // empty treelet: its inverted box must never be entered
                        const float *b = sc.tl_box + 6 * k;
                        float te;
                        ++c.boxes;
                        if (seg_box(s, b[0], b[1], b[2], b[3], b[4], b[5], te)) {
                            ref = root;
                            break;
                        }
                    }
                    if (ref == kNone) res = -1;
                }
            }
            if (res == -3 && ref != kNone) {
                if (ref >= 0) {
                    // a 4-wide record: test the up-to-four children, descend into the
                    // nearest, push the others far to near
                    const Node4 nd = sc.nodes4[ref];
                    float a0, a1, a2, a3;
                    int b0 = nd.ref.x, b1 = nd.ref.y, b2 = nd.ref.z, b3 = nd.ref.w;
                    c.boxes += nd.pad.x;
                    const bool h0 = b0 != kNone && seg_box(s, nd.lox.x, nd.loy.x, nd.loz.x, nd.hix.x, nd.hiy.x, nd.hiz.x, a0);
                    const bool h1 = b1 != kNone && seg_box(s, nd.lox.y, nd.loy.y, nd.loz.y, nd.hix.y, nd.hiy.y, nd.hiz.y, a1);
                    const bool h2 = b2 != kNone && seg_box(s, nd.lox.z, nd.loy.z, nd.loz.z, nd.hix.z, nd.hiy.z, nd.hiz.z, a2);
                    const bool h3 = b3 != kNone && seg_box(s, nd.lox.w, nd.loy.w, nd.loz.w, nd.hix.w, nd.hiy.w, nd.hiz.w, a3);
                    const int nh = (int)h0 + (int)h1 + (int)h2 + (int)h3;
                    if (!h0) a0 = INFINITY;
                    if (!h1) a1 = INFINITY;
                    if (!h2) a2 = INFINITY;
                    if (!h3) a3 = INFINITY;
                    // sorting network on (a, b): hits (finite a) come first, nearest first
                    auto cswap = [](float &x, int &xr, float &y, int &yr) {
                        if (y < x) {
                            const float t = x; x = y; y = t;
                            const int tr = xr; xr = yr; yr = tr;
                        }
                    };
                    cswap(a0, b0, a1, b1);
                    cswap(a2, b2, a3, b3);
                    cswap(a0, b0, a2, b2);
                    cswap(a1, b1, a3, b3);
                    cswap(a1, b1, a2, b2);
                    ref = nh > 0 ? b0 : kNone;
                    // (no array here: a dynamically indexed one would live in scratch memory)
                    auto push = [&](int farc) {
                        if (res != -3) return;
                        if (sp < depth) {
                            stk[(sp++) * kWave] = farc;
                        } else {
                            ++c.fallbacks;
                            int first, count;
                            if (farc < 0) {
                                first = leaf_first(farc);
                                count = leaf_count(farc);
                            } else {
                                const int4 rg = sc.nodes[farc].d;
                                first = rg.z;
                                count = rg.w - rg.z + 1;
                            }
                            const int h = test_range(sc, s, first, count, exA, exB, eps6, f64, c);
                            if (h >= 0) res = h;
                        }
                    };
                    if (nh >= 4) push(b3);
                    if (nh >= 3) push(b2);
                    if (nh >= 2) push(b1);
                } else {
                    const int h = test_range(sc, s, leaf_first(ref), leaf_count(ref), exA, exB, eps6, f64, c);
                    if (h >= 0) res = h;
                    ref = kNone;
                }
            }
        }
        const unsigned long long cl = __ballot(run && res == -1);  // lanes that just turned out clear
        if (cl) {
            if (rule == kAbortAll) {
                if (res == -3) res = -2;
            } else if (rule == kAbortSameKey) {
                unsigned long long m = cl;
                while (m) {
                    const int src = __ffsll((long long)m) - 1;
                    m &= m - 1;
                    const int kc = __shfl(key, src);
                    if (res == -3 && key == kc) res = -2;
                }
            }
        }
    }
    return res;
}

// Per-wave treelet order.  Lane k < 32 holds a 64-bit key for treelet k
// (UINT64_MAX = skip); the wave ranks the keys (index breaks ties) into
// order[0..n).  Returns n.
__device__ inline int wave_rank_order(unsigned long long key, unsigned long long *skey, uint8_t *order) {
    const int lane = lane_id();
    if (lane < kTreelets) skey[lane] = key;
    wave_sync();
    const bool valid = lane < kTreelets && key != ~0ull;
    if (valid) {
        int rank = 0;
        for (int m = 0; m < kTreelets; ++m) {
            const unsigned long long km = skey[m];
            rank += (km < key) || (km == key && m < lane);
        }
        order[rank] = (uint8_t)lane;
    }
    const int n = __popcll(__ballot(valid));
    wave_sync();
    return n;
}

// Key of treelet `lane` for a segment bundle with box [lo, hi]: treelets whose
// box misses the bundle box cannot hold a hit and are skipped.
__device__ inline unsigned long long treelet_key(const SceneDev &sc, int lane, const float lo[3], const float hi[3],
                                                 int mode, unsigned long long learned_code) {
    if (lane >= kTreelets || sc.tl_root[lane] == kNone) return ~0ull;
    const float *b = sc.tl_box + 6 * lane;
    if (b[0] > hi[0] || b[3] < lo[0] || b[1] > hi[1] || b[4] < lo[1] || b[2] > hi[2] || b[5] < lo[2]) return ~0ull;
    float d2 = 0.f;
    for (int k = 0; k < 3; ++k) {
        const float c = 0.5f * (b[k] + b[3 + k]) - 0.5f * (lo[k] + hi[k]);
        d2 += c * c;
    }
    const unsigned dk = __float_as_uint(d2);  // non-negative: bit order = value order
    if (mode == IVM_ORDER_INDEX) return (unsigned long long)lane;
    if (mode == IVM_ORDER_REVERSED) return (unsigned long long)(0xffffffffu - dk);
    if (mode == IVM_ORDER_LEARNED) {
        // learned_code: up to 12 treelet ids, 5 bits each, best first (31 = unused slot
        // only when fewer than 12 are listed, since 31 is also a valid id, a count in
        // the top 4 bits says how many are listed).
        const int listed = (int)(learned_code >> 60);
        for (int m = 0; m < listed && m < 12; ++m)
            if ((int)((learned_code >> (5 * m)) & 31) == lane) return (unsigned long long)m << 32;
        return (1ull << 40) | dk;
    }
    return dk;
}

// ---------------------------------------------------------------------------
// pair cull and scan
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_cull(SceneDev sc, uint64_t *cand, uint32_t *counts, int n_items) {
    const int lane = lane_id();
    const int wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int nwaves = (gridDim.x * blockDim.x) >> 6;
    for (int item = wave; item < n_items; item += nwaves) {
        const int i = item / sc.W, w = item - (item / sc.W) * sc.W;
        const int j = w * 64 + lane;
        bool ok = false;
        if (w * 64 + 63 > i && j > i && j < sc.F) {
            const double *pi = sc.fplane + 6 * i, *pj = sc.fplane + 6 * j;
            bool a = false;
            for (int s = sc.soff[i]; s < sc.soff[i + 1] && !a; ++s) {
                const float4 p = sc.smp[s];
                a = orient(pj, p.x, p.y, p.z) > 0.0;
            }
            if (a) {
                for (int s = sc.soff[j]; s < sc.soff[j + 1] && !ok; ++s) {
                    const float4 q = sc.smp[s];
                    ok = orient(pi, q.x, q.y, q.z) > 0.0;
                }
            }
        }
        const unsigned long long m = __ballot(ok);
        if (lane == 0) {
            cand[item] = m;
            counts[item] = (uint32_t)__popcll(m);
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) counts[n_items] = 0;
}

constexpr int kScanThreads = 1024;
constexpr int kScanPer = 4;
constexpr int kScanBlock = kScanThreads * kScanPer;

__device__ inline uint32_t block_exclusive_scan(uint32_t v, uint32_t *sh, uint32_t *total) {
    const int tid = threadIdx.x;
    sh[tid] = v;
    __syncthreads();
    for (int off = 1; off < kScanThreads; off <<= 1) {
        uint32_t x = tid >= off ? sh[tid - off] : 0u;
        __syncthreads();
        sh[tid] += x;
        __syncthreads();
    }
    uint32_t incl = sh[tid];
    *total = sh[kScanThreads - 1];
    __syncthreads();
    return incl - v;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_blocks(uint32_t *a, int n, uint32_t *bsum) {
    __shared__ uint32_t sh[kScanThreads];
    const int base = blockIdx.x * kScanBlock + threadIdx.x * kScanPer;
    uint32_t v[kScanPer], s = 0;
    for (int m = 0; m < kScanPer; ++m) {
        v[m] = base + m < n ? a[base + m] : 0u;
        s += v[m];
    }
    uint32_t tot;
    uint32_t ex = block_exclusive_scan(s, sh, &tot);
    for (int m = 0; m < kScanPer; ++m) {
        if (base + m < n) a[base + m] = ex;
        ex += v[m];
    }
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_sums(uint32_t *bsum, int nb) {
    __shared__ uint32_t sh[kScanThreads];
    uint32_t carry = 0;
    for (int base = 0; base < nb; base += kScanThreads) {
        const int i = base + threadIdx.x;
        uint32_t v = i < nb ? bsum[i] : 0u;
        uint32_t tot;
        uint32_t ex = block_exclusive_scan(v, sh, &tot);
        if (i < nb) bsum[i] = ex + carry;
        carry += tot;
        __syncthreads();
    }
}

__global__ void k_scan_add(uint32_t *a, int n, const uint32_t *bsum) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] += bsum[i / kScanBlock];
}

static hipError_t exclusive_scan_u32(uint32_t *a, int n, uint32_t *tmp, hipStream_t s) {
    const int nb = (n + kScanBlock - 1) / kScanBlock;
    hipLaunchKernelGGL(k_scan_blocks, dim3(nb), dim3(kScanThreads), 0, s, a, n, tmp);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(kScanThreads), 0, s, tmp, nb);
    hipLaunchKernelGGL(k_scan_add, dim3((n + 255) / 256), dim3(256), 0, s, a, n, (const uint32_t *)tmp);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// persistent pair kernel
// ---------------------------------------------------------------------------

constexpr int kBlock = 256;
constexpr int kWavesPerBlock = kBlock / kWave;

__device__ inline void flush_counters(ivm_stats *st, const Cnt &c, unsigned long long segs,
                                      unsigned long long visible, unsigned long long items) {
    if (!st) return;
    const unsigned long long v = wave_sum_u64(c.boxes), t = wave_sum_u64(c.tests);
    const unsigned long long r = wave_sum_u64(c.rechecks), f = wave_sum_u64(c.fallbacks);
    const unsigned long long sg = wave_sum_u64(segs);
    const unsigned long long tv = wave_sum_u64(c.traversed), ss = wave_sum_u64(c.solid_segs);
    const unsigned long long sp = wave_sum_u64(c.solid_planes);
    if (lane_id() == 0) {
        if (tv) atomicAdd((unsigned long long *)&st->traversed, tv);
        if (ss) atomicAdd((unsigned long long *)&st->solid_segments, ss);
        if (sp) atomicAdd((unsigned long long *)&st->solid_planes, sp);
        atomicAdd((unsigned long long *)&st->box_tests, v);
        atomicAdd((unsigned long long *)&st->tri_tests, t);
        atomicAdd((unsigned long long *)&st->rechecks, r);
        atomicAdd((unsigned long long *)&st->fallbacks, f);
        atomicAdd((unsigned long long *)&st->segments, sg);
        if (visible) atomicAdd((unsigned long long *)&st->pairs_visible, visible);
        if (items) atomicAdd((unsigned long long *)&st->point_items, items);
    }
}

__device__ inline int find_item(const uint32_t *prefix, int n_items, uint32_t g) {
    int lo = 0, hi = n_items - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (prefix[mid] <= g) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__device__ inline void decode_pair(const SceneDev &sc, const uint64_t *cand, const uint32_t *prefix, int n_items,
                                   uint32_t g, int &i, int &j) {
    const int item = find_item(prefix, n_items, g);
    unsigned long long m = cand[item];
    for (uint32_t q = prefix[item]; q < g; ++q) m &= m - 1;
    const int bit = __ffsll((long long)m) - 1;
    i = item / sc.W;
    j = (item - i * sc.W) * 64 + bit;
}

constexpr int kCache = 2;  // recent blockers tested before a traversal
constexpr int kSolidTries = 4;  // distinct solids tried per certificate attempt
constexpr int kScanMaxSolids = 4096;  // scenes with at most this many solids scan them all per pair
constexpr int kScanTries = 6;         // solids from the scan tried per pair (and per point certificate)
constexpr int kScanLinearMax = 256;   // up to this many solids a scan reads them all instead of the grid
constexpr int kScanMaxSolidsPoint = 4096;  // the same scan per (point, facet) in the Tx/Rx kernel
constexpr int kPairChunk = 4;   // consecutive undecided pairs taken by a wave at a time (small jobs)
constexpr int kPairChunkLarge = 32;       // ... when a wave has many pairs to do (better reuse)
constexpr uint32_t kLargePerWave = 2048;  // candidate pairs per wave above which chunks are large

// Single-occluder certificate.  Let H_i, H_j be the convex hulls of the two
// sample sets (valid when the samples lie in their facet's plane, checked at
// build) and C a facet whose triangles tile one convex polygon (also checked).  For fixed q the points p whose open segment
// to q meets C form a convex set, and symmetrically for p fixed; so if every
// segment between hull corners meets C transversally inside (0, 1), every
// segment between the hulls does, and each crosses C's plane strictly, at a point
// of the closed polygon C, i.e. of one of its closed triangles.  Then no
// admissible segment of the pair is clear.  One lane per (corner, corner,
// triangle of C).
__device__ bool certify_blocked(const SceneDev &sc, int i, int j, int C, int *corner, float eps6, bool f64,
                                Cnt &c) {
    const int lane = lane_id();
    const int ni = sc.fhull_n[i], nj = sc.fhull_n[j];
    const int t0 = sc.ftri[2 * C], nt = sc.ftri[2 * C + 1];
    if (ni == 0 || nj == 0 || nt <= 0 || !(sc.fflags[C] & kFacetConvex)) return false;
    const int pairs = ni * nj;  // <= kHullMax^2 = 64
    corner[lane] = 0;
    wave_sync();
    for (int it = lane; it < pairs * nt; it += kWave) {
        const int cp = it / nt, t = it - (it / nt) * nt;
        const int a = cp / nj, b = cp - (cp / nj) * nj;
        const float4 P = sc.smp[sc.fhull[kHullMax * i + a]];
        const float4 Q = sc.smp[sc.fhull[kHullMax * j + b]];
        const Seg s = make_seg(P.x, P.y, P.z, Q.x, Q.y, Q.z);
        ++c.tests;
        const float4 *tr = sc.tri_caller + 3 * (t0 + t);
        if (tri_hit(s, tr[0], tr[1], tr[2], eps6, f64, c.rechecks)) corner[cp] = 1;
    }
    wave_sync();
    const bool missing = lane < pairs && corner[lane] == 0;
    const bool ok = __ballot(missing) == 0ull;
    wave_sync();
    return ok;
}

// a * b < c * d, exact for doubles holding integers of magnitude below 2^52:
// the rounded products order the exact ones unless they tie, and then the
// rounding errors (exact by fma) decide.
__device__ inline bool prod_less(double a, double b, double c, double d) {
    const double p = a * b, q = c * d;
    if (p != q) return p < q;
    return fma(a, b, -p) < fma(c, d, -q);
}

// Solid certificate.  A verified solid s is an open convex prism K (wall
// planes and roof plane; unbounded below) whose walls and roof above its base
// height zb are covered by triangles of its facets.  Every segment between the
// sample hulls H_i and H_j is blocked when
//   (i)   H_i lies strictly outside one face plane of K, and so does H_j;
//   (ii)  every hull corner has z >= zb;
//   (iii) every segment between hull corners passes through K.
// For p outside K the points q whose segment to p meets K form the convex set
// p + [1, inf)(K - p), so (iii) at the corners holds for all of H_i x H_j.  Such
// a segment enters K at a point e with 0 < t < 1; by (ii) e lies at or above
// the base, on a covered face, and every face plane through e is crossed
// strictly (the segment goes from its outside to its inside), so the open
// segment meets a closed covering triangle transversally.  The triangle is not
// of facet i or j: those lie outside K by (i).  One lane per corner pair.
// Plane values are exact FP64 integers in sample units (below 2^51); the
// interval of t inside K is intersected with exact fraction comparisons.
// A verified solid staged in LDS: its wall planes, then (at kSolidMaxPlanes)
// its record (walls, top z, base z, 0), all in sample units.
struct SolidLds {
    int4 pl[kSolidMaxPlanes + 1];
    float4 lo, hi;  // metres: footprint box and (base, top) heights in .z
};

// One load round: lane k < kSolidMaxPlanes fetches plane k, the next lane the
// record; the footprint box comes from the walls' corner points.
__device__ inline void stage_solid(const SceneDev &sc, int s, SolidLds &dst) {
    const int lane = lane_id();
    int4 v = make_int4(0, 0, 0, 0);
    if (lane < kSolidMaxPlanes) v = sc.splane[s * kSolidMaxPlanes + lane];
    else if (lane == kSolidMaxPlanes) v = sc.solid[s];
    if (lane <= kSolidMaxPlanes) dst.pl[lane] = v;
    const int np = __shfl(v.x, kSolidMaxPlanes), top = __shfl(v.y, kSolidMaxPlanes);
    const int base = __shfl(v.z, kSolidMaxPlanes);
    const float m = ldexpf(1.0f, -sc.gs);  // sample units -> metres (exact: integers below 2^24)
    const bool w = lane < np;
    const float x0 = wave_min(w ? (float)v.x * m : INFINITY), x1 = wave_max(w ? (float)v.x * m : -INFINITY);
    const float y0 = wave_min(w ? (float)v.y * m : INFINITY), y1 = wave_max(w ? (float)v.y * m : -INFINITY);
    if (lane == 0) {
        dst.lo = make_float4(x0, y0, (float)base * m, 0.f);
        dst.hi = make_float4(x1, y1, (float)top * m, 0.f);
    }
    wave_sync();
}

// A segment set inside the box [lo, hi] can pass through the open prism only if
// that box reaches into the open footprint box and below the top (a necessary
// test before the exact ones).
__device__ inline bool solid_box_reach(const SolidLds &S, const float lo[3], const float hi[3]) {
    return hi[0] > S.lo.x && lo[0] < S.hi.x && hi[1] > S.lo.y && lo[1] < S.hi.y && lo[2] < S.hi.z;
}

// Swap the staged solid in slot `a` with the one in slot 0 (wave-uniform).
__device__ inline void solid_to_front(int *solids, SolidLds *lds, int a) {
    if (a <= 0) return;
    const int lane = lane_id();
    int4 *x = (int4 *)&lds[0], *y = (int4 *)&lds[a];
    constexpr int n = sizeof(SolidLds) / sizeof(int4);
    int4 vx = make_int4(0, 0, 0, 0), vy = vx;
    if (lane < n) {
        vx = x[lane];
        vy = y[lane];
    }
    const int t0 = solids[0], ta = solids[a];
    wave_sync();
    if (lane < n) {
        x[lane] = vy;
        y[lane] = vx;
    }
    solids[0] = ta;
    solids[a] = t0;
    wave_sync();
}

// Plane value of face k (k == number of walls: the roof) at a point in sample
// units; > 0 outside.
__device__ inline double solid_plane(const SolidLds &S, int k, double x, double y, double z) {
    const int4 R = S.pl[kSolidMaxPlanes];
    if (k < R.x) {
        const int4 p = S.pl[k];
        return (double)p.w * (x - (double)p.x) - (double)p.z * (y - (double)p.y);
    }
    return z - (double)R.y;
}

// Conditions (ii) and (iii) for one segment (ends in sample units): both ends
// at or above the base and some t in [0, 1] with every plane value negative;
// also P strictly outside one face plane (implied by (i) for the certificates;
// it makes the test stand alone for single segments: P is not in the prism,
// so the entry is at t > 0).
__device__ bool solid_segment(const SolidLds &S, double px, double py, double pz, double qx, double qy, double qz,
                              Cnt &c) {
    const int4 R = S.pl[kSolidMaxPlanes];
    if (!(pz >= (double)R.z && qz >= (double)R.z)) return false;
    double Ln = 0.0, Ld = 1.0, Un = 1.0, Ud = 1.0;  // t in (Ln / Ld, Un / Ud)
    bool pout = false;
    for (int k = 0; k <= R.x; ++k) {
        ++c.solid_planes;
        const double va = solid_plane(S, k, px, py, pz);
        const double vb = solid_plane(S, k, qx, qy, qz);
        if (va >= 0.0 && vb >= 0.0) return false;
        pout |= va > 0.0;
        if (va >= 0.0) {  // enters this half-space at t = va / (va - vb)
            const double n = va, dd = va - vb;
            if (prod_less(Ln, dd, n, Ld)) { Ln = n; Ld = dd; }
        } else if (vb >= 0.0) {  // leaves it at t = -va / (vb - va)
            const double n = -va, dd = vb - va;
            if (prod_less(n, Ud, Un, dd)) { Un = n; Ud = dd; }
        }
    }
    return pout && prod_less(Ln, Ud, Un, Ld);
}

// (ends in metres) A segment can be strictly inside the prism somewhere only if its
// box meets the open footprint box, both ends are at or above the base and the
// lower end is below the top: a necessary condition in exact FP32 comparisons
// (the footprint box is the vertices' box) that spares the FP64 steps.
__device__ inline bool solid_segment(const SolidLds &S, float4 P, float4 Q, double u, Cnt &c) {
    const float4 lo = S.lo, hi = S.hi;
    if (fmaxf(P.x, Q.x) <= lo.x || fminf(P.x, Q.x) >= hi.x || fmaxf(P.y, Q.y) <= lo.y || fminf(P.y, Q.y) >= hi.y ||
        fminf(P.z, Q.z) < lo.z || fminf(P.z, Q.z) >= hi.z)
        return false;
    return solid_segment(S, P.x * u, P.y * u, P.z * u, Q.x * u, Q.y * u, Q.z * u, c);
}

// The same test reading solid `sid` from global memory (each lane may test its
// own solid): a necessary condition checked before staging a candidate.
__device__ __forceinline__ bool solid_segment_global(const SceneDev &sc, int sid, float4 P, float4 Q, Cnt &c) {
    const double u = ldexp(1.0, sc.gs);
    const double px = P.x * u, py = P.y * u, pz = P.z * u, qx = Q.x * u, qy = Q.y * u, qz = Q.z * u;
    const int4 R = sc.solid[sid];
    if (R.x <= 0 || !(pz >= (double)R.z && qz >= (double)R.z)) return false;
    double Ln = 0.0, Ld = 1.0, Un = 1.0, Ud = 1.0;
    bool pout = false;
    for (int k = 0; k <= R.x; ++k) {
        ++c.solid_planes;
        double va, vb;
        if (k < R.x) {
            const int4 pl = sc.splane[sid * kSolidMaxPlanes + k];
            va = (double)pl.w * (px - (double)pl.x) - (double)pl.z * (py - (double)pl.y);
            vb = (double)pl.w * (qx - (double)pl.x) - (double)pl.z * (qy - (double)pl.y);
        } else {
            va = pz - (double)R.y;
            vb = qz - (double)R.y;
        }
        if (va >= 0.0 && vb >= 0.0) return false;
        pout |= va > 0.0;
        if (va >= 0.0) {
            const double n = va, dd = va - vb;
            if (prod_less(Ln, dd, n, Ld)) { Ln = n; Ld = dd; }
        } else if (vb >= 0.0) {
            const double n = -va, dd = vb - va;
            if (prod_less(n, Ud, Un, dd)) { Un = n; Ud = dd; }
        }
    }
    return pout && prod_less(Ln, Ud, Un, Ld);
}

// The sample hulls of a pair staged in LDS: hc[0, 8) facet i, hc[8, 16) facet j;
// cc[(side * 4 + cluster) * kHullMax + k] the cluster hulls, ccn their sizes.
struct HullLds {
    float4 hc[2 * kHullMax];
    float4 cc[8 * kHullMax];
    int ccn[8];
    int ni, nj;
};

__device__ inline void stage_hulls(const SceneDev &sc, int i, int j, HullLds &H) {
    const int lane = lane_id();
    const int side = lane >> 5, cl = (lane >> 3) & 3, k = lane & 7, f = side ? j : i;
    const int n = sc.fchull_n[4 * f + cl];
    const int hn = sc.fhull_n[f];
    const int ci = k < n ? sc.fchull[(4 * f + cl) * kHullMax + k] : -1;
    const int hi = (cl == 0 && k < hn) ? sc.fhull[kHullMax * f + k] : -1;
    if (ci >= 0) H.cc[(side * 4 + cl) * kHullMax + k] = sc.smp[ci];
    if (hi >= 0) H.hc[side * kHullMax + k] = sc.smp[hi];
    if (k == 0) H.ccn[side * 4 + cl] = n;
    if (lane == 0) H.ni = hn;
    if (lane == 32) H.nj = hn;
    wave_sync();
}

// Condition (i): each facet's sample hull strictly outside one face plane.
__device__ bool solid_sides(const SolidLds &S, const HullLds &H, double u, Cnt &c) {
    const int lane = lane_id();
    const int ni = H.ni, nj = H.nj;
    const float4 P = H.hc[lane < ni ? lane : 0], Q = H.hc[kHullMax + (lane < nj ? lane : 0)];
    const int np = S.pl[kSolidMaxPlanes].x;
    bool outP = false, outQ = false;
    for (int k = 0; k <= np && !(outP && outQ); ++k) {
        c.solid_planes += lane < max(ni, nj);
        const double va = solid_plane(S, k, P.x * u, P.y * u, P.z * u);
        const double vb = solid_plane(S, k, Q.x * u, Q.y * u, Q.z * u);
        outP |= __ballot(lane < ni && !(va > 0.0)) == 0ull;
        outQ |= __ballot(lane < nj && !(vb > 0.0)) == 0ull;
    }
    return outP && outQ;
}

// Candidate solids under the 2-D segment A -> B: the `npieces` lanes of a group
// split it into pieces (this lane takes piece `piece`) and visit the grid cells
// under each piece's box (all solids, npieces per step, when there are few of
// them or the grid is unusable).  key_of(sid, lo, hi) ranks a solid from its
// footprint box (INFINITY rejects it); each lane keeps its best.  Which solids are found only affects speed.
template <class KeyOf, class Accept>
__device__ inline void scan_solids(const SceneDev &sc, float ax, float ay, float bx, float by, int piece, int npieces,
                                   KeyOf key_of, Accept accept, float &bkey, int &bsol) {
    bkey = INFINITY;
    bsol = -1;
    auto consider = [&](int sid, float4 L, float4 H) {
        const float key = key_of(sid, L, H);
        if (key < bkey && accept(sid)) {
            bkey = key;
            bsol = sid;
        }
    };
    if (sc.gridi[1] && sc.n_solids > kScanLinearMax) {
        const float4 gp = sc.gridp[0];
        const int G = sc.gridi[0];
        const float icw = 1.0f / gp.z, ich = 1.0f / gp.w;  // (cells are a heuristic filter too)
        const float inv = 1.0f / (float)npieces;
        const float t0 = (float)piece * inv, t1 = (float)(piece + 1) * inv;
        const float xa = ax + (bx - ax) * t0, xb = ax + (bx - ax) * t1;
        const float ya = ay + (by - ay) * t0, yb = ay + (by - ay) * t1;
        const int cx0 = min(G - 1, max(0, (int)floorf((fminf(xa, xb) - gp.x) * icw)));
        const int cx1 = min(G - 1, max(0, (int)floorf((fmaxf(xa, xb) - gp.x) * icw)));
        const int cy0 = min(G - 1, max(0, (int)floorf((fminf(ya, yb) - gp.y) * ich)));
        const int cy1 = min(G - 1, max(0, (int)floorf((fmaxf(ya, yb) - gp.y) * ich)));
        for (int cy = cy0; cy <= cy1; ++cy)
            for (int cx = cx0; cx <= cx1; ++cx) {
                const int cell = cy * G + cx;
                const int e1 = sc.gcell_off[cell + 1];
                for (int e = sc.gcell_off[cell]; e < e1; ++e) {
                    const float4 L = sc.gcell_ent[2 * e], H = sc.gcell_ent[2 * e + 1];
                    consider(__float_as_int(L.w), L, H);
                }
            }
    } else {
        for (int b = piece; b < sc.n_solids; b += npieces) consider(b, sc.sbox[2 * b], sc.sbox[2 * b + 1]);
    }
}

// The 2-D segment A -> B with its reciprocal direction, for ranking solids.
struct Ray2 {
    float ax, ay, ix, iy;  // ix = 1 / (bx - ax), 0 when the segment has no x extent
    bool zx, zy;           // no x / y extent
};

__device__ inline Ray2 make_ray2(float ax, float ay, float bx, float by) {
    Ray2 r;
    r.ax = ax;
    r.ay = ay;
    r.zx = bx == ax;
    r.zy = by == ay;
    r.ix = r.zx ? 0.f : 1.0f / (bx - ax);
    r.iy = r.zy ? 0.f : 1.0f / (by - ay);
    return r;
}

// Key of a solid for the segment: how near either end its footprint box starts
// along the segment (INFINITY if the 2-D segment misses the box).  A ranking
// heuristic only: a certificate is always checked exactly afterwards.
__device__ inline float segment_box_key(const Ray2 &r, float4 L, float4 H) {
    float t0 = 0.f, t1 = 1.f;
    if (!r.zx) {
        const float a = (L.x - r.ax) * r.ix, b = (H.x - r.ax) * r.ix;
        t0 = fmaxf(t0, fminf(a, b));
        t1 = fminf(t1, fmaxf(a, b));
    } else if (!(r.ax > L.x && r.ax < H.x)) {
        return INFINITY;
    }
    if (!r.zy) {
        const float a = (L.y - r.ay) * r.iy, b = (H.y - r.ay) * r.iy;
        t0 = fmaxf(t0, fminf(a, b));
        t1 = fminf(t1, fmaxf(a, b));
    } else if (!(r.ay > L.y && r.ay < H.y)) {
        return INFINITY;
    }
    return t0 < t1 ? fminf(t0, 1.f - t1) : INFINITY;
}

// Whole pair: one lane per pair of hull corners (at most 8 x 8).  `reach` gets
// whether any corner segment passes through the prism (a sub-pair bundle holds
// such a corner segment whenever its clusters hold hull corners).
__device__ bool certify_solid(const SolidLds &S, const HullLds &H, double u, Cnt &c, bool *reach = nullptr) {
    const int ni = H.ni, nj = H.nj;
    if (reach) *reach = false;
    if (S.pl[kSolidMaxPlanes].x <= 0 || ni == 0 || nj == 0 || !solid_sides(S, H, u, c)) return false;
    const int lane = lane_id();
    const bool act = lane < ni * nj;
    const int a = act ? lane / nj : 0, b = act ? lane - (lane / nj) * nj : 0;
    Cnt tmp;  // (a per-lane choice between two counter objects would force them into scratch)
    const bool good = solid_segment(S, H.hc[a], H.hc[kHullMax + b], u, tmp);
    if (act) c.solid_planes += tmp.solid_planes;
    if (reach) *reach = __ballot(act && good) != 0ull;
    return __ballot(act && !good) == 0ull;
}

// Per sub-pair (quadrant clusters, as in certify_subpairs): the cluster hulls
// lie inside the facet hulls, so (i) carries over; lanes run over the
// flattened (sub-pair, corner, corner) items.  Returns the certified sub-pairs
// among `todo`.
__device__ unsigned certify_solid_subpairs(const SolidLds &S, const HullLds &H, double u, unsigned todo,
                                           unsigned long long *fail, Cnt &c) {
    if (S.pl[kSolidMaxPlanes].x <= 0 || !todo || H.ni == 0 || H.nj == 0 || !solid_sides(S, H, u, c)) return 0u;
    const int lane = lane_id();
    if (lane < 16) fail[lane] = 0ull;
    wave_sync();
    int total = 0;
    for (int sp = 0; sp < 16; ++sp)
        if ((todo >> sp) & 1u) total += H.ccn[sp >> 2] * H.ccn[4 + (sp & 3)];
    for (int it = lane; it < total; it += kWave) {
        int run = 0, sp = 0, hi = 0, hj = 0;
        for (sp = 0; sp < 16; ++sp) {
            if (!((todo >> sp) & 1u)) continue;
            hi = H.ccn[sp >> 2];
            hj = H.ccn[4 + (sp & 3)];
            if (it < run + hi * hj) break;
            run += hi * hj;
        }
        const int cp = it - run;
        const int a = cp / hj, b = cp - (cp / hj) * hj;
        if (!solid_segment(S, H.cc[(sp >> 2) * kHullMax + a], H.cc[(4 + (sp & 3)) * kHullMax + b], u, c))
            atomicOr(&fail[sp], 1ull);
    }
    wave_sync();
    bool ok = false;
    if (lane < 16 && ((todo >> lane) & 1u)) ok = H.ccn[lane >> 2] * H.ccn[4 + (lane & 3)] > 0 && fail[lane] == 0ull;
    const unsigned res = (unsigned)(__ballot(ok) & 0xffffull);
    wave_sync();
    return res;
}

// Fan certificate: the solid certificate with one side's hull shrunk to a
// single sample.  Every segment from sample p of facet i to H_j passes through
// K when (i) holds for H_i (so for p) and H_j, p and the corners of H_j have
// z >= zb, and the segments from p to the corners of H_j pass through K (the
// convexity argument above with H_i = {p}); the same from a sample of j to the
// corners of H_i.  Lanes run over the (side, sample, corner) items of the
// compacted admissible samples sp[0, np) and sq[0, nq); fi / fj get the
// samples whose fans are certified (bit a = sp[a] / sq[a]).
__device__ void certify_fans(const SolidLds &S, const HullLds &H, const float4 *sp, int np, const float4 *sq, int nq,
                             double u, unsigned long long *fail, unsigned long long &fi, unsigned long long &fj,
                             Cnt &c) {
    fi = fj = 0ull;
    if (S.pl[kSolidMaxPlanes].x <= 0 || H.ni == 0 || H.nj == 0 || !solid_sides(S, H, u, c)) return;
    const int lane = lane_id();
    if (lane < 2) fail[lane] = 0ull;
    wave_sync();
    const int ti = np * H.nj, total = ti + nq * H.ni;
    for (int it = lane; it < total; it += kWave) {
        const bool si = it < ti;
        const int r = si ? it : it - ti;
        const int hc = si ? H.nj : H.ni;
        const int a = r / hc, k = r - a * hc;
        const float4 A = si ? sp[a] : sq[a];
        const float4 B = H.hc[(si ? kHullMax : 0) + k];
        if (!solid_segment(S, A, B, u, c)) atomicOr(&fail[si ? 0 : 1], 1ull << a);
    }
    wave_sync();
    const unsigned long long mi = np >= 64 ? ~0ull : ((1ull << np) - 1ull);
    const unsigned long long mj = nq >= 64 ? ~0ull : ((1ull << nq) - 1ull);
    fi = ~fail[0] & mi;
    fj = ~fail[1] & mj;
    wave_sync();
}

// Up to kSolidTries distinct verified solids among the blockers `hit` of the
// lanes with `blocked`, appended to the wave-uniform list (oldest replaced) and
// staged in LDS.
__device__ inline void remember_solid_ids(const SceneDev &sc, int *solids, int &nsol, int &spos, SolidLds *lds,
                                          int cap, bool blocked, int hit) {
    int sid = blocked ? sc.fsolid[__float_as_int(sc.tri[3 * hit].w)] : -1;
    for (int m = 0; m < nsol; ++m)
        if (sid == solids[m]) sid = -1;
    for (int added = 0; added < cap; ++added) {
        const unsigned long long left = __ballot(sid >= 0);
        if (!left) break;
        const int S0 = __shfl(sid, __ffsll((long long)left) - 1);
        if (sid == S0) sid = -1;
        int slot;
        if (nsol < cap) slot = nsol++;
        else { slot = spos; spos = (spos + 1) % cap; }
        solids[slot] = S0;
        stage_solid(sc, S0, lds[slot]);
    }
}

// Certificate per sub-pair: the samples of each facet are split into 4
// quadrant clusters (scene build) and sub-pair (ci, cj) is certified blocked by
// facet C when every segment between the corners of the two cluster hulls
// meets C (same convexity argument as above).  Lanes run over the flattened
// (sub-pair, corner, corner, triangle) items; returns the certified sub-pairs
// among `todo` (bit 4 ci + cj).
// (Always inlined: an out-of-line call taking the scene view by reference makes
// the pair kernel keep its kernel-argument copy in private memory and read every
// scene array through generic flat loads.)
__device__ __forceinline__ unsigned certify_subpairs(const SceneDev &sc, int i, int j, int C, unsigned todo,
                                                     unsigned long long *bits, float eps6, bool f64, Cnt &c) {
    const int lane = lane_id();
    const int t0 = sc.ftri[2 * C], nt = sc.ftri[2 * C + 1];
    if (nt <= 0 || !todo || !(sc.fflags[C] & kFacetConvex)) return 0u;
    if (lane < 16) bits[lane] = 0ull;
    wave_sync();
    int total = 0;
    for (int sp = 0; sp < 16; ++sp) {
        if (!((todo >> sp) & 1u)) continue;
        total += sc.fchull_n[4 * i + (sp >> 2)] * sc.fchull_n[4 * j + (sp & 3)] * nt;
    }
    for (int it = lane; it < total; it += kWave) {
        int run = 0, sp = 0, hi = 0, hj = 0;
        for (sp = 0; sp < 16; ++sp) {
            if (!((todo >> sp) & 1u)) continue;
            hi = sc.fchull_n[4 * i + (sp >> 2)];
            hj = sc.fchull_n[4 * j + (sp & 3)];
            const int cnt = hi * hj * nt;
            if (it < run + cnt) break;
            run += cnt;
        }
        const int local = it - run;
        const int cp = local / nt, t = local - (local / nt) * nt;
        const int a = cp / hj, b = cp - (cp / hj) * hj;
        const float4 P = sc.smp[sc.fchull[(4 * i + (sp >> 2)) * kHullMax + a]];
        const float4 Q = sc.smp[sc.fchull[(4 * j + (sp & 3)) * kHullMax + b]];
        const Seg sg = make_seg(P.x, P.y, P.z, Q.x, Q.y, Q.z);
        ++c.tests;
        const float4 *tr = sc.tri_caller + 3 * (t0 + t);
        if (tri_hit(sg, tr[0], tr[1], tr[2], eps6, f64, c.rechecks)) atomicOr(&bits[sp], 1ull << cp);
    }
    wave_sync();
    bool ok = false;
    if (lane < 16 && ((todo >> lane) & 1u)) {
        const int n = sc.fchull_n[4 * i + (lane >> 2)] * sc.fchull_n[4 * j + (lane & 3)];
        const unsigned long long full = n >= 64 ? ~0ull : ((1ull << n) - 1ull);
        ok = n > 0 && bits[lane] == full;
    }
    const unsigned res = (unsigned)(__ballot(ok) & 0xffffull);
    wave_sync();
    return res;
}

constexpr int kTile = 64;       // near-field tile capacity (triangle ranks)
constexpr int kFrontier = 128;  // cooperative traversal frontier capacity
// (a tile is gathered only when the bundle box meets at most TraverseOpts::tile_treelets treelets, kDefaultTileTreelets by default)

__device__ inline bool box_overlap(float lx, float ly, float lz, float hx, float hy, float hz, const float lo[3],
                                   const float hi[3]) {
    return !(lx > hi[0] || hx < lo[0] || ly > hi[1] || hy < lo[1] || lz > hi[2] || hz < lo[2]);
}

// Near-field tile: the wave walks the LBVH cooperatively (one frontier node per
// lane per step) against the closed box [lo, hi] of every admissible segment of
// the pair and stages the ranks of all triangles whose leaf boxes meet it,
// except those of facets i and j.  A triangle that meets a segment meets it
// inside that convex box, so all its ancestors' boxes overlap the box too: when
// the walk finishes within capacity the tile holds every possible blocker and a
// segment is decided by scanning the tile alone.  Returns the tile size, or -1
// when the tile would overflow.
__device__ int gather_tile(const SceneDev &sc, int i, int j, const float lo[3], const float hi[3],
                           const uint8_t *order, int n_order, int *frontier, int *tile, int *counters, int cap) {
    const int lane = lane_id();
    if (lane == 0) {
        counters[0] = 0;  // frontier size
        counters[1] = 0;  // tile size
        counters[2] = 0;  // overflow
    }
    wave_sync();
    if (lane < n_order) frontier[atomicAdd(&counters[0], 1)] = sc.tl_root[order[lane]];
    wave_sync();
    while (true) {
        const int nf = counters[0];
        if (nf == 0 || counters[2]) break;
        const int k = min(kWave, nf);
        const int ref = lane < k ? frontier[nf - k + lane] : kNone;
        wave_sync();
        if (lane == 0) counters[0] = nf - k;
        wave_sync();
        auto add_leaf = [&](int leaf) {
            const int first = leaf_first(leaf), cnt = leaf_count(leaf);
            for (int r = first; r < first + cnt; ++r) {
                const int f = __float_as_int(sc.tri[3 * r].w);
                if (f == i || f == j) continue;
                const int at = atomicAdd(&counters[1], 1);
                if (at < cap) tile[at] = r;
                else counters[2] = 1;
            }
        };
        if (ref != kNone) {
            if (ref < 0) {
                add_leaf(ref);
            } else {
                const Node nd = sc.nodes[ref];
                if (box_overlap(nd.a.x, nd.a.y, nd.a.z, nd.a.w, nd.b.x, nd.b.y, lo, hi)) {
                    if (nd.d.x < 0) add_leaf(nd.d.x);
                    else {
                        const int at = atomicAdd(&counters[0], 1);
                        if (at < kFrontier) frontier[at] = nd.d.x;
                        else counters[2] = 1;
                    }
                }
                if (box_overlap(nd.b.z, nd.b.w, nd.c.x, nd.c.y, nd.c.z, nd.c.w, lo, hi)) {
                    if (nd.d.y < 0) add_leaf(nd.d.y);
                    else {
                        const int at = atomicAdd(&counters[0], 1);
                        if (at < kFrontier) frontier[at] = nd.d.y;
                        else counters[2] = 1;
                    }
                }
            }
        }
        wave_sync();
    }
    const int n = counters[2] ? -1 : counters[1];
    wave_sync();
    return n;
}

// Exact any-hit over the tile: the first definite FP32 hit decides; undecided
// tests go to FP64.
__device__ inline int tile_hit(const SceneDev &sc, const Seg &s, const int *tile, int n, float eps6, bool f64, Cnt &c) {
    for (int k = 0; k < n; ++k) {
        const int r = tile[k];
        ++c.tests;
        if (tri_hit(s, sc.tri[3 * r], sc.tri[3 * r + 1], sc.tri[3 * r + 2], eps6, f64, c.rechecks)) return r;
    }
    return -1;
}

// A segment space is a list of rectangles of (admissible p index, admissible q
// index): rect k covers p in [pa, pa + pn) and q in [qb, qb + qn).
struct Rects {
    int n;
    int pa[16], pn[16], qb[16], qn[16], pre[17];
};

// Segment space of the sub-pairs in `todo`: sub-pair (ci, cj) covers the
// admissible samples of cluster ci of i (sP[pco[ci], pco[ci + 1])) times those
// of cluster cj of j.  Written by lane 0.
__device__ inline void set_rects(Rects &R, unsigned todo, const int *pco, const int *qco) {
    if (lane_id() != 0) return;
    int nr = 0, run = 0;
    for (int sp = 0; sp < 16; ++sp) {
        if (!((todo >> sp) & 1u)) continue;
        const int ci = sp >> 2, cj = sp & 3;
        R.pa[nr] = pco[ci];
        R.pn[nr] = pco[ci + 1] - pco[ci];
        R.qb[nr] = qco[cj];
        R.qn[nr] = qco[cj + 1] - qco[cj];
        R.pre[nr] = run;
        run += R.pn[nr] * R.qn[nr];
        ++nr;
    }
    R.pre[nr] = run;
    R.n = nr;
}

__constant__ uint8_t kIdentOrder[kTreelets] = {0,  1,  2,  3,  4,  5,  6,  7,  8,  9,  10, 11, 12, 13, 14, 15,
                                               16, 17, 18, 19, 20, 21, 22, 23, 24, 25, 26, 27, 28, 29, 30, 31};

// The first admissible sample of facet a towards facet b (orient(b, x) > 0),
// taken from position n/2 of a's list (round 0) or its mirror n - 1 - n/2
// (round 1) onwards, wrapping.
__device__ inline bool probe_sample(const SceneDev &sc, int a, int b, int round, float4 &x) {
    const int a0 = sc.soff[a], n = min(sc.soff[a + 1] - a0, kWave);
    const double *pl = sc.fplane + 6 * b;
    for (int t = 0, k = round ? n - 1 - (n >> 1) : n >> 1; t < n; ++t, k = k + 1 == n ? 0 : k + 1) {
        x = sc.smp[a0 + k];
        if (orient(pl, x.x, x.y, x.z) > 0.0) return true;
    }
    return false;
}

// Value of face plane k of verified solid K at x (sample units); k = planes is the top.
__device__ inline double solid_plane_global(const SceneDev &sc, int K, int k, int npl, int top, double x, double y,
                                            double z) {
    if (k < npl) {
        const int4 pl = sc.splane[K * kSolidMaxPlanes + k];
        return (double)pl.w * (x - (double)pl.x) - (double)pl.z * (y - (double)pl.y);
    }
    return z - (double)top;
}

// The whole-pair solid certificate for one lane's pair (i, j) and solid K, all
// steps on this lane: each facet's sample hull strictly outside one face plane,
// and every segment between hull corners through the open prism (the same
// conditions as the wave-wide form, hull corners read from global memory).
__device__ bool certify_pair_lane(const SceneDev &sc, int K, int i, int j, Cnt &c) {
    const int4 R = sc.solid[K];
    const int npl = R.x, ni = sc.fhull_n[i], nj = sc.fhull_n[j];
    if (npl <= 0 || ni == 0 || nj == 0) return false;
    const double u = ldexp(1.0, sc.gs);
    for (int side = 0; side < 2; ++side) {
        const int f = side ? j : i, nh = side ? nj : ni;
        bool out = false;
        for (int k = 0; k <= npl && !out; ++k) {
            bool all = true;
            for (int a = 0; a < nh && all; ++a) {
                const float4 x = sc.smp[sc.fhull[kHullMax * f + a]];
                ++c.solid_planes;
                all = solid_plane_global(sc, K, k, npl, R.y, x.x * u, x.y * u, x.z * u) > 0.0;
            }
            out = all;
        }
        if (!out) return false;
    }
    for (int a = 0; a < ni; ++a) {
        const float4 P = sc.smp[sc.fhull[kHullMax * i + a]];
        for (int b = 0; b < nj; ++b)
            if (!solid_segment_global(sc, K, P, sc.smp[sc.fhull[kHullMax * j + b]], c)) return false;
    }
    return true;
}

// Visibility probes: one admissible segment per candidate pair, 64 pairs per
// traversal (one per lane, treelets in index order).  A clear probe proves its
// pair visible (both bits of M); a blocked one tries the whole-pair certificate
// with the verified solid of the triangle that blocked it, and a certified pair
// is marked done.  Round 0 runs over the candidate pairs, round 1 over the pairs
// round 0 left undecided (und / uprefix), with other samples.  Each wave takes 64 consecutive candidates of one scene; in
// the MULTI form pbase[] is the exclusive prefix of the scenes' candidate
// totals rounded up to multiples of 64.
// Work queue over [0, total) split into `parts` contiguous ranges with a counter
// each (counters[0..parts)).  Workgroups are dispatched to the XCDs round-robin,
// so block b starts on range b % parts, and with one range per XCD the scene
// data its waves touch (neighbouring rows of the matrix) stays in that XCD's L2;
// a wave whose range is used up moves on to the next ranges, so every wave ends
// only when all ranges are empty.  Range bounds are multiples of `align`.
// Takes the next chunk [g0, g1) for the wave; returns false when none is left.
__device__ inline bool take_chunk(uint32_t *counters, int parts, uint32_t total, uint32_t align, uint32_t chunk,
                                  int &tries, uint32_t &g0, uint32_t &g1) {
    const uint32_t units = (total + align - 1) / align;
    while (tries < parts) {
        const int r = (int)((blockIdx.x + (unsigned)tries) % (unsigned)parts);
        const uint32_t lo = (uint32_t)((uint64_t)units * r / parts) * align;
        const uint32_t hi = min(total, (uint32_t)((uint64_t)units * (r + 1) / parts) * align);
        uint32_t off = 0;
        if (lane_id() == 0) off = atomicAdd(&counters[r], chunk);
        off = __shfl(off, 0);
        if (off < hi - lo) {
            g0 = lo + off;
            g1 = min(hi, g0 + chunk);
            return true;
        }
        ++tries;
    }
    return false;
}

template <bool MULTI>
__global__ __launch_bounds__(kBlock) void k_probe_pairs(PairJob one, const PairJob *many, const uint32_t *pbase,
                                                        int n_jobs, uint32_t *queue, int round, TraverseOpts o,
                                                        ivm_stats *st) {
    __shared__ int sStack[kWavesPerBlock][kWave * IVM_MAX_STACK];
    const int wv = threadIdx.x >> 6, lane = lane_id();
    int *stk = &sStack[wv][lane];
    const bool f64 = o.fp64_only != 0;
    Cnt c;
    unsigned long long segs = 0, nvis = 0, ncert = 0;
    const uint32_t total =
        MULTI ? pbase[n_jobs] : ((round ? one.uprefix : one.prefix)[one.n_items] + kWave - 1) / kWave * kWave;
    int tries = 0;
    while (true) {
        uint32_t g0 = 0, g1 = 0;
        if (!take_chunk(queue, o.xcd_parts, total, kWave, kWave, tries, g0, g1)) break;
        int js = 0;
        if (MULTI) {
            int lo = 0, hi = n_jobs - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (pbase[mid] <= g0) lo = mid;
                else hi = mid - 1;
            }
            js = lo;
        }
        const PairJob &J = MULTI ? many[js] : one;
        const SceneDev &sc = J.sc;
        const uint32_t gl = g0 - (MULTI ? pbase[js] : 0u) + (uint32_t)lane;
        const uint64_t *cw = round ? J.und : J.cand;
        const uint32_t *pf = round ? J.uprefix : J.prefix;
        bool act = sc.F >= 2 && gl < pf[J.n_items];
        int i = 0, j = 0;
        float4 P = make_float4(0.f, 0.f, 0.f, 0.f), Q = P;
        if (act) {
            decode_pair(sc, cw, pf, J.n_items, gl, i, j);
            act = probe_sample(sc, i, j, round, P) && probe_sample(sc, j, i, round, Q);
        }
        const Seg sg = make_seg(P.x, P.y, P.z, Q.x, Q.y, Q.z);
        if (act) {
            ++segs;
            ++c.traversed;
        }
        const int hit = any_hit_wave(sc, sg, act, i, j, kIdentOrder, kTreelets, stk, o.stack_depth, o.eps6, f64, c,
                                     0, 0);
        if (act && hit == -1) {
            atomicOr((unsigned long long *)&J.M[(size_t)i * sc.W + (j >> 6)], 1ull << (j & 63));
            atomicOr((unsigned long long *)&J.M[(size_t)j * sc.W + (i >> 6)], 1ull << (i & 63));
            ++nvis;
        }
        if (act && hit >= 0 && sc.n_solids > 0) {
            const int K = sc.fsolid[__float_as_int(sc.tri[3 * hit].w)];
            if (K >= 0 && certify_pair_lane(sc, K, i, j, c)) {
                atomicOr((unsigned long long *)&J.done[(size_t)i * sc.W + (j >> 6)], 1ull << (j & 63));
                ++ncert;
            }
        }
    }
    flush_counters(st, c, segs, wave_sum_u64(nvis), 0);
    const unsigned long long nc = wave_sum_u64(ncert);
    if (st && lane == 0 && nc) atomicAdd((unsigned long long *)&st->solid_certified, nc);
}

// MULTI: the queue index runs over the concatenated candidates of n_jobs scenes
// (base[] = exclusive prefix of their candidate totals); otherwise over `one`.
template <bool MULTI>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(3))) void k_pairs(PairJob one, const PairJob *many, const uint32_t *base, int n_jobs,
                                                  uint32_t *queue, TraverseOpts o, ivm_stats *st) {
    __shared__ float4 sP[kWavesPerBlock][kWave];
    __shared__ float4 sQ[kWavesPerBlock][kWave];
    __shared__ int sStack[kWavesPerBlock][kWave * IVM_MAX_STACK];
    __shared__ unsigned long long sKey[kWavesPerBlock][kTreelets];
    __shared__ uint8_t sOrder[kWavesPerBlock][kTreelets];
    __shared__ int sCorner[kWavesPerBlock][kWave];
    __shared__ int sMiss[kWavesPerBlock][2 * kWave];
    __shared__ unsigned long long sBits[kWavesPerBlock][16];
    __shared__ Rects sR[kWavesPerBlock];
    __shared__ int sTile[kWavesPerBlock][kTile];
    __shared__ int sTileCnt[kWavesPerBlock][4];
    __shared__ SolidLds sSL[kWavesPerBlock][kSolidTries];
    __shared__ HullLds sH[kWavesPerBlock];
    // wave-uniform lists live in LDS: dynamically indexed private arrays would
    // go to scratch memory
    __shared__ int sList[kWavesPerBlock][kCache + kSolidTries + kCache + 10];
    const int wv = threadIdx.x >> 6, lane = lane_id();
    const uint32_t total = MULTI ? base[n_jobs] : one.uprefix[one.n_items];
    int *stk = &sStack[wv][lane];
    int *miss = sMiss[wv];
    Rects &R = sR[wv];
    const bool f64 = o.fp64_only != 0;
    Cnt c;
    unsigned segs = 0, nvis = 0, ncert = 0, nsub = 0, ntiled = 0, nsolid = 0, nfan = 0;  // per-wave counts fit 32 bits
    const unsigned long long lt = (1ull << lane) - 1ull;
    // A wave takes a chunk of consecutive candidates at a time (same facet i,
    // neighbouring j), and keeps its recent blocker triangles and solids from
    // one pair to the next within a scene.
    int *cache = sList[wv];                  // recent blockers (sorted ranks)
    int *solids = cache + kCache;            // verified solids met by traversals
    int *tried = solids + kSolidTries;       // facets tried by a sub-pair certificate
    int *pco = tried + kCache, *qco = pco + 5;  // cluster offsets of the admissible samples
    int ncache = 0, cpos = 0;
    int nsol = 0, sspos = 0;
    int cur_js = -1;
    int vh_i = -1, vh_a = 0, vh_b = 0;  // the wave's last visible pair: facet i and the clear segment's samples
    uint32_t g_next = 0, g_end = 0;
    // decode state: the previous pair's candidate word and its bits from that pair on
    int d_item = 0;
    unsigned long long d_m = 0ull;
    uint32_t d_gl = 0xffffffffu;
    const uint32_t nwaves_all = gridDim.x * (uint32_t)kWavesPerBlock;
    const uint32_t chunk = o.pair_chunk > 0 ? (uint32_t)o.pair_chunk
                           : (total / nwaves_all > kLargePerWave ? (uint32_t)kPairChunkLarge : (uint32_t)kPairChunk);
    int tries = 0;
    while (true) {
        if (g_next >= g_end) {
            uint32_t g0 = 0, g1 = 0;
            if (!take_chunk(queue, o.xcd_parts, total, 1u, chunk, tries, g0, g1)) break;
            g_next = g0;
            g_end = g1;
        }
        const uint32_t g = g_next++;
        int js = 0;
        uint32_t gl = g;
        if (MULTI) {
            int lo = 0, hi = n_jobs - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (base[mid] <= g) lo = mid;
                else hi = mid - 1;
            }
            js = lo;
            gl = g - base[js];
        }
        const PairJob &J = MULTI ? many[js] : one;
        const SceneDev &sc = J.sc;
        if (js != cur_js) {
            cur_js = js;
            vh_i = -1;
            ncache = cpos = nsol = sspos = 0;
            d_m = 0ull;  // (d_gl + 1 wraps to 0, the new scene's first pair: an empty word forces a full decode)
            d_gl = 0xffffffffu;
        }
        // consecutive candidates of one word: the next set bit (a binary search
        // over the prefix only when the word is used up or the chunk jumps)
        // (the pairs the probe kernel left undecided)
        if (gl == d_gl + 1u && (d_m & (d_m - 1ull)) != 0ull) {
            d_m &= d_m - 1ull;
        } else {
            d_item = find_item(J.uprefix, J.n_items, gl);
            d_m = J.und[d_item];
            for (uint32_t q = J.uprefix[d_item]; q < gl; ++q) d_m &= d_m - 1ull;
        }
        d_gl = gl;
        const int jbit = __ffsll((long long)d_m) - 1;
        const int i = d_item / sc.W, j = (d_item - i * sc.W) * 64 + jbit;
        const double *pli = sc.fplane + 6 * i, *plj = sc.fplane + 6 * j;
        const int si0 = sc.soff[i], ni = min(sc.soff[i + 1] - si0, kWave);
        const int sj0 = sc.soff[j], nj = min(sc.soff[j + 1] - sj0, kWave);
        float4 p = lane < ni ? (float4)sc.smp[si0 + lane] : make_float4(0, 0, 0, 0);
        float4 q = lane < nj ? (float4)sc.smp[sj0 + lane] : make_float4(0, 0, 0, 0);
        const bool okp = lane < ni && orient(plj, p.x, p.y, p.z) > 0.0;
        const bool okq = lane < nj && orient(pli, q.x, q.y, q.z) > 0.0;
        p.w = __int_as_float(lane);  // (the sample's index in its facet, for the visible-pair hint)
        q.w = __int_as_float(lane);
        const int clp = lane < ni ? sc.scluster[si0 + lane] : 0;
        const int clq = lane < nj ? sc.scluster[sj0 + lane] : 0;
        // compact admissible samples grouped by cluster: cluster c of i occupies
        // [pco[c], pco[c + 1]) of sP
        pco[0] = qco[0] = 0;
        for (int cl = 0; cl < 4; ++cl) {
            const unsigned long long mpc = __ballot(okp && clp == cl), mqc = __ballot(okq && clq == cl);
            if (okp && clp == cl) sP[wv][pco[cl] + __popcll(mpc & lt)] = p;
            if (okq && clq == cl) sQ[wv][qco[cl] + __popcll(mqc & lt)] = q;
            pco[cl + 1] = pco[cl] + __popcll(mpc);
            qco[cl + 1] = qco[cl] + __popcll(mqc);
        }
        int np = pco[4], nq = qco[4];
        // bounding box of every admissible segment
        float lo[3], hi[3];
        {
            const float big = INFINITY;
            float l0 = big, l1 = big, l2 = big, h0 = -big, h1 = -big, h2 = -big;
            if (okp) { l0 = p.x; l1 = p.y; l2 = p.z; h0 = p.x; h1 = p.y; h2 = p.z; }
            if (okq) {
                l0 = fminf(l0, q.x); l1 = fminf(l1, q.y); l2 = fminf(l2, q.z);
                h0 = fmaxf(h0, q.x); h1 = fmaxf(h1, q.y); h2 = fmaxf(h2, q.z);
            }
            lo[0] = wave_min(l0); lo[1] = wave_min(l1); lo[2] = wave_min(l2);
            hi[0] = wave_max(h0); hi[1] = wave_max(h1); hi[2] = wave_max(h2);
        }
        // the solids that blocked the previous pairs first: a whole-pair certificate
        // costs far less than one traversal batch
        // sub-pairs (quadrant clusters) with admissible samples on both sides
        unsigned todo = 0u;
        int biggest = 0;
        for (int sp = 0; sp < 16; ++sp) {
            const int pn = pco[(sp >> 2) + 1] - pco[sp >> 2], qn = qco[(sp & 3) + 1] - qco[sp & 3];
            if (pn > 0 && qn > 0) todo |= 1u << sp;
            biggest = max(biggest, pn * qn);
        }
        const unsigned all_sub = todo;
        const bool split = biggest >= 2 * kWave;  // sub-pairs worth certifying one by one
        const double gsu = ldexp(1.0, sc.gs);  // metres -> sample units (exact)
        bool hulls = false;                    // sample hulls staged in LDS for this pair
        bool early = false;
        if (!o.exhaustive && sc.n_solids > 0) {
            // only solids whose box reaches the segment box; a solid that certifies
            // the pair moves to the front of the wave's list
            unsigned reach_sub = 0u;
            const float4 Pm = sP[wv][np >> 1], Qm = sQ[wv][nq >> 1];
            for (int m = 0; m < nsol && !early; ++m) {
                if (!solid_box_reach(sSL[wv][m], lo, hi)) continue;
                if (!hulls) {
                    stage_hulls(sc, i, j, sH[wv]);
                    hulls = true;
                }
                bool reach = false;
                early = certify_solid(sSL[wv][m], sH[wv], gsu, c, &reach);
                if (early) solid_to_front(solids, sSL[wv], m);
                else if (reach) reach_sub |= 1u << m;
            }
            // then solids from the whole scene met by the segment joining the centroids
            // of the admissible samples, those nearest to either end first
            if (!early && sc.n_solids <= kScanMaxSolids) {
                const float cpx = wave_sum(okp ? p.x : 0.f) / np, cpy = wave_sum(okp ? p.y : 0.f) / np;
                const float cpz = wave_sum(okp ? p.z : 0.f) / np;
                const float cqx = wave_sum(okq ? q.x : 0.f) / nq, cqy = wave_sum(okq ? q.y : 0.f) / nq;
                const float cqz = wave_sum(okq ? q.z : 0.f) / nq;
                const int own_i = sc.fsolid[i], own_j = sc.fsolid[j];
                const float zlow = fminf(cpz, cqz);
                const Ray2 ray = make_ray2(cpx, cpy, cqx, cqy);
                float bkey;
                int bsol;
                scan_solids(
                    sc, cpx, cpy, cqx, cqy, lane, kWave,
                    [&](int sid, float4 L, float4 H) -> float {
                        if (!(hi[0] > L.x && lo[0] < H.x && hi[1] > L.y && lo[1] < H.y && zlow < H.z && lo[2] >= L.z))
                            return INFINITY;
                        if (sid == own_i || sid == own_j) return INFINITY;
                        for (int m = 0; m < nsol; ++m)
                            if (solids[m] == sid) return INFINITY;
                        return segment_box_key(ray, L, H);
                    },
                    // a solid that certifies the pair blocks every admissible segment, so also
                    // the one between the middle admissible samples (tested for a lane's
                    // best candidate so far only)
                    [](int) -> bool { return true; },
                    bkey, bsol);
                if (bsol >= 0 && !solid_segment_global(sc, bsol, Pm, Qm, c)) bkey = INFINITY;
                for (int tr = 0; tr < kScanTries && !early; ++tr) {
                    const float kmin = wave_min(bkey);
                    if (!(kmin < INFINITY)) break;
                    const unsigned long long win = __ballot(bkey == kmin);
                    const int src = __ffsll((long long)win) - 1;
                    const int sid = __shfl(bsol, src);
                    if (bsol == sid) bkey = INFINITY;  // every lane holding it drops it
                    int slot;
                    if (nsol < kSolidTries) slot = nsol++;
                    else { slot = sspos; sspos = (sspos + 1) % kSolidTries; }
                    reach_sub &= ~(1u << slot);
                    solids[slot] = sid;
                    stage_solid(sc, sid, sSL[wv][slot]);
                    if (!hulls) {
                        stage_hulls(sc, i, j, sH[wv]);
                        hulls = true;
                    }
                    bool reach = false;
                    early = certify_solid(sSL[wv][slot], sH[wv], gsu, c, &reach);
                    if (early) solid_to_front(solids, sSL[wv], slot);
                    else if (reach) reach_sub |= 1u << slot;
                }
            }
            for (int m = 0; m < nsol && !early && split; ++m) {
                if (!((reach_sub >> m) & 1u)) continue;
                todo &= ~certify_solid_subpairs(sSL[wv][m], sH[wv], gsu, todo, sBits[wv], c);
                early = todo == 0u;
            }
            // a pair that several solids block (no single one certifies it): fans of
            // one sample against the other facet's hull, by each solid that reaches
            // the bundle; a segment is blocked when either end's fan is certified, so
            // the segment space shrinks to the samples of uncertified fans on both
            // sides (small sample sets only: the cluster sub-pairs serve large ones)
            if (!early && !split && reach_sub) {
                unsigned long long ci = 0ull, cj = 0ull;
                for (int m = 0; m < nsol; ++m) {
                    if (!((reach_sub >> m) & 1u)) continue;
                    unsigned long long fi, fj;
                    certify_fans(sSL[wv][m], sH[wv], sP[wv], np, sQ[wv], nq, gsu, sBits[wv], fi, fj, c);
                    ci |= fi;
                    cj |= fj;
                }
                if (ci | cj) {
                    const bool kp = lane < np && !((ci >> lane) & 1ull);
                    const bool kq = lane < nq && !((cj >> lane) & 1ull);
                    const float4 vp = sP[wv][lane < np ? lane : 0], vq = sQ[wv][lane < nq ? lane : 0];
                    const unsigned long long bp = __ballot(kp), bq = __ballot(kq);
                    wave_sync();
                    if (kp) sP[wv][__popcll(bp & lt)] = vp;
                    if (kq) sQ[wv][__popcll(bq & lt)] = vq;
                    wave_sync();
                    np = __popcll(bp);
                    nq = __popcll(bq);
                    early = np == 0 || nq == 0;
                    ++nfan;
                }
            }
        }
        if (early) {
            ++nsolid;
            continue;
        }
        unsigned long long lcode = 0;
        if (o.order_mode == IVM_ORDER_LEARNED && J.learned) lcode = J.learned[gl];  // (per undecided pair)
        const int n_order = wave_rank_order(treelet_key(sc, lane, lo, hi, o.order_mode, lcode), sKey[wv], sOrder[wv]);
        // near-field tile (the miss queue's storage doubles as the walk frontier)
        // (only for bundles meeting few treelets: a long bundle would overflow the tile anyway)
        const int ntile = (o.no_tile || n_order > o.tile_treelets)
                              ? -1
                              : gather_tile(sc, i, j, lo, hi, sOrder[wv], n_order, sMiss[wv], sTile[wv], sTileCnt[wv],
                                            o.tile_cap);
        ntiled += ntile >= 0;
        // the segment space: the whole product (one rectangle, spread order over
        // all of it) unless some sub-pairs are already certified
        if (todo != all_sub) {
            set_rects(R, todo, pco, qco);
            ++nsub;
        } else if (lane == 0) {
            R.n = 1;
            R.pa[0] = 0; R.pn[0] = np; R.qb[0] = 0; R.qn[0] = nq;
            R.pre[0] = 0; R.pre[1] = np * nq;
        }
        wave_sync();
        int nseg = R.pre[R.n];
        bool vis = false, done = false, first_traversal = true;
        int nmiss = 0;
        // a first batch of one segment: between the samples at the positions of the
        // clear segment of the wave's last visible pair with the same facet i
        bool hint_batch = false;
        if (vh_i == i && !o.exhaustive && nseg > 1) {
            const unsigned long long ma = __ballot(lane < np && __float_as_int(sP[wv][lane].w) == vh_a);
            const unsigned long long mb = __ballot(lane < nq && __float_as_int(sQ[wv][lane].w) == vh_b);
            if (ma && mb) {
                if (lane == 0) miss[0] = (__ffsll((long long)ma) - 1) | ((__ffsll((long long)mb) - 1) << 8);
                nmiss = 1;
                hint_batch = true;
                wave_sync();
            }
        }
        for (int base = 0; !done; base += kWave) {
            const bool more = base < nseg && !hint_batch;
            if (more) {
                // cache pass: each lane takes one segment in spread order (the first
                // batch pairs many different p with many q) and tests the recent blockers
                const int sidx = base + lane;
                bool need = false;
                int ab = 0;
                if (sidx < nseg) {
                    int k = 0;
                    while (k + 1 < R.n && sidx >= R.pre[k + 1]) ++k;
                    const int local = sidx - R.pre[k], pn = R.pn[k], qn = R.qn[k];
                    // (local + 1/2) / pn sits >= 1/(2 pn) >= 1/128 away from an integer and
                    // local < 4096, so the float product's error (< 2e-3) cannot move the floor
                    const int qa = (int)(((float)local + 0.5f) * __builtin_amdgcn_rcpf((float)pn));
                    const int al = local - qa * pn;
                    const int t = qa + al;
                    const int bl = t - qn * (int)(((float)t + 0.5f) * __builtin_amdgcn_rcpf((float)qn));
                    const int a = R.pa[k] + al, b = R.qb[k] + bl;
                    ab = a | (b << 8);
                    ++segs;
                    need = true;
                    if (ncache > 0 && !o.exhaustive) {
                        const float4 P = sP[wv][a], Q = sQ[wv][b];
                        const Seg sg = make_seg(P.x, P.y, P.z, Q.x, Q.y, Q.z);
                        for (int m = 0; m < ncache && need; ++m) {
                            const int r = cache[m];
                            const int fr = __float_as_int(sc.tri[3 * r].w);
                            if (fr == i || fr == j) continue;  // kept from another pair
                            ++c.tests;
                            if (tri_hit(sg, sc.tri[3 * r], sc.tri[3 * r + 1], sc.tri[3 * r + 2], o.eps6, f64,
                                        c.rechecks))
                                need = false;
                        }
                        // then the solids met so far, segment by segment
                        for (int m = 0; m < nsol && need; ++m)
                            if (solid_segment(sSL[wv][m], P, Q, gsu, c)) {
                                need = false;
                                ++c.solid_segs;
                            }
                    }
                }
                const unsigned long long nm = __ballot(need);
                if (need) miss[nmiss + __popcll(nm & lt)] = ab;
                nmiss += __popcll(nm);
                wave_sync();
            }
            // the misses of each cache pass are traversed at once rather than collected
            // into full batches: their blockers then serve the next passes (fewer misses
            // in all), and a visible pair ends at its first clear segment sooner
            while (!done && nmiss > 0) {
                const int k = min(kWave, nmiss);
                int hit = -1;
                bool clear = false;
                {
                    const int ab = lane < k ? miss[nmiss - k + lane] : 0;
                    const float4 P = sP[wv][ab & 255], Q = sQ[wv][ab >> 8];
                    const Seg sg = make_seg(P.x, P.y, P.z, Q.x, Q.y, Q.z);
                    if (lane < k) ++c.traversed;
                    if (ntile >= 0) {
                        if (lane < k) hit = tile_hit(sc, sg, sTile[wv], ntile, o.eps6, f64, c);
                    } else {
                        hit = any_hit_wave(sc, sg, lane < k, i, j, sOrder[wv], n_order, stk, o.stack_depth, o.eps6, f64,
                                           c, kAbortAll, 0);
                    }
                    clear = lane < k && hit == -1;
                    const unsigned long long cm = __ballot(clear);
                    if (cm) {
                        const int abv = __shfl(ab, __ffsll((long long)cm) - 1);
                        vh_i = i;
                        vh_a = __float_as_int(sP[wv][abv & 255].w);
                        vh_b = __float_as_int(sQ[wv][abv >> 8].w);
                    }
                }
                nmiss -= k;
                wave_sync();
                if (__ballot(clear)) {
                    vis = done = true;
                    break;
                }
                if (sc.n_solids > 0) remember_solid_ids(sc, solids, nsol, sspos, sSL[wv], kSolidTries, lane < k, hit);
                // remember up to kCache distinct new blockers
                unsigned long long fm = __ballot(lane < k);
                for (int added = 0; fm && added < kCache; ++added) {
                    const int src = __ffsll((long long)fm) - 1;
                    fm &= fm - 1;
                    const int r = __shfl(hit, src);
                    bool dup = false;
                    for (int m = 0; m < ncache; ++m) dup |= cache[m] == r;
                    if (dup) continue;
                    if (ncache < kCache) cache[ncache++] = r;
                    else { cache[cpos] = r; cpos = (cpos + 1) % kCache; }
                }
                if (first_traversal && !hint_batch && nseg > kWave && !o.exhaustive) {
                    first_traversal = false;
                    // the first traversal batch is all blocked: try to prove the whole pair
                    // blocked by the facet that blocked its first lane, then its last lane's
                    // first by the verified solids met by this batch, then by single facets
                    bool blocked = false;
                    if (nsol > 0 && !hulls) {
                        stage_hulls(sc, i, j, sH[wv]);
                        hulls = true;
                    }
                    for (int m = 0; m < nsol && !blocked; ++m) blocked = certify_solid(sSL[wv][m], sH[wv], gsu, c);
                    if (blocked) {
                        ++nsolid;
                        done = true;
                        break;
                    }
                    const int C1 = __float_as_int(sc.tri[3 * __shfl(hit, 0)].w);
                    const int C2 = __float_as_int(sc.tri[3 * __shfl(hit, k - 1)].w);
                    blocked = certify_blocked(sc, i, j, C1, sCorner[wv], o.eps6, f64, c);
                    if (!blocked && C2 != C1) blocked = certify_blocked(sc, i, j, C2, sCorner[wv], o.eps6, f64, c);
                    if (blocked) {
                        ++ncert;
                        done = true;
                        break;
                    }
                    // then sub-pair by sub-pair with every solid and facet seen blocking so
                    // far; the uncertified sub-pairs become the new segment space
                    if (split) {
                        const unsigned before = todo;
                        for (int m = 0; m < nsol && todo; ++m)
                            todo &= ~certify_solid_subpairs(sSL[wv][m], sH[wv], gsu, todo, sBits[wv], c);
                        if (!todo) {
                            ++nsolid;
                            done = true;
                            break;
                        }
                        int ntried = 0;
                        for (int m = 0; m < ncache && todo; ++m) {
                            const int C = __float_as_int(sc.tri[3 * cache[m]].w);
                            bool seen = false;
                            for (int u = 0; u < ntried; ++u) seen |= tried[u] == C;
                            if (seen) continue;
                            tried[ntried++] = C;
                            todo &= ~certify_subpairs(sc, i, j, C, todo, sBits[wv], o.eps6, f64, c);
                        }
                        if (!todo) {
                            ++ncert;
                            done = true;
                            break;
                        }
                        if (todo != before) {
                            if (before == all_sub) ++nsub;
                            set_rects(R, todo, pco, qco);
                            wave_sync();
                            nseg = R.pre[R.n];
                            base = -kWave;  // restart the cache passes over the new space
                            nmiss = 0;
                            break;
                        }
                    }
                }
            }
            if (hint_batch) {
                // (the hint's batch is over: the pass over the segments starts)
                hint_batch = false;
                base -= kWave;
                continue;
            }
            if (!more && nmiss == 0) done = true;
        }
        if (vis && lane == 0) {
            atomicOr((unsigned long long *)&J.M[(size_t)i * sc.W + (j >> 6)], 1ull << (j & 63));
            atomicOr((unsigned long long *)&J.M[(size_t)j * sc.W + (i >> 6)], 1ull << (i & 63));
            ++nvis;
        }
        wave_sync();
    }
    flush_counters(st, c, segs, nvis, 0);
    if (st && lane == 0 && ncert) atomicAdd((unsigned long long *)&st->certified, (unsigned long long)ncert);
    if (st && lane == 0 && (nsub + nfan))
        atomicAdd((unsigned long long *)&st->subpair_runs, (unsigned long long)(nsub + nfan));
    if (st && lane == 0 && ntiled) atomicAdd((unsigned long long *)&st->tiled_pairs, (unsigned long long)ntiled);
    if (st && lane == 0 && nsolid) atomicAdd((unsigned long long *)&st->solid_certified, (unsigned long long)nsolid);
}

// Hit records for the occluder-ordering network: for each listed pair, the set
// of treelets holding a triangle that meets at least one admissible segment.
// Treelets already in the set are not searched again, so each segment runs one
// any-hit search per treelet still open.
__global__ __launch_bounds__(kBlock) void k_labels(SceneDev sc, int n, const int32_t *I, const int32_t *J,
                                                   uint32_t *labels, TraverseOpts o) {
    __shared__ float4 sP[kWavesPerBlock][kWave];
    __shared__ float4 sQ[kWavesPerBlock][kWave];
    __shared__ int sStack[kWavesPerBlock][kWave * IVM_MAX_STACK];
    __shared__ unsigned long long sKey[kWavesPerBlock][kTreelets];
    __shared__ uint8_t sOrder[kWavesPerBlock][kTreelets];
    __shared__ uint8_t sRem[kWavesPerBlock][kTreelets];
    const int wv = threadIdx.x >> 6, lane = lane_id();
    int *stk = &sStack[wv][lane];
    const bool f64 = o.fp64_only != 0;
    const unsigned long long lt = (1ull << lane) - 1ull;
    Cnt c;
    const int wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int nwaves = (gridDim.x * blockDim.x) >> 6;
    for (int k = wave; k < n; k += nwaves) {
        int i = min(I[k], J[k]), j = max(I[k], J[k]);
        if (i < 0 || j >= sc.F || i == j) {
            if (lane == 0) labels[k] = 0u;
            continue;
        }
        const double *pli = sc.fplane + 6 * i, *plj = sc.fplane + 6 * j;
        const int si0 = sc.soff[i], ni = min(sc.soff[i + 1] - si0, kWave);
        const int sj0 = sc.soff[j], nj = min(sc.soff[j + 1] - sj0, kWave);
        const float4 p = lane < ni ? (float4)sc.smp[si0 + lane] : make_float4(0, 0, 0, 0);
        const float4 q = lane < nj ? (float4)sc.smp[sj0 + lane] : make_float4(0, 0, 0, 0);
        const bool okp = lane < ni && orient(plj, p.x, p.y, p.z) > 0.0;
        const bool okq = lane < nj && orient(pli, q.x, q.y, q.z) > 0.0;
        const unsigned long long mp = __ballot(okp), mq = __ballot(okq);
        const int np = __popcll(mp), nq = __popcll(mq);
        if (okp) sP[wv][__popcll(mp & lt)] = p;
        if (okq) sQ[wv][__popcll(mq & lt)] = q;
        float lo[3], hi[3];
        {
            const float big = INFINITY;
            float l0 = big, l1 = big, l2 = big, h0 = -big, h1 = -big, h2 = -big;
            if (okp) { l0 = p.x; l1 = p.y; l2 = p.z; h0 = p.x; h1 = p.y; h2 = p.z; }
            if (okq) {
                l0 = fminf(l0, q.x); l1 = fminf(l1, q.y); l2 = fminf(l2, q.z);
                h0 = fmaxf(h0, q.x); h1 = fmaxf(h1, q.y); h2 = fmaxf(h2, q.z);
            }
            lo[0] = wave_min(l0); lo[1] = wave_min(l1); lo[2] = wave_min(l2);
            hi[0] = wave_max(h0); hi[1] = wave_max(h1); hi[2] = wave_max(h2);
        }
        const int n_order = wave_rank_order(treelet_key(sc, lane, lo, hi, IVM_ORDER_INDEX, 0ull), sKey[wv], sOrder[wv]);
        unsigned mask = 0u;
        const int nseg = np * nq;
        for (int base = 0; base < nseg; base += kWave) {
            const bool open = lane < n_order && !((mask >> sOrder[wv][lane]) & 1u);
            const unsigned long long om = __ballot(open);
            if (open) sRem[wv][__popcll(om & lt)] = sOrder[wv][lane];
            wave_sync();
            const int nrem = __popcll(om);
            if (nrem == 0) break;
            const int sidx = base + lane;
            const bool act = sidx < nseg;
            Seg sg = make_seg(0, 0, 0, 0, 0, 0);
            if (act) {
                const int a = sidx / nq, b = sidx - (sidx / nq) * nq;
                const float4 P = sP[wv][a], Q = sQ[wv][b];
                sg = make_seg(P.x, P.y, P.z, Q.x, Q.y, Q.z);
            }
            for (int r = 0; r < nrem; ++r) {
                bool hit = false;
                if (act) hit = any_hit(sc, sg, i, j, &sRem[wv][r], 1, stk, o.stack_depth, o.eps6, f64, c) >= 0;
                if (__ballot(hit)) mask |= 1u << sRem[wv][r];
            }
            wave_sync();
        }
        if (lane == 0) labels[k] = mask;
    }
}

hipError_t launch_pair_labels(Scene &scn, const TraverseOpts &o, int n, const int32_t *I, const int32_t *J,
                              uint32_t *labels, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_labels, dim3(o.grid_blocks), dim3(kBlock), 0, s, scn.dev, n, I, J, labels, o);
    return hipGetLastError();
}

__global__ void k_pair_stats(ivm_stats *st, const uint32_t *prefix, int n_items, int F) {
    if (threadIdx.x == 0 && blockIdx.x == 0 && st) {
        atomicAdd((unsigned long long *)&st->pairs_candidate, (unsigned long long)prefix[n_items]);
        atomicAdd((unsigned long long *)&st->pairs_total, (unsigned long long)F * (F - 1) / 2);
    }
}

__global__ void k_fill_u32(uint32_t *p, uint32_t v, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}
__global__ void k_fill_u64(uint64_t *p, uint64_t v, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}

hipError_t launch_fill_u32(uint32_t *p, uint32_t v, size_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    unsigned b = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(k_fill_u32, dim3(b > 4096 ? 4096 : b), dim3(256), 0, s, p, v, n);
    return hipGetLastError();
}
hipError_t launch_fill_u64(uint64_t *p, uint64_t v, size_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    unsigned b = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(k_fill_u64, dim3(b > 4096 ? 4096 : b), dim3(256), 0, s, p, v, n);
    return hipGetLastError();
}

int device_cu_count() {
    static int cus = 0;
    if (!cus) {
        int dev = 0;
        hipGetDevice(&dev);
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) == hipSuccess) cus = prop.multiProcessorCount;
        if (cus <= 0) cus = 256;
    }
    return cus;
}

PairJob make_pair_job(Scene &scn, uint64_t *M, bool learned) {
    char *ws = (char *)scn.ws;
    const Layout &L = scn.lay;
    PairJob j;
    j.sc = scn.dev;
    j.cand = (const uint64_t *)(ws + L.cand);
    j.prefix = (const uint32_t *)(ws + L.prefix);
    j.n_items = scn.n_items;
    j.M = M;
    j.learned = learned && L.learned_bytes ? (const uint64_t *)(ws + L.learned) : nullptr;
    j.done = (uint64_t *)(ws + L.done);
    j.und = (const uint64_t *)(ws + L.und);
    j.uprefix = (const uint32_t *)(ws + L.uprefix);
    return j;
}

// Zero M, cull every unordered pair by orientation, scan the candidate counts
// and reset the scene's queue counter.
hipError_t launch_cull_scan(Scene &scn, uint64_t *M, ivm_stats *stats, hipStream_t s) {
    const SceneDev &sc = scn.dev;
    char *ws = (char *)scn.ws;
    const Layout &L = scn.lay;
    uint64_t *cand = (uint64_t *)(ws + L.cand);
    uint32_t *prefix = (uint32_t *)(ws + L.prefix);
    const int n_items = scn.n_items;
    hipError_t e;
    if ((e = launch_fill_u64(M, 0ull, (size_t)sc.F * sc.W, s)) != hipSuccess) return e;
    if ((e = launch_fill_u64((uint64_t *)(ws + L.done), 0ull, (size_t)sc.F * sc.W, s)) != hipSuccess) return e;
    if ((e = launch_fill_u32((uint32_t *)(ws + L.queue), 0u, 64, s)) != hipSuccess) return e;
    const unsigned blocks = (unsigned)((n_items + 3) / 4);
    hipLaunchKernelGGL(k_cull, dim3(blocks > 65535u ? 65535u : (blocks ? blocks : 1u)), dim3(256), 0, s, sc, cand,
                       prefix, n_items);
    if ((e = exclusive_scan_u32(prefix, n_items + 1, (uint32_t *)(ws + L.scan_tmp), s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_pair_stats, dim3(1), dim3(64), 0, s, stats, (const uint32_t *)prefix, n_items, sc.F);
    return hipGetLastError();
}

// The candidates no probe has decided: und = cand & ~(M | done), word by word,
// and their counts (scanned into uprefix afterwards).
__global__ void k_undecided(int n_items, const uint64_t *cand, const uint64_t *M, const uint64_t *done, uint64_t *und,
                            uint32_t *counts) {
    const int w = blockIdx.x * blockDim.x + threadIdx.x;
    if (w < n_items) {
        const uint64_t u = cand[w] & ~(M[w] | done[w]);
        und[w] = u;
        counts[w] = (uint32_t)__popcll(u);
    }
    if (w == 0) counts[n_items] = 0;
}

hipError_t launch_undecided(Scene &scn, uint64_t *M, hipStream_t s) {
    char *ws = (char *)scn.ws;
    const Layout &L = scn.lay;
    const int n = scn.n_items;
    uint32_t *up = (uint32_t *)(ws + L.uprefix);
    hipLaunchKernelGGL(k_undecided, dim3((unsigned)((n + 256) / 256)), dim3(256), 0, s, n, (const uint64_t *)(ws + L.cand),
                       (const uint64_t *)M, (const uint64_t *)(ws + L.done), (uint64_t *)(ws + L.und), up);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return exclusive_scan_u32(up, n + 1, (uint32_t *)(ws + L.scan_tmp), s);
}

// base[0, n]: exclusive prefix of the scenes' candidate totals (all candidates, or
// the undecided ones); base[n + 1, 2n + 1]: the same with each total rounded up to
// a multiple of 64 (the probe queue).
__global__ void k_job_base(const PairJob *jobs, int n, uint32_t *base, int undecided) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    uint32_t run = 0, prun = 0;
    for (int k = 0; k < n; ++k) {
        base[k] = run;
        base[n + 1 + k] = prun;
        const uint32_t cnt =
            jobs[k].sc.F >= 2 ? (undecided ? jobs[k].uprefix : jobs[k].prefix)[jobs[k].n_items] : 0u;
        run += cnt;
        prun += (cnt + kWave - 1) / kWave * kWave;
    }
    base[n] = run;
    base[2 * n + 1] = prun;
}

hipError_t launch_job_base(const PairJob *d_jobs, int n_jobs, uint32_t *d_base, bool undecided, hipStream_t s) {
    hipLaunchKernelGGL(k_job_base, dim3(1), dim3(64), 0, s, d_jobs, n_jobs, d_base, undecided ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_probe_jobs(const PairJob *d_jobs, const uint32_t *d_base, int n_jobs, uint32_t *d_queue, int round,
                             const TraverseOpts &o, ivm_stats *stats, hipStream_t s) {
    PairJob none{};
    hipLaunchKernelGGL(k_probe_pairs<true>, dim3(o.grid_blocks), dim3(kBlock), 0, s, none, d_jobs, d_base + n_jobs + 1,
                       n_jobs, d_queue + kQueueProbe + kXcdParts * round, round, o, stats);
    return hipGetLastError();
}

hipError_t launch_pair_jobs(const PairJob *d_jobs, const uint32_t *d_base, int n_jobs, uint32_t *d_queue,
                            const TraverseOpts &o, ivm_stats *stats, hipStream_t s) {
    PairJob none{};
    hipLaunchKernelGGL(k_pairs<true>, dim3(o.grid_blocks), dim3(kBlock), 0, s, none, d_jobs, d_base, n_jobs,
                       d_queue + kQueuePairs, o, stats);
    return hipGetLastError();
}

hipError_t launch_matrix(Scene &scn, const TraverseOpts &o, uint64_t *M, ivm_stats *stats,
                         const uint8_t * /*unused*/, hipStream_t s) {
    const SceneDev &sc = scn.dev;
    char *ws = (char *)scn.ws;
    const Layout &L = scn.lay;
    hipError_t e;
    if (sc.F < 2) return launch_fill_u64(M, 0ull, (size_t)sc.F * sc.W, s);
    if ((e = launch_cull_scan(scn, M, stats, s)) != hipSuccess) return e;
    const bool learned = o.order_mode == IVM_ORDER_LEARNED && L.learned_bytes && scn.model;
    const PairJob job = make_pair_job(scn, M, learned);
    if (o.events && (e = hipEventRecord(o.events[0], s)) != hipSuccess) return e;
    // probe rounds, each followed by the compaction of the still-undecided pairs
    // (the exhaustive baseline runs no probe and takes every candidate)
    for (int round = 0; round < kProbeRounds && !o.exhaustive; ++round) {
        hipLaunchKernelGGL(k_probe_pairs<false>, dim3(o.grid_blocks), dim3(kBlock), 0, s, job,
                           (const PairJob *)nullptr, (const uint32_t *)nullptr, 1,
                           (uint32_t *)(ws + L.queue) + kQueueProbe + kXcdParts * round, round, o, stats);
        if ((e = launch_undecided(scn, M, s)) != hipSuccess) return e;
    }
    if (o.exhaustive && (e = launch_undecided(scn, M, s)) != hipSuccess) return e;
    // the learned treelet order of the undecided pairs (network inference)
    if (learned && (e = launch_learned_order(scn, *scn.model, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_pairs<false>, dim3(o.grid_blocks), dim3(kBlock), 0, s, job, (const PairJob *)nullptr,
                       (const uint32_t *)nullptr, 1, (uint32_t *)(ws + L.queue) + kQueuePairs, o, stats);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (o.events && (e = hipEventRecord(o.events[1], s)) != hipSuccess) return e;
    return hipSuccess;
}

// ---------------------------------------------------------------------------
// Tx/Rx points and line of sight
// ---------------------------------------------------------------------------


// Work units are (job, side, chunk of 64 consecutive samples, block of U
// consecutive snapshots); a wave takes the next unit from a counter
// until none is left (units differ in cost by orders of magnitude: chunks of
// facets seen from the trajectory need traversals).  Within a unit the wave follows its chunk of samples along the
// trajectory from one point to the next.  A lane keeps a hint for its sample:
// what decided it at an earlier point of the unit (a verified solid or a
// triangle that blocked it, or clear), and a blocker hint is tested first; the
// next point is a few centimetres away and the same blocker nearly always
// blocks again.  A hint only orders the exact tests: every bit of every point
// is decided by tests at that point.  The samples left then go through the
// wave's recent blockers and solids and the point certificates, and the rest
// into the probe and miss queues, which are traversed in full 64-lane batches
// that mix points of the unit (an entry carries its snapshot) and are drained
// at the unit's end.  Swept certificates cover kSweptBlock points at a time.  Samples of facets already known visible from the point
// are skipped (a set bit is never cleared, so a stale read only costs work).
__device__ inline void remember_blockers(int *cache, int &ncache, int &cpos, unsigned long long fm, int hit) {
    for (int added = 0; fm && added < kCache; ++added) {
        const int src = __ffsll((long long)fm) - 1;
        fm &= fm - 1;
        const int r = __shfl(hit, src);
        bool dup = false;
        for (int m = 0; m < ncache; ++m) dup |= cache[m] == r;
        if (dup) continue;
        if (ncache < kCache) cache[ncache++] = r;
        else { cache[cpos] = r; cpos = (cpos + 1) % kCache; }
    }
}

// Solids that blocked recent segments from the current point X, staged in LDS
// and tested segment by segment (X strictly outside one face plane, so a
// segment from X that passes through the prism enters it at 0 < t < 1, see the
// solid certificate).  A sample's own facet never blocks it: if it is a face of
// the solid the sample lies on that face plane while X is strictly in front,
// and the segment stays outside the prism.
constexpr int kSolidCache = 2;

// A lane's hint: a verified solid (>= 0), none, clear (its sample was seen
// from an earlier point), or triangle h (-(h + 3)).
constexpr int kHintNone = -1, kHintClear = -2;
constexpr int kSweptMinLeft = 8;  // points a unit must still hold for a swept certificate to be tried
static_assert(kSweptBlock <= kWave, "a swept box's points are reduced one per lane");
constexpr int kNoUpdate = (int)0x80000000;  // (a slot of the hint-update buffer with nothing new)

// The hint left by a traversal that found triangle `hit`: its facet's verified
// solid if there is one (a solid also blocks segments that pass beside this
// particular triangle), else the triangle.
__device__ inline int hint_of_hit(const SceneDev &sc, int hit) {
    const int K = sc.fsolid[__float_as_int(sc.tri[3 * hit].w)];
    return K >= 0 ? K : -(hit + 3);
}

// Swept solid test: the segments from every point X of the box [bl, bh] to
// sample Q pass through verified solid sid.  The box lies strictly outside one
// face plane of the prism (tested at the corner where that plane's value is
// least, the value being linear), so every X does; the segment from each box
// corner to Q passes through the prism, both ends at or above the base.  For
// fixed Q the points X whose open segment to Q meets the open prism form a
// convex set (for X a combination of two such points, the same combination of
// their segments' points in the prism lies on the open segment from X), so the
// whole box is covered, and from each X the segment enters the prism at
// 0 < t < 1, above the base, through a covered face.  The corners' coordinates
// are those of on-grid points, so every plane value stays exact.
__device__ bool swept_solid(const SceneDev &sc, int sid, float4 bl, float4 bh, float4 Q, Cnt &c) {
    const double u = ldexp(1.0, sc.gs);
    const int4 R = sc.solid[sid];
    if (R.x <= 0) return false;
    bool sep = false;
    for (int k = 0; k <= R.x && !sep; ++k) {
        ++c.solid_planes;
        if (k < R.x) {
            const int4 pl = sc.splane[sid * kSolidMaxPlanes + k];
            const double x = (double)(pl.w > 0 ? bl.x : bh.x) * u, y = (double)(pl.z < 0 ? bl.y : bh.y) * u;
            sep = (double)pl.w * (x - (double)pl.x) - (double)pl.z * (y - (double)pl.y) > 0.0;
        } else {
            sep = (double)bl.z * u - (double)R.y > 0.0;
        }
    }
    if (!sep) return false;
    const int nx = bl.x == bh.x ? 1 : 2, ny = bl.y == bh.y ? 1 : 2, nz = bl.z == bh.z ? 1 : 2;
    for (int k = 0; k < nx * ny * nz; ++k) {
        const float4 X = make_float4((k % nx) ? bh.x : bl.x, ((k / nx) % ny) ? bh.y : bl.y, (k / (nx * ny)) ? bh.z : bl.z,
                                     0.f);
        if (!solid_segment_global(sc, sid, X, Q, c)) return false;
    }
    return true;
}

// Set the visible bit of facet f in row n of the table at `base` for the lanes
// with `clear`.  Entries of one point and facet are usually adjacent, so only a
// lane whose nearest clear lane below holds another point or facet issues the
// atomic (repeats would only cost memory traffic).
__device__ inline void mark_visible(uint64_t *base, int W, bool clear, int n, int f) {
    const int lane = lane_id();
    const unsigned long long below = __ballot(clear) & ((1ull << lane) - 1ull);
    const int prev = below ? 63 - __clzll((long long)below) : lane;
    const int fprev = __shfl(f, prev), nprev = __shfl(n, prev);
    if (clear && (prev == lane || fprev != f || nprev != n))
        atomicOr((unsigned long long *)&base[(size_t)n * W + (f >> 6)], 1ull << (f & 63));
}

// Point certificate: every segment from X to the sample hull of facet f passes
// through solid K (X strictly outside one face plane, X and the hull corners at
// or above the base; for fixed X the q whose segment meets K form a convex set),
// so no sample of f is visible from X.  The candidates come from a scan of the
// scene's solid boxes met by the segment from X to f's box centre, nearest to
// either end first; they are staged in the wave's solid cache slots.  One lane
// per hull corner.
__device__ bool certify_point_facet(const SceneDev &sc, int f, float4 X, SolidLds *lds, int *scache, int &nsc,
                                    int &spos, int &sid_out, Cnt &c) {
    const int lane = lane_id();
    const int nh = sc.fhull_n[f];
    if (nh == 0) return false;
    const double gu = ldexp(1.0, sc.gs);
    const float4 corner = sc.smp[sc.fhull[kHullMax * f + (lane < nh ? lane : 0)]];
    const float4 corner0 = sc.smp[sc.fhull[kHullMax * f]];
    const float *fb = sc.fbox + 6 * f;
    const float cx = 0.5f * (fb[0] + fb[3]), cy = 0.5f * (fb[1] + fb[4]);
    const float bx0 = fminf(X.x, fb[0]), bx1 = fmaxf(X.x, fb[3]), by0 = fminf(X.y, fb[1]), by1 = fmaxf(X.y, fb[4]);
    const float bz0 = fminf(X.z, fb[2]);
    const int own = sc.fsolid[f];
    const Ray2 ray = make_ray2(X.x, X.y, cx, cy);
    float bkey;
    int bsol;
    scan_solids(
        sc, X.x, X.y, cx, cy, lane, kWave,
        [&](int sid, float4 L, float4 H) -> float {
            if (!(bx1 > L.x && bx0 < H.x && by1 > L.y && by0 < H.y && bz0 < H.z && bz0 >= L.z)) return INFINITY;
            if (sid == own) return INFINITY;
            for (int m = 0; m < nsc; ++m)
                if (scache[m] == sid) return INFINITY;
            return segment_box_key(ray, L, H);
        },
        // a certifying solid blocks the segment to the first hull corner in particular
        [](int) -> bool { return true; },
        bkey, bsol);
    if (bsol >= 0 && !solid_segment_global(sc, bsol, X, corner0, c)) bkey = INFINITY;
    for (int tr = 0; tr < kScanTries; ++tr) {
        const float kmin = wave_min(bkey);
        if (!(kmin < INFINITY)) break;
        const int src = __ffsll((long long)__ballot(bkey == kmin)) - 1;
        const int sid = __shfl(bsol, src);
        if (bsol == sid) bkey = INFINITY;  // every lane holding it drops it
        int slot;
        if (nsc < kSolidCache) slot = nsc++;
        else { slot = spos; spos = (spos + 1) % kSolidCache; }
        scache[slot] = sid;
        stage_solid(sc, sid, lds[slot]);
        Cnt tmp;
        const bool good = lane < nh && solid_segment(lds[slot], X, corner, gu, tmp);
        c.solid_planes += tmp.solid_planes;
        if (__ballot(lane < nh && !good) == 0ull) {
            sid_out = sid;
            return true;
        }
    }
    return false;
}

// The same certificate for nf = 2..4 facets at once: lane group g (64 / 4 or
// 64 / 2 lanes, aligned) scans and tests for facet f_g, the hull corners read
// from global memory.  Returns bit g set when f_g is proven blocked from X;
// sid_out holds, on the lanes of a certified group, the certifying solid.
__device__ unsigned certify_point_facets(const SceneDev &sc, int nf, int f0, int f1, int f2, int f3, float4 X,
                                         const int *scache, int nsc, int &sid_out, Cnt &c) {
    const int lane = lane_id();
    const int gs = nf <= 2 ? 32 : 16;               // lanes per group
    const int g = lane / gs, r = lane - g * gs;
    const unsigned long long gm = (gs == 32 ? 0xffffffffull : 0xffffull) << (g * gs);
    const bool live = g < nf;
    const int f = g == 0 ? f0 : (g == 1 ? f1 : (g == 2 ? f2 : f3));
    const int fs = live ? f : f0;                    // (idle groups read facet f0's data)
    const int nh = live ? sc.fhull_n[fs] : 0;
    // (hull entries exist only for nh > 0: no index is read otherwise)
    const float4 none = make_float4(0.f, 0.f, 0.f, 0.f);
    const float4 corner = nh > 0 ? sc.smp[sc.fhull[kHullMax * fs + (r < nh ? r : 0)]] : none;
    const float4 corner0 = nh > 0 ? sc.smp[sc.fhull[kHullMax * fs]] : none;
    const float *fb = sc.fbox + 6 * fs;
    const float cx = 0.5f * (fb[0] + fb[3]), cy = 0.5f * (fb[1] + fb[4]);
    const float bx0 = fminf(X.x, fb[0]), bx1 = fmaxf(X.x, fb[3]), by0 = fminf(X.y, fb[1]), by1 = fmaxf(X.y, fb[4]);
    const float bz0 = fminf(X.z, fb[2]);
    const int own = sc.fsolid[fs];
    const Ray2 ray = make_ray2(X.x, X.y, cx, cy);
    float bkey = INFINITY;
    int bsol = -1;
    if (nh > 0)
        scan_solids(
            sc, X.x, X.y, cx, cy, r, gs,
            [&](int sid, float4 L, float4 H) -> float {
                if (!(bx1 > L.x && bx0 < H.x && by1 > L.y && by0 < H.y && bz0 < H.z && bz0 >= L.z)) return INFINITY;
                if (sid == own) return INFINITY;
                for (int m = 0; m < nsc; ++m)
                    if (scache[m] == sid) return INFINITY;
                return segment_box_key(ray, L, H);
            },
            [](int) -> bool { return true; }, bkey, bsol);
    // a certifying solid blocks the segment to the first hull corner in particular
    if (bsol >= 0 && !solid_segment_global(sc, bsol, X, corner0, c)) bkey = INFINITY;
    bool done = false;  // this lane's group is certified
    sid_out = -1;
    unsigned res = 0u;
    for (int tr = 0; tr < kScanTries; ++tr) {
        float kmin = bkey;
        for (int o = gs >> 1; o > 0; o >>= 1) kmin = fminf(kmin, __shfl_xor(kmin, o));
        const bool has = nh > 0 && !done && kmin < INFINITY;
        if (!__ballot(has)) break;
        const unsigned long long eq = __ballot(has && bkey == kmin) & gm;
        const int src = eq ? __ffsll((long long)eq) - 1 : lane;
        const int sid = __shfl(bsol, src);
        if (has && bsol == sid) bkey = INFINITY;  // every lane of the group holding it drops it
        const bool act = has && r < nh;
        const bool good = act && solid_segment_global(sc, sid, X, corner, c);
        const unsigned long long bad = __ballot(act && !good) & gm;
        if (has && bad == 0ull) {
            done = true;
            sid_out = sid;
        }
        const unsigned long long dm = __ballot(done && r == 0);
        for (int q = 0; q < nf; ++q)
            if ((dm >> (q * gs)) & 1ull) res |= 1u << q;
    }
    return res;
}

template <bool MULTI>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(3))) void k_points(PointJob one, const PointJob *many, int n_jobs,
                                                   long long n_units, unsigned long long *counter, TraverseOpts o,
                                                   ivm_stats *st) {
    __shared__ int sStack[kWavesPerBlock][kWave * IVM_MAX_STACK];
    __shared__ unsigned long long sKey[kWavesPerBlock][kTreelets];
    __shared__ uint8_t sOrder[kWavesPerBlock][kTreelets];
    __shared__ int sMiss[kWavesPerBlock][2 * kWave];
    __shared__ SolidLds sSL[kWavesPerBlock][kSolidCache];
    __shared__ int sList[kWavesPerBlock][kCache + kSolidCache];
    // probe queue [0, np): the probe sample (snapshot * 64 + lane) and the facet's
    // other missing samples at that snapshot (lane bits); then [np, np + nexp):
    // facets whose probe was blocked, with the blocking triangle in place of the
    // sample.  Miss queue entries are snapshot * 64 + lane.
    __shared__ int sProbe[kWavesPerBlock][2 * kWave];
    __shared__ unsigned long long sPMask[kWavesPerBlock][2 * kWave];
    __shared__ int sPSnap[kWavesPerBlock][2 * kWave];
    __shared__ int sUpd[kWavesPerBlock][kWave];  // hints found by a traversal batch, by sample lane
    // (the wave index made explicitly wave-uniform: everything derived from it
    // then lives in scalar registers)
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)), lane = lane_id();
    int *stk = &sStack[wv][lane];
    int *miss = sMiss[wv];
    const bool f64 = o.fp64_only != 0;
    const unsigned long long lt = (1ull << lane) - 1ull;
    Cnt c;
    unsigned long long segs = 0, items = 0;
    int *cache = sList[wv], *scache = cache + kCache;  // wave-uniform lists in LDS
    int ncache = 0, cpos = 0, nmiss = 0, n_order = 0;
    unsigned long long nsolidf = 0;  // (point, facet) pairs certified by a solid
    int nsc = 0, spos = 0;
    int np = 0, nexp = 0;
    const bool probing = !o.exhaustive;
    sUpd[wv][lane] = kNoUpdate;
    // the current unit's chunk and side, and its job's points and table (row 0)
    int cur_chunk = 0, cur_side = 0;
    const float *pts = nullptr;
    uint64_t *out = nullptr;
    int hint = kHintNone;
    float xx = 0.f, xy = 0.f, xz = 0.f;  // the current point
    long long pt = 0, ord_pt = -1;       // the current point (a wave-local count), the point sOrder was ranked for
    // Runs the traversals the queues call for: full batches of misses; the other
    // missing samples of a facet whose probe was blocked (less those the probe's
    // blocking triangle also blocks) into the miss queue; batches of up to 64
    // probes, one sample per (point, facet), where a clear probe shows its facet
    // visible from its point at once.  `fin` empties the queues.
    auto pump = [&](const PointJob &JK, bool fin) __attribute__((always_inline)) {
        const SceneDev &S = JK.sc;
        const int base = cur_chunk * kWave;
        while (true) {
            const bool do_miss = nmiss >= kWave || (fin && nmiss > 0 && nexp == 0);
            if (!do_miss && nexp > 0) {
                const int e = np + nexp - 1;
                const unsigned long long m = sPMask[wv][e];
                const int h = sProbe[wv][e], ne = sPSnap[wv][e];
                --nexp;
                bool keep = (m >> lane) & 1ull;
                if (keep) {
                    const float *X = pts + 3 * ne;
                    const float4 P = S.smp[base + lane];
                    const Seg sg3 = make_seg(X[0], X[1], X[2], P.x, P.y, P.z);
                    ++c.tests;
                    keep = !tri_hit(sg3, S.tri[3 * h], S.tri[3 * h + 1], S.tri[3 * h + 2], o.eps6, f64, c.rechecks);
                    if (!keep) hint = hint_of_hit(S, h);
                }
                const unsigned long long km = __ballot(keep);
                if (keep) miss[nmiss + __popcll(km & lt)] = ne * kWave + lane;
                nmiss += __popcll(km);
                wave_sync();
                continue;
            }
            if (!do_miss && !(np >= kWave || (fin && np > 0))) break;
            if (ord_pt != pt) {
                // treelet order for the current point, nearest treelet box first (a
                // heuristic only; the batch's other points are close by)
                ord_pt = pt;
                const float xq[3] = {xx, xy, xz};
                const int mode = o.order_mode == IVM_ORDER_LEARNED ? IVM_ORDER_PLAIN : o.order_mode;
                unsigned long long tk = ~0ull;
                if (lane < kTreelets && S.tl_root[lane] != kNone) {
                    const float *b = S.tl_box + 6 * lane;
                    float d2 = 0.f;
                    for (int q = 0; q < 3; ++q) {
                        const float cq = fmaxf(fmaxf(b[q] - xq[q], xq[q] - b[3 + q]), 0.f);
                        d2 += cq * cq;
                    }
                    const unsigned dk = __float_as_uint(d2);
                    tk = mode == IVM_ORDER_INDEX ? (unsigned long long)lane
                         : (mode == IVM_ORDER_REVERSED ? (unsigned long long)(0xffffffffu - dk) : dk);
                }
                n_order = wave_rank_order(tk, sKey[wv], sOrder[wv]);
            }
            const int k = min(kWave, do_miss ? nmiss : np);
            const bool act = lane < k;
            const int q = (do_miss ? nmiss : np) - (act ? k - lane : 1);
            const int code = do_miss ? miss[q] : sProbe[wv][q];
            const unsigned long long pm = do_miss || !act ? 0ull : sPMask[wv][q];
            const int ne = code >> 6, sl = code & (kWave - 1);
            const int f = S.sfacet[base + sl];
            const float4 Pq = S.smp[base + sl];
            const float *X = pts + 3 * ne;
            const Seg sg = make_seg(X[0], X[1], X[2], Pq.x, Pq.y, Pq.z);
            if (act) ++c.traversed;
            // (the key names the point and the facet: the facet by its first sample's lane in the chunk)
            const int key_pf = (ne << 6) | max(S.soff[f] - base, 0);
            const int hit = any_hit_wave(S, sg, act, f, f, sOrder[wv], n_order, stk, o.stack_depth, o.eps6, f64, c,
                                         kAbortSameKey, key_pf);
            const bool clear = hit == -1;
            if (do_miss) nmiss -= k;
            else np -= k;
            wave_sync();
            mark_visible(out, S.W, clear, ne, f);
            if (act && (clear || hit >= 0)) sUpd[wv][sl] = clear ? kHintClear : hint_of_hit(S, hit);
            remember_blockers(cache, ncache, cpos, __ballot(hit >= 0), hit);
            if (S.n_solids > 0) remember_solid_ids(S, scache, nsc, spos, sSL[wv], kSolidCache, hit >= 0, hit);
            if (!do_miss) {
                // (another probe of the same point and facet that is clear settles it)
                bool vis = clear;
                for (unsigned long long cm = __ballot(clear); cm; cm &= cm - 1) {
                    const int src = __ffsll((long long)cm) - 1;
                    vis |= __shfl(f, src) == f && __shfl(ne, src) == ne;
                }
                const bool blk = act && hit >= 0 && !vis && pm != 0ull;
                const unsigned long long bm = __ballot(blk);
                if (blk) {
                    const int pos = np + __popcll(bm & lt);
                    sProbe[wv][pos] = hit;
                    sPMask[wv][pos] = pm;
                    sPSnap[wv][pos] = ne;
                }
                nexp = __popcll(bm);
            }
            wave_sync();
            // the batch's hints go to the lanes that own the samples
            const int u = sUpd[wv][lane];
            if (u != kNoUpdate) {
                hint = u;
                sUpd[wv][lane] = kNoUpdate;
            }
            wave_sync();
        }
    };
    while (true) {
        unsigned long long ut = 0ull;
        if (lane == 0) ut = atomicAdd(counter, 1ull);
        const long long u = (long long)__shfl(ut, 0);
        if (u >= n_units) break;
        int js = 0;
        if (MULTI) {
            int lo = 0, hi = n_jobs - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (many[mid].unit_base <= u) lo = mid;
                else hi = mid - 1;
            }
            js = lo;
        }
        const PointJob &J = MULTI ? many[js] : one;
        const SceneDev &sc = J.sc;
        const int N = J.N, U = J.U, nb = (N + U - 1) / U, nch = (sc.S + kWave - 1) / kWave;
        const long long local = u - J.unit_base;
        const int kx = (int)(local / nb), blk = (int)(local - (long long)kx * nb);
        cur_side = kx / nch;
        cur_chunk = kx - cur_side * nch;
        pts = cur_side ? J.rx : J.tx;
        out = cur_side ? J.rxv : J.txv;
        ncache = cpos = nsc = spos = 0;
        hint = kHintNone;
        const int sidx = cur_chunk * kWave + lane;
        const int fl = sidx < sc.S ? sc.sfacet[sidx] : -1;  // the facet of this lane's sample (-1 = none)
        const int own = fl >= 0 ? sc.fsolid[fl] : -1;       // the solid the sample's facet belongs to
        const int n0 = blk * U, n1 = min(N, n0 + U);
        float4 bl = make_float4(0.f, 0.f, 0.f, 0.f), bh = bl;
        bool swept = false, tried = false;
        int nb1 = n0;  // end of the current swept box's points
        for (int n = n0; n < n1; ++n) {
            if (n == nb1) {
                // the box of the next kSweptBlock points, for swept certificates: a lane
                // whose hint solid blocks its sample from the whole box skips its other points
                nb1 = min(n1, n + kSweptBlock);
                const bool in = lane < nb1 - n;
                const float *Xb = pts + 3 * (in ? n + lane : n);
                // (wave-uniform: kept in scalar registers)
                auto uni = [](float v) { return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v))); };
                bl = make_float4(uni(wave_min(Xb[0])), uni(wave_min(Xb[1])), uni(wave_min(Xb[2])), 0.f);
                bh = make_float4(uni(wave_max(Xb[0])), uni(wave_max(Xb[1])), uni(wave_max(Xb[2])), 0.f);
                swept = tried = false;
            }
            xx = pts[3 * n];
            xy = pts[3 * n + 1];
            xz = pts[3 * n + 2];
            ++pt;
            const float4 X4 = make_float4(xx, xy, xz, 0.f);
            const uint64_t *row = out + (size_t)n * sc.W;
            bool need = false;
            const float4 P = fl >= 0 ? (float4)sc.smp[sidx] : make_float4(0.f, 0.f, 0.f, 0.f);
            bool by_solid = false;  // decided by a solid at this point
            if (fl >= 0 && !swept)
                need = orient(sc.fplane + 6 * fl, xx, xy, xz) > 0.0 && !((row[fl >> 6] >> (fl & 63)) & 1ull);
            segs += __popcll(__ballot(need));  // (a wave-uniform count)
            if (need) {
                if (!o.exhaustive) {
                    // the hint first
                    if (hint >= 0) {
                        if (solid_segment_global(sc, hint, X4, P, c)) {
                            need = false;
                            by_solid = true;
                            ++c.solid_segs;
                        } else {
                            hint = kHintNone;
                        }
                    } else if (hint <= -3) {
                        const int r = -(hint + 3);
                        const Seg sg = make_seg(xx, xy, xz, P.x, P.y, P.z);
                        ++c.tests;
                        if (tri_hit(sg, sc.tri[3 * r], sc.tri[3 * r + 1], sc.tri[3 * r + 2], o.eps6, f64, c.rechecks))
                            need = false;
                        else
                            hint = kHintNone;
                    }
                    // then the wave's recent solids and blockers
                    for (int m = 0; m < nsc && need; ++m) {
                        if (solid_segment(sSL[wv][m], X4, P, ldexp(1.0, sc.gs), c)) {
                            need = false;
                            by_solid = true;
                            hint = scache[m];
                            ++c.solid_segs;
                        }
                    }
                    if (need && ncache > 0) {
                        const Seg sg = make_seg(xx, xy, xz, P.x, P.y, P.z);
                        for (int k = 0; k < ncache && need; ++k) {
                            const int r = cache[k];
                            if (__float_as_int(sc.tri[3 * r].w) == fl) continue;
                            ++c.tests;
                            if (tri_hit(sg, sc.tri[3 * r], sc.tri[3 * r + 1], sc.tri[3 * r + 2], o.eps6, f64, c.rechecks)) {
                                need = false;
                                hint = -(r + 3);
                            }
                        }
                    }
                }
            }
            // one swept certificate per lane and unit, while enough points remain
            if (by_solid && !tried && hint != own && n + kSweptMinLeft < nb1) {
                tried = true;
                swept = swept_solid(sc, hint, bl, bh, P, c);
            }
            unsigned long long nm = __ballot(need);
            // a facet left with misses: try to prove it blocked from X by a solid of the
            // scene (not a facet seen from an earlier point: it goes to its probe)
            if (nm && !o.exhaustive && sc.n_solids > 0 && sc.n_solids <= kScanMaxSolidsPoint) {
                bool seen = false;
                for (unsigned long long hc = __ballot(need && hint == kHintClear); hc;) {
                    const int fc = __shfl(fl, __ffsll((long long)hc) - 1);
                    seen |= fl == fc;
                    hc &= ~__ballot(fl == fc);
                }
                unsigned long long left = nm & ~__ballot(seen);
                while (left) {
                    // up to four facets at once, one lane group each
                    int fq0 = -1, fq1 = -1, fq2 = -1, fq3 = -1;
                    int nf = 0;
                    for (; nf < 4 && left; ++nf) {
                        const int fc = __shfl(fl, __ffsll((long long)left) - 1);
                        left &= ~__ballot(need && fl == fc);
                        if (nf == 0) fq0 = fc;
                        else if (nf == 1) fq1 = fc;
                        else if (nf == 2) fq2 = fc;
                        else fq3 = fc;
                    }
                    if (nf == 1) {
                        int sid = -1;
                        if (certify_point_facet(sc, fq0, X4, sSL[wv], scache, nsc, spos, sid, c)) {
                            if (fl == fq0 && need) {
                                need = false;
                                hint = sid;
                            }
                            ++nsolidf;
                        }
                    } else {
                        int sid_g;
                        const unsigned ok = certify_point_facets(sc, nf, fq0, fq1, fq2, fq3, X4, scache, nsc, sid_g, c);
                        const int gs = nf <= 2 ? 32 : 16;
                        for (int q = 0; q < nf; ++q) {
                            if (!((ok >> q) & 1u)) continue;
                            const int fcq = q == 0 ? fq0 : (q == 1 ? fq1 : (q == 2 ? fq2 : fq3));
                            // the certifying solid joins the wave's solid cache
                            const int sid = __shfl(sid_g, q * gs);
                            if (fl == fcq && need) {
                                need = false;
                                hint = sid;
                            }
                            ++nsolidf;
                            bool cached = false;
                            for (int m = 0; m < nsc; ++m) cached |= scache[m] == sid;
                            if (!cached) {
                                int slot;
                                if (nsc < kSolidCache) slot = nsc++;
                                else { slot = spos; spos = (spos + 1) % kSolidCache; }
                                scache[slot] = sid;
                                stage_solid(sc, sid, sSL[wv][slot]);
                            }
                        }
                    }
                }
                nm = __ballot(need);
            }
            if (nm) ++items;
            if (probing) {
                // one probe per facet left with misses: the sample seen from an earlier
                // point if there is one, else the middle missing sample (np < 64 here,
                // and a chunk adds at most 64)
                for (unsigned long long left = nm; left;) {
                    const int fc = __shfl(fl, __ffsll((long long)left) - 1);
                    const bool mine = need && fl == fc;
                    const unsigned long long mf = __ballot(mine);
                    left &= ~mf;
                    const unsigned long long mc = __ballot(mine && hint == kHintClear);
                    const unsigned long long mm = __ballot(mine && __popcll(mf & lt) == (__popcll(mf) >> 1));
                    const int pick = __ffsll((long long)(mc ? mc : mm)) - 1;
                    if (lane == pick) {
                        sProbe[wv][np] = n * kWave + lane;
                        sPMask[wv][np] = mf & ~(1ull << lane);
                        sPSnap[wv][np] = n;
                    }
                    ++np;
                }
            } else {
                if (need) miss[nmiss + __popcll(nm & lt)] = n * kWave + lane;
                nmiss += __popcll(nm);
            }
            wave_sync();
            // (the unit's last point empties the queues)
            pump(J, n + 1 == n1);
        }
    }
    flush_counters(st, c, lane == 0 ? segs : 0ull, 0, items);
    if (st && lane == 0 && nsolidf) atomicAdd((unsigned long long *)&st->solid_certified, nsolidf);
}

__global__ __launch_bounds__(kBlock) void k_los(SceneDev sc, int N, const float *tx, const float *rx, uint8_t *los,
                                                TraverseOpts o) {
    __shared__ int sStack[kWavesPerBlock][kWave * IVM_MAX_STACK];
    const int wv = threadIdx.x >> 6, lane = lane_id();
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    Cnt c;
    if (n < N) {
        const Seg s = make_seg(tx[3 * n], tx[3 * n + 1], tx[3 * n + 2], rx[3 * n], rx[3 * n + 1], rx[3 * n + 2]);
        const bool hit = any_hit(sc, s, -1, -1, kIdentOrder, kTreelets, &sStack[wv][lane], o.stack_depth, o.eps6,
                                 o.fp64_only != 0, c) >= 0;
        los[n] = hit ? 0 : 1;
    }
}

// On-grid and exactness-budget check of Tx/Rx positions (see ivm.h).
__global__ void k_check_points(SceneDev sc, int N, const float *tx, const float *rx) {
    const int id = blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= 2 * N) return;
    const float *X = (id < N ? tx + 3 * id : rx + 3 * (id - N));
    const double sscale = ldexp(1.0, sc.gs);
    double D = 0.0;
    int bad = 0;
    for (int k = 0; k < 3; ++k) {
        const double y = (double)X[k] * sscale;
        if (!(fabs(y) < 16777216.0) || y != floor(y)) bad |= kStGrid;
        const double lo = fmin(sc.extent[k], y), hi = fmax(sc.extent[3 + k], y);
        D = fmax(D, (hi - lo) / sscale);
    }
    const double E = sc.extent[6];
    const int g = sc.g, kk = sc.gs - sc.g;
    const double bound = (6.0 * D * E * E + 12.0 * D * D * E) * ldexp(1.0, 3 * g + 2 * kk);
    if (!(bound < 9007199254740992.0) || !(D * sscale < 16777216.0)) bad |= kStGrid;
    if (bad) atomicOr(sc.status, bad);
}

// Work units of the Tx/Rx kernel: (side, chunk of 64 samples, block of U snapshots).
long long point_units(const Scene &scn, int N, int U) {
    const int nch = (scn.dev.S + kWave - 1) / kWave;
    return (scn.dev.S > 0 && scn.dev.F > 0 && N > 0) ? (long long)2 * nch * ((N + U - 1) / U) : 0;
}

// Snapshots per Tx/Rx work unit for jobs with S[k] samples and N[k] snapshots:
// the longest of kSweptBlock, 2 kSweptBlock, ..., kUnitMax that still leaves at
// least 16 units per wave (a wave's hints start afresh with each unit, and the
// last units taken set the tail of the launch).
int point_unit_len(const int *S, const int *N, int n_jobs, int grid_blocks) {
    const long long waves = (long long)grid_blocks * kWavesPerBlock;
    int best = kSweptBlock;
    for (int U = 2 * kSweptBlock; U <= kUnitMax; U *= 2) {
        long long units = 0;
        for (int k = 0; k < n_jobs; ++k)
            if (S[k] > 0 && N[k] > 0) units += 2ll * ((S[k] + kWave - 1) / kWave) * ((N[k] + U - 1) / U);
        if (units < 16 * waves) break;
        best = U;
    }
    return best;
}

PointJob make_point_job(Scene &scn, int N, const float *tx, const float *rx, uint64_t *txv, uint64_t *rxv,
                        long long unit_base, int U) {
    PointJob j;
    j.sc = scn.dev;
    j.N = N;
    j.tx = tx;
    j.rx = rx;
    j.txv = txv;
    j.rxv = rxv;
    j.unit_base = unit_base;
    j.U = U;
    return j;
}

// Zero the tables and check the positions (on grid, within the exactness budget).
hipError_t launch_points_prep(Scene &scn, int N, const float *tx, const float *rx, uint64_t *txv, uint64_t *rxv,
                              hipStream_t s) {
    const SceneDev &sc = scn.dev;
    hipError_t e;
    if ((e = launch_fill_u64(txv, 0ull, (size_t)N * sc.W, s)) != hipSuccess) return e;
    if ((e = launch_fill_u64(rxv, 0ull, (size_t)N * sc.W, s)) != hipSuccess) return e;
    if (N > 0) hipLaunchKernelGGL(k_check_points, dim3((2 * N + 255) / 256), dim3(256), 0, s, sc, N, tx, rx);
    return hipGetLastError();
}

hipError_t launch_los(Scene &scn, const TraverseOpts &o, int N, const float *tx, const float *rx, uint8_t *los,
                      hipStream_t s) {
    if (N <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_los, dim3((N + kBlock - 1) / kBlock), dim3(kBlock), 0, s, scn.dev, N, tx, rx, los, o);
    return hipGetLastError();
}

// Edge visibility for first-order diffraction (Section III-B: the receiver's
// diffracting edge is found the way a reflecting face is).  Edge e, where facets
// fa and fb meet, is seen from X when X lies strictly on the visible side of fa
// or of fb and the segment from X to one of the edge's s sample points meets no
// triangle outside fa and fb.  One wave per (side, 64 / G edges, block of
// kEdgeBlock consecutive snapshots): G consecutive lanes (G = s rounded up to a
// power of two) hold the samples of one edge, and the wave follows them along
// the trajectory with the table kernel's tools: each lane first tests the solid
// or triangle that blocked its sample at the previous point and tries one swept
// certificate for the box of the block's points.  The rest goes into two queues
// of (point, lane) entries traversed in full 64-lane batches that mix the block's
// points: one probe per (point, edge), the sample seen from an earlier point,
// whose edge's other samples follow only if it is blocked (less those its
// blocking triangle also blocks); and, for edges with no such sample, all their
// samples at once (a clear lane stops the others of its point and edge).  Hints
// only order exact tests.
constexpr int kEdgeBlock = kSweptBlock;

__global__ __launch_bounds__(kBlock) void k_edges(SceneDev sc, int N, int E, int s, int G, int We, const int *efac,
                                                  const float *esmp, const float *tx, const float *rx,
                                                  uint64_t *txe, uint64_t *rxe, TraverseOpts o) {
    __shared__ int sStack[kWavesPerBlock][kWave * IVM_MAX_STACK];
    __shared__ unsigned long long sKey[kWavesPerBlock][kTreelets];
    __shared__ uint8_t sOrder[kWavesPerBlock][kTreelets];
    __shared__ int sMiss[kWavesPerBlock][2 * kWave];
    __shared__ int sProbe[kWavesPerBlock][2 * kWave];
    __shared__ unsigned long long sPMask[kWavesPerBlock][2 * kWave];
    __shared__ int sPSnap[kWavesPerBlock][2 * kWave];
    __shared__ int sUpd[kWavesPerBlock][kWave];
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)), lane = lane_id();
    const int per_wave = kWave / G;
    const long long nch = (E + per_wave - 1) / per_wave;
    const int nb = (N + kEdgeBlock - 1) / kEdgeBlock;
    const long long q = (long long)blockIdx.x * kWavesPerBlock + wv;
    if (q >= 2LL * nch * nb) return;  // (wave-uniform)
    // consecutive waves take consecutive blocks of one chunk (the same scene data)
    const int blk = (int)(q % nb);
    const long long kx = q / nb;
    const int side = (int)(kx / nch);
    const int chunk = (int)(kx - (long long)side * nch);
    const int grp = lane / G, j = lane % G;
    const int e = chunk * per_wave + grp;
    const unsigned long long gm = (G == kWave ? ~0ull : ((1ull << G) - 1ull)) << (grp * G);
    const float *pts = side ? rx : tx;
    uint64_t *out = side ? rxe : txe;
    int fa = -1, fb = -1;
    bool valid = e < E && j < s;
    if (valid) {
        fa = efac[2 * e];
        fb = efac[2 * e + 1];
        valid = fa >= 0 && fa < sc.F && fb >= -1 && fb < sc.F && fb != fa;
    }
    const int exb = fb >= 0 ? fb : fa;
    const int own_a = valid ? sc.fsolid[fa] : -1, own_b = valid && fb >= 0 ? sc.fsolid[fb] : -1;
    float4 P = make_float4(0.f, 0.f, 0.f, 0.f);
    if (valid) {
        const float *pp = esmp + 3 * ((size_t)e * s + j);
        P = make_float4(pp[0], pp[1], pp[2], 0.f);
    }
    const int n0 = blk * kEdgeBlock, n1 = min(N, n0 + kEdgeBlock);
    // the box of the block's points (swept certificates) and a treelet order from
    // its first point (a heuristic only)
    float4 bl, bh;
    {
        const float *Xb = pts + 3 * (lane < n1 - n0 ? n0 + lane : n0);
        auto uni = [](float v) { return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v))); };
        bl = make_float4(uni(wave_min(Xb[0])), uni(wave_min(Xb[1])), uni(wave_min(Xb[2])), 0.f);
        bh = make_float4(uni(wave_max(Xb[0])), uni(wave_max(Xb[1])), uni(wave_max(Xb[2])), 0.f);
    }
    int n_order;
    {
        const float xq[3] = {pts[3 * n0], pts[3 * n0 + 1], pts[3 * n0 + 2]};
        unsigned long long tk = ~0ull;
        if (lane < kTreelets && sc.tl_root[lane] != kNone) {
            const float *b = sc.tl_box + 6 * lane;
            float d2 = 0.f;
            for (int k = 0; k < 3; ++k) {
                const float cq = fmaxf(fmaxf(b[k] - xq[k], xq[k] - b[3 + k]), 0.f);
                d2 += cq * cq;
            }
            tk = __float_as_uint(d2);
        }
        n_order = wave_rank_order(tk, sKey[wv], sOrder[wv]);
    }
    int *stk = &sStack[wv][lane];
    int *miss = sMiss[wv];
    const bool f64 = o.fp64_only != 0;
    const unsigned long long lt = (1ull << lane) - 1ull;
    Cnt c;
    int hint = kHintNone;
    bool swept = false, tried = false;
    int np = 0, nexp = 0, nmiss = 0;
    sUpd[wv][lane] = kNoUpdate;
    // Runs the traversals the queues call for (entries are point offset * 64 +
    // lane): full batches of misses; the other samples of an edge whose probe was
    // blocked (less those its blocking triangle also blocks) into the miss queue;
    // batches of up to 64 probes.  `fin` empties the queues.
    auto pump = [&](bool fin) __attribute__((always_inline)) {
        while (true) {
            const bool do_miss = nmiss >= kWave || (fin && nmiss > 0 && nexp == 0);
            if (!do_miss && nexp > 0) {
                const int ex = np + nexp - 1;
                const unsigned long long m = sPMask[wv][ex];
                const int h = sProbe[wv][ex], d = sPSnap[wv][ex];
                --nexp;
                bool keep = (m >> lane) & 1ull;
                if (keep) {
                    const float *X = pts + 3 * (n0 + d);
                    const Seg sg3 = make_seg(X[0], X[1], X[2], P.x, P.y, P.z);
                    ++c.tests;
                    keep = !tri_hit(sg3, sc.tri[3 * h], sc.tri[3 * h + 1], sc.tri[3 * h + 2], o.eps6, f64, c.rechecks);
                    if (!keep) hint = hint_of_hit(sc, h);
                }
                const unsigned long long km = __ballot(keep);
                if (keep) miss[nmiss + __popcll(km & lt)] = d * kWave + lane;
                nmiss += __popcll(km);
                wave_sync();
                continue;
            }
            if (!do_miss && !(np >= kWave || (fin && np > 0))) break;
            const int k = min(kWave, do_miss ? nmiss : np);
            const bool act = lane < k;
            const int q = (do_miss ? nmiss : np) - (act ? k - lane : 1);
            const int code = do_miss ? miss[q] : sProbe[wv][q];
            const unsigned long long pm = do_miss || !act ? 0ull : sPMask[wv][q];
            const int d = code >> 6, sl = code & (kWave - 1);
            // the entry's lane: its edge, sample and side facets
            const float Px = __shfl(P.x, sl), Py = __shfl(P.y, sl), Pz = __shfl(P.z, sl);
            const int ea = __shfl(fa, sl), eb = __shfl(exb, sl), eg = sl / G;
            const float *X = pts + 3 * (n0 + d);
            const Seg sg = make_seg(X[0], X[1], X[2], Px, Py, Pz);
            if (act) ++c.traversed;
            const int hit = any_hit_wave(sc, sg, act, ea, eb, sOrder[wv], n_order, stk, o.stack_depth, o.eps6, f64, c,
                                         kAbortSameKey, d * kWave + eg);
            const bool clear = act && hit == -1;
            if (do_miss) nmiss -= k;
            else np -= k;
            wave_sync();
            const int ee = chunk * per_wave + eg;
            if (clear) atomicOr((unsigned long long *)(out + (size_t)(n0 + d) * We + (ee >> 6)), 1ull << (ee & 63));
            if (act && (clear || hit >= 0)) sUpd[wv][sl] = clear ? kHintClear : hint_of_hit(sc, hit);
            if (!do_miss) {
                const bool blk = act && hit >= 0 && pm != 0ull;
                const unsigned long long bm = __ballot(blk);
                if (blk) {
                    const int pos = np + __popcll(bm & lt);
                    sProbe[wv][pos] = hit;
                    sPMask[wv][pos] = pm;
                    sPSnap[wv][pos] = d;
                }
                nexp = __popcll(bm);
            }
            wave_sync();
            const int u = sUpd[wv][lane];
            if (u != kNoUpdate) {
                hint = u;
                sUpd[wv][lane] = kNoUpdate;
            }
            wave_sync();
        }
    };
    for (int n = n0; n < n1; ++n) {
        const float xx = pts[3 * n], xy = pts[3 * n + 1], xz = pts[3 * n + 2];
        const float4 X4 = make_float4(xx, xy, xz, 0.f);
        bool need = valid && !swept &&
                    (orient(sc.fplane + 6 * (size_t)fa, xx, xy, xz) > 0.0 ||
                     (fb >= 0 && orient(sc.fplane + 6 * (size_t)fb, xx, xy, xz) > 0.0));
        bool by_solid = false;
        if (need && !o.exhaustive) {
            if (hint >= 0) {
                if (solid_segment_global(sc, hint, X4, P, c)) {
                    need = false;
                    by_solid = true;
                } else {
                    hint = kHintNone;
                }
            } else if (hint <= -3) {
                const int r = -(hint + 3);
                const Seg sg = make_seg(xx, xy, xz, P.x, P.y, P.z);
                ++c.tests;
                if (tri_hit(sg, sc.tri[3 * r], sc.tri[3 * r + 1], sc.tri[3 * r + 2], o.eps6, f64, c.rechecks))
                    need = false;
                else
                    hint = kHintNone;
            }
        }
        if (by_solid && !tried && hint != own_a && hint != own_b && n + kSweptMinLeft < n1) {
            tried = true;
            swept = swept_solid(sc, hint, bl, bh, P, c);
        }
        // one probe per edge with a sample seen before; the other edges' samples all
        const unsigned long long clm = __ballot(need && hint == kHintClear);
        const unsigned long long nmm = __ballot(need);
        const unsigned long long mine = clm & gm;
        const bool probe = mine != 0ull && lane == __ffsll((long long)mine) - 1;
        const bool direct = need && (clm & gm) == 0ull;
        const unsigned long long pb = __ballot(probe), db = __ballot(direct);
        if (probe) {
            const int pos = np + __popcll(pb & lt);
            sProbe[wv][pos] = (n - n0) * kWave + lane;
            sPMask[wv][pos] = nmm & gm & ~(1ull << lane);
        }
        if (direct) miss[nmiss + __popcll(db & lt)] = (n - n0) * kWave + lane;
        np += __popcll(pb);
        nmiss += __popcll(db);
        wave_sync();
        pump(n + 1 == n1);
    }
}

// Edge rows of the matrix: edges are visibility nodes beside faces (Sections I
// and II-A), and the face seen for diffraction is the face seen for reflection
// (Section III-B).  A node is a facet (its samples; side facets {f}) or an edge
// (its samples; side facets {fa, fb}, fb = -1 for an edge of one facet).  Edge e
// and node v see each other when some sample p of e and q of v have q strictly
// in front of fa or fb, p strictly in front of one of v's side facets, and the
// open segment (p, q) meets no triangle outside the side facets of both.
//
// One lane per (row edge, target node, edge sample): G consecutive lanes (G = s
// rounded up to a power of two) hold one edge-target pair, so a wave covers
// 64 / G targets of one row.  A lane walks the target's samples in order,
// tests the verified solid and the triangle that blocked its previous segment
// before a traversal (a solid that holds one of the four side facets is never
// tested: its faces would include excluded triangles), and
// stops at the first clear segment or when another lane of its group has found
// one (a flag in LDS); a ballot over the group sets the target's bit.
__global__ __launch_bounds__(kBlock) void k_edge_rows(SceneDev sc, int E, int s, int G, const int *efac,
                                                      const float *esmp, int n_rows, const int *rows, uint64_t *ef,
                                                      uint64_t *ee, TraverseOpts o) {
    __shared__ int sStack[kWavesPerBlock][kWave * IVM_MAX_STACK];
    __shared__ volatile int sDone[kWavesPerBlock][kWave];
    const int wv = threadIdx.x >> 6, lane = lane_id();
    const int per_wave = kWave / G, n_targets = sc.F + E;
    const long long nb = (n_targets + per_wave - 1) / per_wave;
    const long long qw = (long long)blockIdx.x * kWavesPerBlock + wv;
    if (qw >= (long long)n_rows * nb) return;  // (wave-uniform)
    const int k = (int)(qw / nb), grp = lane / G, a = lane % G;
    const int target = (int)(qw % nb) * per_wave + grp;
    const int e = rows[k];
    volatile int *done = sDone[wv];
    done[lane] = 0;
    bool clear = false;
    const bool row_ok = e >= 0 && e < E;
    if (row_ok && target < n_targets && a < s && target != sc.F + e) {
        const int fa = efac[2 * e], fb = efac[2 * e + 1];
        const float *p = esmp + 3 * ((size_t)e * s + a);
        int ta, tb;  // the target's side facets
        int q0, nq;  // its samples: facet samples [q0, q0 + nq) or edge samples of edge q0
        const bool is_edge = target >= sc.F;
        if (is_edge) {
            ta = efac[2 * (target - sc.F)];
            tb = efac[2 * (target - sc.F) + 1];
            q0 = target - sc.F;
            nq = s;
        } else {
            ta = target;
            tb = -1;
            q0 = sc.soff[target];
            nq = sc.soff[target + 1] - q0;
        }
        const bool sides_ok = fa >= 0 && fa < sc.F && fb >= -1 && fb < sc.F && ta >= 0 && ta < sc.F && tb >= -1 &&
                              tb < sc.F;
        const bool p_front = sides_ok && (orient(sc.fplane + 6 * (size_t)ta, p[0], p[1], p[2]) > 0.0 ||
                                          (tb >= 0 && orient(sc.fplane + 6 * (size_t)tb, p[0], p[1], p[2]) > 0.0));
        if (p_front) {
            const Ex4 ex{fa, fb, ta, tb};
            int last = -1, lsol = -1;  // the triangle that blocked the previous segment, and its verified solid
            // (a solid that holds one of the four side facets is never used: its faces
            // would include excluded triangles)
            const int sa = sc.fsolid[fa], sb = fb >= 0 ? sc.fsolid[fb] : -1;
            const int sta = sc.fsolid[ta], stb = tb >= 0 ? sc.fsolid[tb] : -1;
            const float4 P4 = make_float4(p[0], p[1], p[2], 0.f);
            Cnt c;
            for (int b = 0; b < nq && !done[grp]; ++b) {
                float qx, qy, qz;
                if (is_edge) {
                    const float *q = esmp + 3 * ((size_t)q0 * s + b);
                    qx = q[0];
                    qy = q[1];
                    qz = q[2];
                } else {
                    const float4 q = sc.smp[q0 + b];
                    qx = q.x;
                    qy = q.y;
                    qz = q.z;
                }
                if (!(orient(sc.fplane + 6 * (size_t)fa, qx, qy, qz) > 0.0 ||
                      (fb >= 0 && orient(sc.fplane + 6 * (size_t)fb, qx, qy, qz) > 0.0)))
                    continue;
                if (lsol >= 0 && solid_segment_global(sc, lsol, P4, make_float4(qx, qy, qz, 0.f), c)) continue;
                const Seg sg = make_seg(p[0], p[1], p[2], qx, qy, qz);
                if (last >= 0 && tri_hit(sg, sc.tri[3 * last], sc.tri[3 * last + 1], sc.tri[3 * last + 2], o.eps6,
                                         o.fp64_only != 0, c.rechecks))
                    continue;
                const int h = any_hit_ex(sc, sg, ex, kIdentOrder, kTreelets, &sStack[wv][lane], o.stack_depth, o.eps6,
                                         o.fp64_only != 0, c);
                if (h < 0) {
                    clear = true;
                    done[grp] = 1;
                    break;
                }
                last = h;
                const int K = sc.fsolid[__float_as_int(sc.tri[3 * h].w)];
                if (K >= 0 && K != sa && K != sb && K != sta && K != stb) lsol = K;
            }
        }
    }
    const unsigned long long bal = __ballot(clear);
    if (a == 0 && row_ok && target < n_targets) {
        const unsigned long long gm = (G == kWave ? ~0ull : ((1ull << G) - 1ull)) << lane;
        if (bal & gm) {
            if (target < sc.F)
                atomicOr((unsigned long long *)(ef + (size_t)k * sc.W + (target >> 6)), 1ull << (target & 63));
            else
                atomicOr((unsigned long long *)(ee + (size_t)k * ((E + 63) / 64) + ((target - sc.F) >> 6)),
                         1ull << ((target - sc.F) & 63));
        }
    }
}

__global__ void k_check_rows(int E, int n_rows, const int *rows, int *status) {
    const int id = blockIdx.x * blockDim.x + threadIdx.x;
    if (id < n_rows && !(rows[id] >= 0 && rows[id] < E)) atomicOr(status, kStInvalid);
}

// Edge inputs: facet ids in range and distinct, every sample on the sample grid
// and inside the scene's box (so the exactness budget of the scene covers it).
__global__ void k_check_edges(SceneDev sc, int E, int s, const int *efac, const float *esmp) {
    const int id = blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= E * s) return;
    const int e = id / s;
    int bad = 0;
    if (id % s == 0) {
        const int fa = efac[2 * e], fb = efac[2 * e + 1];
        if (!(fa >= 0 && fa < sc.F && fb >= -1 && fb < sc.F && fb != fa)) bad |= kStInvalid;
    }
    const double sscale = ldexp(1.0, sc.gs);
    for (int k = 0; k < 3; ++k) {
        const double y = (double)esmp[3 * (size_t)id + k] * sscale;
        if (!(fabs(y) < 16777216.0) || y != floor(y) || y < sc.extent[k] || y > sc.extent[3 + k]) bad |= kStGrid;
    }
    if (bad) atomicOr(sc.status, bad);
}

// First-order diffraction candidates per snapshot: popcount(tx edges & rx edges).
__global__ __launch_bounds__(256) void k_edge_counts(int N, int We, const uint64_t *txe, const uint64_t *rxe,
                                                     int64_t *counts) {
    const int lane = threadIdx.x & 63;
    const int n = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (n >= N) return;  // (wave-uniform)
    unsigned long long c = 0;
    for (int w = lane; w < We; w += 64) c += __popcll(txe[(size_t)n * We + w] & rxe[(size_t)n * We + w]);
    c = wave_sum_u64(c);
    if (lane == 0) counts[n] = (int64_t)c;
}

hipError_t launch_edges(Scene &scn, const TraverseOpts &o, int N, int E, int s, const int *efac, const float *esmp,
                        const float *tx, const float *rx, uint64_t *txe, uint64_t *rxe, int64_t *counts,
                        hipStream_t st) {
    const SceneDev &sc = scn.dev;
    const int We = (E + 63) / 64;
    hipError_t e;
    if (N > 0 && We > 0) {
        if ((e = launch_fill_u64(txe, 0ull, (size_t)N * We, st)) != hipSuccess) return e;
        if ((e = launch_fill_u64(rxe, 0ull, (size_t)N * We, st)) != hipSuccess) return e;
    }
    if (N > 0 && E > 0) {
        hipLaunchKernelGGL(k_check_points, dim3((2 * N + 255) / 256), dim3(256), 0, st, sc, N, tx, rx);
        const long long items = (long long)E * s;
        hipLaunchKernelGGL(k_check_edges, dim3((unsigned)((items + 255) / 256)), dim3(256), 0, st, sc, E, s, efac,
                           esmp);
        int G = 1;
        while (G < s) G <<= 1;
        const long long per_wave = kWave / G;
        const long long waves = 2LL * ((E + per_wave - 1) / per_wave) * ((N + kEdgeBlock - 1) / kEdgeBlock);
        hipLaunchKernelGGL(k_edges, dim3((unsigned)((waves + kWavesPerBlock - 1) / kWavesPerBlock)), dim3(kBlock), 0,
                           st, sc, N, E, s, G, We, efac, esmp, tx, rx, txe, rxe, o);
    }
    if (counts && N > 0) {
        if (We > 0) {
            hipLaunchKernelGGL(k_edge_counts, dim3((unsigned)((N + 3) / 4)), dim3(256), 0, st, N, We, txe, rxe,
                               counts);
        } else if ((e = launch_fill_u64((uint64_t *)counts, 0ull, (size_t)N, st)) != hipSuccess) {
            return e;
        }
    }
    return hipGetLastError();
}

hipError_t launch_edge_rows(Scene &scn, const TraverseOpts &o, int E, int s, const int *efac, const float *esmp,
                            int n_rows, const int *rows, uint64_t *ef, uint64_t *ee, hipStream_t st) {
    const SceneDev &sc = scn.dev;
    const int We = (E + 63) / 64;
    hipError_t e;
    if (n_rows <= 0) return hipSuccess;
    if ((e = launch_fill_u64(ef, 0ull, (size_t)n_rows * sc.W, st)) != hipSuccess) return e;
    if (We > 0 && (e = launch_fill_u64(ee, 0ull, (size_t)n_rows * We, st)) != hipSuccess) return e;
    if (E <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_check_rows, dim3((unsigned)((n_rows + 255) / 256)), dim3(256), 0, st, E, n_rows, rows,
                       sc.status);
    const long long items = (long long)E * s;
    hipLaunchKernelGGL(k_check_edges, dim3((unsigned)((items + 255) / 256)), dim3(256), 0, st, sc, E, s, efac, esmp);
    int G = 1;
    while (G < s) G <<= 1;
    const long long per_wave = kWave / G;
    const long long waves = (long long)n_rows * ((sc.F + E + per_wave - 1) / per_wave);
    hipLaunchKernelGGL(k_edge_rows, dim3((unsigned)((waves + kWavesPerBlock - 1) / kWavesPerBlock)), dim3(kBlock), 0,
                       st, sc, E, s, G, efac, esmp, n_rows, rows, ef, ee, o);
    return hipGetLastError();
}

hipError_t launch_point_jobs(const PointJob *d_jobs, int n_jobs, long long total_units, uint32_t *d_queue,
                             const TraverseOpts &o, ivm_stats *stats, hipStream_t s) {
    if (total_units <= 0) return hipSuccess;
    PointJob none{};
    // (the unit counter is cleared with the rest of the queue slots at the batch's start)
    hipLaunchKernelGGL(k_points<true>, dim3(o.grid_blocks), dim3(kBlock), 0, s, none, d_jobs, n_jobs, total_units,
                       (unsigned long long *)(d_queue + kQueuePoints), o, stats);
    return hipGetLastError();
}

hipError_t launch_points(Scene &scn, const TraverseOpts &o, int N, const float *tx, const float *rx, uint64_t *txv,
                         uint64_t *rxv, uint8_t *los, ivm_stats *stats, hipStream_t s) {
    hipError_t e;
    if ((e = launch_points_prep(scn, N, tx, rx, txv, rxv, s)) != hipSuccess) return e;
    if (N == 0) return hipSuccess;
    if (o.events && (e = hipEventRecord(o.events[0], s)) != hipSuccess) return e;
    const int U = point_unit_len(&scn.dev.S, &N, 1, o.grid_blocks);
    const long long units = point_units(scn, N, U);
    if (units > 0) {
        const PointJob job = make_point_job(scn, N, tx, rx, txv, rxv, 0, U);
        uint32_t *ctr = (uint32_t *)((char *)scn.ws + scn.lay.queue) + kQueuePoints;
        if ((e = launch_fill_u32(ctr, 0u, 2, s)) != hipSuccess) return e;
        hipLaunchKernelGGL(k_points<false>, dim3(o.grid_blocks), dim3(kBlock), 0, s, job, (const PointJob *)nullptr, 1,
                           units, (unsigned long long *)ctr, o, stats);
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (o.events && (e = hipEventRecord(o.events[1], s)) != hipSuccess) return e;
    return launch_los(scn, o, N, tx, rx, los, s);
}

}  // namespace ivm
