// solids.hip -- build-time checks behind the bundle certificates.
//
// Two facts make it sound to decide a whole bundle of segments at once:
//   * a facet whose triangles tile one convex polygon (k_facet_convex): the
//     segments between two convex point sets that all cross such a polygon at
//     their corners all cross it;
//   * a verified solid (k_solid_verify): a vertical convex prism whose walls and
//     roof are covered by the triangles of one facet group.  A segment that
//     starts outside the prism, stays at or above its base and passes through
//     its interior crosses a wall or the roof transversally at a point of a
//     covering triangle (its first entry point), so it is blocked (Section II-B:
//     a third face between two faces blocks them).
// Every test here is exact integer arithmetic in sample-grid units: vertex and
// sample coordinates are integers below 2^24 there (checked at validation), so
// differences stay below 2^25, 2-D cross products below 2^51 and the sums below
// 2^58 fit int64.
#include <climits>

#include "ivm_internal.h"

namespace ivm {
namespace {

inline int nblk(long long n, int b) { return (int)((n + b - 1) / b); }

struct I2 {
    long long x, y;
};

__device__ inline long long cross2(long long ax, long long ay, long long bx, long long by) { return ax * by - ay * bx; }

// Vertex coordinate in sample units, or false when off the grid / too large
// (such scenes fail validation; the check only keeps this kernel in range).
__device__ inline bool to_units(float v, float scale, long long *out) {
    const float y = v * scale;
    if (!(fabsf(y) < 16777216.0f) || y != floorf(y)) return false;
    *out = (long long)y;
    return true;
}

// Interior-disjointness of two triangles in 2-D: some edge line of either one
// has the first triangle on one closed side and the second on the other.
// Zero-area triangles never overlap anything.
__device__ bool tri_disjoint(const I2 *A, const I2 *B) {
    const I2 *T[2] = {A, B};
    for (int w = 0; w < 2; ++w) {
        const I2 *P = T[w], *Q = T[1 - w];
        const long long o = cross2(P[1].x - P[0].x, P[1].y - P[0].y, P[2].x - P[0].x, P[2].y - P[0].y);
        if (o == 0) return true;
        const int sg = o > 0 ? 1 : -1;
        for (int e = 0; e < 3; ++e) {
            const I2 a = P[e], b = P[(e + 1) % 3];
            bool sep = true;
            for (int v = 0; v < 3 && sep; ++v) {
                const long long c = cross2(b.x - a.x, b.y - a.y, Q[v].x - a.x, Q[v].y - a.y);
                sep = (sg > 0 ? c <= 0 : c >= 0);
            }
            if (sep) return true;
        }
    }
    return false;
}

__device__ inline long long tri_area2(const I2 *P) {
    const long long o = cross2(P[1].x - P[0].x, P[1].y - P[0].y, P[2].x - P[0].x, P[2].y - P[0].y);
    return o < 0 ? -o : o;
}

// Convexity of each facet: the 2-D convex hull (projection dropping the
// normal's largest axis) of its vertices has exactly the summed area of its
// triangles and the triangles have pairwise disjoint interiors, so their union
// is that hull (a closed set covering a convex body up to measure zero is the
// body).  One thread per facet.
__global__ void k_facet_convex(ivm_scene_desc d, const int *ffirst, const double *fplane, int *fflags) {
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= d.n_facets) return;
    int flags = 0;
    const int t0 = ffirst[2 * f], nt = ffirst[2 * f + 1];
    const double n0 = fabs(fplane[6 * f + 3]), n1 = fabs(fplane[6 * f + 4]), n2 = fabs(fplane[6 * f + 5]);
    const int drop = (n0 >= n1 && n0 >= n2) ? 0 : (n1 >= n2 ? 1 : 2);
    const int ax = drop == 0 ? 1 : 0, ay = drop == 2 ? 1 : 2;
    const float ss = ldexpf(1.0f, d.grid_sample_log2);
    I2 tv[kConvexMaxTris][3];
    bool ok = nt > 0 && nt <= kConvexMaxTris && t0 != INT_MAX && t0 + nt <= d.n_triangles &&
              !(n0 == 0.0 && n1 == 0.0 && n2 == 0.0);
    long long sum = 0;
    for (int t = 0; ok && t < nt; ++t) {
        for (int c = 0; c < 3 && ok; ++c) {
            int vi = d.tri_vertices[3 * (t0 + t) + c];
            if (vi < 0 || vi >= d.n_vertices) { ok = false; break; }
            ok = to_units(d.vertices[3 * vi + ax], ss, &tv[t][c].x) && to_units(d.vertices[3 * vi + ay], ss, &tv[t][c].y);
        }
        if (ok) sum += tri_area2(tv[t]);
    }
    if (ok) {
        for (int a = 0; a < nt && ok; ++a)
            for (int b = a + 1; b < nt && ok; ++b) ok = tri_disjoint(tv[a], tv[b]);
    }
    if (ok) {
        // Andrew's monotone chain over the 3 nt vertices
        I2 pts[3 * kConvexMaxTris];
        int np = 0;
        for (int t = 0; t < nt; ++t)
            for (int c = 0; c < 3; ++c) pts[np++] = tv[t][c];
        for (int m = 1; m < np; ++m) {
            const I2 x = pts[m];
            int k = m - 1;
            while (k >= 0 && (pts[k].x > x.x || (pts[k].x == x.x && pts[k].y > x.y))) {
                pts[k + 1] = pts[k];
                --k;
            }
            pts[k + 1] = x;
        }
        I2 h[2 * 3 * kConvexMaxTris + 1];
        int nh = 0;
        auto turn = [](I2 o, I2 a, I2 b) { return cross2(a.x - o.x, a.y - o.y, b.x - o.x, b.y - o.y); };
        for (int m = 0; m < np; ++m) {
            while (nh >= 2 && turn(h[nh - 2], h[nh - 1], pts[m]) <= 0) --nh;
            h[nh++] = pts[m];
        }
        for (int m = np - 2, lo = nh + 1; m >= 0; --m) {
            while (nh >= lo && turn(h[nh - 2], h[nh - 1], pts[m]) <= 0) --nh;
            h[nh++] = pts[m];
        }
        if (nh > 1) --nh;
        long long hull2 = 0;
        for (int m = 1; m + 1 < nh; ++m) hull2 += turn(h[0], h[m], h[m + 1]);
        if (hull2 > 0 && hull2 == sum) flags |= kFacetConvex;
    }
    fflags[f] = flags;
}

// counting sort of facets by solid id: counts, exclusive offsets, scatter
__global__ void k_solid_count(int F, int n_solids, const int32_t *hint, int *cnt, int *fsolid) {
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= F) return;
    fsolid[f] = -1;
    const int s = hint[f];
    if (s >= 0 && s < n_solids) atomicAdd(&cnt[s], 1);
}

__global__ __launch_bounds__(1024) void k_solid_scan(int n, const int *cnt, int *off) {
    __shared__ int part[1024];
    const int t = threadIdx.x;
    const int chunk = (n + 1023) / 1024;
    const int b = t * chunk, e = min(n, b + chunk);
    int acc = 0;
    for (int k = b; k < e; ++k) acc += cnt[k];
    part[t] = acc;
    __syncthreads();
    for (int step = 1; step < 1024; step <<= 1) {
        const int v = t >= step ? part[t - step] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    int run = t > 0 ? part[t - 1] : 0;
    for (int k = b; k < e; ++k) {
        off[k] = run;
        run += cnt[k];
    }
    if (t == 1023) off[n] = part[1023];
}

__global__ void k_solid_scatter(int F, int n_solids, const int32_t *hint, const int *off, int *fill, int *fac) {
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= F) return;
    const int s = hint[f];
    if (s >= 0 && s < n_solids) fac[off[s] + atomicAdd(&fill[s], 1)] = f;
}

__device__ inline int half_plane(long long x, long long y) { return (y < 0 || (y == 0 && x < 0)) ? 1 : 0; }

// angle(a) < angle(b) on [0, 2 pi)
__device__ inline bool angle_less(long long ax, long long ay, long long bx, long long by) {
    const int ha = half_plane(ax, ay), hb = half_plane(bx, by);
    if (ha != hb) return ha < hb;
    return cross2(ax, ay, bx, by) > 0;
}

// The prism check, one 64-lane block per solid group.  Lane 0 classifies the
// facets and checks the closed convex footprint and the areas; all lanes test
// the triangle pairs for overlapping interiors.
__global__ __launch_bounds__(64) void k_solid_verify(ivm_scene_desc d, const int *ffirst, const double *fplane,
                                                     const int *off, const int *fac, int4 *rec, int4 *planes,
                                                     float4 *sbox, int *fsolid, int *n_verified) {
    const int s = blockIdx.x, lane = threadIdx.x;
    __shared__ int mem[kSolidMaxFacets];
    __shared__ long long tv[kSolidMaxTris][9];   // x, y, z of the three vertices
    __shared__ int tgrp[kSolidMaxTris];          // -1 roof, k >= 0 wall plane k
    __shared__ long long pd[kSolidMaxPlanes][2], pref[kSolidMaxPlanes][2], pu[kSolidMaxPlanes][2],
        pv[kSolidMaxPlanes][2];
    __shared__ int succ[kSolidMaxPlanes];
    __shared__ int nt_tot, npl, fail, m;
    __shared__ long long H, ZB;
    if (lane == 0) {
        m = off[s + 1] - off[s];
        fail = (m <= 0 || m > kSolidMaxFacets) ? 1 : 0;
        nt_tot = 0;
        npl = 0;
    }
    __syncthreads();
    if (!fail && lane < m) mem[lane] = fac[off[s] + lane];
    __syncthreads();
    if (lane == 0 && !fail) {
        for (int a = 1; a < m; ++a) {  // members in facet order (deterministic plane order)
            const int x = mem[a];
            int k = a - 1;
            while (k >= 0 && mem[k] > x) {
                mem[k + 1] = mem[k];
                --k;
            }
            mem[k + 1] = x;
        }
        const float ss = ldexpf(1.0f, d.grid_sample_log2);
        long long h = LLONG_MIN, zb = LLONG_MAX;
        bool roof = false;
        for (int q = 0; q < m && !fail; ++q) {
            const int f = mem[q];
            const int t0 = ffirst[2 * f], nt = ffirst[2 * f + 1];
            const double nx = fplane[6 * f + 3], ny = fplane[6 * f + 4], nz = fplane[6 * f + 5];
            const bool is_roof = nx == 0.0 && ny == 0.0 && nz > 0.0;
            const bool is_wall = nz == 0.0 && (nx != 0.0 || ny != 0.0);
            if (nt <= 0 || t0 == INT_MAX || t0 + nt > d.n_triangles || nt_tot + nt > kSolidMaxTris ||
                !(is_roof || is_wall)) {
                fail = 1;
                break;
            }
            const int first = nt_tot;
            for (int t = 0; t < nt && !fail; ++t) {
                for (int c = 0; c < 3 && !fail; ++c) {
                    const int vi = d.tri_vertices[3 * (t0 + t) + c];
                    if (vi < 0 || vi >= d.n_vertices) { fail = 1; break; }
                    for (int k = 0; k < 3; ++k)
                        if (!to_units(d.vertices[3 * vi + k], ss, &tv[nt_tot][3 * c + k])) fail = 1;
                    h = max(h, tv[nt_tot][3 * c + 2]);
                    zb = min(zb, tv[nt_tot][3 * c + 2]);
                }
                ++nt_tot;
            }
            if (fail) break;
            if (is_roof) {
                roof = true;
                for (int t = first; t < nt_tot; ++t) tgrp[t] = -1;
                continue;
            }
            // wall: horizontal direction from two vertices of the first triangle with distinct (x, y),
            // turned so that the outward normal is (d.y, -d.x) (exact sign from the FP64 normal)
            const long long *v = tv[first];
            long long dx = v[3] - v[0], dy = v[4] - v[1];
            if (dx == 0 && dy == 0) { dx = v[6] - v[0]; dy = v[7] - v[1]; }
            if (dx == 0 && dy == 0) { fail = 1; break; }
            const int lam = dy != 0 ? ((nx > 0.0) == (dy > 0) ? 1 : -1) : ((ny > 0.0) == (dx < 0) ? 1 : -1);
            if (lam < 0) { dx = -dx; dy = -dy; }
            int k = 0;
            for (; k < npl; ++k) {
                if (cross2(pd[k][0], pd[k][1], dx, dy) == 0 && pd[k][0] * dx + pd[k][1] * dy > 0 &&
                    cross2(pd[k][0], pd[k][1], v[0] - pref[k][0], v[1] - pref[k][1]) == 0)
                    break;
            }
            if (k == npl) {
                if (npl == kSolidMaxPlanes) { fail = 1; break; }
                pd[k][0] = dx; pd[k][1] = dy;
                pref[k][0] = v[0]; pref[k][1] = v[1];
                ++npl;
            }
            for (int t = first; t < nt_tot; ++t) tgrp[t] = k;
        }
        if (!fail && (!roof || npl < 3 || h <= zb)) fail = 1;
        // roof triangles at the top height; wall vertices on their lines; wall extents
        for (int k = 0; k < npl && !fail; ++k) {
            long long smin = LLONG_MAX, smax = LLONG_MIN;
            for (int t = 0; t < nt_tot; ++t) {
                if (tgrp[t] != k) continue;
                for (int c = 0; c < 3; ++c) {
                    const long long x = tv[t][3 * c], y = tv[t][3 * c + 1];
                    if (cross2(pd[k][0], pd[k][1], x - pref[k][0], y - pref[k][1]) != 0) fail = 1;
                    const long long sp = pd[k][0] * (x - pref[k][0]) + pd[k][1] * (y - pref[k][1]);
                    if (sp < smin) { smin = sp; pu[k][0] = x; pu[k][1] = y; }
                    if (sp > smax) { smax = sp; pv[k][0] = x; pv[k][1] = y; }
                }
            }
            if (smax <= smin) fail = 1;
        }
        for (int t = 0; t < nt_tot && !fail; ++t)
            if (tgrp[t] < 0 && (tv[t][2] != h || tv[t][5] != h || tv[t][8] != h)) fail = 1;
        // footprint: the wall traces chain head to tail into one convex loop turning once
        for (int k = 0; k < npl && !fail; ++k) {
            int found = -1, count = 0;
            for (int q = 0; q < npl; ++q)
                if (pu[q][0] == pv[k][0] && pu[q][1] == pv[k][1]) { found = q; ++count; }
            if (count != 1) fail = 1;
            succ[k] = found;
        }
        if (!fail) {
            int cur = 0, wraps = 0;
            unsigned seen = 0u;
            for (int step = 0; step < npl && !fail; ++step) {
                const int nx2 = succ[cur];
                if ((seen >> cur) & 1u) fail = 1;
                seen |= 1u << cur;
                if (cross2(pd[cur][0], pd[cur][1], pd[nx2][0], pd[nx2][1]) <= 0) fail = 1;
                if (angle_less(pd[nx2][0], pd[nx2][1], pd[cur][0], pd[cur][1])) ++wraps;
                cur = nx2;
            }
            if (cur != 0 || wraps != 1) fail = 1;
        }
        if (!fail) {
            // twice the footprint area, relative to the first corner
            long long area2 = 0;
            for (int k = 0; k < npl; ++k) {
                const int q = succ[k];
                area2 += cross2(pu[k][0] - pu[0][0], pu[k][1] - pu[0][1], pu[q][0] - pu[0][0], pu[q][1] - pu[0][1]);
            }
            // roof: inside the footprint, areas add up to it
            long long roof2 = 0;
            for (int t = 0; t < nt_tot && !fail; ++t) {
                if (tgrp[t] >= 0) continue;
                I2 P[3];
                for (int c = 0; c < 3; ++c) {
                    P[c].x = tv[t][3 * c];
                    P[c].y = tv[t][3 * c + 1];
                    for (int k = 0; k < npl; ++k)
                        if (cross2(pd[k][0], pd[k][1], P[c].x - pu[k][0], P[c].y - pu[k][1]) < 0) fail = 1;
                }
                roof2 += tri_area2(P);
            }
            if (roof2 != area2) fail = 1;
            // walls: (along-wall axis, z) areas add up to the edge x [base, top] rectangle
            for (int k = 0; k < npl && !fail; ++k) {
                const int axk = (pd[k][0] >= 0 ? pd[k][0] : -pd[k][0]) >= (pd[k][1] >= 0 ? pd[k][1] : -pd[k][1]) ? 0 : 1;
                long long w2 = 0;
                for (int t = 0; t < nt_tot; ++t) {
                    if (tgrp[t] != k) continue;
                    I2 P[3];
                    for (int c = 0; c < 3; ++c) {
                        P[c].x = tv[t][3 * c + axk];
                        P[c].y = tv[t][3 * c + 2];
                    }
                    w2 += tri_area2(P);
                }
                long long len = pv[k][axk] - pu[k][axk];
                if (len < 0) len = -len;
                if (w2 != 2 * len * (h - zb)) fail = 1;
            }
        }
        H = h;
        ZB = zb;
    }
    __syncthreads();
    // overlapping interiors inside one face (roof, or one wall plane)
    if (!fail) {
        const int n = nt_tot;
        bool bad = false;
        for (int it = lane; it < n * n; it += 64) {
            const int a = it / n, b = it - (it / n) * n;
            if (b <= a || tgrp[a] != tgrp[b]) continue;
            const int g = tgrp[a];
            int axk = 0, ayk = 1;
            if (g >= 0) {
                axk = (pd[g][0] >= 0 ? pd[g][0] : -pd[g][0]) >= (pd[g][1] >= 0 ? pd[g][1] : -pd[g][1]) ? 0 : 1;
                ayk = 2;
            }
            I2 A[3], B[3];
            for (int c = 0; c < 3; ++c) {
                A[c].x = tv[a][3 * c + axk];
                A[c].y = tv[a][3 * c + ayk];
                B[c].x = tv[b][3 * c + axk];
                B[c].y = tv[b][3 * c + ayk];
            }
            if (!tri_disjoint(A, B)) bad = true;
        }
        if (bad) atomicOr(&fail, 1);
    }
    __syncthreads();
    const bool ok = !fail;
    if (lane == 0) {
        rec[s] = make_int4(ok ? npl : 0, ok ? (int)H : 0, ok ? (int)ZB : 0, 0);
        if (ok) atomicAdd(n_verified, 1);
        // footprint box and heights in metres (exact: sample-grid integers below 2^24)
        float4 lo = make_float4(INFINITY, INFINITY, INFINITY, 0.f), hi = make_float4(-INFINITY, -INFINITY, -INFINITY, 0.f);
        if (ok) {
            const float mu = ldexpf(1.0f, -d.grid_sample_log2);
            for (int k = 0; k < npl; ++k) {
                lo.x = fminf(lo.x, (float)pu[k][0] * mu);
                lo.y = fminf(lo.y, (float)pu[k][1] * mu);
                hi.x = fmaxf(hi.x, (float)pu[k][0] * mu);
                hi.y = fmaxf(hi.y, (float)pu[k][1] * mu);
            }
            lo.z = (float)ZB * mu;
            hi.z = (float)H * mu;
        }
        sbox[2 * s] = lo;
        sbox[2 * s + 1] = hi;
    }
    if (ok) {
        if (lane < npl) planes[s * kSolidMaxPlanes + lane] = make_int4((int)pu[lane][0], (int)pu[lane][1],
                                                                       (int)pd[lane][0], (int)pd[lane][1]);
        if (lane < m) fsolid[mem[lane]] = s;
    }
}

// Grid extent from the verified solids' boxes (one block).
__global__ __launch_bounds__(1024) void k_grid_extent(int ns, const float4 *sbox, int G, float4 *gridp, int *gridi) {
    __shared__ float red[4][1024];
    const int t = threadIdx.x;
    float x0 = INFINITY, y0 = INFINITY, x1 = -INFINITY, y1 = -INFINITY;
    for (int s = t; s < ns; s += 1024) {
        const float4 lo = sbox[2 * s], hi = sbox[2 * s + 1];
        if (lo.x <= hi.x) {
            x0 = fminf(x0, lo.x); y0 = fminf(y0, lo.y);
            x1 = fmaxf(x1, hi.x); y1 = fmaxf(y1, hi.y);
        }
    }
    red[0][t] = x0; red[1][t] = y0; red[2][t] = -x1; red[3][t] = -y1;
    __syncthreads();
    for (int w = 512; w >= 1; w >>= 1) {
        if (t < w)
            for (int k = 0; k < 4; ++k) red[k][t] = fminf(red[k][t], red[k][t + w]);
        __syncthreads();
    }
    if (t == 0) {
        const float a = red[0][0], b = red[1][0], c = -red[2][0], e = -red[3][0];
        const bool ok = a <= c && b <= e;
        const float cw = ok ? fmaxf((c - a) / G, 1e-3f) : 1.f, ch = ok ? fmaxf((e - b) / G, 1e-3f) : 1.f;
        gridp[0] = make_float4(ok ? a : 0.f, ok ? b : 0.f, cw, ch);
        gridi[0] = G;
        gridi[1] = ok ? 1 : 0;
        gridi[2] = 0;
        gridi[3] = 0;
    }
}

__device__ inline bool grid_cells(const float4 *gridp, int G, float4 lo, float4 hi, int &cx0, int &cx1, int &cy0,
                                  int &cy1) {
    const float4 gp = gridp[0];
    const float icw = 1.0f / gp.z, ich = 1.0f / gp.w;  // the lookup computes cells the same way
    cx0 = min(G - 1, max(0, (int)floorf((lo.x - gp.x) * icw)));
    cx1 = min(G - 1, max(0, (int)floorf((hi.x - gp.x) * icw)));
    cy0 = min(G - 1, max(0, (int)floorf((lo.y - gp.y) * ich)));
    cy1 = min(G - 1, max(0, (int)floorf((hi.y - gp.y) * ich)));
    return (cx1 - cx0 + 1) * (cy1 - cy0 + 1) <= kGridMaxCellsPerSolid;
}

// Count, then fill, the cells each verified solid's footprint box overlaps.
__global__ void k_grid_insert(int ns, const float4 *sbox, const float4 *gridp, const int *gridi, const int *off,
                              int *cnt, int *list, int cap) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= ns || !gridi[1]) return;
    const float4 lo = sbox[2 * s], hi = sbox[2 * s + 1];
    if (!(lo.x <= hi.x)) return;
    const int G = gridi[0];
    int cx0, cx1, cy0, cy1;
    if (!grid_cells(gridp, G, lo, hi, cx0, cx1, cy0, cy1)) return;
    for (int cy = cy0; cy <= cy1; ++cy)
        for (int cx = cx0; cx <= cx1; ++cx) {
            const int cell = cy * G + cx;
            if (!off) {
                atomicAdd(&cnt[cell], 1);
            } else {
                const int pos = off[cell] + atomicAdd(&cnt[cell], 1);
                if (pos < cap) list[pos] = s;
            }
        }
}

// Sort each cell's list (deterministic order) and mark the grid unusable on overflow.
__global__ void k_grid_finish(int ncell, const int *off, int *list, int cap, int *gridi) {
    const int cell = blockIdx.x * blockDim.x + threadIdx.x;
    if (cell == 0) {
        gridi[2] = off[ncell];
        if (off[ncell] > cap) gridi[1] = 0;
    }
    if (cell >= ncell || off[ncell] > cap) return;
    const int a = off[cell], b = off[cell + 1];
    for (int m = a + 1; m < b; ++m) {
        const int x = list[m];
        int k = m - 1;
        while (k >= a && list[k] > x) {
            list[k + 1] = list[k];
            --k;
        }
        list[k + 1] = x;
    }
}

// The cell entries with each solid's footprint box inline (one load per entry in
// the scans instead of an id and then a box).
__global__ void k_grid_entries(int cap, const int *list, const float4 *sbox, const int *gridi, float4 *ent) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= cap || !gridi[1] || e >= gridi[2]) return;
    const int s = list[e];
    const float4 lo = sbox[2 * s], hi = sbox[2 * s + 1];
    ent[2 * e] = make_float4(lo.x, lo.y, lo.z, __int_as_float(s));
    ent[2 * e + 1] = make_float4(hi.x, hi.y, hi.z, 0.f);
}

__global__ void k_fill_i32(int *p, int v, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

}  // namespace

hipError_t launch_solids(Scene &sc, hipStream_t s) {
    const ivm_scene_desc &d = sc.desc;
    char *ws = (char *)sc.ws;
    const Layout &L = sc.lay;
    const int F = d.n_facets;
    const int *ffirst = (const int *)(ws + L.ffirst);
    const double *fplane = (const double *)(ws + L.fplane);
    int *fflags = (int *)(ws + L.fflags);
    int *fsolid = (int *)(ws + L.fsolid);
    int *nver = (int *)(ws + L.sol_nver);
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, s, nver, 0, 1);
    if (F > 0) {
        hipLaunchKernelGGL(k_facet_convex, dim3(nblk(F, 128)), dim3(128), 0, s, d, ffirst, fplane, fflags);
        hipLaunchKernelGGL(k_fill_i32, dim3(nblk(F, 256)), dim3(256), 0, s, fsolid, -1, F);
    }
    const int ns = d.n_solids;
    if (F > 0 && ns > 0 && d.facet_solid) {
        int *cnt = (int *)(ws + L.sol_cnt), *fill = cnt + (ns + 1);
        int *off = (int *)(ws + L.sol_off), *fac = (int *)(ws + L.sol_fac);
        hipLaunchKernelGGL(k_fill_i32, dim3(nblk(2 * (ns + 1), 256)), dim3(256), 0, s, cnt, 0, 2 * (ns + 1));
        hipLaunchKernelGGL(k_solid_count, dim3(nblk(F, 256)), dim3(256), 0, s, F, ns, d.facet_solid, cnt, fsolid);
        hipLaunchKernelGGL(k_solid_scan, dim3(1), dim3(1024), 0, s, ns, (const int *)cnt, off);
        hipLaunchKernelGGL(k_solid_scatter, dim3(nblk(F, 256)), dim3(256), 0, s, F, ns, d.facet_solid,
                           (const int *)off, fill, fac);
        hipLaunchKernelGGL(k_solid_verify, dim3(ns), dim3(64), 0, s, d, ffirst, fplane, (const int *)off,
                           (const int *)fac, (int4 *)(ws + L.sol_rec), (int4 *)(ws + L.sol_plane),
                           (float4 *)(ws + L.sol_box), fsolid, nver);
        // grid over the verified solids' footprints
        const int G = solid_grid_dim(ns), ncell = G * G, cap = kGridEntriesPerSolid * ns + 1024;
        float4 *gridp = (float4 *)(ws + L.grid_p);
        int *gridi = (int *)(ws + L.grid_p + sizeof(float4));
        int *gcnt = (int *)(ws + L.grid_cnt), *goff = (int *)(ws + L.grid_off), *glist = (int *)(ws + L.grid_list);
        const float4 *sbox = (const float4 *)(ws + L.sol_box);
        hipLaunchKernelGGL(k_grid_extent, dim3(1), dim3(1024), 0, s, ns, sbox, G, gridp, gridi);
        hipLaunchKernelGGL(k_fill_i32, dim3(nblk(2 * ncell, 256)), dim3(256), 0, s, gcnt, 0, 2 * ncell);
        hipLaunchKernelGGL(k_grid_insert, dim3(nblk(ns, 256)), dim3(256), 0, s, ns, sbox, (const float4 *)gridp,
                           (const int *)gridi, (const int *)nullptr, gcnt, glist, cap);
        hipLaunchKernelGGL(k_solid_scan, dim3(1), dim3(1024), 0, s, ncell, (const int *)gcnt, goff);
        hipLaunchKernelGGL(k_grid_insert, dim3(nblk(ns, 256)), dim3(256), 0, s, ns, sbox, (const float4 *)gridp,
                           (const int *)gridi, (const int *)goff, gcnt + ncell, glist, cap);
        hipLaunchKernelGGL(k_grid_finish, dim3(nblk(ncell, 256)), dim3(256), 0, s, ncell, (const int *)goff, glist,
                           cap, gridi);
        hipLaunchKernelGGL(k_grid_entries, dim3(nblk(cap, 256)), dim3(256), 0, s, cap, (const int *)glist, sbox,
                           (const int *)gridi, (float4 *)(ws + L.grid_ent));
    } else {
        hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, s, (int *)(ws + L.grid_p + sizeof(float4)), 0, 4);
    }
    return hipGetLastError();
}

}  // namespace ivm
