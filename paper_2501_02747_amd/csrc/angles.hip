// angles.hip -- angular bouncing ranges of the visible facet pairs.
//
// Section II-A reads the 3-D scene in 2-D views (a horizontal one for vertical
// faces, a vertical one otherwise) in which every face is a segment; Section
// II-B, eq. 1, takes at an end B of the reference face the angle between BA
// (along the face) and BF (towards an end F of the aim face) as the arccos of
// their normalised dot product, and eq. 2 records an angle of 180 degrees or
// more, measured from the face towards its visible side, as 0.
//
// For a visible pair (i, j) the view looks along d, the line where the two
// planes meet (n_i x n_j), or for parallel planes the vertical (vertical
// facets), x (horizontal facets) or the horizontal line in facet i's plane; the
// first non-zero component of d in the order z, x, y is positive.  d lies in
// both planes, so each facet projects to a segment: facet i's ends are its
// vertices with the smallest (A) and largest (B) value of (d x n_i) . v, facet
// j's ends E, F those of (d x n_j) . v.  omega = the angles at B between BA and
// BE, BF (sorted); mu = those at A between AB and AE, AF (sorted).  An angle is
// that of the two vectors projected on the plane normal to d:
//   cos = (dd u.v - (u.d)(v.d)) / sqrt((dd u.u - (u.d)^2)(dd v.v - (v.d)^2)),
// each of the three integer terms exact (128-bit) and rounded once to FP64; an
// aim vertex not strictly in front of facet i (eq. 2) gives 0.  Vertices that
// tie in the extreme value differ only along d, so they give the same angles.
//
// Coordinates are integers in vertex-grid units (exact from the FP32 records).
// A pair whose terms could leave the 128-bit range (checked per pair from the
// bit lengths of d and of the scene's extent) gets NaN and raises a status bit
// that the entry point reports as IVM_ERR_GRID.
//
// Layout: one wave per row of M; lanes own words of the row; a wave scan of the
// words' popcounts places each set bit's pair in the row-major output (CSR
// offsets from a row-count pass and one block scan).
#include "ivm_internal.h"

namespace ivm {
namespace {

typedef __int128 i128;

struct V3 {
    long long x, y, z;
};
struct W3 {
    i128 x, y, z;
};

__device__ inline long long to_grid(float v, float scale) { return (long long)(v * scale); }

__device__ inline V3 sub3(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ inline W3 widen(V3 a) { return {(i128)a.x, (i128)a.y, (i128)a.z}; }
__device__ inline i128 dotw(W3 a, W3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ inline W3 crossw(W3 a, W3 b) {
    return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__device__ inline i128 iabs(i128 v) { return v < 0 ? -v : v; }
__device__ inline int bitlen(i128 v) {
    unsigned long long hi = (unsigned long long)((unsigned __int128)v >> 64), lo = (unsigned long long)v;
    return hi ? 128 - __clzll((long long)hi) : (lo ? 64 - __clzll((long long)lo) : 0);
}

// Vertex m (0..2) of caller triangle t in grid units: a, a + e1, a + e2.
__device__ inline V3 tri_vertex(const SceneDev &sc, int t, int m, float scale) {
    const float4 a = sc.tri_caller[3 * (size_t)t];
    float x = a.x, y = a.y, z = a.z;
    if (m > 0) {
        const float4 e = sc.tri_caller[3 * (size_t)t + m];
        x += e.x;
        y += e.y;
        z += e.z;
    }
    return {to_grid(x, scale), to_grid(y, scale), to_grid(z, scale)};
}

// Normal (b - a) x (c - a) of the facet's first triangle, grid units.
__device__ inline W3 facet_normal(const SceneDev &sc, int f, float scale) {
    const int t = sc.ftri[2 * f];
    const V3 a = tri_vertex(sc, t, 0, scale), b = tri_vertex(sc, t, 1, scale), c = tri_vertex(sc, t, 2, scale);
    return crossw(widen(sub3(b, a)), widen(sub3(c, a)));
}

// The pair's view direction (see the file comment).
__device__ inline W3 view_direction(W3 ni, W3 nj) {
    W3 d = crossw(ni, nj);
    if (d.x == 0 && d.y == 0 && d.z == 0) {
        if (ni.z == 0)
            d = {0, 0, 1};
        else if (ni.x == 0 && ni.y == 0)
            d = {1, 0, 0};
        else
            d = {-ni.y, ni.x, 0};
    }
    const i128 lead = d.z != 0 ? d.z : (d.x != 0 ? d.x : d.y);
    if (lead < 0) d = {-d.x, -d.y, -d.z};
    return d;
}

// Ends of facet f along t (relative to the point o): argmin and argmax of t.(v - o).
__device__ inline void facet_ends(const SceneDev &sc, int f, W3 t, V3 o, float scale, V3 &lo, V3 &hi) {
    const int t0 = sc.ftri[2 * f], nt = sc.ftri[2 * f + 1];
    i128 kmin = 0, kmax = 0;
    bool first = true;
    for (int k = 0; k < nt; ++k)
        for (int m = 0; m < 3; ++m) {
            const V3 v = tri_vertex(sc, t0 + k, m, scale);
            const i128 key = dotw(t, widen(sub3(v, o)));
            if (first || key < kmin) {
                kmin = key;
                lo = v;
            }
            if (first || key > kmax) {
                kmax = key;
                hi = v;
            }
            first = false;
        }
}

constexpr double kRadPerDeg = 3.14159265358979323846 / 180.0;

// Angle (degrees) at `at` between (other - at) and (P - at) in the view normal
// to d; 0 unless P is strictly in front of facet i (plane point a_i, normal n_i).
__device__ inline double view_angle(V3 at, V3 other, V3 P, V3 a_i, W3 n_i, W3 d, i128 dd) {
#pragma clang fp contract(off)
    if (dotw(widen(sub3(P, a_i)), n_i) <= 0) return 0.0;
    const W3 u = widen(sub3(other, at)), v = widen(sub3(P, at));
    const i128 ud = dotw(u, d), vd = dotw(v, d);
    const i128 uv = dd * dotw(u, v) - ud * vd;
    const i128 uu = dd * dotw(u, u) - ud * ud;
    const i128 vv = dd * dotw(v, v) - vd * vd;
    const double c = (double)uv / sqrt((double)uu * (double)vv);
    return acos(fmin(1.0, fmax(-1.0, c))) / kRadPerDeg;
}

__global__ __launch_bounds__(256) void k_angle_counts(int F, int W, const uint64_t *M, int64_t *counts) {
    const int lane = threadIdx.x & 63;
    const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (row >= F) return;  // (wave-uniform)
    unsigned long long c = 0;
    const uint64_t *r = M + (size_t)row * W;
    for (int w = lane; w < W; w += 64) {
        uint64_t b = r[w];
        if (w == W - 1 && (F & 63)) b &= (1ull << (F & 63)) - 1ull;  // padding names no facet
        c += __popcll(b);
    }
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o);
    if (lane == 0) counts[row + 1] = (int64_t)c;
}

constexpr int kScanT = 1024;

// In-place inclusive scan of a[1..n] with a[0] = 0 (one block).
__global__ __launch_bounds__(kScanT) void k_angle_scan(int64_t *a, int n) {
    __shared__ int64_t sh[kScanT];
    const int t = threadIdx.x;
    const int per = (n + kScanT - 1) / kScanT;
    const int b0 = 1 + min(n, t * per), b1 = 1 + min(n, t * per + per);
    int64_t s = 0;
    for (int k = b0; k < b1; ++k) s += a[k];
    sh[t] = s;
    __syncthreads();
    for (int o = 1; o < kScanT; o <<= 1) {
        const int64_t add = t >= o ? sh[t - o] : 0;
        __syncthreads();
        sh[t] += add;
        __syncthreads();
    }
    int64_t run = sh[t] - s;
    for (int k = b0; k < b1; ++k) {
        run += a[k];
        a[k] = run;
    }
    if (t == 0) a[0] = 0;
}

__global__ __launch_bounds__(256) void k_angles(SceneDev sc, const uint64_t *M, const int64_t *offsets, int32_t *cols,
                                                double *ranges) {
    const int lane = threadIdx.x & 63;
    const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= sc.F) return;  // (wave-uniform)
    const int W = sc.W;
    const float scale = (float)(1 << sc.g);
    const uint64_t *row = M + (size_t)i * W;
    const W3 n_i = facet_normal(sc, i, scale);
    const V3 a_i = tri_vertex(sc, sc.ftri[2 * i], 0, scale);
    // bit length of the largest coordinate difference of the scene, vertex-grid units
    double ext = 0.0;
    for (int k = 0; k < 3; ++k) ext = fmax(ext, sc.extent[3 + k] - sc.extent[k]);
    const int ext_bits = bitlen((i128)ceil(ldexp(ext, sc.g - sc.gs)));
    int64_t base = offsets[i];
    for (int w0 = 0; w0 < W; w0 += 64) {
        const int w = w0 + lane;
        uint64_t bits = w < W ? row[w] : 0ull;
        if (w == W - 1 && (sc.F & 63)) bits &= (1ull << (sc.F & 63)) - 1ull;  // padding names no facet
        // place this lane's bits after those of the lanes before it
        unsigned long long incl = __popcll(bits);
        for (int o = 1; o < 64; o <<= 1) {
            const unsigned long long up = __shfl_up(incl, o);
            if (lane >= o) incl += up;
        }
        const unsigned long long total = __shfl(incl, 63);
        int64_t pos = base + (int64_t)(incl - __popcll(bits));
        while (bits) {
            const int j = w * 64 + __ffsll((long long)bits) - 1;
            bits &= bits - 1;
            const W3 n_j = facet_normal(sc, j, scale);
            const W3 d = view_direction(n_i, n_j);
            const int bd = max(bitlen(iabs(d.x)), max(bitlen(iabs(d.y)), bitlen(iabs(d.z))));
            const int bn = max(bitlen(iabs(n_i.x)), max(bitlen(iabs(n_i.y)), bitlen(iabs(n_i.z))));
            const int bm = max(bitlen(iabs(n_j.x)), max(bitlen(iabs(n_j.y)), bitlen(iabs(n_j.z))));
            double *o = ranges + 4 * (size_t)pos;
            cols[pos] = j;
            ++pos;
            // dd u.v and (u.d)(v.d) below 2^(2 bd + 2 ext + 4); t.(v - o) below 2^(bd + bn + ext + 3)
            if (2 * bd + 2 * ext_bits + 5 > 126 || bd + max(bn, bm) + ext_bits + 4 > 126) {
                o[0] = o[1] = o[2] = o[3] = __builtin_nan("");
                atomicOr(sc.status, kStAngleRange);
                continue;
            }
            const i128 dd = dotw(d, d);
            V3 A, B, E, Fv;
            facet_ends(sc, i, crossw(d, n_i), a_i, scale, A, B);
            facet_ends(sc, j, crossw(d, n_j), a_i, scale, E, Fv);
            double w1 = view_angle(B, A, E, a_i, n_i, d, dd), w2 = view_angle(B, A, Fv, a_i, n_i, d, dd);
            double m1 = view_angle(A, B, E, a_i, n_i, d, dd), m2 = view_angle(A, B, Fv, a_i, n_i, d, dd);
            o[0] = fmin(w1, w2);
            o[1] = fmax(w1, w2);
            o[2] = fmin(m1, m2);
            o[3] = fmax(m1, m2);
        }
        base += (int64_t)total;
    }
}

}  // namespace

hipError_t launch_angle_offsets(const SceneDev &sc, const uint64_t *M, int64_t *offsets, hipStream_t s) {
    hipLaunchKernelGGL(k_angle_counts, dim3((unsigned)((sc.F + 3) / 4)), dim3(256), 0, s, sc.F, sc.W, M, offsets);
    hipLaunchKernelGGL(k_angle_scan, dim3(1), dim3(kScanT), 0, s, offsets, sc.F);
    return hipGetLastError();
}

hipError_t launch_angles(const SceneDev &sc, const uint64_t *M, const int64_t *offsets, int32_t *cols,
                         double *ranges, hipStream_t s) {
    hipLaunchKernelGGL(k_angles, dim3((unsigned)((sc.F + 3) / 4)), dim3(256), 0, s, sc, M, offsets, cols, ranges);
    return hipGetLastError();
}

}  // namespace ivm
