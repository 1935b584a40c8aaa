// paths.hip -- exact image-method validation of the image-tree candidates.
//
// A candidate walk f1 -> ... -> fk is a specular path from T to R (Section
// III-A: the image method; Section III-B: the image tree the table prunes;
// Section IV-B: the pruned tree yields the same valid rays) when
//   * T mirrored successively in the planes of f1, ..., fk gives images
//     I1, ..., Ik, and tracing back from R, with target = R at first: for
//     m = k .. 1 the target lies strictly in front of f_m's plane and I_m
//     strictly behind it, and the point P_m where the segment (target, I_m)
//     meets the plane lies in the closed facet f_m (in one of its triangles);
//     then target = P_m;
//   * every leg T -> P_1 -> ... -> P_k -> R misses (open segment, closed
//     triangles) every triangle outside the facets at the leg's two ends.
//
// The points are rational.  They are carried as homogeneous integer vectors
// (X, W), W > 0, in sample-grid units, with 512-bit two's complement integers;
// reflection in the plane (a, n), n the facet's first-triangle normal divided
// by the gcd of its components:
//   X' = X (n.n) - 2 ((X - a W).n) n,  W' = W (n.n);
// the plane point between target (Xt, Wt) in front and image (Xi, Wi) behind,
// with alpha = (Xt - a Wt).n > 0 and beta = (Xi - a Wi).n < 0:
//   P = (alpha Xi - beta Xt,  alpha Wi - beta Wt).
// Every decision is a sign of such an integer expression, so it is exact; a
// product that could leave 512 bits marks the walk undecided and raises a
// status bit (the entry point reports IVM_ERR_GRID).
//
// A leg is tested against the triangles of the BVH leaves whose boxes, widened
// by an absolute margin, its FP64 approximation crosses (a superset of those
// the exact leg meets).  Each segment/triangle test first runs in FP64 on the
// approximate end points with an error bound covering their perturbation and
// the rounding of the test; a comparison within the bound sends the test to
// the exact integer form:
//   D = Xq Wp - Xp Wq, S = Xp - a Wp, h = D x e2, det' = e1.h, u' = S.h,
//   g = S x e1, v' = D.g, t' = e2.g;
//   hit iff det' > 0 and u' >= 0, v' >= 0, u' + v' <= det' Wp, 0 < t', t' Wq < det'
//   (mirrored for det' < 0), which is the division-free Moller-Trumbore test of
//   the segment (Xp / Wp, Xq / Wq) scaled by positive factors.
#include "ivm_internal.h"

namespace ivm {
namespace {

constexpr int kL = 8;  // 64-bit limbs per integer (512 bits)
constexpr int kMaxOrder = 4;

struct BigI {
    uint64_t w[kL];
};

__device__ inline BigI bi_from(long long v) {
    BigI r;
    r.w[0] = (uint64_t)v;
    const uint64_t ext = v < 0 ? ~0ull : 0ull;
    for (int k = 1; k < kL; ++k) r.w[k] = ext;
    return r;
}

__device__ inline BigI bi_from128(__int128 v) {
    BigI r;
    r.w[0] = (uint64_t)v;
    r.w[1] = (uint64_t)((unsigned __int128)v >> 64);
    const uint64_t ext = v < 0 ? ~0ull : 0ull;
    for (int k = 2; k < kL; ++k) r.w[k] = ext;
    return r;
}

__device__ inline bool bi_isneg(const BigI &a) { return (long long)a.w[kL - 1] < 0; }

__device__ inline bool bi_iszero(const BigI &a) {
    uint64_t o = 0;
    for (int k = 0; k < kL; ++k) o |= a.w[k];
    return o == 0;
}

__device__ inline int bi_sign(const BigI &a) { return bi_isneg(a) ? -1 : (bi_iszero(a) ? 0 : 1); }

__device__ inline BigI bi_add(const BigI &a, const BigI &b) {
    BigI r;
    uint64_t c = 0;
    for (int k = 0; k < kL; ++k) {
        const uint64_t s = a.w[k] + c;
        const uint64_t c1 = s < c;
        r.w[k] = s + b.w[k];
        c = c1 + (r.w[k] < s);
    }
    return r;
}

__device__ inline BigI bi_neg(const BigI &a) {
    BigI r;
    uint64_t c = 1;
    for (int k = 0; k < kL; ++k) {
        r.w[k] = ~a.w[k] + c;
        c = (c && r.w[k] == 0) ? 1 : 0;
    }
    return r;
}

__device__ inline BigI bi_sub(const BigI &a, const BigI &b) { return bi_add(a, bi_neg(b)); }

__device__ inline int bi_bitlen_mag(const BigI &m) {  // of a non-negative value
    for (int k = kL - 1; k >= 0; --k)
        if (m.w[k]) return 64 * k + 64 - __clzll((long long)m.w[k]);
    return 0;
}

// a * b; sets *ovf when |a| |b| could reach 2^(64 kL - 8) (sums of up to 2^6
// such products then still fit).
__device__ inline BigI bi_mul(const BigI &a, const BigI &b, bool *ovf) {
    const bool na = bi_isneg(a), nb = bi_isneg(b);
    const BigI A = na ? bi_neg(a) : a, B = nb ? bi_neg(b) : b;
    const int la = bi_bitlen_mag(A), lb = bi_bitlen_mag(B);
    BigI r;
    for (int k = 0; k < kL; ++k) r.w[k] = 0;
    if (la == 0 || lb == 0) return r;
    if (la + lb > 64 * kL - 8) {  // products stay below 2^504, so sums of a few stay in range
        *ovf = true;
        return r;
    }
    const int ka = (la + 63) >> 6, kb = (lb + 63) >> 6;
    for (int i = 0; i < ka; ++i) {
        uint64_t carry = 0;
        for (int j = 0; j < kb && i + j < kL; ++j) {
            const uint64_t lo = A.w[i] * B.w[j], hi = __umul64hi(A.w[i], B.w[j]);
            uint64_t s = r.w[i + j] + lo;
            uint64_t c = s < lo;
            s += carry;
            c += s < carry;
            r.w[i + j] = s;
            carry = hi + c;
        }
        if (i + kb < kL) r.w[i + kb] += carry;
    }
    return (na != nb) ? bi_neg(r) : r;
}

__device__ inline double bi_to_double(const BigI &a) {
    const bool n = bi_isneg(a);
    const BigI m = n ? bi_neg(a) : a;
    int top = kL - 1;
    while (top > 0 && m.w[top] == 0) --top;
    double v = (double)m.w[top];
    if (top >= 1) v = fma(v, 18446744073709551616.0, (double)m.w[top - 1]);
    if (top >= 2) v = fma(v, 18446744073709551616.0, (double)m.w[top - 2]);
    const int shift = 64 * (top >= 2 ? top - 2 : 0);
    v = ldexp(v, shift);
    return n ? -v : v;
}

struct HP {  // homogeneous point (x / w, y / w, z / w), w > 0
    BigI x, y, z, w;
};

struct I3 {
    long long x, y, z;
};

__device__ inline long long gcd_ll(long long a, long long b) {
    a = a < 0 ? -a : a;
    b = b < 0 ? -b : b;
    while (b) {
        const long long t = a % b;
        a = b;
        b = t;
    }
    return a;
}

__device__ inline I3 reduce(I3 n) {
    long long g = gcd_ll(gcd_ll(n.x, n.y), n.z);
    if (g > 1) {
        n.x /= g;
        n.y /= g;
        n.z /= g;
    }
    return n;
}

__device__ inline I3 cross_ll(I3 a, I3 b) {
    return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}

// Sample-grid integer of a float coordinate (exact: |x| 2^gs < 2^24 on the grid).
__device__ inline long long sgrid(float v, float su) { return (long long)(v * su); }

// Vertex m of caller triangle t in sample units.
__device__ inline I3 tri_vertex_s(const SceneDev &sc, int t, int m, float su) {
    const float4 a = sc.tri_caller[3 * (size_t)t];
    float x = a.x, y = a.y, z = a.z;
    if (m > 0) {
        const float4 e = sc.tri_caller[3 * (size_t)t + m];
        x += e.x;
        y += e.y;
        z += e.z;
    }
    return {sgrid(x, su), sgrid(y, su), sgrid(z, su)};
}

// Plane point and reduced normal of facet f.
__device__ inline void facet_plane(const SceneDev &sc, int f, float su, I3 &a, I3 &n) {
    const int t = sc.ftri[2 * f];
    a = tri_vertex_s(sc, t, 0, su);
    const I3 b = tri_vertex_s(sc, t, 1, su), c = tri_vertex_s(sc, t, 2, su);
    n = reduce(cross_ll({b.x - a.x, b.y - a.y, b.z - a.z}, {c.x - a.x, c.y - a.y, c.z - a.z}));
}

// (X - a W) . n
__device__ inline BigI plane_value(const HP &P, I3 a, I3 n, bool *ovf) {
    const BigI sx = bi_sub(P.x, bi_mul(P.w, bi_from(a.x), ovf));
    const BigI sy = bi_sub(P.y, bi_mul(P.w, bi_from(a.y), ovf));
    const BigI sz = bi_sub(P.z, bi_mul(P.w, bi_from(a.z), ovf));
    return bi_add(bi_add(bi_mul(sx, bi_from(n.x), ovf), bi_mul(sy, bi_from(n.y), ovf)), bi_mul(sz, bi_from(n.z), ovf));
}

__device__ inline HP reflect(const HP &P, I3 a, I3 n, bool *ovf) {
    const BigI nn = bi_from128((__int128)n.x * n.x + (__int128)n.y * n.y + (__int128)n.z * n.z);
    const BigI k1 = plane_value(P, a, n, ovf);
    const BigI k2 = bi_add(k1, k1);  // 2 (X - aW).n
    HP r;
    r.x = bi_sub(bi_mul(P.x, nn, ovf), bi_mul(k2, bi_from(n.x), ovf));
    r.y = bi_sub(bi_mul(P.y, nn, ovf), bi_mul(k2, bi_from(n.y), ovf));
    r.z = bi_sub(bi_mul(P.z, nn, ovf), bi_mul(k2, bi_from(n.z), ovf));
    r.w = bi_mul(P.w, nn, ovf);
    return r;
}

// (X - v W) . m with m given as 128-bit components.
__device__ inline BigI rel_dot(const HP &P, I3 v, __int128 mx, __int128 my, __int128 mz, bool *ovf) {
    const BigI sx = bi_sub(P.x, bi_mul(P.w, bi_from(v.x), ovf));
    const BigI sy = bi_sub(P.y, bi_mul(P.w, bi_from(v.y), ovf));
    const BigI sz = bi_sub(P.z, bi_mul(P.w, bi_from(v.z), ovf));
    return bi_add(bi_add(bi_mul(sx, bi_from128(mx), ovf), bi_mul(sy, bi_from128(my), ovf)),
                  bi_mul(sz, bi_from128(mz), ovf));
}

// P in the closed facet f: in one of its triangles (edge tests against the
// triangle's own normal, as (b - a) x (P - a) . n_t >= 0 = (P - a) . (n_t x (b - a))).
__device__ inline bool in_facet(const SceneDev &sc, const HP &P, int f, float su, bool *ovf) {
    const int t0 = sc.ftri[2 * f], nt = sc.ftri[2 * f + 1];
    for (int t = t0; t < t0 + nt; ++t) {
        const I3 a = tri_vertex_s(sc, t, 0, su), b = tri_vertex_s(sc, t, 1, su), c = tri_vertex_s(sc, t, 2, su);
        const I3 nt3 = reduce(cross_ll({b.x - a.x, b.y - a.y, b.z - a.z}, {c.x - a.x, c.y - a.y, c.z - a.z}));
        const I3 ed[3] = {{b.x - a.x, b.y - a.y, b.z - a.z}, {c.x - b.x, c.y - b.y, c.z - b.z},
                          {a.x - c.x, a.y - c.y, a.z - c.z}};
        const I3 base[3] = {a, b, c};
        bool inside = true;
        for (int k = 0; k < 3 && inside; ++k) {
            const __int128 mx = (__int128)nt3.y * ed[k].z - (__int128)nt3.z * ed[k].y;
            const __int128 my = (__int128)nt3.z * ed[k].x - (__int128)nt3.x * ed[k].z;
            const __int128 mz = (__int128)nt3.x * ed[k].y - (__int128)nt3.y * ed[k].x;
            inside = bi_sign(rel_dot(P, base[k], mx, my, mz, ovf)) >= 0;
        }
        if (inside) return true;
    }
    return false;
}

struct DPt {
    double x, y, z;
};

__device__ inline DPt approx(const HP &P) {
    const double w = bi_to_double(P.w);
    return {bi_to_double(P.x) / w, bi_to_double(P.y) / w, bi_to_double(P.z) / w};
}

// Exact segment/triangle test of the leg (P, Q) against the triangle with
// corner A and edges E1, E2 (sample units).
__device__ bool segtri_exact(const HP &P, const HP &Q, I3 A, I3 E1, I3 E2, bool *ovf) {
    const BigI Dx = bi_sub(bi_mul(Q.x, P.w, ovf), bi_mul(P.x, Q.w, ovf));
    const BigI Dy = bi_sub(bi_mul(Q.y, P.w, ovf), bi_mul(P.y, Q.w, ovf));
    const BigI Dz = bi_sub(bi_mul(Q.z, P.w, ovf), bi_mul(P.z, Q.w, ovf));
    const BigI Sx = bi_sub(P.x, bi_mul(P.w, bi_from(A.x), ovf));
    const BigI Sy = bi_sub(P.y, bi_mul(P.w, bi_from(A.y), ovf));
    const BigI Sz = bi_sub(P.z, bi_mul(P.w, bi_from(A.z), ovf));
    const BigI e1x = bi_from(E1.x), e1y = bi_from(E1.y), e1z = bi_from(E1.z);
    const BigI e2x = bi_from(E2.x), e2y = bi_from(E2.y), e2z = bi_from(E2.z);
    // h = D x e2
    const BigI hx = bi_sub(bi_mul(Dy, e2z, ovf), bi_mul(Dz, e2y, ovf));
    const BigI hy = bi_sub(bi_mul(Dz, e2x, ovf), bi_mul(Dx, e2z, ovf));
    const BigI hz = bi_sub(bi_mul(Dx, e2y, ovf), bi_mul(Dy, e2x, ovf));
    const BigI det = bi_add(bi_add(bi_mul(e1x, hx, ovf), bi_mul(e1y, hy, ovf)), bi_mul(e1z, hz, ovf));
    const int sd = bi_sign(det);
    if (sd == 0) return false;
    const BigI u = bi_add(bi_add(bi_mul(Sx, hx, ovf), bi_mul(Sy, hy, ovf)), bi_mul(Sz, hz, ovf));
    // g = S x e1
    const BigI gx = bi_sub(bi_mul(Sy, e1z, ovf), bi_mul(Sz, e1y, ovf));
    const BigI gy = bi_sub(bi_mul(Sz, e1x, ovf), bi_mul(Sx, e1z, ovf));
    const BigI gz = bi_sub(bi_mul(Sx, e1y, ovf), bi_mul(Sy, e1x, ovf));
    const BigI v = bi_add(bi_add(bi_mul(Dx, gx, ovf), bi_mul(Dy, gy, ovf)), bi_mul(Dz, gz, ovf));
    const BigI t = bi_add(bi_add(bi_mul(e2x, gx, ovf), bi_mul(e2y, gy, ovf)), bi_mul(e2z, gz, ovf));
    const BigI detw = bi_mul(det, P.w, ovf), tw = bi_mul(t, Q.w, ovf);
    const BigI uv = bi_add(u, v);
    if (sd > 0)
        return bi_sign(u) >= 0 && bi_sign(v) >= 0 && bi_sign(bi_sub(detw, uv)) >= 0 && bi_sign(t) > 0 &&
               bi_sign(bi_sub(det, tw)) > 0;
    return bi_sign(u) <= 0 && bi_sign(v) <= 0 && bi_sign(bi_sub(uv, detw)) >= 0 && bi_sign(t) < 0 &&
           bi_sign(bi_sub(tw, det)) > 0;
}

// FP64 test on the approximate end points (error per coordinate <= err), then
// the exact one when a comparison falls within the error bound.
__device__ bool segtri_leg(const HP &P, const HP &Q, DPt p, DPt q, double err, I3 A, I3 E1, I3 E2, bool *ovf,
                           unsigned &exact) {
#pragma clang fp contract(off)
    const double dx = q.x - p.x, dy = q.y - p.y, dz = q.z - p.z;
    const double sx = p.x - (double)A.x, sy = p.y - (double)A.y, sz = p.z - (double)A.z;
    const double ex = (double)E1.x, ey = (double)E1.y, ez = (double)E1.z;
    const double fx = (double)E2.x, fy = (double)E2.y, fz = (double)E2.z;
    const double hx = dy * fz - dz * fy, hy = dz * fx - dx * fz, hz = dx * fy - dy * fx;
    const double det = ex * hx + ey * hy + ez * hz;
    const double u = sx * hx + sy * hy + sz * hz;
    const double gx = sy * ez - sz * ey, gy = sz * ex - sx * ez, gz = sx * ey - sy * ex;
    const double v = dx * gx + dy * gy + dz * gz;
    const double t = fx * gx + fy * gy + fz * gz;
    // magnitudes and error bounds: perturbations (d by 2 err, s by err) plus
    // rounding (kappa of each term's magnitude)
    const double D = fmax(fabs(dx), fmax(fabs(dy), fabs(dz))), S = fmax(fabs(sx), fmax(fabs(sy), fabs(sz)));
    const double e1m = fmax(fabs(ex), fmax(fabs(ey), fabs(ez))), e2m = fmax(fabs(fx), fmax(fabs(fy), fabs(fz)));
    const double kappa = 0x1p-46, dd = 2.0 * err, ds = err;
    const double b_det = 6.0 * e1m * e2m * (dd + kappa * D);
    const double b_u = 6.0 * e2m * (S * dd + D * ds + dd * ds + kappa * S * D);
    const double b_v = 6.0 * e1m * (S * dd + D * ds + dd * ds + kappa * S * D);
    const double b_t = 6.0 * e1m * e2m * (ds + kappa * S);
    const double sg = det > 0.0 ? 1.0 : -1.0;
    const double w = sg * det - sg * u - sg * v, x = sg * det - sg * t;
    const double b_w = 2.0 * (b_det + b_u + b_v), b_x = 2.0 * (b_det + b_t);
    if (fabs(det) > 2.0 * b_det) {
        // a definite miss on any one comparison, or a definite hit on all
        if (sg * u < -2.0 * b_u || sg * v < -2.0 * b_v || w < -b_w || sg * t < -2.0 * b_t || x < -b_x) return false;
        if (sg * u > 2.0 * b_u && sg * v > 2.0 * b_v && w > b_w && sg * t > 2.0 * b_t && x > b_x) return true;
    }
    ++exact;
    return segtri_exact(P, Q, A, E1, E2, ovf);
}

constexpr int kPathStack = 32;

// Conservative slab test of the FP64 leg against a box widened by `pad`.
__device__ inline bool leg_box(DPt p, DPt q, const float *lo, const float *hi, double pad) {
    double t0 = 0.0, t1 = 1.0;
    const double P[3] = {p.x, p.y, p.z}, Q[3] = {q.x, q.y, q.z};
    for (int k = 0; k < 3; ++k) {
        const double l = (double)lo[k] - pad, h = (double)hi[k] + pad, d = Q[k] - P[k];
        if (fabs(d) < 1e-300) {
            if (P[k] < l || P[k] > h) return false;
            continue;
        }
        double a = (l - P[k]) / d, b = (h - P[k]) / d;
        if (a > b) {
            const double s = a;
            a = b;
            b = s;
        }
        t0 = fmax(t0, a);
        t1 = fmin(t1, b);
    }
    return t0 <= t1 + 1e-9;
}

// Is the open leg (P, Q) clear of every triangle outside facets exA, exB?
__device__ bool leg_clear(const SceneDev &sc, const HP &P, const HP &Q, int exA, int exB, float su, bool *ovf,
                          unsigned &tests, unsigned &exact) {
    DPt p = approx(P), q = approx(Q);
    // metres -> sample units for the tests; boxes stay in metres
    const double C = fmax(fmax(fabs(p.x), fabs(p.y)), fmax(fmax(fabs(p.z), fabs(q.x)), fmax(fabs(q.y), fabs(q.z))));
    const double err = 0x1p-48 * C + 1e-300;  // per-coordinate error of the approximations (sample units)
    const double inv = 1.0 / (double)su;
    const DPt pm = {p.x * inv, p.y * inv, p.z * inv}, qm = {q.x * inv, q.y * inv, q.z * inv};
    const double pad = (err + 0x1p-40 * C) * inv;
    int stk[kPathStack];
    for (int k = 0; k < kTreelets; ++k) {
        const int root = sc.tl_root[k];
        if (root == 0x7fffffff) continue;
        if (!leg_box(pm, qm, sc.tl_box + 6 * k, sc.tl_box + 6 * k + 3, pad)) continue;
        int sp = 0;
        int ref = root;
        while (true) {
            if (ref < 0) {  // leaf: its triangles
                const int first = leaf_first(ref), cnt = leaf_count(ref);
                for (int r = first; r < first + cnt; ++r) {
                    const float4 A = sc.tri[3 * r];
                    const int f = __float_as_int(A.w);
                    if (f == exA || f == exB) continue;
                    const float4 B = sc.tri[3 * r + 1], Cc = sc.tri[3 * r + 2];
                    ++tests;
                    if (segtri_leg(P, Q, p, q, err, {sgrid(A.x, su), sgrid(A.y, su), sgrid(A.z, su)},
                                   {sgrid(B.x, su), sgrid(B.y, su), sgrid(B.z, su)},
                                   {sgrid(Cc.x, su), sgrid(Cc.y, su), sgrid(Cc.z, su)}, ovf, exact))
                        return false;
                }
                if (sp == 0) break;
                ref = stk[--sp];
                continue;
            }
            const Node nd = sc.nodes[ref];
            const float l0[3] = {nd.a.x, nd.a.y, nd.a.z}, h0[3] = {nd.a.w, nd.b.x, nd.b.y};
            const float l1[3] = {nd.b.z, nd.b.w, nd.c.x}, h1[3] = {nd.c.y, nd.c.z, nd.c.w};
            const bool b0 = leg_box(pm, qm, l0, h0, pad), b1 = leg_box(pm, qm, l1, h1, pad);
            if (b0 && b1) {
                if (sp < kPathStack) {
                    stk[sp++] = nd.d.y;
                } else {  // full stack: the far subtree's triangles one by one
                    int first, count;
                    if (nd.d.y < 0) {
                        first = leaf_first(nd.d.y);
                        count = leaf_count(nd.d.y);
                    } else {
                        const int4 rg = sc.nodes[nd.d.y].d;
                        first = rg.z;
                        count = rg.w - rg.z + 1;
                    }
                    for (int r = first; r < first + count; ++r) {
                        const float4 A = sc.tri[3 * r];
                        const int f = __float_as_int(A.w);
                        if (f == exA || f == exB) continue;
                        const float4 B = sc.tri[3 * r + 1], Cc = sc.tri[3 * r + 2];
                        ++tests;
                        if (segtri_leg(P, Q, p, q, err, {sgrid(A.x, su), sgrid(A.y, su), sgrid(A.z, su)},
                                       {sgrid(B.x, su), sgrid(B.y, su), sgrid(B.z, su)},
                                       {sgrid(Cc.x, su), sgrid(Cc.y, su), sgrid(Cc.z, su)}, ovf, exact))
                            return false;
                    }
                }
                ref = nd.d.x;
            } else if (b0) {
                ref = nd.d.x;
            } else if (b1) {
                ref = nd.d.y;
            } else {
                if (sp == 0) break;
                ref = stk[--sp];
            }
        }
    }
    return true;
}

__device__ inline HP hp_point(const float *x, float su) {
    HP r;
    r.x = bi_from(sgrid(x[0], su));
    r.y = bi_from(sgrid(x[1], su));
    r.z = bi_from(sgrid(x[2], su));
    r.w = bi_from(1);
    return r;
}

// 1 valid, 0 not, 2 undecided (a product left the integer range).
__device__ int validate_walk(const SceneDev &sc, const float *T, const float *R, const int *walk, int k,
                             unsigned &tests, unsigned &exact) {
    const float su = (float)(1 << sc.gs);
    bool ovf = false;
    HP img[kMaxOrder + 1];
    I3 pa[kMaxOrder], pn[kMaxOrder];
    img[0] = hp_point(T, su);
    for (int m = 0; m < k; ++m) {
        facet_plane(sc, walk[m], su, pa[m], pn[m]);
        img[m + 1] = reflect(img[m], pa[m], pn[m], &ovf);
    }
    HP pts[kMaxOrder];
    HP target = hp_point(R, su);
    for (int m = k - 1; m >= 0; --m) {
        const HP &I = img[m + 1];
        const BigI alpha = plane_value(target, pa[m], pn[m], &ovf);
        const BigI beta = plane_value(I, pa[m], pn[m], &ovf);
        if (ovf) return 2;
        if (!(bi_sign(alpha) > 0 && bi_sign(beta) < 0)) return 0;
        HP P;
        P.x = bi_sub(bi_mul(alpha, I.x, &ovf), bi_mul(beta, target.x, &ovf));
        P.y = bi_sub(bi_mul(alpha, I.y, &ovf), bi_mul(beta, target.y, &ovf));
        P.z = bi_sub(bi_mul(alpha, I.z, &ovf), bi_mul(beta, target.z, &ovf));
        P.w = bi_sub(bi_mul(alpha, I.w, &ovf), bi_mul(beta, target.w, &ovf));
        const bool inside = in_facet(sc, P, walk[m], su, &ovf);
        if (ovf) return 2;
        if (!inside) return 0;
        pts[m] = P;
        target = P;
    }
    // legs T -> P_1 -> ... -> P_k -> R, each clear of triangles outside its end facets
    for (int m = 0; m <= k; ++m) {
        const HP A = m == 0 ? hp_point(T, su) : pts[m - 1];
        const HP B = m == k ? hp_point(R, su) : pts[m];
        const int exA = m == 0 ? -1 : walk[m - 1], exB = m == k ? -1 : walk[m];
        const bool clear = leg_clear(sc, A, B, exA, exB, su, &ovf, tests, exact);
        if (ovf) return 2;
        if (!clear) return 0;
    }
    return 1;
}

// One thread per int32 element of the lists; the thread at the first element
// of a k-tuple validates that walk and writes its verdict to all k elements.
__global__ __launch_bounds__(128) void k_validate(SceneDev sc, int N, int K, const float *tx, const float *rx,
                                                  const int64_t *offsets, const int32_t *paths, long long n_elems,
                                                  uint8_t *valid, int64_t *valid_counts, unsigned long long *stats) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    unsigned tests = 0, exact = 0;
    if (e < n_elems) {
        // list (n, k) holding element e: the last list start <= e (lists may be empty)
        int lo = 0, hi = N * K - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (offsets[mid] <= e) lo = mid;
            else hi = mid - 1;
        }
        const int n = lo / K, k = lo % K + 1;
        const long long rel = e - offsets[lo];
        if (rel % k == 0) {
            int walk[kMaxOrder];
            bool ok_ids = true;
            for (int m = 0; m < k; ++m) {
                walk[m] = paths[e + m];
                ok_ids &= walk[m] >= 0 && walk[m] < sc.F && (m == 0 || walk[m] != walk[m - 1]);
            }
            int v = 0;
            if (ok_ids) v = validate_walk(sc, tx + 3 * (size_t)n, rx + 3 * (size_t)n, walk, k, tests, exact);
            else atomicOr(sc.status, kStInvalid);
            if (v == 2) atomicOr(sc.status, kStPathRange);
            for (int m = 0; m < k; ++m) valid[e + m] = (uint8_t)v;
            if (v == 1 && valid_counts) atomicAdd((unsigned long long *)&valid_counts[(size_t)n * K + k - 1], 1ull);
        }
    }
    if (stats) {
        if (tests) atomicAdd(&stats[0], (unsigned long long)tests);
        if (exact) atomicAdd(&stats[1], (unsigned long long)exact);
    }
}

// Tx / Rx positions on the sample grid (so their integers are exact).
__global__ void k_check_positions(int N, const float *tx, const float *rx, float su, int *status) {
    const int id = blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= 6 * N) return;
    const float v = (id < 3 * N ? tx[id] : rx[id - 3 * N]) * su;
    if (!(fabsf(v) < 16777216.0f) || v != floorf(v)) atomicOr(status, kStGrid);
}

}  // namespace

hipError_t launch_validate_paths(const SceneDev &sc, int N, int K, const float *tx, const float *rx,
                                 const int64_t *offsets, const int32_t *paths, long long n_elems, uint8_t *valid,
                                 int64_t *valid_counts, unsigned long long *stats, hipStream_t s) {
    if (valid_counts) {
        hipError_t e = launch_fill_u64((uint64_t *)valid_counts, 0ull, (size_t)N * K, s);
        if (e != hipSuccess) return e;
    }
    if (N > 0)
        hipLaunchKernelGGL(k_check_positions, dim3((unsigned)((6 * N + 255) / 256)), dim3(256), 0, s, N, tx, rx,
                           (float)(1 << sc.gs), sc.status);
    if (n_elems <= 0) return hipGetLastError();
    hipLaunchKernelGGL(k_validate, dim3((unsigned)((n_elems + 127) / 128)), dim3(128), 0, s, sc, N, K, tx, rx,
                       offsets, paths, n_elems, valid, valid_counts, stats);
    return hipGetLastError();
}

}  // namespace ivm
