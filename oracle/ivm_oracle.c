/*
 * ivm_oracle.c -- plain FP64 brute-force oracle for facet inter-visibility.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the bench's
 * CPU-baseline leg may load this library.  It shares no code, header or
 * constant with the GPU library and must never be used as a fallback for it.
 *
 * What it computes (the paper's pre-processing, Sections II-B and III-B, read
 * as an exact 3-D decision over deterministic per-facet sample points):
 *
 *   orient(i, x)  = (x - a_i) . ((b_i - a_i) x (c_i - a_i)), with (a_i, b_i, c_i)
 *                   the first triangle of facet i.  Positive = the visible side
 *                   (Section II-B, eq. 2: only the side facing away from the
 *                   building is visible; rays never leave a face's back side).
 *   admissible(p in S_i, q in S_j)  iff  orient(i, q) > 0 and orient(j, p) > 0.
 *   segtri(p, q, t): open segment (p, q) meets closed triangle t transversally
 *                   (Moller-Trumbore 1997, division-free form).
 *   clear(p, q; i, j) iff no triangle outside facets i and j meets (p, q)
 *                   (Section II-B: reference and aim face see each other only
 *                   when no other obstacle lies between; a third face blocks).
 *   M[i][j] = exists admissible clear (p, q); M[i][i] = 0.
 *   vis_X(f) = orient(f, X) > 0 and exists p in S_f with (X, p) clear of every
 *                   triangle outside f (Section III-B, Table II: the transmitter
 *                   searches its visible reference faces).
 *   LoS(T, R) = (T, R) clear of every triangle.
 *
 * Every coordinate lies on a dyadic grid that keeps these degree-3 polynomials
 * exact in FP64, so this file computes the exact predicate; ivo_exact_audit()
 * re-evaluates them in 128-bit integers to prove it on given inputs.
 *
 * Build: gcc -O3 -ffp-contract=off -fopenmp -shared -fPIC (no fast-math).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int F, T, S;
    double *ta, *tb, *tc;     /* triangle vertices, T x 3 each */
    int *tfacet;              /* T */
    int *soff;                /* F + 1 */
    double *smp;              /* S x 3 */
    double *fa, *fn;          /* facet plane: point a_i and normal n_i, F x 3 */
} ivo_scene;

static void sub3(const double *x, const double *y, double *r) {
    r[0] = x[0] - y[0]; r[1] = x[1] - y[1]; r[2] = x[2] - y[2];
}
static void cross3(const double *x, const double *y, double *r) {
    r[0] = x[1] * y[2] - x[2] * y[1];
    r[1] = x[2] * y[0] - x[0] * y[2];
    r[2] = x[0] * y[1] - x[1] * y[0];
}
static double dot3(const double *x, const double *y) {
    return x[0] * y[0] + x[1] * y[1] + x[2] * y[2];
}

/* ---- scene setup ------------------------------------------------------- */

ivo_scene *ivo_create(int F, int T, int S, const float *vertices, const int32_t *tri_vertices,
                      const int32_t *tri_facet, const int32_t *sample_offsets, const float *samples) {
    ivo_scene *s = (ivo_scene *)calloc(1, sizeof(ivo_scene));
    s->F = F; s->T = T; s->S = S;
    s->ta = (double *)malloc(sizeof(double) * 3 * (size_t)(T > 0 ? T : 1));
    s->tb = (double *)malloc(sizeof(double) * 3 * (size_t)(T > 0 ? T : 1));
    s->tc = (double *)malloc(sizeof(double) * 3 * (size_t)(T > 0 ? T : 1));
    s->tfacet = (int *)malloc(sizeof(int) * (size_t)(T > 0 ? T : 1));
    s->soff = (int *)malloc(sizeof(int) * (size_t)(F + 1));
    s->smp = (double *)malloc(sizeof(double) * 3 * (size_t)(S > 0 ? S : 1));
    s->fa = (double *)calloc(3 * (size_t)(F > 0 ? F : 1), sizeof(double));
    s->fn = (double *)calloc(3 * (size_t)(F > 0 ? F : 1), sizeof(double));
    for (int t = 0; t < T; ++t) {
        for (int c = 0; c < 3; ++c) {
            s->ta[3 * t + c] = (double)vertices[3 * tri_vertices[3 * t + 0] + c];
            s->tb[3 * t + c] = (double)vertices[3 * tri_vertices[3 * t + 1] + c];
            s->tc[3 * t + c] = (double)vertices[3 * tri_vertices[3 * t + 2] + c];
        }
        s->tfacet[t] = tri_facet[t];
    }
    for (int f = 0; f <= F; ++f) s->soff[f] = sample_offsets[f];
    for (int i = 0; i < 3 * S; ++i) s->smp[i] = (double)samples[i];
    /* facet plane from its first triangle (the lowest triangle index tagged f) */
    int *seen = (int *)calloc((size_t)(F > 0 ? F : 1), sizeof(int));
    for (int t = 0; t < T; ++t) {
        int f = tri_facet[t];
        if (f < 0 || f >= F || seen[f]) continue;
        seen[f] = 1;
        double e1[3], e2[3];
        sub3(&s->tb[3 * t], &s->ta[3 * t], e1);
        sub3(&s->tc[3 * t], &s->ta[3 * t], e2);
        cross3(e1, e2, &s->fn[3 * f]);
        memcpy(&s->fa[3 * f], &s->ta[3 * t], 3 * sizeof(double));
    }
    free(seen);
    return s;
}

void ivo_free(ivo_scene *s) {
    if (!s) return;
    free(s->ta); free(s->tb); free(s->tc); free(s->tfacet); free(s->soff); free(s->smp);
    free(s->fa); free(s->fn); free(s);
}

/* ---- predicates ---------------------------------------------------------- */

/* Open segment (p, q) against closed triangle (a, b, c), Moller-Trumbore without
 * division: with d = q - p, e1 = b - a, e2 = c - a, s = p - a,
 *   det = e1.(d x e2), u = s.(d x e2), v = d.(s x e1), t = e2.(s x e1);
 * a hit needs det != 0 (a segment parallel to the plane never hits), and after
 * normalising by the sign of det: u >= 0, v >= 0, u + v <= det, 0 < t < det. */
int ivo_segtri(const double *p, const double *q, const double *a, const double *b, const double *c) {
    double d[3], e1[3], e2[3], s[3], h[3], g[3];
    sub3(q, p, d);
    sub3(b, a, e1);
    sub3(c, a, e2);
    cross3(d, e2, h);
    double det = dot3(e1, h);
    if (det == 0.0) return 0;
    sub3(p, a, s);
    double u = dot3(s, h);
    cross3(s, e1, g);
    double v = dot3(d, g);
    double t = dot3(e2, g);
    if (det > 0.0)
        return u >= 0.0 && v >= 0.0 && u + v <= det && t > 0.0 && t < det;
    return u <= 0.0 && v <= 0.0 && u + v >= det && t < 0.0 && t > det;
}

double ivo_orient(const ivo_scene *s, int f, const double *x) {
    double r[3];
    sub3(x, &s->fa[3 * f], r);
    return dot3(r, &s->fn[3 * f]);
}

/* 1 iff the open segment (p, q) misses every triangle whose facet is neither ex1 nor ex2. */
int ivo_segment_clear(const ivo_scene *s, const double *p, const double *q, int ex1, int ex2) {
    for (int t = 0; t < s->T; ++t) {
        int f = s->tfacet[t];
        if (f == ex1 || f == ex2) continue;
        if (ivo_segtri(p, q, &s->ta[3 * t], &s->tb[3 * t], &s->tc[3 * t])) return 0;
    }
    return 1;
}

/* Directed pair: p runs over S_i (outer), q over S_j (inner). */
int ivo_pair_directed(const ivo_scene *s, int i, int j) {
    if (i == j) return 0;
    for (int a = s->soff[i]; a < s->soff[i + 1]; ++a) {
        const double *p = &s->smp[3 * a];
        if (!(ivo_orient(s, j, p) > 0.0)) continue;
        for (int b = s->soff[j]; b < s->soff[j + 1]; ++b) {
            const double *q = &s->smp[3 * b];
            if (!(ivo_orient(s, i, q) > 0.0)) continue;
            if (ivo_segment_clear(s, p, q, i, j)) return 1;
        }
    }
    return 0;
}

/* Canonical direction: p on the lower-numbered facet. */
int ivo_pair(const ivo_scene *s, int i, int j) {
    return i < j ? ivo_pair_directed(s, i, j) : ivo_pair_directed(s, j, i);
}

/* Full F x F byte matrix.  audit != 0 evaluates (j, i) independently as well and
 * returns the number of pairs whose two directions disagree. */
int64_t ivo_matrix(const ivo_scene *s, uint8_t *M, int audit, int nthreads) {
    int F = s->F;
    int64_t mismatches = 0;
    memset(M, 0, (size_t)F * (size_t)F);
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : mismatches)
    for (int i = 0; i < F; ++i) {
        for (int j = i + 1; j < F; ++j) {
            int r = ivo_pair_directed(s, i, j);
            M[(size_t)i * F + j] = (uint8_t)r;
            M[(size_t)j * F + i] = (uint8_t)r;
            if (audit && ivo_pair_directed(s, j, i) != r) mismatches++;
        }
    }
    return mismatches;
}

/* Selected pairs (I[k], J[k]) -> out[k]. */
void ivo_pairs(const ivo_scene *s, int n, const int32_t *I, const int32_t *J, uint8_t *out,
               int nthreads) {
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel for schedule(dynamic, 1)
    for (int k = 0; k < n; ++k) out[k] = (uint8_t)ivo_pair(s, I[k], J[k]);
}

/* Point-facet visibility: X sees facet f. */
int ivo_point_visible(const ivo_scene *s, const double *X, int f) {
    if (!(ivo_orient(s, f, X) > 0.0)) return 0;
    for (int a = s->soff[f]; a < s->soff[f + 1]; ++a)
        if (ivo_segment_clear(s, X, &s->smp[3 * a], f, -1)) return 1;
    return 0;
}

/* Per-snapshot table: tx_vis/rx_vis are N x F bytes, los N bytes. */
void ivo_txrx(const ivo_scene *s, int N, const float *tx, const float *rx, uint8_t *tx_vis,
              uint8_t *rx_vis, uint8_t *los, int nthreads) {
    int F = s->F;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel for schedule(dynamic, 1)
    for (int n = 0; n < N; ++n) {
        double T[3] = {tx[3 * n], tx[3 * n + 1], tx[3 * n + 2]};
        double R[3] = {rx[3 * n], rx[3 * n + 1], rx[3 * n + 2]};
        for (int f = 0; f < F; ++f) {
            tx_vis[(size_t)n * F + f] = (uint8_t)ivo_point_visible(s, T, f);
            rx_vis[(size_t)n * F + f] = (uint8_t)ivo_point_visible(s, R, f);
        }
        los[n] = (uint8_t)ivo_segment_clear(s, T, R, -1, -1);
    }
}

/* Selected (point, facet) entries: X is K x 3, out[k] = vis_{X_k}(f_k). */
void ivo_point_facets(const ivo_scene *s, int K, const float *X, const int32_t *f, uint8_t *out,
                      int nthreads) {
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel for schedule(dynamic, 4)
    for (int k = 0; k < K; ++k) {
        double P[3] = {X[3 * k], X[3 * k + 1], X[3 * k + 2]};
        out[k] = (uint8_t)ivo_point_visible(s, P, f[k]);
    }
}

/* LoS for K point pairs. */
void ivo_los(const ivo_scene *s, int K, const float *A, const float *B, uint8_t *out) {
    for (int k = 0; k < K; ++k) {
        double P[3] = {A[3 * k], A[3 * k + 1], A[3 * k + 2]};
        double Q[3] = {B[3 * k], B[3 * k + 1], B[3 * k + 2]};
        out[k] = (uint8_t)ivo_segment_clear(s, P, Q, -1, -1);
    }
}

/* All-hit occluder labels for a pair (i, j): bit m of the result is set iff some
 * triangle in group m (group_of_tri[t] in [0, 32)) meets at least one admissible
 * segment of the pair.  Used to label training records for the occluder ordering. */
uint32_t ivo_pair_occluder_groups(const ivo_scene *s, int i, int j, const int32_t *group_of_tri) {
    uint32_t mask = 0;
    int lo = i < j ? i : j, hi = i < j ? j : i;
    for (int a = s->soff[lo]; a < s->soff[lo + 1]; ++a) {
        const double *p = &s->smp[3 * a];
        if (!(ivo_orient(s, hi, p) > 0.0)) continue;
        for (int b = s->soff[hi]; b < s->soff[hi + 1]; ++b) {
            const double *q = &s->smp[3 * b];
            if (!(ivo_orient(s, lo, q) > 0.0)) continue;
            for (int t = 0; t < s->T; ++t) {
                int f = s->tfacet[t];
                if (f == lo || f == hi) continue;
                if (ivo_segtri(p, q, &s->ta[3 * t], &s->tb[3 * t], &s->tc[3 * t]))
                    mask |= 1u << group_of_tri[t];
            }
        }
    }
    return mask;
}

void ivo_pairs_occluder_groups(const ivo_scene *s, int n, const int32_t *I, const int32_t *J,
                               const int32_t *group_of_tri, uint32_t *out, int nthreads) {
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel for schedule(dynamic, 1)
    for (int k = 0; k < n; ++k) out[k] = ivo_pair_occluder_groups(s, I[k], J[k], group_of_tri);
}

/* ---- edge rows of the matrix ---------------------------------------------
 * Edges are visibility nodes beside faces (Sections I and II-A); the face seen
 * for diffraction is the face seen for reflection (Section III-B).  A node is a
 * facet (its samples, side facets {f}) or a building edge (its samples, side
 * facets {fa, fb}, fb = -1 for an edge of one facet).  A point x is on a node's
 * visible side when it is strictly in front of one of its side facets.  Nodes u
 * and v see each other when some sample p of u and q of v have q on u's visible
 * side, p on v's visible side, and the open segment (p, q) meets no triangle of
 * a facet outside the side facets of u and v.  For two facets this is the
 * matrix definition above. */

static int ivo_front_of(const ivo_scene *s, const int *side, const double *x) {
    for (int k = 0; k < 2; ++k)
        if (side[k] >= 0 && ivo_orient(s, side[k], x) > 0.0) return 1;
    return 0;
}

static int ivo_clear_ex4(const ivo_scene *s, const double *p, const double *q, const int *ex) {
    for (int t = 0; t < s->T; ++t) {
        int f = s->tfacet[t];
        if (f == ex[0] || f == ex[1] || f == ex[2] || f == ex[3]) continue;
        if (ivo_segtri(p, q, &s->ta[3 * t], &s->tb[3 * t], &s->tc[3 * t])) return 0;
    }
    return 1;
}

/* Node u (samples P[np], side facets su[2]) against node v (Q[nq], sv[2]). */
int ivo_node_pair(const ivo_scene *s, const double *P, int np, const int *su, const double *Q, int nq,
                  const int *sv) {
    const int ex[4] = {su[0], su[1], sv[0], sv[1]};
    for (int a = 0; a < np; ++a) {
        const double *p = &P[3 * a];
        if (!ivo_front_of(s, sv, p)) continue;
        for (int b = 0; b < nq; ++b) {
            const double *q = &Q[3 * b];
            if (!ivo_front_of(s, su, q)) continue;
            if (ivo_clear_ex4(s, p, q, ex)) return 1;
        }
    }
    return 0;
}

/* Rows of the edge part of the matrix for the edges rows[0..n): ef[k][f] for
 * every facet f and ee[k][e'] for every edge e' (0 on the diagonal).  Edge e
 * has facets efac[2e], efac[2e+1] and samples esmp[(e*se + j)*3 ..]. */
void ivo_edge_rows(const ivo_scene *s, int E, const int32_t *efac, const float *esmp, int se, int n,
                   const int32_t *rows, uint8_t *ef, uint8_t *ee, int nthreads) {
    double *ES = (double *)malloc(sizeof(double) * 3 * (size_t)(E * se > 0 ? E * se : 1));
    for (int k = 0; k < 3 * E * se; ++k) ES[k] = (double)esmp[k];
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel for schedule(dynamic, 1) collapse(2)
    for (int k = 0; k < n; ++k) {
        for (int c = 0; c < s->F + E; ++c) {
            const int e = rows[k];
            const int su[2] = {efac[2 * e], efac[2 * e + 1]};
            if (c < s->F) {
                const int sv[2] = {c, -1};
                ef[(size_t)k * s->F + c] = (uint8_t)ivo_node_pair(
                    s, &ES[3 * (size_t)e * se], se, su, &s->smp[3 * (size_t)s->soff[c]], s->soff[c + 1] - s->soff[c], sv);
            } else {
                const int e2 = c - s->F;
                const int sv[2] = {efac[2 * e2], efac[2 * e2 + 1]};
                ee[(size_t)k * E + e2] = e2 == e ? 0 : (uint8_t)ivo_node_pair(s, &ES[3 * (size_t)e * se], se, su,
                                                                              &ES[3 * (size_t)e2 * se], se, sv);
            }
        }
    }
    free(ES);
}

/* ---- exactness audit ------------------------------------------------------
 * Re-evaluates the segment/triangle predicate with 128-bit integers on the
 * sample grid (unit 2^-gs m) and compares every comparison with the FP64
 * evaluation above.  Returns the number of segment/triangle combinations whose
 * FP64 outcome for any of the comparisons differs from the exact one, or -1
 * if an input is off the grid. */
typedef __int128 i128;

static int to_grid(double x, double scale, int64_t *out) {
    double y = x * scale;
    if (y != floor(y) || fabs(y) > 9.0e15) return 0;
    *out = (int64_t)y;
    return 1;
}

static int sgn128(i128 x) { return (x > 0) - (x < 0); }
static int sgnd(double x) { return (x > 0.0) - (x < 0.0); }

int64_t ivo_exact_audit(int n, const float *P, const float *Q, const float *A, const float *B,
                        const float *C, int grid_log2, int64_t *n_zero_det) {
    double scale = ldexp(1.0, grid_log2);
    int64_t bad = 0, zeros = 0;
    for (int k = 0; k < n; ++k) {
        int64_t ip[3], iq[3], ia[3], ib[3], ic[3];
        double dp[3], dq[3], da[3], db[3], dc[3];
        for (int c = 0; c < 3; ++c) {
            dp[c] = P[3 * k + c]; dq[c] = Q[3 * k + c];
            da[c] = A[3 * k + c]; db[c] = B[3 * k + c]; dc[c] = C[3 * k + c];
            if (!to_grid(dp[c], scale, &ip[c]) || !to_grid(dq[c], scale, &iq[c]) ||
                !to_grid(da[c], scale, &ia[c]) || !to_grid(db[c], scale, &ib[c]) ||
                !to_grid(dc[c], scale, &ic[c]))
                return -1;
        }
        /* exact */
        i128 d[3], e1[3], e2[3], s[3], h[3], g[3];
        for (int c = 0; c < 3; ++c) {
            d[c] = (i128)iq[c] - ip[c];
            e1[c] = (i128)ib[c] - ia[c];
            e2[c] = (i128)ic[c] - ia[c];
            s[c] = (i128)ip[c] - ia[c];
        }
        h[0] = d[1] * e2[2] - d[2] * e2[1];
        h[1] = d[2] * e2[0] - d[0] * e2[2];
        h[2] = d[0] * e2[1] - d[1] * e2[0];
        g[0] = s[1] * e1[2] - s[2] * e1[1];
        g[1] = s[2] * e1[0] - s[0] * e1[2];
        g[2] = s[0] * e1[1] - s[1] * e1[0];
        i128 det = e1[0] * h[0] + e1[1] * h[1] + e1[2] * h[2];
        i128 u = s[0] * h[0] + s[1] * h[1] + s[2] * h[2];
        i128 v = d[0] * g[0] + d[1] * g[1] + d[2] * g[2];
        i128 t = e2[0] * g[0] + e2[1] * g[1] + e2[2] * g[2];
        int ex[6] = {sgn128(det), sgn128(u), sgn128(v), sgn128(det - u - v), sgn128(t), sgn128(det - t)};
        /* FP64, same formulas as ivo_segtri */
        double fd[3], fe1[3], fe2[3], fs[3], fh[3], fg[3];
        sub3(dq, dp, fd); sub3(db, da, fe1); sub3(dc, da, fe2); sub3(dp, da, fs);
        cross3(fd, fe2, fh);
        cross3(fs, fe1, fg);
        double fdet = dot3(fe1, fh), fu = dot3(fs, fh), fv = dot3(fd, fg), ft = dot3(fe2, fg);
        int fp[6] = {sgnd(fdet), sgnd(fu), sgnd(fv), sgnd(fdet - fu - fv), sgnd(ft), sgnd(fdet - ft)};
        int ok = 1;
        for (int c = 0; c < 6; ++c) ok &= (ex[c] == fp[c]);
        /* also the final hit decision must agree */
        int hit_exact;
        if (ex[0] == 0) hit_exact = 0;
        else if (ex[0] > 0) hit_exact = ex[1] >= 0 && ex[2] >= 0 && ex[3] >= 0 && ex[4] > 0 && ex[5] > 0;
        else hit_exact = ex[1] <= 0 && ex[2] <= 0 && ex[3] <= 0 && ex[4] < 0 && ex[5] < 0;
        ok &= (hit_exact == ivo_segtri(dp, dq, da, db, dc));
        if (!ok) bad++;
        if (ex[0] == 0) zeros++;
    }
    if (n_zero_det) *n_zero_det = zeros;
    return bad;
}

/* Orientation exactness audit: 128-bit (x - a).((b - a) x (c - a)) vs FP64. */
int64_t ivo_orient_audit(int n, const float *X, const float *A, const float *B, const float *C,
                         int grid_log2) {
    double scale = ldexp(1.0, grid_log2);
    int64_t bad = 0;
    for (int k = 0; k < n; ++k) {
        int64_t ix[3], ia[3], ib[3], ic[3];
        double dx[3], da[3], db[3], dc[3];
        for (int c = 0; c < 3; ++c) {
            dx[c] = X[3 * k + c]; da[c] = A[3 * k + c]; db[c] = B[3 * k + c]; dc[c] = C[3 * k + c];
            if (!to_grid(dx[c], scale, &ix[c]) || !to_grid(da[c], scale, &ia[c]) ||
                !to_grid(db[c], scale, &ib[c]) || !to_grid(dc[c], scale, &ic[c]))
                return -1;
        }
        i128 e1[3], e2[3], r[3], nrm[3];
        for (int c = 0; c < 3; ++c) {
            e1[c] = (i128)ib[c] - ia[c]; e2[c] = (i128)ic[c] - ia[c]; r[c] = (i128)ix[c] - ia[c];
        }
        nrm[0] = e1[1] * e2[2] - e1[2] * e2[1];
        nrm[1] = e1[2] * e2[0] - e1[0] * e2[2];
        nrm[2] = e1[0] * e2[1] - e1[1] * e2[0];
        i128 o = r[0] * nrm[0] + r[1] * nrm[1] + r[2] * nrm[2];
        double fe1[3], fe2[3], fr[3], fn[3];
        sub3(db, da, fe1); sub3(dc, da, fe2); sub3(dx, da, fr);
        cross3(fe1, fe2, fn);
        if (sgn128(o) != sgnd(dot3(fr, fn))) bad++;
    }
    return bad;
}

int ivo_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
