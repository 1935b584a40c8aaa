// Interface relations of the inter-visibility matrix (Section II-B, Table I:
// for a reference face and an aim face that see each other, whether their
// planes are parallel (PAR) or perpendicular (PER); relations between vertical
// faces belong to the horizontal view, those involving horizontal faces to a
// vertical one).  One wave per matrix row, the lanes over its words.
//
// The facet normals of the plane records are cross products of vertex
// differences: exact FP64 multiples of 2^-2g below 2^50 after scaling, so the
// scaled integers are exact and the cross and dot products of two normals are
// decided in 128-bit integers.
#include "ivm_internal.h"

namespace ivm {
namespace {

struct INormal {
    long long x, y, z;
};

__device__ inline INormal int_normal(const SceneDev &sc, int f, double s2) {
    const double *n = sc.fplane + 6 * f + 3;
    return {(long long)(n[0] * s2), (long long)(n[1] * s2), (long long)(n[2] * s2)};
}

__global__ __launch_bounds__(256) void k_relations(SceneDev sc, const uint64_t *M, uint64_t *par, uint64_t *per,
                                                   int8_t *cls) {
    const int i = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (i >= sc.F) return;  // (wave-uniform)
    const double s2 = ldexp(1.0, 2 * sc.g);  // metres^2 -> vertex-grid units^2 (exact)
    const INormal a = int_normal(sc, i, s2);
    if (lane == 0) cls[i] = (int8_t)(a.z == 0 ? 0 : (a.x == 0 && a.y == 0 ? 1 : 2));
    for (int w = lane; w < sc.W; w += 64) {
        uint64_t m = M[(size_t)i * sc.W + w], p = 0ull, q = 0ull;
        while (m) {
            const int bit = __ffsll((long long)m) - 1;
            m &= m - 1ull;
            const INormal b = int_normal(sc, w * 64 + bit, s2);
            const __int128 cx = (__int128)a.y * b.z - (__int128)a.z * b.y;
            const __int128 cy = (__int128)a.z * b.x - (__int128)a.x * b.z;
            const __int128 cz = (__int128)a.x * b.y - (__int128)a.y * b.x;
            const __int128 dot = (__int128)a.x * b.x + (__int128)a.y * b.y + (__int128)a.z * b.z;
            if (cx == 0 && cy == 0 && cz == 0) p |= 1ull << bit;
            if (dot == 0) q |= 1ull << bit;
        }
        par[(size_t)i * sc.W + w] = p;
        per[(size_t)i * sc.W + w] = q;
    }
}

}  // namespace

hipError_t launch_relations(const SceneDev &sc, const uint64_t *M, uint64_t *par, uint64_t *per, int8_t *cls,
                            hipStream_t s) {
    if (sc.F <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_relations, dim3((unsigned)((sc.F + 3) / 4)), dim3(256), 0, s, sc, M, par, per, cls);
    return hipGetLastError();
}

}  // namespace ivm
