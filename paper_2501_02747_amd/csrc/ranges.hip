// Ray creation and suppression points along a sampled trajectory, the
// visibility ranges between them and their coherence times (Section III-C: the
// visibility change nodes of the inter-visibility table of a mobile Tx / Rx;
// Section III-D, eq. 8: T_c,l = d_l / v_l, the smaller of the Tx-side and
// Rx-side values when both move; eq. 9: the mean over the ranges).
//
// One block: its threads count the creations and suppressions of every
// snapshot (XOR of consecutive table rows, W words per side), then one thread
// walks the snapshots in order for the ranges, route distances and times.
// The sequential part is O(N) with FP64 steps in a fixed order (no contraction)
// so that its results do not depend on the launch.
#include "ivm_internal.h"

namespace ivm {
namespace {

constexpr int kRangeThreads = 1024;

// Route distance from snapshot n - 1 to snapshot n of one side (metres).
__device__ inline double route_step(const float *X, int n) {
#pragma clang fp contract(off)
    const double dx = (double)X[3 * n] - (double)X[3 * n - 3];
    const double dy = (double)X[3 * n + 1] - (double)X[3 * n - 2];
    const double dz = (double)X[3 * n + 2] - (double)X[3 * n - 1];
    double q = dx * dx;
    q = q + dy * dy;
    q = q + dz * dz;
    return sqrt(q);
}

__device__ inline bool side_change(const int *ev, int n, int s) {
    const int *e = ev + 5 * n;
    return n > 0 && (e[2 * s] != 0 || e[2 * s + 1] != 0 || e[4] != 0);
}

__global__ __launch_bounds__(kRangeThreads) void k_ranges(int N, int W, const uint64_t *tv, const uint64_t *rv,
                                                          const uint8_t *los, const float *tx, const float *rx,
                                                          double dt, int *events, int *starts, double *tc,
                                                          double *dist, int *n_ranges, double *mean) {
#pragma clang fp contract(off)
    for (int n = threadIdx.x; n < N; n += blockDim.x) {
        int c[5] = {0, 0, 0, 0, 0};
        if (n > 0) {
            for (int s = 0; s < 2; ++s) {
                const uint64_t *cur = (s ? rv : tv) + (size_t)n * W, *prev = cur - W;
                for (int w = 0; w < W; ++w) {
                    c[2 * s] += __popcll(cur[w] & ~prev[w]);      // created
                    c[2 * s + 1] += __popcll(prev[w] & ~cur[w]);  // suppressed
                }
            }
            c[4] = (int)(los[n] != 0) - (int)(los[n - 1] != 0);
        }
        for (int k = 0; k < 5; ++k) events[5 * n + k] = c[k];
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    // combined ranges: a start at 0 and at every change of either side
    int L = 0;
    for (int n = 0; n < N; ++n)
        if (n == 0 || side_change(events, n, 0) || side_change(events, n, 1)) {
            starts[L] = n;
            tc[L] = INFINITY;
            ++L;
        }
    // each side's ranges [a, e) (the last to N - 1): d / v with v = d / ((e - a) dt),
    // given to the combined ranges that start inside
    for (int s = 0; s < 2; ++s) {
        const float *X = s ? rx : tx;
        int a = 0, l = 0;
        for (int n = 1; n <= N; ++n) {
            if (n < N && !side_change(events, n, s)) continue;
            const int e = n < N ? n : N - 1;
            double d = 0.0;
            for (int k = a + 1; k <= e; ++k) d = d + route_step(X, k);
            double t = INFINITY;
            if (d > 0.0) {
                const double v = d / ((double)(e - a) * dt);
                t = d / v;
            }
            const int hi = n < N ? n : N;
            for (; l < L && starts[l] < hi; ++l) tc[l] = fmin(tc[l], t);
            a = n;
        }
    }
    // each side's route distance over each combined range, and the mean of the finite times
    double acc = 0.0;
    int nf = 0;
    for (int l = 0; l < L; ++l) {
        const int e = l + 1 < L ? starts[l + 1] : N - 1;
        for (int s = 0; s < 2; ++s) {
            const float *X = s ? rx : tx;
            double d = 0.0;
            for (int k = starts[l] + 1; k <= e; ++k) d = d + route_step(X, k);
            dist[2 * l + s] = d;
        }
        if (tc[l] != INFINITY) {
            acc = acc + tc[l];
            ++nf;
        }
    }
    *n_ranges = L;
    *mean = nf > 0 ? acc / (double)nf : INFINITY;
}

}  // namespace

hipError_t launch_ranges(const SceneDev &sc, int N, const uint64_t *tv, const uint64_t *rv, const uint8_t *los,
                         const float *tx, const float *rx, double dt, int *events, int *starts, double *tc,
                         double *dist, int *n_ranges, double *mean, hipStream_t s) {
    hipLaunchKernelGGL(k_ranges, dim3(1), dim3(kRangeThreads), 0, s, N, sc.W, tv, rv, los, tx, rx, dt, events, starts,
                       tc, dist, n_ranges, mean);
    return hipGetLastError();
}

}  // namespace ivm
