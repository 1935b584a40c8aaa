// Ray creation and suppression points along a sampled trajectory, the
// visibility ranges between them and their coherence times (Section III-C: the
// visibility change nodes of the inter-visibility table of a mobile Tx / Rx;
// Section III-D, eq. 8: T_c,l = d_l / v_l, the smaller of the Tx-side and
// Rx-side values when both move; eq. 9: the mean over the ranges).
//
// One wave per snapshot counts its creations and suppressions (XOR of
// consecutive table rows, the lanes over the W words of each side) and its
// route steps; then one block of 1024 threads numbers the combined ranges and
// each side's ranges with block scans, and one thread per range sums its route
// steps in snapshot order (FP64, no contraction), so every result is the
// sequential one whatever the launch.
#include <mutex>

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

// Exclusive scan of one int per thread over the block; returns the total.
__device__ inline int block_scan(int v, int *sh, int &excl) {
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int o = 1; o < kRangeThreads; o <<= 1) {
        const int add = t >= o ? sh[t - o] : 0;
        __syncthreads();
        sh[t] += add;
        __syncthreads();
    }
    excl = sh[t] - v;
    const int total = sh[kRangeThreads - 1];
    __syncthreads();
    return total;
}

// Workspace layout (N snapshots): flags int32[N] (bit 0 Tx side, bit 1 Rx side
// changes at n), steps double[N][2], side range starts int32[2][N], side times
// double[2][N], side range index of each snapshot int32[2][N].
struct RangeWs {
    int *flags;
    double *step;
    int *sstart;
    double *stime;
    int *sidx;
};

__device__ inline RangeWs ws_layout(void *ws, int N) {
    char *p = (char *)ws;
    RangeWs w;
    w.step = (double *)p;
    p += sizeof(double) * 2 * (size_t)N;
    w.stime = (double *)p;
    p += sizeof(double) * 2 * (size_t)N;
    w.flags = (int *)p;
    p += sizeof(int) * (size_t)N;
    w.sstart = (int *)p;
    p += sizeof(int) * 2 * (size_t)N;
    w.sidx = (int *)p;
    return w;
}

__global__ __launch_bounds__(256) void k_range_events(int N, int W, const uint64_t *tv, const uint64_t *rv,
                                                     const uint8_t *los, const float *tx, const float *rx, void *ws,
                                                     int *events) {
#pragma clang fp contract(off)
    const RangeWs w = ws_layout(ws, N);
    const int n = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (n >= N) return;  // (wave-uniform)
    unsigned c[4] = {0u, 0u, 0u, 0u};
    if (n > 0)
        for (int s = 0; s < 2; ++s) {
            const uint64_t *cur = (s ? rv : tv) + (size_t)n * W, *prev = cur - W;
            for (int k = lane; k < W; k += 64) {
                c[2 * s] += __popcll(cur[k] & ~prev[k]);      // created
                c[2 * s + 1] += __popcll(prev[k] & ~cur[k]);  // suppressed
            }
        }
    for (int k = 0; k < 4; ++k)
        for (int o = 32; o > 0; o >>= 1) c[k] += __shfl_xor(c[k], o);
    if (lane == 0) {
        const int dl = n > 0 ? (int)(los[n] != 0) - (int)(los[n - 1] != 0) : 0;
        for (int k = 0; k < 4; ++k) events[5 * n + k] = (int)c[k];
        events[5 * n + 4] = dl;
        const bool ct = (c[0] | c[1]) != 0u || dl != 0, cr = (c[2] | c[3]) != 0u || dl != 0;
        w.flags[n] = (ct ? 1 : 0) | (cr ? 2 : 0);
        w.step[2 * n] = n > 0 ? route_step(tx, n) : 0.0;
        w.step[2 * n + 1] = n > 0 ? route_step(rx, n) : 0.0;
    }
}

__global__ __launch_bounds__(kRangeThreads) void k_ranges(int N, double dt, void *ws, int *starts, double *tc,
                                                          double *dist, int *n_ranges, double *mean) {
#pragma clang fp contract(off)
    __shared__ int sh[kRangeThreads];
    const RangeWs w = ws_layout(ws, N);
    const int t = threadIdx.x;
    // number the ranges: thread t owns snapshots [n0, n1); a range starts at 0 and
    // at every change (combined: either side; side s: its own bit)
    const int per = (N + kRangeThreads - 1) / kRangeThreads;
    const int n0 = min(N, t * per), n1 = min(N, n0 + per);
    int cnt[3] = {0, 0, 0};
    for (int n = n0; n < n1; ++n) {
        const int f = w.flags[n];
        cnt[0] += n == 0 || f != 0;
        cnt[1] += n == 0 || (f & 1);
        cnt[2] += n == 0 || (f & 2);
    }
    int base[3], tot[3];
    for (int k = 0; k < 3; ++k) tot[k] = block_scan(cnt[k], sh, base[k]);
    for (int n = n0; n < n1; ++n) {
        const int f = w.flags[n];
        if (n == 0 || f != 0) starts[base[0]++] = n;
        for (int s = 0; s < 2; ++s) {
            if (n == 0 || (f & (1 << s))) w.sstart[s * N + base[1 + s]++] = n;
            w.sidx[s * N + n] = base[1 + s] - 1;
        }
    }
    __syncthreads();
    const int L = tot[0];
    // each side's range r: [sstart[r], next start) (the last to N - 1): d / v with
    // v = d / ((e - a) dt); a side that does not move sets no limit
    for (int s = 0; s < 2; ++s)
        for (int r = t; r < tot[1 + s]; r += kRangeThreads) {
            const int a = w.sstart[s * N + r];
            const int e = r + 1 < tot[1 + s] ? w.sstart[s * N + r + 1] : N - 1;
            double d = 0.0;
            for (int k = a + 1; k <= e; ++k) d = d + w.step[2 * k + s];
            double time = INFINITY;
            if (d > 0.0) {
                const double v = d / ((double)(e - a) * dt);
                time = d / v;
            }
            w.stime[s * N + r] = time;
        }
    __syncthreads();
    // each combined range: the smaller side time of the side ranges containing it,
    // and each side's route distance over it
    for (int l = t; l < L; l += kRangeThreads) {
        const int a = starts[l];
        const int e = l + 1 < L ? starts[l + 1] : N - 1;
        tc[l] = fmin(w.stime[w.sidx[a]], w.stime[N + w.sidx[N + a]]);
        for (int s = 0; s < 2; ++s) {
            double d = 0.0;
            for (int k = a + 1; k <= e; ++k) d = d + w.step[2 * k + s];
            dist[2 * l + s] = d;
        }
    }
    __syncthreads();
    if (t == 0) {  // the mean of the finite times (eq. 9), in range order
        double acc = 0.0;
        int nf = 0;
        for (int l0 = 0; l0 < L; l0 += 32) {
            double buf[32];  // (independent loads first, then the additions in order)
#pragma unroll
            for (int j = 0; j < 32; ++j) buf[j] = l0 + j < L ? tc[l0 + j] : INFINITY;
#pragma unroll
            for (int j = 0; j < 32; ++j)
                if (buf[j] != INFINITY) {
                    acc = acc + buf[j];
                    ++nf;
                }
        }
        *n_ranges = L;
        *mean = nf > 0 ? acc / (double)nf : INFINITY;
    }
}

}  // namespace

size_t ranges_workspace_bytes(int N) { return (size_t)N * (4 * sizeof(double) + 5 * sizeof(int)) + 256; }

// Scratch of the allocation-free variant: room for kRangesNoAllocMaxSnap
// snapshots, one copy per GPU for the life of the process.  Host code never
// passes `scratch` itself to a kernel (on the host the name is a stand-in, not
// a device address); it uses the address hipGetSymbolAddress reports for the
// current device, looked up once per device.
constexpr size_t kRangesScratchBytes = (size_t)kRangesNoAllocMaxSnap * (4 * sizeof(double) + 5 * sizeof(int)) + 256;
static_assert(kRangesNoAllocMaxSnap == IVM_RANGES_NOALLOC_MAX_SNAP, "allocation-free limit");
static __device__ __align__(256) unsigned char scratch[kRangesScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t ranges_scratch(void **out) {
    *out = nullptr;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

hipError_t launch_ranges(const SceneDev &sc, int N, const uint64_t *tv, const uint64_t *rv, const uint8_t *los,
                         const float *tx, const float *rx, double dt, void *ws, int *events, int *starts, double *tc,
                         double *dist, int *n_ranges, double *mean, hipStream_t s) {
    hipLaunchKernelGGL(k_range_events, dim3((unsigned)((N + 3) / 4)), dim3(256), 0, s, N, sc.W, tv, rv, los, tx, rx, ws,
                       events);
    hipLaunchKernelGGL(k_ranges, dim3(1), dim3(kRangeThreads), 0, s, N, dt, ws, starts, tc, dist, n_ranges, mean);
    return hipGetLastError();
}

}  // namespace ivm
