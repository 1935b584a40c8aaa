// candidates.hip -- image-tree reflection candidates from the bit tables.
//
// Section III-B (Table II): the transmitter is the parent node, the facets it
// sees are the reference faces, and the matrix row of a reference face lists the
// aim faces.  A reflection path of order k is a walk f1 -> ... -> fk with
// tx_vis(f1), M[f_m][f_m+1] and rx_vis(fk); order 0 is line of sight.
//   order 1: popcount(tx & rx)
//   order 2: sum over f1 in tx of popcount(M[f1] & rx)
// One wave per snapshot; lanes stride over the W words of a row.  The work is
// a bandwidth-bound stream of |tx| rows of M per snapshot.
#include "ivm_internal.h"

namespace ivm {

__device__ inline unsigned long long wsum(unsigned long long v) {
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

__global__ __launch_bounds__(256) void k_cand_count(int F, int W, const uint64_t *M, int N, const uint64_t *txv,
                                                    const uint64_t *rxv, const uint8_t *los, int K, int64_t *counts) {
    const int lane = threadIdx.x & 63;
    const int wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int nwaves = (gridDim.x * blockDim.x) >> 6;
    for (int n = wave; n < N; n += nwaves) {
        const uint64_t *t = txv + (size_t)n * W, *r = rxv + (size_t)n * W;
        unsigned long long c1 = 0, c2 = 0;
        for (int w = lane; w < W; w += 64) c1 += __popcll(t[w] & r[w]);
        if (K >= 2) {
            for (int w0 = 0; w0 < W; ++w0) {
                unsigned long long tw = t[w0];
                while (tw) {
                    const int f = w0 * 64 + __ffsll((long long)tw) - 1;
                    tw &= tw - 1;
                    if (f >= F) break;  // padding bits of the caller's table name no row
                    const uint64_t *row = M + (size_t)f * W;
                    for (int w = lane; w < W; w += 64) c2 += __popcll(row[w] & r[w]);
                }
            }
        }
        c1 = wsum(c1);
        c2 = wsum(c2);
        if (lane == 0) {
            int64_t *o = counts + (size_t)n * (K + 1);
            o[0] = los[n] ? 1 : 0;
            o[1] = (int64_t)c1;
            if (K >= 2) o[2] = (int64_t)c2;
        }
    }
}

// offsets[n*K + k-1] = start of list (n, k) in int32 elements; offsets[N*K] = total.
__global__ __launch_bounds__(1024) void k_cand_offsets(int N, int K, const int64_t *counts, int64_t *offsets) {
    __shared__ long long sh[1024];
    const int L = N * K;
    long long carry = 0;
    for (int base = 0; base < L; base += 1024) {
        const int i = base + threadIdx.x;
        long long v = 0;
        if (i < L) {
            const int n = i / K, k = i - (i / K) * K + 1;
            v = counts[(size_t)n * (K + 1) + k] * k;
        }
        sh[threadIdx.x] = v;
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) {
            long long x = threadIdx.x >= off ? sh[threadIdx.x - off] : 0;
            __syncthreads();
            sh[threadIdx.x] += x;
            __syncthreads();
        }
        if (i < L) offsets[i] = carry + sh[threadIdx.x] - v;
        carry += sh[1023];
        __syncthreads();
    }
    if (threadIdx.x == 0) offsets[L] = carry;
}

// Exclusive wave prefix of a per-lane count.
__device__ inline unsigned wave_excl(unsigned v, unsigned *total) {
    const int lane = threadIdx.x & 63;
    unsigned x = v;
    for (int o = 1; o < 64; o <<= 1) {
        unsigned y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    *total = __shfl(x, 63);
    return x - v;
}

__global__ __launch_bounds__(256) void k_cand_fill(int F, int W, const uint64_t *M, int N, const uint64_t *txv,
                                                   const uint64_t *rxv, int K, const int64_t *offsets, int32_t *paths) {
    const int lane = threadIdx.x & 63;
    const int wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int nwaves = (gridDim.x * blockDim.x) >> 6;
    for (int n = wave; n < N; n += nwaves) {
        const uint64_t *t = txv + (size_t)n * W, *r = rxv + (size_t)n * W;
        // order 1
        {
            int32_t *out = paths + offsets[(size_t)n * K + 0];
            unsigned base = 0;
            for (int w0 = 0; w0 < W; w0 += 64) {
                const int w = w0 + lane;
                unsigned long long word = w < W ? (t[w] & r[w]) : 0ull;
                unsigned tot;
                unsigned pos = base + wave_excl((unsigned)__popcll(word), &tot);
                while (word) {
                    out[pos++] = w * 64 + __ffsll((long long)word) - 1;
                    word &= word - 1;
                }
                base += tot;
            }
        }
        if (K >= 2) {
            int32_t *out = paths + offsets[(size_t)n * K + 1];
            unsigned base = 0;
            for (int v0 = 0; v0 < W; ++v0) {
                unsigned long long tw = t[v0];
                while (tw) {
                    const int f1 = v0 * 64 + __ffsll((long long)tw) - 1;
                    tw &= tw - 1;
                    if (f1 >= F) break;
                    const uint64_t *row = M + (size_t)f1 * W;
                    for (int w0 = 0; w0 < W; w0 += 64) {
                        const int w = w0 + lane;
                        unsigned long long word = w < W ? (row[w] & r[w]) : 0ull;
                        unsigned tot;
                        unsigned pos = base + wave_excl((unsigned)__popcll(word), &tot);
                        while (word) {
                            out[2 * pos] = f1;
                            out[2 * pos + 1] = w * 64 + __ffsll((long long)word) - 1;
                            ++pos;
                            word &= word - 1;
                        }
                        base += tot;
                    }
                }
            }
        }
    }
}

static unsigned waves_grid(int N) {
    long long b = ((long long)N + 3) / 4;
    if (b < 1) b = 1;
    if (b > 8192) b = 8192;
    return (unsigned)b;
}

hipError_t launch_candidates_count(const SceneDev &d, const uint64_t *M, int N, const uint64_t *txv,
                                   const uint64_t *rxv, const uint8_t *los, int K, int64_t *counts, hipStream_t s) {
    if (N <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_cand_count, dim3(waves_grid(N)), dim3(256), 0, s, d.F, d.W, M, N, txv, rxv, los, K, counts);
    return hipGetLastError();
}

hipError_t launch_candidates_offsets(int N, int K, const int64_t *counts, int64_t *offsets, hipStream_t s) {
    hipLaunchKernelGGL(k_cand_offsets, dim3(1), dim3(1024), 0, s, N, K, counts, offsets);
    return hipGetLastError();
}

hipError_t launch_candidates_fill(const SceneDev &d, const uint64_t *M, int N, const uint64_t *txv,
                                  const uint64_t *rxv, int K, const int64_t *offsets, int32_t *paths, hipStream_t s) {
    if (N <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_cand_fill, dim3(waves_grid(N)), dim3(256), 0, s, d.F, d.W, M, N, txv, rxv, K, offsets, paths);
    return hipGetLastError();
}

}  // namespace ivm
