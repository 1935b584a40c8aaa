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
//
// Orders 3 and 4 (the higher orders the paper iterates to, Section II-C and
// Section IV-C) count walks through two vectors held in LDS, one block per
// snapshot: v[g] = popcount(M[g] & rx), the walks g -> ... of one step that end
// on an Rx-visible facet, and u[g] = sum over f in tx of M[f][g], the walks from
// the Tx side that reach g in one step.  Then
//   order 2 = sum over g in tx of v[g]
//   order 3 = sum over g of u[g] v[g]
//   order 4 = sum over g of u[g] (sum over h in M[g] of v[h])
// which is t^T M^(k-1) r written out; no symmetry of M is assumed.  Every term
// is a non-negative integer, so the int64 sums are exact below 2^63 (F^4 bounds
// them; F <= 40960 keeps F^4 < 2^63).
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

constexpr int kHighThreads = 512;
constexpr int kLanesPerRow = 8, kRowsPerWave = 64 / kLanesPerRow;

// LDS of k_cand_high for F facets: u as 16-bit halves of uint32 words (LDS
// atomics are 32-bit; a count never exceeds F < 2^16, so halves never carry),
// v as uint16 (a row popcount never exceeds F).
__host__ __device__ inline size_t cand_high_lds(int F) {
    const size_t uw = ((size_t)F + 1) / 2;
    return 4 * uw + 2 * (((size_t)F + 1) & ~(size_t)1);
}

__device__ inline unsigned long long block_sum_u64(unsigned long long v, unsigned long long *sh) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    v = wsum(v);
    if (lane == 0) sh[wv] = v;
    __syncthreads();
    unsigned long long s = 0;
    for (int k = 0; k < kHighThreads / 64; ++k) s += sh[k];
    __syncthreads();
    return s;
}

__global__ __launch_bounds__(kHighThreads) void k_cand_high(int F, int W, const uint64_t *M, int N,
                                                            const uint64_t *txv, const uint64_t *rxv,
                                                            const uint8_t *los, int K, int64_t *counts) {
    extern __shared__ __align__(16) unsigned char lds[];
    __shared__ unsigned long long red[kHighThreads / 64];
    const int Fh = (F + 1) / 2;
    unsigned *u = (unsigned *)lds;
    unsigned short *v = (unsigned short *)(lds + 4 * (size_t)Fh);
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, nw = kHighThreads / 64;
    const int grp = lane / kLanesPerRow, sub = lane % kLanesPerRow;
    for (int n = blockIdx.x; n < N; n += gridDim.x) {
        const uint64_t *t = txv + (size_t)n * W, *r = rxv + (size_t)n * W;
        for (int i = tid; i < Fh; i += kHighThreads) u[i] = 0u;
        __syncthreads();
        // one pass over the rows: v[g], and the rows of Tx-visible facets pushed into
        // u.  Eight lanes share a row, so a wave keeps eight rows' loads in flight.
        for (int g0 = wv * kRowsPerWave; g0 < F; g0 += nw * kRowsPerWave) {
            const int g = g0 + grp;
            unsigned c = 0;
            if (g < F) {
                const uint64_t *row = M + (size_t)g * W;
                const bool in_t = (t[g >> 6] >> (g & 63)) & 1ull;
                for (int w = sub; w < W; w += kLanesPerRow) {
                    const uint64_t m = row[w];
                    c += (unsigned)__popcll(m & r[w]);
                    if (in_t) {
                        uint64_t b = m;
                        while (b) {
                            const int h = w * 64 + __ffsll((long long)b) - 1;
                            b &= b - 1;
                            if (h >= F) break;
                            atomicAdd(&u[h >> 1], 1u << (16 * (h & 1)));
                        }
                    }
                }
            }
            for (int o = kLanesPerRow / 2; o > 0; o >>= 1) c += __shfl_xor(c, o);
            if (g < F && sub == 0) v[g] = (unsigned short)c;
        }
        __syncthreads();
        unsigned long long c1 = 0, c2 = 0, c3 = 0, c4 = 0;
        if (wv == 0)
            for (int w = lane; w < W; w += 64) c1 += __popcll(t[w] & r[w]);
        for (int g = tid; g < F; g += kHighThreads) {
            const unsigned ug = (u[g >> 1] >> (16 * (g & 1))) & 0xffffu;
            const unsigned vg = v[g];
            c3 += (unsigned long long)ug * vg;
            if ((t[g >> 6] >> (g & 63)) & 1ull) c2 += vg;
        }
        if (K >= 4)
            for (int g0 = wv * kRowsPerWave; g0 < F; g0 += nw * kRowsPerWave) {
                const int g = g0 + grp;
                if (g >= F) continue;
                const unsigned ug = (u[g >> 1] >> (16 * (g & 1))) & 0xffffu;
                if (ug == 0u) continue;
                const uint64_t *row = M + (size_t)g * W;
                unsigned long long sv = 0;
                for (int w = sub; w < W; w += kLanesPerRow) {
                    uint64_t b = row[w];
                    while (b) {
                        const int h = w * 64 + __ffsll((long long)b) - 1;
                        b &= b - 1;
                        if (h >= F) break;
                        sv += v[h];
                    }
                }
                c4 += (unsigned long long)ug * sv;  // (each lane its words' share; summed below)
            }
        c1 = block_sum_u64(c1, red);
        c2 = block_sum_u64(c2, red);
        c3 = block_sum_u64(c3, red);
        c4 = block_sum_u64(c4, red);
        if (tid == 0) {
            int64_t *o = counts + (size_t)n * (K + 1);
            o[0] = los[n] ? 1 : 0;
            o[1] = (int64_t)c1;
            o[2] = (int64_t)c2;
            o[3] = (int64_t)c3;
            if (K >= 4) o[4] = (int64_t)c4;
        }
        // (block_sum_u64 ends on a barrier: u may be cleared for the next snapshot)
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

// Calls fn(f) for every set bit f < F of a row, in increasing order (all lanes
// read the same words, so the loop is wave-uniform).
template <class Fn>
__device__ __attribute__((always_inline)) inline void for_bits(const uint64_t *row, int W, int F, Fn &&fn) {
    for (int w = 0; w < W; ++w) {
        uint64_t b = row[w];
        while (b) {
            const int f = w * 64 + __ffsll((long long)b) - 1;
            b &= b - 1;
            if (f >= F) return;
            fn(f);
        }
    }
}

// Appends the K-tuples (pre..., h) for every set bit h of row & r, in increasing
// h, at out + K * base (base counts tuples and advances past them).
template <int K>
__device__ __attribute__((always_inline)) inline void emit_row(const uint64_t *row, const uint64_t *r, int W,
                                                               const int (&pre)[K - 1], int32_t *out,
                                                               unsigned long long &base) {
    const int lane = threadIdx.x & 63;
    for (int w0 = 0; w0 < W; w0 += 64) {
        const int w = w0 + lane;
        unsigned long long word = w < W ? (row[w] & r[w]) : 0ull;
        unsigned tot;
        unsigned long long pos = base + wave_excl((unsigned)__popcll(word), &tot);
        while (word) {
            int32_t *o = out + (size_t)K * pos;
#pragma unroll
            for (int m = 0; m < K - 1; ++m) o[m] = pre[m];
            o[K - 1] = w * 64 + __ffsll((long long)word) - 1;
            ++pos;
            word &= word - 1;
        }
        base += tot;
    }
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
            unsigned long long base = 0;
            for (int w0 = 0; w0 < W; w0 += 64) {
                const int w = w0 + lane;
                unsigned long long word = w < W ? (t[w] & r[w]) : 0ull;
                unsigned tot;
                unsigned long long pos = base + wave_excl((unsigned)__popcll(word), &tot);
                while (word) {
                    out[pos++] = w * 64 + __ffsll((long long)word) - 1;
                    word &= word - 1;
                }
                base += tot;
            }
        }
        if (K >= 2) {
            int32_t *out = paths + offsets[(size_t)n * K + 1];
            unsigned long long base = 0;
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
                        unsigned long long pos = base + wave_excl((unsigned)__popcll(word), &tot);
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
        // orders 3 and 4: the prefixes walk the rows in increasing order, so the
        // tuples come out in lexicographic order
        if (K >= 3) {
            int32_t *out = paths + offsets[(size_t)n * K + 2];
            unsigned long long base = 0;
            for_bits(t, W, F, [&](int f1) {
                for_bits(M + (size_t)f1 * W, W, F, [&](int f2) {
                    const int pre[2] = {f1, f2};
                    emit_row<3>(M + (size_t)f2 * W, r, W, pre, out, base);
                });
            });
        }
        if (K >= 4) {
            int32_t *out = paths + offsets[(size_t)n * K + 3];
            unsigned long long base = 0;
            for_bits(t, W, F, [&](int f1) {
                for_bits(M + (size_t)f1 * W, W, F, [&](int f2) {
                    for_bits(M + (size_t)f2 * W, W, F, [&](int f3) {
                        const int pre[3] = {f1, f2, f3};
                        emit_row<4>(M + (size_t)f3 * W, r, W, pre, out, base);
                    });
                });
            });
        }
    }
}

static unsigned waves_grid(int N) {
    long long b = ((long long)N + 3) / 4;
    if (b < 1) b = 1;
    if (b > 8192) b = 8192;
    return (unsigned)b;
}

bool candidates_high_fits(int F) {
    if (F < 1 || F > kCandHighMaxF) return false;
    int dev = 0, lds = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
        return false;
    return cand_high_lds(F) + 64 * sizeof(unsigned long long) <= (size_t)lds;
}

hipError_t launch_candidates_count(const SceneDev &d, const uint64_t *M, int N, const uint64_t *txv,
                                   const uint64_t *rxv, const uint8_t *los, int K, int64_t *counts, hipStream_t s) {
    if (N <= 0) return hipSuccess;
    if (K >= 3) {
        const size_t lds = cand_high_lds(d.F);
        if (lds > 65536) {
            const hipError_t e = hipFuncSetAttribute((const void *)k_cand_high,
                                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            if (e != hipSuccess) return e;
        }
        const unsigned grid = (unsigned)(N < 8192 ? N : 8192);
        hipLaunchKernelGGL(k_cand_high, dim3(grid), dim3(kHighThreads), lds, s, d.F, d.W, M, N, txv, rxv, los, K,
                           counts);
        return hipGetLastError();
    }
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
