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
// Section IV-C) are t^T M^(k-1) r written out with u = M^T t and v = M r:
//   order 2 = sum over g of u[g] r[g]
//   order 3 = sum over g of u[g] v[g]
//   order 4 = sum over h of (sum over g of u[g] M[g][h]) v[h]
// computed for a slab of snapshots at a time as integer matrix products on the
// matrix cores (below); no symmetry of M is assumed.  Every term is a
// non-negative integer, so the int64 sums are exact below 2^63 (F^4 bounds
// them; F <= 40960 keeps F^4 < 2^63 and u below 2^16).
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

// ---------------------------------------------------------------------------
// orders 3 and 4 on the matrix cores
// ---------------------------------------------------------------------------
// Over a slab of snapshots the walk counts are bilinear forms of three dense
// integer products (T, R: the slab's Tx and Rx rows; every factor is 0/1 but U):
//   U = T M      U[n][g] = sum_f t_n[f] M[f][g]   (u of snapshot n)
//   V = R M^T    V[n][g] = sum_h M[g][h] r_n[h]   (v of snapshot n)
//   X = U M      X[n][h] = sum_g U[n][g] M[g][h]
// order 2 = sum_g U r, order 3 = sum_g U V, order 4 = sum_h X V.  Each product
// runs on v_mfma_i32_16x16x64_i8 (i8 x i8, exact int32 sums): the 0/1 operands
// are bit rows expanded to bytes, and U < 2^16 enters X as two byte planes
// a - 128 and b - 128 (U = a + 256 b), so X = X_a + 256 X_b + 32896 c[h] with
// c[h] = sum_g M[g][h].  Every operand is read along its K index: M^T (bits,
// zero-padded to Fp = 64 W rows) is built once per call.
//
// Tile: a block of 4 waves owns 64 snapshots x 256 facets; wave w the 64
// facets of bit word 4 blockIdx.y + w, as 4 x 4 MFMA tiles of 16 x 16.  One K
// step is one bit word (64 facets).  The 64-row A panel of a step (expanded
// bits, or the byte planes of U) is staged once per block in LDS, double
// buffered; each wave expands its own B bits in registers.  MFMA operands:
// lane l holds row (or column) l % 16 and bytes 16 (l / 16) .. +15 of the K
// step, byte v being K index 16 (l / 16) + v in both operands (the unit sums
// over every byte pair alike); the result holds D[4 (l / 16) + v][l % 16].

typedef int i32x4 __attribute__((ext_vector_type(4)));

constexpr int kHiRows = 64;             // snapshots per block
constexpr int kXcds = 8;                // XCDs of the MI355X (blocks reach them round-robin)
constexpr int kHiWaves = 4;             // bit words (64 facets each) per block
#ifndef IVM_HI_KS
#define IVM_HI_KS 4
#endif
#ifndef IVM_HI_XCT
#define IVM_HI_XCT 2
#endif
#ifndef IVM_HI_UCT
#define IVM_HI_UCT 2
#endif
constexpr int kHiKs = IVM_HI_KS;        // bit words (64 facets each) per K step
constexpr int kHiXct = IVM_HI_XCT;      // column tiles of 16 per wave in the X product
constexpr int kHiUct = IVM_HI_UCT;      // column tiles of 16 per wave in the U and V products

// 16 bits -> 16 bytes of 0/1 (byte v = bit v): each nibble spread by one
// 24-bit multiply (shifts 0, 7, 14, 21 place bit m at bit 8 m, no carries).
__device__ inline i32x4 expand16(unsigned c) {
    i32x4 r;
    r[0] = (int)(((c & 15u) * 0x204081u) & 0x01010101u);
    r[1] = (int)((((c >> 4) & 15u) * 0x204081u) & 0x01010101u);
    r[2] = (int)((((c >> 8) & 15u) * 0x204081u) & 0x01010101u);
    r[3] = (int)((((c >> 12) & 15u) * 0x204081u) & 0x01010101u);
    return r;
}

// Scratch of the products inside the scene's pair scratch (see hi_slab).
struct HiScratch {
    uint64_t *mt;     // M^T bits, Fp x W words (rows >= F and bits >= F zero)
    int *csum;        // c[h] = popcount(M^T row h), Fp
    int8_t *ua, *ub;  // byte planes of U, NBp x Fp
    uint16_t *v;      // V, NBp x Fp
    int nbp;          // slab rows (a multiple of kHiRows)
};

// M^T and its row popcounts: wave (hw, chunk) transposes 64 x 64 blocks of
// rows 64 gw .. +63 (gw over its chunk of words) and bit word hw by ballots.
__global__ __launch_bounds__(256) void k_hi_transpose(int F, int W, int chunks, const uint64_t *M, uint64_t *mt,
                                                      int *csum) {
    const int lane = threadIdx.x & 63;
    const int wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (wave >= W * chunks) return;
    const int hw = wave / chunks, ch = wave - (wave / chunks) * chunks;
    const int per = (W + chunks - 1) / chunks, g0 = ch * per, g1 = min(W, g0 + per);
    const int hb = F - 64 * hw;  // valid bits of word hw
    const uint64_t hmask = hb >= 64 ? ~0ull : (hb > 0 ? (1ull << hb) - 1ull : 0ull);
    int cnt = 0;
    for (int gw = g0; gw < g1; ++gw) {
        const int g = 64 * gw + lane;
        const uint64_t x = g < F ? (M[(size_t)g * W + hw] & hmask) : 0ull;
        uint64_t mine = 0;
        for (int b = 0; b < 64; ++b) {
            const uint64_t col = __ballot((x >> b) & 1ull);
            if (lane == b) mine = col;
        }
        mt[(size_t)(64 * hw + lane) * W + gw] = mine;
        cnt += __popcll(mine);
    }
    if (g1 > g0) atomicAdd(&csum[64 * hw + lane], cnt);
}

// counts[n][0] = line of sight, [1] = popcount(t & r), [2..K] = 0 (the product
// kernels add into them).
__global__ __launch_bounds__(256) void k_hi_init(int F, int W, int N, const uint64_t *txv, const uint64_t *rxv,
                                                 const uint8_t *los, int K, int64_t *counts) {
    const int lane = threadIdx.x & 63;
    const int n = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (n >= N) return;
    const uint64_t tail = (F & 63) ? (1ull << (F & 63)) - 1ull : ~0ull;
    unsigned long long c1 = 0;
    for (int w = lane; w < W; w += 64) {
        uint64_t x = txv[(size_t)n * W + w] & rxv[(size_t)n * W + w];
        if (w == W - 1) x &= tail;
        c1 += __popcll(x);
    }
    c1 = wsum(c1);
    if (lane == 0) {
        int64_t *o = counts + (size_t)n * (K + 1);
        o[0] = los[n] ? 1 : 0;
        o[1] = (int64_t)c1;
        for (int k = 2; k <= K; ++k) o[k] = 0;
    }
}

// Sums of 16 lanes (one result row group) of a wave.
__device__ inline unsigned long long sum16(unsigned long long x) {
    for (int o = 8; o >= 1; o >>= 1) x += __shfl_xor(x, o);
    return x;
}

// Adds a wave's per-row partial sums (lane l: rows 16 i + 4 (l / 16) + v) into
// the block's LDS row sums.
__device__ inline void add_rows(unsigned long long (&p)[4][4], unsigned long long *rows) {
    const int lane = threadIdx.x & 63;
    for (int i = 0; i < 4; ++i)
        for (int v = 0; v < 4; ++v) {
            const unsigned long long s = sum16(p[i][v]);
            if ((lane & 15) == 0) atomicAdd(&rows[16 * i + 4 * (lane >> 4) + v], s);
        }
}

// U and V of a slab (rows n0 .. n0 + nb - 1), their byte planes and V stored,
// orders 2 and 3 added into counts.  A K step is KS bit words; a block covers
// 64 snapshots x 256 facets, each wave CT column tiles of 16.
template <int KS, int CT>
__global__ __launch_bounds__(64 * 16 / CT) void k_hi_uv(int F, int W, int N, int n0, int nb, const uint64_t *txv,
                                                         const uint64_t *rxv, const uint64_t *M, HiScratch hs, int K,
                                                         int64_t *counts) {
    constexpr int kThreads = 64 * 16 / CT;
    constexpr int kPitch = 64 * KS + 16;                   // LDS bytes per panel row (conflict-free 16-byte reads)
    constexpr int kItems = 2 * kHiRows * KS / kThreads;    // panel words a thread expands per step
    static_assert(kItems >= 1 && 2 * kHiRows * KS % kThreads == 0, "panel split");
    extern __shared__ __align__(16) unsigned char lds_hi[];
    unsigned char *panel = lds_hi;                    // [buffer][T, R][row][kPitch]
    unsigned long long *rows = (unsigned long long *)(lds_hi + 4 * kHiRows * kPitch);  // [2][kHiRows]
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int rb = blockIdx.x * kHiRows;              // slab row of the block
    const int c0 = 256 * blockIdx.y + 16 * CT * wv;   // the wave's first column (facet)
    const bool active = c0 < 64 * W;
    const size_t Fp = (size_t)64 * W;
    const uint64_t tail = (F & 63) ? (1ull << (F & 63)) - 1ull : ~0ull;
    if (tid < 2 * kHiRows) rows[tid] = 0ull;
    // panel producer: item -> (source, row, word of the step)
    const uint64_t *psrc[kItems];
    int pdst[kItems], psw[kItems];
    bool prow[kItems];
    for (int p = 0; p < kItems; ++p) {
        const int it = tid + kThreads * p, src = it / (kHiRows * KS), r = (it / KS) % kHiRows;
        psw[p] = it % KS;
        prow[p] = rb + r < nb;
        psrc[p] = (src ? rxv : txv) + (size_t)(prow[p] ? n0 + rb + r : 0) * W;
        pdst[p] = src * kHiRows * kPitch + r * kPitch + 64 * psw[p];
    }
    // B rows of the wave: column g = c0 + 16 j + (lane & 15)
    const int q = lane >> 4, c16 = lane & 15;
    const uint64_t *bt[CT], *bm[CT];
    bool bmv[CT];
    for (int j = 0; j < CT; ++j) {
        const int g = (active ? c0 : 0) + 16 * j + c16;
        bt[j] = hs.mt + (size_t)g * W;
        bmv[j] = active && g < F;
        bm[j] = M + (size_t)(bmv[j] ? g : 0) * W;
    }
    i32x4 accU[4][CT], accV[4][CT];
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < CT; ++j) {
            accU[i][j] = i32x4{0, 0, 0, 0};
            accV[i][j] = i32x4{0, 0, 0, 0};
        }
    // raw bit words: the panel's (pa) and the wave's B rows (wt: M^T rows, wm: M
    // rows); each B word is reloaded with the next step's right after it has
    // been expanded, so one register set carries a step of load latency
    uint64_t pa[kItems], wt[CT][KS], wm[CT][KS];
    auto fetch_a = [&](int kw0) {
        for (int p = 0; p < kItems; ++p) {
            const int kw = kw0 + psw[p];
            uint64_t x = (prow[p] && kw < W) ? psrc[p][kw] : 0ull;
            if (kw == W - 1) x &= tail;
            pa[p] = x;
        }
    };
    auto fetch_b = [&](int j, int kw, uint64_t &t, uint64_t &m) {
        t = (active && kw < W) ? bt[j][kw] : 0ull;
        uint64_t x = (bmv[j] && kw < W) ? bm[j][kw] : 0ull;
        if (kw == W - 1) x &= tail;
        m = x;
    };
    fetch_a(0);
    for (int s = 0; s < KS; ++s)
        for (int j = 0; j < CT; ++j) fetch_b(j, s, wt[j][s], wm[j][s]);
    const int steps = (W + KS - 1) / KS;
    for (int st = 0; st < steps; ++st) {
        unsigned char *pb = panel + (st & 1) * 2 * kHiRows * kPitch;
        for (int p = 0; p < kItems; ++p) {
            i32x4 *dst = (i32x4 *)(pb + pdst[p]);
            const uint64_t x = pa[p];
            dst[0] = expand16((unsigned)x & 0xffffu);
            dst[1] = expand16((unsigned)(x >> 16) & 0xffffu);
            dst[2] = expand16((unsigned)(x >> 32) & 0xffffu);
            dst[3] = expand16((unsigned)(x >> 48));
        }
        fetch_a((st + 1) * KS);
        __syncthreads();
        // (words past W and the columns of an inactive wave are zero operands:
        // their products add nothing, and the loop stays branch-free so the
        // accumulators keep their registers)
        for (int s = 0; s < KS; ++s) {
            i32x4 bU[CT], bV[CT];
            for (int j = 0; j < CT; ++j) {
                bU[j] = expand16((unsigned)(wt[j][s] >> (16 * q)) & 0xffffu);
                bV[j] = expand16((unsigned)(wm[j][s] >> (16 * q)) & 0xffffu);
                fetch_b(j, (st + 1) * KS + s, wt[j][s], wm[j][s]);
            }
            for (int i = 0; i < 4; ++i) {
                const int off = (16 * i + c16) * kPitch + 64 * s + 16 * q;
                const i32x4 aT = *(const i32x4 *)(pb + off);
                const i32x4 aR = *(const i32x4 *)(pb + kHiRows * kPitch + off);
                for (int j = 0; j < CT; ++j) {
                    accU[i][j] = __builtin_amdgcn_mfma_i32_16x16x64_i8(aT, bU[j], accU[i][j], 0, 0, 0);
                    accV[i][j] = __builtin_amdgcn_mfma_i32_16x16x64_i8(aR, bV[j], accV[i][j], 0, 0, 0);
                }
            }
        }
    }
    if (active) {
        const int cw = c0 >> 6, cb = c0 & 63;   // the R word of the wave's columns, their first bit
        unsigned long long p2[4][4], p3[4][4];
        for (int i = 0; i < 4; ++i)
            for (int v = 0; v < 4; ++v) {
                const int r = 16 * i + 4 * q + v, rl = rb + r;
                unsigned long long s2 = 0, s3 = 0;
                if (rl < nb) {
                    const uint64_t rw = rxv[(size_t)(n0 + rl) * W + cw];
                    for (int j = 0; j < CT; ++j) {
                        const int g = c0 + 16 * j + c16;
                        const unsigned u = (unsigned)accU[i][j][v], vv = (unsigned)accV[i][j][v];
                        if (g < F) {
                            if ((rw >> (cb + 16 * j + c16)) & 1ull) s2 += u;
                            s3 += (unsigned long long)u * vv;
                        }
                        const size_t e = (size_t)rl * Fp + g;
                        hs.ua[e] = (int8_t)((int)(u & 255u) - 128);
                        hs.ub[e] = (int8_t)((int)(u >> 8) - 128);
                        hs.v[e] = (uint16_t)vv;
                    }
                }
                p2[i][v] = s2;
                p3[i][v] = s3;
            }
        add_rows(p2, rows);
        add_rows(p3, rows + kHiRows);
    }
    __syncthreads();
    if (tid < kHiRows && rb + tid < nb) {
        int64_t *o = counts + (size_t)(n0 + rb + tid) * (K + 1);
        atomicAdd((unsigned long long *)&o[2], rows[tid]);
        atomicAdd((unsigned long long *)&o[3], rows[kHiRows + tid]);
    }
}

template <int KS>
constexpr size_t hi_lds() { return (size_t)4 * kHiRows * (64 * KS + 16) + 2 * kHiRows * sizeof(unsigned long long); }

// X = U M of a slab from the byte planes of U; order 4 added into counts.  A
// block covers 64 snapshots x 256 facets; each wave CT column tiles of 16
// (256 / (16 CT) waves), so fewer accumulators per wave allow two waves per SIMD.
template <int KS, int CT>
__global__ __launch_bounds__(64 * 16 / CT) void k_hi_x(int F, int W, int n0, int nb, int ncb, HiScratch hs, int K,
                                                        int64_t *counts) {
    constexpr int kThreads = 64 * 16 / CT;
    constexpr int kPitch = 64 * KS + 16;
    constexpr int kItems = 2 * kHiRows * KS * 4 / kThreads;  // 16-byte panel chunks a thread stages per step
    static_assert(2 * kHiRows * KS * 4 % kThreads == 0, "panel split");
    extern __shared__ __align__(16) unsigned char lds_hi[];
    unsigned char *panel = lds_hi;                    // [buffer][plane a, plane b][row][kPitch]
    unsigned long long *rows = (unsigned long long *)(lds_hi + 4 * kHiRows * kPitch);
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    // tiles (row block, column block) in row-major order, a contiguous run of
    // them per XCD (blocks reach the 8 XCDs round-robin by index): the column
    // blocks of one row block run together on one XCD and share its L2 copy of
    // the row block's byte planes
    const int tiles = gridDim.x, per = tiles / kXcds, extra = tiles % kXcds;
    const int xcd = blockIdx.x % kXcds, k = blockIdx.x / kXcds;
    const int t = xcd * per + (xcd < extra ? xcd : extra) + k;
    const int rb = (t / ncb) * kHiRows;
    const int c0 = 256 * (t % ncb) + 16 * CT * wv;   // the wave's first column
    const bool active = c0 < 64 * W;
    const size_t Fp = (size_t)64 * W;
    if (tid < kHiRows) rows[tid] = 0ull;
    // panel producer: chunk -> (plane, row, 16 bytes of the step); rows < nbp are in the slab
    const int8_t *psrc[kItems];
    int pdst[kItems], pk[kItems];
    for (int p = 0; p < kItems; ++p) {
        const int it = tid + kThreads * p, pl = it / (kHiRows * KS * 4), r = (it / (KS * 4)) % kHiRows,
                  c = it % (KS * 4);
        pk[p] = c >> 2;                                // word of the step
        psrc[p] = (pl ? hs.ub : hs.ua) + (size_t)(rb + r) * Fp + 16 * c;
        pdst[p] = pl * kHiRows * kPitch + r * kPitch + 16 * c;
    }
    const int q = lane >> 4, c16 = lane & 15;
    const uint64_t *bt[CT];
    for (int j = 0; j < CT; ++j) bt[j] = hs.mt + (size_t)((active ? c0 : 0) + 16 * j + c16) * W;
    i32x4 accA[4][CT], accB[4][CT];
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < CT; ++j) {
            accA[i][j] = i32x4{0, 0, 0, 0};
            accB[i][j] = i32x4{0, 0, 0, 0};
        }
    i32x4 pa[kItems];
    uint64_t wt[CT][KS];
    auto fetch_a = [&](int kw0) {
        for (int p = 0; p < kItems; ++p)
            pa[p] = kw0 + pk[p] < W ? *(const i32x4 *)(psrc[p] + 64 * (size_t)kw0) : i32x4{0, 0, 0, 0};
    };
    fetch_a(0);
    for (int s = 0; s < KS; ++s)
        for (int j = 0; j < CT; ++j) wt[j][s] = (active && s < W) ? bt[j][s] : 0ull;
    const int steps = (W + KS - 1) / KS;
    for (int st = 0; st < steps; ++st) {
        unsigned char *pb = panel + (st & 1) * 2 * kHiRows * kPitch;
        for (int p = 0; p < kItems; ++p) *(i32x4 *)(pb + pdst[p]) = pa[p];
        fetch_a((st + 1) * KS);
        __syncthreads();
        for (int s = 0; s < KS; ++s) {  // (zero operands past W and for an inactive wave)
            i32x4 b[CT];
            for (int j = 0; j < CT; ++j) {
                b[j] = expand16((unsigned)(wt[j][s] >> (16 * q)) & 0xffffu);
                const int kw = (st + 1) * KS + s;
                wt[j][s] = (active && kw < W) ? bt[j][kw] : 0ull;
            }
            for (int i = 0; i < 4; ++i) {
                const int off = (16 * i + c16) * kPitch + 64 * s + 16 * q;
                const i32x4 a0 = *(const i32x4 *)(pb + off);
                const i32x4 a1 = *(const i32x4 *)(pb + kHiRows * kPitch + off);
                for (int j = 0; j < CT; ++j) {
                    accA[i][j] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a0, b[j], accA[i][j], 0, 0, 0);
                    accB[i][j] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a1, b[j], accB[i][j], 0, 0, 0);
                }
            }
        }
    }
    if (active) {
        unsigned long long p4[4][4];
        long long cs[CT];
        for (int j = 0; j < CT; ++j) cs[j] = 32896ll * hs.csum[c0 + 16 * j + c16];
        for (int i = 0; i < 4; ++i)
            for (int v = 0; v < 4; ++v) {
                const int rl = rb + 16 * i + 4 * q + v;
                unsigned long long s4 = 0;
                if (rl < nb)
                    for (int j = 0; j < CT; ++j) {
                        const int h = c0 + 16 * j + c16;
                        if (h < F) {
                            const long long x = (long long)accA[i][j][v] + 256ll * accB[i][j][v] + cs[j];
                            s4 += (unsigned long long)x * hs.v[(size_t)rl * Fp + h];
                        }
                    }
                p4[i][v] = s4;
            }
        add_rows(p4, rows);
    }
    __syncthreads();
    if (tid < kHiRows && rb + tid < nb)
        atomicAdd((unsigned long long *)&counts[(size_t)(n0 + rb + tid) * (K + 1) + 4], rows[tid]);
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

bool candidates_high_fits(int F) { return F >= 1 && F <= kCandHighMaxF; }

// The products' scratch inside the scene's pair scratch [cand, hi_end): M^T,
// c, then a slab of U planes and V as large as the rest holds (the layout
// guarantees kHiMinSlab snapshots), never more than N needs.
static bool hi_scratch(const Scene &sc, int N, HiScratch &hs) {
    const size_t W = (size_t)sc.dev.W, Fp = 64 * W;
    const size_t cap = sc.lay.hi_end - sc.lay.cand, fixed = Fp * W * 8 + Fp * 4;
    if (cap < fixed + (size_t)kHiRows * Fp * 4) return false;
    size_t nbp = (cap - fixed) / (4 * Fp) / kHiRows * kHiRows;
    const size_t need = ((size_t)N + kHiRows - 1) / kHiRows * kHiRows;
    if (nbp > need) nbp = need;
    char *p = (char *)sc.ws + sc.lay.cand;
    hs.mt = (uint64_t *)p;
    p += Fp * W * 8;
    hs.csum = (int *)p;
    p += Fp * 4;
    hs.ua = (int8_t *)p;
    p += nbp * Fp;
    hs.ub = (int8_t *)p;
    p += nbp * Fp;
    hs.v = (uint16_t *)p;
    hs.nbp = (int)nbp;
    return true;
}

hipError_t launch_candidates_high(const Scene &sc, const uint64_t *M, int N, const uint64_t *txv,
                                  const uint64_t *rxv, const uint8_t *los, int K, int64_t *counts, hipStream_t s) {
    if (N <= 0) return hipSuccess;
    const SceneDev &d = sc.dev;
    HiScratch hs;
    if (K < 3 || K > 4 || !candidates_high_fits(d.F) || !hi_scratch(sc, N, hs)) return hipErrorInvalidValue;
    hipError_t e = launch_fill_u32((uint32_t *)hs.csum, 0u, (size_t)64 * d.W, s);
    if (e != hipSuccess) return e;
    int chunks = (2048 + d.W - 1) / d.W;  // about 2048 transposing waves
    if (chunks > d.W) chunks = d.W;
    const long long tw = (long long)d.W * chunks;
    hipLaunchKernelGGL(k_hi_transpose, dim3((unsigned)((tw + 3) / 4)), dim3(256), 0, s, d.F, d.W, chunks, M, hs.mt,
                       hs.csum);
    hipLaunchKernelGGL(k_hi_init, dim3((unsigned)(((long long)N + 3) / 4)), dim3(256), 0, s, d.F, d.W, N, txv, rxv,
                       los, K, counts);
    constexpr size_t lds = hi_lds<kHiKs>();
    if ((e = hipFuncSetAttribute((const void *)k_hi_uv<kHiKs, kHiUct>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds)) !=
            hipSuccess ||
        (e = hipFuncSetAttribute((const void *)k_hi_x<kHiKs, kHiXct>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds)) !=
            hipSuccess)
        return e;
    const unsigned gy = (unsigned)((d.W + kHiWaves - 1) / kHiWaves);
    for (int n0 = 0; n0 < N; n0 += hs.nbp) {
        const int nb = N - n0 < hs.nbp ? N - n0 : hs.nbp;
        const dim3 grid((unsigned)((nb + kHiRows - 1) / kHiRows), gy);
        hipLaunchKernelGGL((k_hi_uv<kHiKs, kHiUct>), grid, dim3(64 * 16 / kHiUct), lds, s, d.F, d.W, N, n0, nb, txv, rxv, M, hs, K, counts);
        if (K >= 4)
            hipLaunchKernelGGL((k_hi_x<kHiKs, kHiXct>), dim3(grid.x * gy), dim3(64 * 16 / kHiXct), lds, s, d.F, d.W, n0,
                               nb, (int)gy, hs, K, counts);
    }
    return hipGetLastError();
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
