// mlp.hip -- the occluder-ordering network: pair features, GEMMs on BF16 MFMA
// (FP32 accumulation) or FP32 VALU, BCE-with-logits, Adam, and in-matrix
// inference that turns 32 treelet scores into a traversal order.
//
// The MFMA micro-kernel uses v_mfma_f32_16x16x16_bf16: lane l supplies
// A[l % 16][4 (l / 16) + v] and B[4 (l / 16) + v][l % 16] (v = 0..3) and
// receives D[4 (l / 16) + v][l % 16].
#include <cmath>

#include "ivm_internal.h"

namespace ivm {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// FP32 -> BF16, round to nearest even (inputs are finite).
__device__ inline short to_bf16(float x) {
    unsigned u = __float_as_uint(x);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (short)(u >> 16);
}

// ---------------------------------------------------------------------------
// pair features
// ---------------------------------------------------------------------------

__device__ inline void pair_features(const SceneDev &sc, int i, int j, float *x) {
    const float *fi = sc.ffeat + 8 * i, *fj = sc.ffeat + 8 * j;
    const float c0x = sc.fnorm[0], c0y = sc.fnorm[1], c0z = sc.fnorm[2], hs = sc.fnorm[3];
    for (int k = 0; k < 3; ++k) {
        x[k] = fi[k];
        x[3 + k] = fj[k];
        x[6 + k] = fi[3 + k];
        x[9 + k] = fj[3 + k];
    }
    x[12] = fi[6];
    x[13] = fj[6];
    const float dx = fj[0] - fi[0], dy = fj[1] - fi[1], dz = fj[2] - fi[2];
    const float dist = sqrtf(dx * dx + dy * dy + dz * dz);
    x[14] = dist;
    const float *bi = sc.fbox + 6 * i, *bj = sc.fbox + 6 * j;
    const float c0[3] = {c0x, c0y, c0z};
    for (int k = 0; k < 3; ++k) {
        x[15 + k] = (fminf(bi[k], bj[k]) - c0[k]) / hs;
        x[18 + k] = (fmaxf(bi[3 + k], bj[3 + k]) - c0[k]) / hs;
    }
    const float inv = dist > 0.f ? 1.0f / dist : 0.f;
    x[21] = dx * inv;
    x[22] = dy * inv;
    x[23] = dz * inv;
}

__global__ void k_pair_features(SceneDev sc, int n, const int32_t *I, const int32_t *J, float *X) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    int i = I[k], j = J[k];
    if (i < 0 || j < 0 || i >= sc.F || j >= sc.F) {
        for (int m = 0; m < kIn; ++m) X[(size_t)k * kIn + m] = 0.f;
        return;
    }
    float x[kIn];
    pair_features(sc, i, j, x);
    for (int m = 0; m < kIn; ++m) X[(size_t)k * kIn + m] = x[m];
}

hipError_t launch_pair_features(const SceneDev &d, int n, const int32_t *I, const int32_t *J, float *X, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_pair_features, dim3((n + 255) / 256), dim3(256), 0, s, d, n, I, J, X);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// GEMM: C[m][n] (+)= sum_k A(m, k) B(k, n) (+ bias[n], ReLU), strided operands
// ---------------------------------------------------------------------------

struct GemmArgs {
    int M, N, K;
    const float *A;
    int sam, sak;
    const float *B;
    int sbk, sbn;
    float *C;
    int ldc;
    const float *bias;
    int relu;
};

__global__ __launch_bounds__(256) void k_gemm_bf16(GemmArgs g) {
    const int lane = threadIdx.x & 63;
    const int wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int tn_count = (g.N + 15) / 16;
    const int tiles = ((g.M + 15) / 16) * tn_count;
    if (wave >= tiles) return;
    const int tm = wave / tn_count, tn = wave - (wave / tn_count) * tn_count;
    const int row = tm * 16 + (lane & 15), col = tn * 16 + (lane & 15), kq = 4 * (lane >> 4);
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < g.K; k0 += 16) {
        bf16x4 a, b;
        for (int v = 0; v < 4; ++v) {
            const int k = k0 + kq + v;
            a[v] = (row < g.M && k < g.K) ? to_bf16(g.A[(size_t)row * g.sam + (size_t)k * g.sak]) : (short)0;
            b[v] = (col < g.N && k < g.K) ? to_bf16(g.B[(size_t)k * g.sbk + (size_t)col * g.sbn]) : (short)0;
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
    }
    for (int v = 0; v < 4; ++v) {
        const int m = tm * 16 + kq + v;
        if (m < g.M && col < g.N) {
            float val = acc[v] + (g.bias ? g.bias[col] : 0.f);
            if (g.relu) val = fmaxf(val, 0.f);
            g.C[(size_t)m * g.ldc + col] = val;
        }
    }
}

__global__ void k_gemm_f32(GemmArgs g) {
    const long long id = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (id >= (long long)g.M * g.N) return;
    const int m = (int)(id / g.N), n = (int)(id - (id / g.N) * g.N);
    float acc = 0.f;
    for (int k = 0; k < g.K; ++k) acc = fmaf(g.A[(size_t)m * g.sam + (size_t)k * g.sak], g.B[(size_t)k * g.sbk + (size_t)n * g.sbn], acc);
    float val = acc + (g.bias ? g.bias[n] : 0.f);
    if (g.relu) val = fmaxf(val, 0.f);
    g.C[(size_t)m * g.ldc + n] = val;
}

static hipError_t gemm(const Model &md, const GemmArgs &g, hipStream_t s) {
    if (g.M <= 0 || g.N <= 0) return hipSuccess;
    if (md.precision == IVM_MODEL_FP32) {
        const long long n = (long long)g.M * g.N;
        hipLaunchKernelGGL(k_gemm_f32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, g);
    } else {
        const int tiles = ((g.M + 15) / 16) * ((g.N + 15) / 16);
        hipLaunchKernelGGL(k_gemm_bf16, dim3((tiles + 3) / 4), dim3(256), 0, s, g);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// loss, element-wise backward steps, bias gradients, Adam
// ---------------------------------------------------------------------------

// loss += mean BCE-with-logits; dz = (sigmoid(z) - y) / (n * 32)
__global__ void k_bce(int n, const float *z, const float *y, float *dz, float *loss) {
    __shared__ float red[256];
    const int id = blockIdx.x * blockDim.x + threadIdx.x;
    const int tot = n * kOut;
    float l = 0.f;
    if (id < tot) {
        const float zz = z[id], yy = y[id];
        l = fmaxf(zz, 0.f) - zz * yy + log1pf(expf(-fabsf(zz)));
        dz[id] = (1.0f / (1.0f + expf(-zz)) - yy) / (float)tot;
    }
    red[threadIdx.x] = l;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0 && loss) atomicAdd(loss, red[0] / (float)tot);
}

// dz *= (h > 0): ReLU derivative from the stored activation
__global__ void k_relu_mask(int n, float *dz, const float *h) {
    const int id = blockIdx.x * blockDim.x + threadIdx.x;
    if (id < n && !(h[id] > 0.f)) dz[id] = 0.f;
}

// db[c] = sum over rows of dz[r][c]
__global__ void k_colsum(int rows, int cols, const float *dz, float *db) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= cols) return;
    float acc = 0.f;
    for (int r = 0; r < rows; ++r) acc += dz[(size_t)r * cols + c];
    db[c] = acc;
}

__global__ void k_adam(int n, float *p, const float *g, float *m, float *v, float lr, float bc1, float bc2) {
    const int id = blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= n) return;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float gg = g[id];
    const float mm = b1 * m[id] + (1.f - b1) * gg;
    const float vv = b2 * v[id] + (1.f - b2) * gg * gg;
    m[id] = mm;
    v[id] = vv;
    p[id] -= lr * (mm / bc1) / (sqrtf(vv / bc2) + eps);
}

__global__ void k_zero_f32(float *p, int n) {
    const int id = blockIdx.x * blockDim.x + threadIdx.x;
    if (id < n) p[id] = 0.f;
}

size_t model_workspace_bytes(int max_batch) {
    const size_t P = kParams, B = (size_t)(max_batch > 0 ? max_batch : 1);
    size_t floats = 4 * P + B * (3 * kHid + kOut + 2 * kHid) + 64;
    return (floats * sizeof(float) + 255) & ~size_t(255);
}

void model_bind(Model &m, void *ws, int max_batch, int precision) {
    float *f = (float *)ws;
    const size_t P = kParams, B = (size_t)max_batch;
    m.max_batch = max_batch;
    m.precision = precision;
    m.params = f; f += P;
    m.grad = f; f += P;
    m.m = f; f += P;
    m.v = f; f += P;
    m.h0 = f; f += B * kHid;
    m.h1 = f; f += B * kHid;
    m.h2 = f; f += B * kHid;
    m.logits = f; f += B * kOut;
    m.d0 = f; f += B * kHid;
    m.d1 = f; f += B * kHid;
    m.loss = f;
    m.step = 0;
}

static GemmArgs fwd_args(int n, const float *H, int kin, const float *W, const float *b, float *out, int nout, int relu) {
    GemmArgs g{};
    g.M = n; g.N = nout; g.K = kin;
    g.A = H; g.sam = kin; g.sak = 1;
    g.B = W; g.sbk = 1; g.sbn = kin;
    g.C = out; g.ldc = nout; g.bias = b; g.relu = relu;
    return g;
}

hipError_t model_forward(Model &m, int n, const float *X, hipStream_t s) {
    const float *P = m.params;
    hipError_t e;
    if ((e = gemm(m, fwd_args(n, X, kIn, P + kOffW0, P + kOffB0, m.h0, kHid, 1), s)) != hipSuccess) return e;
    if ((e = gemm(m, fwd_args(n, m.h0, kHid, P + kOffW1, P + kOffB1, m.h1, kHid, 1), s)) != hipSuccess) return e;
    if ((e = gemm(m, fwd_args(n, m.h1, kHid, P + kOffW2, P + kOffB2, m.h2, kHid, 1), s)) != hipSuccess) return e;
    return gemm(m, fwd_args(n, m.h2, kHid, P + kOffW3, P + kOffB3, m.logits, kOut, 0), s);
}

// dW = dZ^T H (nout x kin), db = column sums of dZ, and (when dH != nullptr) dH = dZ W.
static hipError_t layer_backward(Model &m, int n, const float *dZ, int nout, const float *H, int kin, const float *W,
                                 float *dW, float *db, float *dH, hipStream_t s) {
    GemmArgs g{};
    g.M = nout; g.N = kin; g.K = n;
    g.A = dZ; g.sam = 1; g.sak = nout;
    g.B = H; g.sbk = kin; g.sbn = 1;
    g.C = dW; g.ldc = kin; g.bias = nullptr; g.relu = 0;
    hipError_t e = gemm(m, g, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_colsum, dim3((nout + 127) / 128), dim3(128), 0, s, n, nout, dZ, db);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (dH) {
        GemmArgs h{};
        h.M = n; h.N = kin; h.K = nout;
        h.A = dZ; h.sam = nout; h.sak = 1;
        h.B = W; h.sbk = kin; h.sbn = 1;
        h.C = dH; h.ldc = kin; h.bias = nullptr; h.relu = 0;
        if ((e = gemm(m, h, s)) != hipSuccess) return e;
    }
    return hipSuccess;
}

// Forward, loss (added to m.loss, which the caller zeroes) and gradient into `grad`.
hipError_t model_backward(Model &m, int n, const float *X, const float *Y, float *grad, hipStream_t s) {
    hipError_t e;
    if ((e = model_forward(m, n, X, s)) != hipSuccess) return e;
    const float *P = m.params;
    const int tot = n * kOut;
    // dZ3 in d1 (n x 32)
    hipLaunchKernelGGL(k_bce, dim3((tot + 255) / 256), dim3(256), 0, s, n, m.logits, Y, m.d1, m.loss);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // layer 3: dW3, db3, dH2 -> d0
    if ((e = layer_backward(m, n, m.d1, kOut, m.h2, kHid, P + kOffW3, grad + kOffW3, grad + kOffB3, m.d0, s)) != hipSuccess)
        return e;
    hipLaunchKernelGGL(k_relu_mask, dim3((n * kHid + 255) / 256), dim3(256), 0, s, n * kHid, m.d0, m.h2);
    // layer 2: dH1 -> d1
    if ((e = layer_backward(m, n, m.d0, kHid, m.h1, kHid, P + kOffW2, grad + kOffW2, grad + kOffB2, m.d1, s)) != hipSuccess)
        return e;
    hipLaunchKernelGGL(k_relu_mask, dim3((n * kHid + 255) / 256), dim3(256), 0, s, n * kHid, m.d1, m.h1);
    // layer 1: dH0 -> d0
    if ((e = layer_backward(m, n, m.d1, kHid, m.h0, kHid, P + kOffW1, grad + kOffW1, grad + kOffB1, m.d0, s)) != hipSuccess)
        return e;
    hipLaunchKernelGGL(k_relu_mask, dim3((n * kHid + 255) / 256), dim3(256), 0, s, n * kHid, m.d0, m.h0);
    // layer 0: no input gradient
    return layer_backward(m, n, m.d0, kHid, X, kIn, P + kOffW0, grad + kOffW0, grad + kOffB0, nullptr, s);
}

hipError_t model_adam(Model &m, float lr, hipStream_t s) {
    m.step += 1;
    const float bc1 = 1.0f - powf(0.9f, (float)m.step), bc2 = 1.0f - powf(0.999f, (float)m.step);
    hipLaunchKernelGGL(k_adam, dim3((kParams + 255) / 256), dim3(256), 0, s, kParams, m.params, m.grad, m.m, m.v, lr,
                       bc1, bc2);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// inference inside the matrix call: 16 candidate pairs per wave
// ---------------------------------------------------------------------------

__device__ inline void decode_candidate(const SceneDev &sc, const uint64_t *cand, const uint32_t *prefix, int n_items,
                                        uint32_t g, int &i, int &j) {
    int lo = 0, hi = n_items - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (prefix[mid] <= g) lo = mid;
        else hi = mid - 1;
    }
    unsigned long long m = cand[lo];
    for (uint32_t q = prefix[lo]; q < g; ++q) m &= m - 1;
    const int bit = __ffsll((long long)m) - 1;
    i = lo / sc.W;
    j = (lo - i * sc.W) * 64 + bit;
}

__device__ inline void wave_fence() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// In-call inference for the learned order.  Each block stages the network in
// LDS once: every weight rounded to BF16 (the rounding the MFMA inputs get
// anyway; biases are read in FP32 from global memory), rows padded so that the
// 16 rows an MFMA step reads fall in different LDS banks; then its kLearnWaves
// waves score 16 pairs at a time with the same 16 x 16 x 16 BF16 MFMA steps in
// the same order as the training forward pass.  Hidden activations are kept as
// BF16 (each is rounded to BF16 as the next layer's input), the scores as FP32.
// learned[g] = top-12 treelets by score, 5 bits each (best first), count in the
// top 4 bits.  NaN scores rank as -inf; ties go to the lower treelet index.
constexpr int kLearnWaves = 5;
constexpr int kRowIn = kIn + 4;     // padded row of W0 (BF16 elements)
constexpr int kRowHid = kHid + 16;  // padded rows of W1..W3 and of the activations: 72 words, 8 banks apart
constexpr int kLdsW0 = 0, kLdsW1 = kLdsW0 + kHid * kRowIn, kLdsW2 = kLdsW1 + kHid * kRowHid;
constexpr int kLdsW3 = kLdsW2 + kHid * kRowHid, kLdsWEnd = kLdsW3 + kOut * kRowHid;
constexpr size_t kLearnLds = sizeof(short) * kLdsWEnd + sizeof(short) * kLearnWaves * 2 * 16 * kRowHid +
                             sizeof(float) * kLearnWaves * 16 * kOut;

// act: [16][kRowHid] BF16 rows (LDS); W: [nout][ldw] BF16 (LDS); b: FP32 biases.
// Writes out_bf[16][kRowHid] (BF16, + bias, ReLU) or, for the last layer, out_f[16][kOut] (FP32).
__device__ inline void mlp_layer16_lds(const short *act, int kin, const short *W, int ldw, const float *b, int nout,
                                       short *out_bf, float *out_f, bool relu) {
    const int lane = threadIdx.x & 63;
    const int r = lane & 15, kq = 4 * (lane >> 4);
    for (int n0 = 0; n0 < nout; n0 += 16) {
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        for (int k0 = 0; k0 < kin; k0 += 16) {
            bf16x4 a, bb;
            if (k0 + 16 <= kin) {
                a = *(const bf16x4 *)(act + r * kRowHid + k0 + kq);
                bb = *(const bf16x4 *)(W + (n0 + r) * ldw + k0 + kq);
            } else {
                for (int v = 0; v < 4; ++v) {
                    const int k = k0 + kq + v;
                    a[v] = k < kin ? act[r * kRowHid + k] : (short)0;
                    bb[v] = k < kin ? W[(n0 + r) * ldw + k] : (short)0;
                }
            }
            acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, bb, acc, 0, 0, 0);
        }
        for (int v = 0; v < 4; ++v) {
            float val = acc[v] + b[n0 + r];
            if (relu) val = fmaxf(val, 0.f);
            if (out_f) out_f[(kq + v) * kOut + n0 + r] = val;
            else out_bf[(kq + v) * kRowHid + n0 + r] = to_bf16(val);
        }
    }
}

__global__ __launch_bounds__(64 * kLearnWaves) void k_learned(SceneDev sc, const uint64_t *cand,
                                                              const uint32_t *prefix, int n_items, const float *params,
                                                              uint64_t *learned) {
    extern __shared__ __align__(16) unsigned char lds[];
    short *sW = (short *)lds;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    short *actA = (short *)(lds + sizeof(short) * kLdsWEnd) + wv * 2 * 16 * kRowHid;
    short *actB = actA + 16 * kRowHid;
    float *outS = (float *)(lds + sizeof(short) * kLdsWEnd + sizeof(short) * kLearnWaves * 2 * 16 * kRowHid) +
                  wv * 16 * kOut;
    // stage the four weight matrices into their padded rows
    auto stage = [&](int off, int rows, int cols, int dst, int ld) {
        for (int k = threadIdx.x; k < rows * cols; k += blockDim.x) {
            const int rr = k / cols, cc = k - rr * cols;
            sW[dst + rr * ld + cc] = to_bf16(params[off + k]);
        }
    };
    stage(kOffW0, kHid, kIn, kLdsW0, kRowIn);
    stage(kOffW1, kHid, kHid, kLdsW1, kRowHid);
    stage(kOffW2, kHid, kHid, kLdsW2, kRowHid);
    stage(kOffW3, kOut, kHid, kLdsW3, kRowHid);
    __syncthreads();
    const uint32_t total = prefix[n_items];
    const uint32_t stride = gridDim.x * (uint32_t)kLearnWaves * 16u;
    for (uint32_t g0 = (blockIdx.x * (uint32_t)kLearnWaves + (uint32_t)wv) * 16u; g0 < total; g0 += stride) {
        if (lane < 16) {
            float x[kIn];
            if (g0 + lane < total) {
                int i, j;
                decode_candidate(sc, cand, prefix, n_items, g0 + lane, i, j);
                pair_features(sc, i, j, x);
            } else {
                for (int m = 0; m < kIn; ++m) x[m] = 0.f;
            }
            for (int m = 0; m < kIn; ++m) actA[lane * kRowHid + m] = to_bf16(x[m]);
        }
        wave_fence();
        mlp_layer16_lds(actA, kIn, sW + kLdsW0, kRowIn, params + kOffB0, kHid, actB, nullptr, true);
        wave_fence();
        mlp_layer16_lds(actB, kHid, sW + kLdsW1, kRowHid, params + kOffB1, kHid, actA, nullptr, true);
        wave_fence();
        mlp_layer16_lds(actA, kHid, sW + kLdsW2, kRowHid, params + kOffB2, kHid, actB, nullptr, true);
        wave_fence();
        mlp_layer16_lds(actB, kHid, sW + kLdsW3, kRowHid, params + kOffB3, kOut, nullptr, outS, false);
        wave_fence();
        for (int p = 0; p < 16 && g0 + p < total; ++p) {
            float sv = lane < kOut ? outS[p * kOut + lane] : -INFINITY;
            if (sv != sv) sv = -INFINITY;
            unsigned long long code = 0;
            if (lane < kOut) {
                int rank = 0;
                for (int m = 0; m < kOut; ++m) {
                    float sm = outS[p * kOut + m];
                    if (sm != sm) sm = -INFINITY;
                    rank += (sm > sv) || (sm == sv && m < lane);
                }
                if (rank < 12) code = (unsigned long long)lane << (5 * rank);
            }
            for (int o = 32; o >= 1; o >>= 1) code |= __shfl_xor(code, o);
            if (lane == 0) learned[g0 + p] = code | (12ull << 60);
        }
        wave_fence();
    }
}

hipError_t launch_learned_order(Scene &scn, const Model &m, hipStream_t s) {
    char *ws = (char *)scn.ws;
    const Layout &L = scn.lay;
    hipError_t e = hipFuncSetAttribute((const void *)k_learned, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)kLearnLds);
    if (e != hipSuccess) return e;
    // one block per CU (the staged network fills most of its LDS), over the pairs
    // the probes left undecided (the ones the pair kernel visits)
    hipLaunchKernelGGL(k_learned, dim3(device_cu_count()), dim3(64 * kLearnWaves), kLearnLds, s, scn.dev,
                       (const uint64_t *)(ws + L.und), (const uint32_t *)(ws + L.uprefix), scn.n_items,
                       (const float *)m.params, (uint64_t *)(ws + L.learned));
    return hipGetLastError();
}

}  // namespace ivm
