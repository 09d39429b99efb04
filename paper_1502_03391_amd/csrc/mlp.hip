// Warm-start network kernels for gfx950: BF16 matrix-core GEMM with FP32
// accumulation and fused epilogues, MSE loss and gradient, bias gradients,
// Adam, and the landmark feature gather.
//
// The network maps an out-of-sample object's dissimilarities to a fixed set
// of in-sample landmark objects (every modality) to a starting point y for
// the Section 3 out-of-sample iteration.  Layers: z = h W + b, h' = GELU(z)
// (exact x Phi(x)) except after the last layer.  Weights are FP32 masters
// with BF16 copies for the products; activations and the gradients used as
// product operands are stored in BF16; accumulation is FP32.
#include "fjofc_internal.h"

#include <cstdlib>

#include <algorithm>

namespace fjofc {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));

// FP32 -> BF16, round to nearest even (finite inputs).
__device__ __forceinline__ uint16_t f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float gelu(float z) {
    return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f));
}

__device__ __forceinline__ float gelu_grad(float z) {
    return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) +
           z * 0.39894228040143268f * expf(-0.5f * z * z);
}

// C (M x N) = A (M x K) B (K x N), both operands k-contiguous: A(m, k) =
// A[m lda + k], B(k, n) = Bt[n ldb + k] (the library keeps transposed BF16
// copies of weights, activations and gradients, so every product reads
// both operands this way).  A workgroup of 2 x 2 wavefronts covers 64 x 64
// outputs (one wavefront, 32 x 32, for small products), each wavefront
// 32 x 32 as 2 x 2 tiles of the gfx950 BF16 matrix instruction 16x16x32
// (FP32 accumulation).  Operand layout of that
// instruction: lane l supplies A[l % 16][8 (l / 16) + e] and
// B[8 (l / 16) + e][l % 16], e = 0..7 (16 contiguous bytes of a k-row), and
// receives C[4 (l / 16) + v][l % 16], v = 0..3.  Fragments are loaded
// straight from global memory (L2-resident at these sizes), three K steps
// ahead of the one being multiplied.
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
constexpr int GB = 64, GK = 32, GNB = 4;

union Frag {
    uint4 u;
    bf8 v;
    uint16_t h[8];
};

// Elements p[r ld + k .. k + 7], zero past R rows or K columns.  VEC: rows
// are 16-byte aligned, so a whole in-range chunk is one 16-byte load.
template <bool VEC>
__device__ __forceinline__ bf8 load_frag(const uint16_t *__restrict__ p, long ld, int r, int R,
                                         int k, int K) {
    Frag f;
    if (VEC && r < R && k + 8 <= K) {
        f.u = *reinterpret_cast<const uint4 *>(p + (long)r * ld + k);
    } else {
#pragma unroll
        for (int e = 0; e < 8; ++e)
            f.h[e] = (r < R && k + e < K) ? p[(long)r * ld + k + e] : (uint16_t)0;
    }
    return f.v;
}

// The epilogue of a wavefront's 32 x 32 outputs (acc[i][j] holds rows
// m0 + 16 i + 4 (lane / 16) + v, column n0 + 16 j + lane % 16).
template <int EPI>
__device__ __forceinline__ void gemm_store(const f4 (&acc)[2][2], int M, int N, int m0, int n0,
                                           int lane, const GemmEpi &e) {
    const int li = lane & 15;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int col = n0 + 16 * j + li;
            const int rb = m0 + 16 * i + 4 * (lane >> 4);
            if (col >= N) continue;
            uint16_t hb[4];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = rb + v;
                hb[v] = 0;
                if (row >= M) continue;
                const long o = (long)row * e.ldc + col;
                const float x = acc[i][j][v];
                if (EPI == GEMM_HIDDEN) {
                    const float z = x + e.bias[col];
                    e.outf[o] = z;
                    hb[v] = f2bf(gelu(z));
                    e.outb[o] = hb[v];
                } else if (EPI == GEMM_LAST) {
                    e.outf[o] = x + e.bias[col];
                } else if (EPI == GEMM_BWD) {
                    const float g = x * gelu_grad(e.Z[o]);
                    e.outf[o] = g;
                    hb[v] = f2bf(g);
                    e.outb[o] = hb[v];
                } else {
                    e.outf[o] = x;
                }
            }
            if ((EPI == GEMM_HIDDEN || EPI == GEMM_BWD) && e.outbT) {
                uint16_t *t = e.outbT + (long)col * e.ldt + rb;
                if (rb + 4 <= M && (e.ldt & 3) == 0) {
                    uint2 w;
                    w.x = (uint32_t)hb[0] | ((uint32_t)hb[1] << 16);
                    w.y = (uint32_t)hb[2] | ((uint32_t)hb[3] << 16);
                    *reinterpret_cast<uint2 *>(t) = w;
                } else {
#pragma unroll
                    for (int v = 0; v < 4; ++v)
                        if (rb + v < M) t[v] = hb[v];
                }
            }
        }
}

// WM x WN wavefronts per workgroup (a 32 WM x 32 WN output tile).
template <int EPI, bool VEC, int WM, int WN>
__global__ __launch_bounds__(WAVE *WM *WN) void gemm_kernel(int M, int N, int K,
                                                            const uint16_t *__restrict__ A,
                                                            long lda,
                                                            const uint16_t *__restrict__ Bt,
                                                            long ldb, GemmEpi e) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int m0 = blockIdx.y * (32 * WM) + (wv / WN) * 32;
    const int n0 = blockIdx.x * (32 * WN) + (wv % WN) * 32;
    const int li = lane & 15, lk = (lane >> 4) * 8;
    f4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
    // ring of GNB register stages: the loads of K step s + GNB - 1 are issued
    // before step s is multiplied
    bf8 a[GNB][2], b[GNB][2];
#pragma unroll
    for (int st = 0; st < GNB - 1; ++st)
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            a[st][i] = load_frag<VEC>(A, lda, m0 + 16 * i + li, M, st * GK + lk, K);
            b[st][i] = load_frag<VEC>(Bt, ldb, n0 + 16 * i + li, N, st * GK + lk, K);
        }
    for (int k0 = 0; k0 < K; k0 += GNB * GK) {
#pragma unroll
        for (int u = 0; u < GNB; ++u) {
            const int kk = k0 + u * GK;
            if (kk >= K) break;
            const int kn = kk + (GNB - 1) * GK, un = (u + GNB - 1) % GNB;
            if (kn < K) {
#pragma unroll
                for (int i = 0; i < 2; ++i) {
                    a[un][i] = load_frag<VEC>(A, lda, m0 + 16 * i + li, M, kn + lk, K);
                    b[un][i] = load_frag<VEC>(Bt, ldb, n0 + 16 * i + li, N, kn + lk, K);
                }
            }
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[u][i], b[u][j], acc[i][j],
                                                                        0, 0, 0);
        }
    }
    gemm_store<EPI>(acc, M, N, m0, n0, lane, e);
}

// Split K: a workgroup of GSK wavefronts per 32 x 32 output tile, wavefront
// w multiplying the w-th quarter of K (in GK steps, all of its loads issued
// ahead through the same register ring), the partial tiles then added
// through LDS in a fixed order (0 + (1 + (2 + 3))) before wavefront 0's
// epilogue.  Small products (few output tiles, K of a few hundred) are
// otherwise a chain of dependent K steps on too few wavefronts.
constexpr int GSK = 4;
template <int EPI, bool VEC>
__global__ __launch_bounds__(WAVE *GSK) void gemm_sk_kernel(int M, int N, int K,
                                                           const uint16_t *__restrict__ A,
                                                           long lda,
                                                           const uint16_t *__restrict__ Bt,
                                                           long ldb, GemmEpi e) {
    __shared__ f4 red[GSK - 1][4][WAVE];
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int m0 = blockIdx.y * 32, n0 = blockIdx.x * 32;
    const int li = lane & 15, lk = (lane >> 4) * 8;
    const int steps = (K + GK - 1) / GK;
    const int per = (steps + GSK - 1) / GSK;
    const int kb = wv * per * GK, ke = min(K, kb + per * GK);
    f4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
    bf8 a[GNB][2], b[GNB][2];
#pragma unroll
    for (int st = 0; st < GNB - 1; ++st)
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            a[st][i] = load_frag<VEC>(A, lda, m0 + 16 * i + li, M, kb + st * GK + lk, ke);
            b[st][i] = load_frag<VEC>(Bt, ldb, n0 + 16 * i + li, N, kb + st * GK + lk, ke);
        }
    for (int k0 = kb; k0 < ke; k0 += GNB * GK) {
#pragma unroll
        for (int u = 0; u < GNB; ++u) {
            const int kk = k0 + u * GK;
            if (kk >= ke) break;
            const int kn = kk + (GNB - 1) * GK, un = (u + GNB - 1) % GNB;
            if (kn < ke) {
#pragma unroll
                for (int i = 0; i < 2; ++i) {
                    a[un][i] = load_frag<VEC>(A, lda, m0 + 16 * i + li, M, kn + lk, ke);
                    b[un][i] = load_frag<VEC>(Bt, ldb, n0 + 16 * i + li, N, kn + lk, ke);
                }
            }
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[u][i], b[u][j], acc[i][j],
                                                                        0, 0, 0);
        }
    }
    if (wv > 0) {
#pragma unroll
        for (int q = 0; q < 4; ++q) red[wv - 1][q][lane] = acc[q >> 1][q & 1];
    }
    __syncthreads();
    if (wv != 0) return;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        f4 t = red[GSK - 2][q][lane];
#pragma unroll
        for (int w = GSK - 3; w >= 0; --w) t = red[w][q][lane] + t;
        acc[q >> 1][q & 1] += t;
    }
    gemm_store<EPI>(acc, M, N, m0, n0, lane, e);
}

// out (C x R) = transpose of in (R x C), BF16, through a 32 x 33 LDS tile.
__global__ __launch_bounds__(256) void transpose16_kernel(const uint16_t *__restrict__ in,
                                                          long ld_in, int R, int C,
                                                          uint16_t *__restrict__ out,
                                                          long ld_out) {
    __shared__ uint16_t t[32][33];
    const int c0 = blockIdx.x * 32, r0 = blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (int q = ty; q < 32; q += 8) {
        const int r = r0 + q, c = c0 + tx;
        t[q][tx] = (r < R && c < C) ? in[(long)r * ld_in + c] : (uint16_t)0;
    }
    __syncthreads();
    for (int q = ty; q < 32; q += 8) {
        const int c = c0 + q, r = r0 + tx;
        if (c < C && r < R) out[(long)c * ld_out + r] = t[tx][q];
    }
}

// MSE over the batch and outputs: g = 2 (out - y) / (B k) (FP32 and BF16,
// and BF16 transposed when GbT is given); each workgroup adds its part of
// sum (out - y)^2 in FP64 into part[blockIdx.x] (fixed order inside).
constexpr int MSE_BLOCKS = 64;
__global__ __launch_bounds__(256) void mse_kernel(const float *__restrict__ out,
                                                  const float *__restrict__ y, int B, int k,
                                                  float *__restrict__ G, uint16_t *__restrict__ Gb,
                                                  uint16_t *__restrict__ GbT, long ldt,
                                                  double *__restrict__ part) {
    __shared__ double sh[256];
    const long tot = (long)B * k;
    const float sc = 2.0f / (float)tot;
    double s = 0.0;
    for (long q = blockIdx.x * 256L + threadIdx.x; q < tot; q += 256L * gridDim.x) {
        const float d = out[q] - y[q];
        s += (double)d * d;
        const float g = sc * d;
        G[q] = g;
        const uint16_t gb = f2bf(g);
        Gb[q] = gb;
        if (GbT) GbT[(q % k) * ldt + q / k] = gb;
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// loss = (sum of the MSE_BLOCKS parts, in order) / (B k).
__global__ void mse_finish_kernel(const double *__restrict__ part, long tot,
                                  double *__restrict__ loss, int accumulate) {
    double s = 0.0;
    for (int q = 0; q < MSE_BLOCKS; ++q) s += part[q];
    loss[0] = accumulate ? loss[0] + s / (double)tot : s / (double)tot;
}

// Bias gradient: column sums of G (B x N), two passes.  Pass 1: workgroup
// (column block of 32, row slice) sums its rows in FP64 with 8 row groups
// and writes one partial per column and slice; pass 2 adds the slices in
// order.  The result does not depend on scheduling.
constexpr int CS_COLS = 32, CS_GROUPS = 8, CS_SLICES = 16;
__global__ __launch_bounds__(CS_COLS *CS_GROUPS) void colsum_part_kernel(
    const float *__restrict__ G, int B, int N, double *__restrict__ part) {
    __shared__ double sh[CS_GROUPS][CS_COLS];
    const int cl = threadIdx.x % CS_COLS, g = threadIdx.x / CS_COLS;
    const int c = blockIdx.x * CS_COLS + cl;
    const int rows = (B + CS_SLICES - 1) / CS_SLICES;
    const int r0 = blockIdx.y * rows, r1 = min(B, r0 + rows);
    double s0 = 0.0, s1 = 0.0;
    if (c < N) {
        int r = r0 + g;
        for (; r + CS_GROUPS < r1; r += 2 * CS_GROUPS) {
            s0 += (double)G[(long)r * N + c];
            s1 += (double)G[(long)(r + CS_GROUPS) * N + c];
        }
        if (r < r1) s0 += (double)G[(long)r * N + c];
    }
    sh[g][cl] = s0 + s1;
    __syncthreads();
    if (g == 0 && c < N) {
        double t = 0.0;
        for (int q = 0; q < CS_GROUPS; ++q) t += sh[q][cl];
        part[(long)blockIdx.y * N + c] = t;
    }
}

__global__ void colsum_finish_kernel(const double *__restrict__ part, int N,
                                     float *__restrict__ db) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= N) return;
    double t = 0.0;
    for (int q = 0; q < CS_SLICES; ++q) t += part[(long)q * N + c];
    db[c] = (float)t;
}

// Adam with bias correction on the FP32 masters; refreshes the BF16 copy.
__global__ void adam_kernel(float *__restrict__ p, const float *__restrict__ g,
                            float *__restrict__ m, float *__restrict__ v,
                            uint16_t *__restrict__ p16, long n, float lr, float b1, float b2,
                            float eps, float c1, float c2) {
    for (long q = blockIdx.x * (long)blockDim.x + threadIdx.x; q < n;
         q += (long)gridDim.x * blockDim.x) {
        const float gq = g[q];
        const float mq = b1 * m[q] + (1.0f - b1) * gq;
        const float vq = b2 * v[q] + (1.0f - b2) * gq * gq;
        m[q] = mq;
        v[q] = vq;
        const float pq = p[q] - lr * (mq / c1) / (sqrtf(vq / c2) + eps);
        p[q] = pq;
        p16[q] = f2bf(pq);
    }
}

__global__ void to_bf16_kernel(const float *__restrict__ x, uint16_t *__restrict__ y, long n) {
    for (long q = blockIdx.x * (long)blockDim.x + threadIdx.x; q < n;
         q += (long)gridDim.x * blockDim.x)
        y[q] = f2bf(x[q]);
}

// Landmark features of new objects: x[o][i L + l] =
// bf16((delta_new[o][i][lm[l]] - mu[i L + l]) * inv_sd[i L + l]).
__global__ void features_kernel(const float *__restrict__ dnew, int k, int m, int n,
                                const int *__restrict__ lm, int L, const float *__restrict__ mu,
                                const float *__restrict__ isd, uint16_t *__restrict__ x) {
    const long tot = (long)k * m * L;
    for (long q = blockIdx.x * (long)blockDim.x + threadIdx.x; q < tot;
         q += (long)gridDim.x * blockDim.x) {
        const long o = q / ((long)m * L);
        const int f = (int)(q - o * m * L);
        const int i = f / L, l = f - i * L;
        const int j = min(max(lm[l], 0), n - 1);  // indices are validated by the caller
        const float d = dnew[(o * m + i) * n + j];
        x[q] = f2bf((d - mu[f]) * isd[f]);
    }
}

// Start configuration of the out-of-sample iteration from the network's
// consensus point: Y[o][i][c] = out[o][c] for every modality i.
__global__ void broadcast_kernel(const float *__restrict__ out, int B, int m, int d, int P,
                                 float *__restrict__ Y) {
    const long tot = (long)B * m * d;
    for (long q = blockIdx.x * (long)blockDim.x + threadIdx.x; q < tot;
         q += (long)gridDim.x * blockDim.x) {
        const long o = q / ((long)m * d);
        const int c = P == d ? (int)(q % d) : (int)(q - o * m * d);
        Y[q] = out[o * P + c];
    }
}

// Per-feature statistics of an N x F FP32 matrix (row-major), for the
// standardisation of the network's inputs.  Pass 0: slice partials of the
// column sums; pass 1: slice partials of the squared deviations from the
// FP64 mean.  Slice s takes rows s, s + STAT_SLICES, ...; consecutive threads
// read consecutive features of a row.  All sums FP64, fixed order.
constexpr int STAT_SLICES = 256;
template <int PASS>
__global__ __launch_bounds__(256) void colstats_part_kernel(const float *__restrict__ raw,
                                                            long N, int F,
                                                            const double *__restrict__ mean,
                                                            double *__restrict__ part) {
    const int f = blockIdx.x * 256 + threadIdx.x;
    if (f >= F) return;
    const double c = PASS == 0 ? 0.0 : mean[f];
    double a0 = 0.0, a1 = 0.0;
    long r = blockIdx.y;
    for (; r + STAT_SLICES < N; r += 2 * STAT_SLICES) {
        const double x0 = (double)raw[r * F + f] - c;
        const double x1 = (double)raw[(r + STAT_SLICES) * F + f] - c;
        a0 += PASS == 0 ? x0 : x0 * x0;
        a1 += PASS == 0 ? x1 : x1 * x1;
    }
    if (r < N) {
        const double x0 = (double)raw[r * F + f] - c;
        a0 += PASS == 0 ? x0 : x0 * x0;
    }
    part[(long)blockIdx.y * F + f] = a0 + a1;
}

// Pass 0: mean[f] = sum / N (FP64) and mu[f] = FP32 mean.  Pass 1:
// inv_sd[f] = 1 / max(sqrt(sum / (N - 1)), min_sd) (N = 1: 1 / min_sd).
template <int PASS>
__global__ void colstats_finish_kernel(const double *__restrict__ part, long N, int F,
                                       double min_sd, double *__restrict__ mean,
                                       float *__restrict__ out) {
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= F) return;
    double t = 0.0;
    for (int q = 0; q < STAT_SLICES; ++q) t += part[(long)q * F + f];
    if (PASS == 0) {
        mean[f] = t / (double)N;
        out[f] = (float)(t / (double)N);
    } else {
        const double sd = N > 1 ? sqrt(t / (double)(N - 1)) : 0.0;
        out[f] = (float)(1.0 / fmax(sd, min_sd));
    }
}

// Consensus point of each new object: out[o][c] = (1/m) sum_i Y[o][i][c]
// (FP64 sum in modality order).
__global__ void consensus_kernel(const float *__restrict__ Y, int k, int m, int d,
                                 float *__restrict__ out) {
    const long tot = (long)k * d;
    for (long q = blockIdx.x * (long)blockDim.x + threadIdx.x; q < tot;
         q += (long)gridDim.x * blockDim.x) {
        const long o = q / d;
        const int c = (int)(q - o * d);
        double t = 0.0;
        for (int i = 0; i < m; ++i) t += (double)Y[(o * m + i) * d + c];
        out[q] = (float)(t / m);
    }
}

}  // namespace

hipError_t launch_broadcast(const float *out, int B, int m, int d, int P, float *Y,
                            hipStream_t s) {
    const long tot = (long)B * m * d;
    const unsigned nb = (unsigned)std::min<long>(4096, (tot + 255) / 256);
    broadcast_kernel<<<nb > 0 ? nb : 1, 256, 0, s>>>(out, B, m, d, P, Y);
    return hipGetLastError();
}

template <int EPI, int WM, int WN>
static hipError_t gemm_epi(bool vec, int M, int N, int K, const uint16_t *A, long lda,
                           const uint16_t *Bt, long ldb, const GemmEpi &e, hipStream_t s) {
    const dim3 grid((unsigned)((N + 32 * WN - 1) / (32 * WN)),
                    (unsigned)((M + 32 * WM - 1) / (32 * WM)));
    if (vec)
        gemm_kernel<EPI, true, WM, WN><<<grid, WAVE * WM * WN, 0, s>>>(M, N, K, A, lda, Bt, ldb, e);
    else
        gemm_kernel<EPI, false, WM, WN><<<grid, WAVE * WM * WN, 0, s>>>(M, N, K, A, lda, Bt, ldb, e);
    return hipGetLastError();
}

template <int EPI>
static hipError_t gemm_sk(bool vec, int M, int N, int K, const uint16_t *A, long lda,
                          const uint16_t *Bt, long ldb, const GemmEpi &e, hipStream_t s) {
    const dim3 grid((unsigned)((N + 31) / 32), (unsigned)((M + 31) / 32));
    if (vec)
        gemm_sk_kernel<EPI, true><<<grid, WAVE * GSK, 0, s>>>(M, N, K, A, lda, Bt, ldb, e);
    else
        gemm_sk_kernel<EPI, false><<<grid, WAVE * GSK, 0, s>>>(M, N, K, A, lda, Bt, ldb, e);
    return hipGetLastError();
}

enum { GEMM_FORM_ONE = 0, GEMM_FORM_WIDE = 1, GEMM_FORM_SPLITK = 2 };

template <int EPI>
static hipError_t gemm_waves(int form, bool vec, int M, int N, int K, const uint16_t *A,
                             long lda, const uint16_t *Bt, long ldb, const GemmEpi &e,
                             hipStream_t s) {
    if (form == GEMM_FORM_WIDE) return gemm_epi<EPI, 2, 2>(vec, M, N, K, A, lda, Bt, ldb, e, s);
    if (form == GEMM_FORM_SPLITK) return gemm_sk<EPI>(vec, M, N, K, A, lda, Bt, ldb, e, s);
    return gemm_epi<EPI, 1, 1>(vec, M, N, K, A, lda, Bt, ldb, e, s);
}

// Workgroups of 2 x 2 wavefronts (64 x 64 outputs) when that already gives
// at least two workgroups per CU.  Otherwise each 32 x 32 tile gets a
// workgroup of four wavefronts splitting K (K of at least four steps), or
// one wavefront.  FJOFC_GEMM_WAVES ("1", "4" or "k") forces one of the
// three.
constexpr long GEMM_WIDE_MIN_TILES = 512;

int gemm_form(int M, int N, int K) {
    if (const char *v = std::getenv("FJOFC_GEMM_WAVES")) {
        if (v[0] == '1') return GEMM_FORM_ONE;
        if (v[0] == '4') return GEMM_FORM_WIDE;
        if (v[0] == 'k') return GEMM_FORM_SPLITK;
    }
    if ((long)((M + GB - 1) / GB) * ((N + GB - 1) / GB) >= GEMM_WIDE_MIN_TILES)
        return GEMM_FORM_WIDE;
    return K >= GSK * GK ? GEMM_FORM_SPLITK : GEMM_FORM_ONE;
}

hipError_t launch_gemm(int epi, int M, int N, int K, const uint16_t *A, long lda,
                       const uint16_t *Bt, long ldb, const GemmEpi &e, hipStream_t s) {
    if (M <= 0 || N <= 0) return hipSuccess;
    const int wide = gemm_form(M, N, K);
    const bool vec = (lda % 8 == 0) && (ldb % 8 == 0) &&
                     ((reinterpret_cast<uintptr_t>(A) | reinterpret_cast<uintptr_t>(Bt)) & 15) == 0;
    switch (epi) {
    case GEMM_HIDDEN: return gemm_waves<GEMM_HIDDEN>(wide, vec, M, N, K, A, lda, Bt, ldb, e, s);
    case GEMM_LAST: return gemm_waves<GEMM_LAST>(wide, vec, M, N, K, A, lda, Bt, ldb, e, s);
    case GEMM_BWD: return gemm_waves<GEMM_BWD>(wide, vec, M, N, K, A, lda, Bt, ldb, e, s);
    default: return gemm_waves<GEMM_STORE>(wide, vec, M, N, K, A, lda, Bt, ldb, e, s);
    }
}

hipError_t launch_transpose16(const uint16_t *in, long ld_in, int R, int C, uint16_t *out,
                              long ld_out, hipStream_t s) {
    if (R <= 0 || C <= 0) return hipSuccess;
    const dim3 grid((unsigned)((C + 31) / 32), (unsigned)((R + 31) / 32));
    transpose16_kernel<<<grid, 256, 0, s>>>(in, ld_in, R, C, out, ld_out);
    return hipGetLastError();
}

hipError_t launch_mse(const float *out, const float *y, int B, int k, float *G, uint16_t *Gb,
                      uint16_t *GbT, long ldt, double *loss, double *scratch, hipStream_t s,
                      bool accumulate) {
    mse_kernel<<<MSE_BLOCKS, 256, 0, s>>>(out, y, B, k, G, Gb, GbT, ldt, scratch);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !loss) return e;
    mse_finish_kernel<<<1, 1, 0, s>>>(scratch, (long)B * k, loss, accumulate ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_colsum(const float *G, int B, int N, float *db, double *scratch,
                         hipStream_t s) {
    if (N <= 0) return hipSuccess;
    const dim3 grid((unsigned)((N + CS_COLS - 1) / CS_COLS), CS_SLICES);
    colsum_part_kernel<<<grid, CS_COLS * CS_GROUPS, 0, s>>>(G, B, N, scratch);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    colsum_finish_kernel<<<(unsigned)((N + 255) / 256), 256, 0, s>>>(scratch, N, db);
    return hipGetLastError();
}

hipError_t launch_adam(float *p, const float *g, float *m, float *v, uint16_t *p16, long n,
                       float lr, float b1, float b2, float eps, float c1, float c2,
                       hipStream_t s) {
    const unsigned nb = (unsigned)std::min<long>(4096, (n + 255) / 256);
    adam_kernel<<<nb, 256, 0, s>>>(p, g, m, v, p16, n, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

hipError_t launch_to_bf16(const float *x, uint16_t *y, long n, hipStream_t s) {
    const unsigned nb = (unsigned)std::min<long>(4096, (n + 255) / 256);
    to_bf16_kernel<<<nb > 0 ? nb : 1, 256, 0, s>>>(x, y, n);
    return hipGetLastError();
}

hipError_t launch_features(const float *dnew, int k, int m, int n, const int *lm, int L,
                           const float *mu, const float *isd, uint16_t *x, hipStream_t s) {
    const long tot = (long)k * m * L;
    const unsigned nb = (unsigned)std::min<long>(8192, (tot + 255) / 256);
    features_kernel<<<nb > 0 ? nb : 1, 256, 0, s>>>(dnew, k, m, n, lm, L, mu, isd, x);
    return hipGetLastError();
}

hipError_t launch_colstats(const float *raw, long N, int F, double min_sd, float *mu,
                           float *inv_sd, double *scratch, hipStream_t s) {
    // scratch: STAT_SLICES * F partials, then F FP64 means
    double *part = scratch, *mean = scratch + (long)STAT_SLICES * F;
    const dim3 grid((unsigned)((F + 255) / 256), STAT_SLICES);
    const unsigned nf = (unsigned)((F + 255) / 256);
    colstats_part_kernel<0><<<grid, 256, 0, s>>>(raw, N, F, mean, part);
    colstats_finish_kernel<0><<<nf, 256, 0, s>>>(part, N, F, min_sd, mean, mu);
    colstats_part_kernel<1><<<grid, 256, 0, s>>>(raw, N, F, mean, part);
    colstats_finish_kernel<1><<<nf, 256, 0, s>>>(part, N, F, min_sd, mean, inv_sd);
    return hipGetLastError();
}

size_t colstats_scratch_doubles(int F) { return (size_t)(STAT_SLICES + 1) * F; }

hipError_t launch_consensus(const float *Y, int k, int m, int d, float *out, hipStream_t s) {
    const long tot = (long)k * d;
    const unsigned nb = (unsigned)std::min<long>(4096, (tot + 255) / 256);
    consensus_kernel<<<nb > 0 ? nb : 1, 256, 0, s>>>(Y, k, m, d, out);
    return hipGetLastError();
}

}  // namespace fjofc
