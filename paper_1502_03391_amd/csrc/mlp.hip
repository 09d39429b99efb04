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

#include <algorithm>

namespace fjofc {
namespace {

typedef short s4 __attribute__((ext_vector_type(4)));
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

// C (M x N) = A (M x K) B (K x N), A(m,k) = A[m sam + k sak],
// B(k,n) = B[k sbk + n sbn].  64 x 64 tile per workgroup of four
// wavefronts (2 x 2, 32 x 32 each as 2 x 2 MFMA 16x16x16 tiles), K in steps
// of 32 staged through LDS (B stored transposed so both operands are read
// as 4 consecutive BF16 per lane).  Operand layouts of the 16x16x16 BF16
// MFMA: lane l holds A[l % 16][4 (l / 16) + j], B[4 (l / 16) + j][l % 16],
// and receives C[4 (l / 16) + j][l % 16], j = 0..3.
constexpr int GB = 64, GK = 32, GPAD = 4;

template <int EPI>
__global__ __launch_bounds__(256) void gemm_kernel(int M, int N, int K,
                                                   const uint16_t *__restrict__ A, long sam,
                                                   long sak, const uint16_t *__restrict__ B,
                                                   long sbk, long sbn, GemmEpi e) {
    __shared__ uint16_t As[GB][GK + GPAD];
    __shared__ uint16_t Bs[GB][GK + GPAD];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int wm = wv >> 1, wn = wv & 1;
    const int m0 = blockIdx.y * GB, n0 = blockIdx.x * GB;
    f4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < K; k0 += GK) {
#pragma unroll
        for (int q = 0; q < (GB * GK) / 256; ++q) {
            const int idx = tid + 256 * q;
            // A tile, k fastest (coalesced when sak == 1)
            const int ar = idx / GK, ac = idx % GK;
            const int gm = m0 + ar, gk = k0 + ac;
            As[ar][ac] = (gm < M && gk < K) ? A[(long)gm * sam + (long)gk * sak] : (uint16_t)0;
            // B tile, n fastest (coalesced when sbn == 1), stored [n][k]
            const int br = idx / GB, bc = idx % GB;
            const int gk2 = k0 + br, gn = n0 + bc;
            Bs[bc][br] = (gk2 < K && gn < N) ? B[(long)gk2 * sbk + (long)gn * sbn] : (uint16_t)0;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < GK / 16; ++kk) {
            s4 a[2], b[2];
#pragma unroll
            for (int i = 0; i < 2; ++i)
                a[i] = *reinterpret_cast<const s4 *>(&As[wm * 32 + i * 16 + (lane & 15)]
                                                        [kk * 16 + 4 * (lane >> 4)]);
#pragma unroll
            for (int j = 0; j < 2; ++j)
                b[j] = *reinterpret_cast<const s4 *>(&Bs[wn * 32 + j * 16 + (lane & 15)]
                                                        [kk * 16 + 4 * (lane >> 4)]);
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[i], b[j], acc[i][j],
                                                                          0, 0, 0);
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = m0 + wm * 32 + i * 16 + 4 * (lane >> 4) + r;
                const int col = n0 + wn * 32 + j * 16 + (lane & 15);
                if (row >= M || col >= N) continue;
                const long o = (long)row * e.ldc + col;
                const float v = acc[i][j][r];
                if (EPI == GEMM_HIDDEN) {
                    const float z = v + e.bias[col];
                    e.outf[o] = z;
                    e.outb[o] = f2bf(gelu(z));
                } else if (EPI == GEMM_LAST) {
                    e.outf[o] = v + e.bias[col];
                } else if (EPI == GEMM_BWD) {
                    const float g = v * gelu_grad(e.Z[o]);
                    e.outf[o] = g;
                    e.outb[o] = f2bf(g);
                } else {
                    e.outf[o] = v;
                }
            }
}

// MSE over the batch and outputs: g = 2 (out - y) / (B k) (FP32 and BF16),
// loss = mean (out - y)^2 (FP64, fixed-order reduction).
__global__ __launch_bounds__(256) void mse_kernel(const float *__restrict__ out,
                                                  const float *__restrict__ y, int B, int k,
                                                  float *__restrict__ G, uint16_t *__restrict__ Gb,
                                                  double *__restrict__ loss) {
    __shared__ double sh[256];
    const long tot = (long)B * k;
    const float sc = 2.0f / (float)tot;
    double s = 0.0;
    for (long q = threadIdx.x; q < tot; q += 256) {
        const float d = out[q] - y[q];
        s += (double)d * d;
        const float g = sc * d;
        G[q] = g;
        Gb[q] = f2bf(g);
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0 && loss) loss[0] = sh[0] / (double)tot;
}

// Bias gradient: column sums of G (B x N).  A workgroup owns 64 columns;
// its 16 row groups (rows r = g, g + 16, ...) accumulate in FP64 and are
// added in a fixed order, so the result does not depend on scheduling.
constexpr int CS_COLS = 64, CS_GROUPS = 16;
__global__ __launch_bounds__(CS_COLS *CS_GROUPS) void colsum_kernel(
    const float *__restrict__ G, int B, int N, float *__restrict__ db) {
    __shared__ double part[CS_GROUPS][CS_COLS];
    const int cl = threadIdx.x % CS_COLS, g = threadIdx.x / CS_COLS;
    const int c = blockIdx.x * CS_COLS + cl;
    double s = 0.0;
    if (c < N)
        for (int r = g; r < B; r += CS_GROUPS) s += (double)G[(long)r * N + c];
    part[g][cl] = s;
    __syncthreads();
    if (g == 0 && c < N) {
        double t = 0.0;
        for (int q = 0; q < CS_GROUPS; ++q) t += part[q][cl];
        db[c] = (float)t;
    }
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

}  // namespace

hipError_t launch_broadcast(const float *out, int B, int m, int d, int P, float *Y,
                            hipStream_t s) {
    const long tot = (long)B * m * d;
    const unsigned nb = (unsigned)std::min<long>(4096, (tot + 255) / 256);
    broadcast_kernel<<<nb > 0 ? nb : 1, 256, 0, s>>>(out, B, m, d, P, Y);
    return hipGetLastError();
}

hipError_t launch_gemm(int epi, int M, int N, int K, const uint16_t *A, long sam, long sak,
                       const uint16_t *B, long sbk, long sbn, const GemmEpi &e, hipStream_t s) {
    if (M <= 0 || N <= 0) return hipSuccess;
    const dim3 grid((unsigned)((N + GB - 1) / GB), (unsigned)((M + GB - 1) / GB)), block(256);
    switch (epi) {
    case GEMM_HIDDEN: gemm_kernel<GEMM_HIDDEN><<<grid, block, 0, s>>>(M, N, K, A, sam, sak, B, sbk, sbn, e); break;
    case GEMM_LAST: gemm_kernel<GEMM_LAST><<<grid, block, 0, s>>>(M, N, K, A, sam, sak, B, sbk, sbn, e); break;
    case GEMM_BWD: gemm_kernel<GEMM_BWD><<<grid, block, 0, s>>>(M, N, K, A, sam, sak, B, sbk, sbn, e); break;
    default: gemm_kernel<GEMM_STORE><<<grid, block, 0, s>>>(M, N, K, A, sam, sak, B, sbk, sbn, e); break;
    }
    return hipGetLastError();
}

hipError_t launch_mse(const float *out, const float *y, int B, int k, float *G, uint16_t *Gb,
                      double *loss, hipStream_t s) {
    mse_kernel<<<1, 256, 0, s>>>(out, y, B, k, G, Gb, loss);
    return hipGetLastError();
}

hipError_t launch_colsum(const float *G, int B, int N, float *db, hipStream_t s) {
    if (N <= 0) return hipSuccess;
    colsum_kernel<<<(unsigned)((N + CS_COLS - 1) / CS_COLS), CS_COLS * CS_GROUPS, 0, s>>>(G, B, N, db);
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

}  // namespace fjofc
