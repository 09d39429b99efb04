// Kernels of the paper's initialisation (Algorithm 1 step 1, Algorithm 2's
// first lines): classical MDS of a dissimilarity matrix A (the mean of the
// Delta_i, or one Delta_i) needs the top eigenpairs of
//     P = -1/2 J (A o A) J,     J = I_n - 1 1^T / n,
// found here by subspace iteration on a block of K centred vectors V: each
// step needs W = (A o A) V, formed by streaming A once (full rows, squared
// on the fly); J is applied on the K columns (the host folds the column
// means into the orthonormalisation).  Small K x K and d x d eigenproblems
// run on the host in FP64; these kernels provide the n-long products.
#include "fjofc_internal.h"
#include "wave_ops.h"

#include <algorithm>

namespace fjofc {
namespace {

constexpr int CM_BLOCK = 256;
constexpr int CM_WAVES = CM_BLOCK / WAVE;
constexpr int CM_ROWS = 4;  // rows of W per workgroup

// W[j][c] = sum_l (scale sum_s A_s[j][l])^2 V[l][c] for the CM_ROWS rows
// j0.. of this workgroup; the 256 threads split l (coalesced row reads).
template <int K>
__global__ __launch_bounds__(CM_BLOCK) void sqprod_kernel(DeltaPtrs dp, int nsrc, float scale,
                                                          int n, const float *__restrict__ V,
                                                          float *__restrict__ W) {
    constexpr int VP = CM_ROWS * K;  // multiple of 16
    __shared__ float red[CM_WAVES][VP];
    const int tid = threadIdx.x, lane = tid & (WAVE - 1), wv = tid / WAVE;
    const int j0 = blockIdx.x * CM_ROWS;
    float acc[CM_ROWS][K];
#pragma unroll
    for (int r = 0; r < CM_ROWS; ++r)
#pragma unroll
        for (int c = 0; c < K; ++c) acc[r][c] = 0.f;
    for (int l = tid; l < n; l += CM_BLOCK) {
        float v[K];
#pragma unroll
        for (int c = 0; c < K; c += 4) {
            const float4 q = *reinterpret_cast<const float4 *>(V + (size_t)l * K + c);
            v[c] = q.x;
            v[c + 1] = q.y;
            v[c + 2] = q.z;
            v[c + 3] = q.w;
        }
#pragma unroll
        for (int r = 0; r < CM_ROWS; ++r) {
            const int j = j0 + r;
            float a = 0.f;
            if (j < n)
                for (int s = 0; s < nsrc; ++s) a += dp.p[s][(size_t)j * n + l];
            a *= scale;
            const float a2 = a * a;
#pragma unroll
            for (int c = 0; c < K; ++c) acc[r][c] = fmaf(a2, v[c], acc[r][c]);
        }
    }
    float p[VP];
#pragma unroll
    for (int q = 0; q < VP; ++q) p[q] = acc[q / K][q % K];
    float c8[VP / 8];
    wave::reduce_scatter8<VP>(p, c8, lane);
    if ((lane & 7) == 0) {
        const int base = wave::scatter8_base(lane, VP);
#pragma unroll
        for (int r = 0; r < VP / 8; ++r) red[wv][base + r] = c8[r];
    }
    __syncthreads();
    if (tid < VP) {
        float s = 0.f;
        for (int w = 0; w < CM_WAVES; ++w) s += red[w][tid];
        const int j = j0 + tid / K;
        if (j < n) W[(size_t)j * K + tid % K] = s;
    }
}

__device__ __forceinline__ double wave_sum_d(double v) {
    const int lane = threadIdx.x & (WAVE - 1);
#pragma unroll
    for (int s = 32; s >= 1; s >>= 1) {
        int2 p = *reinterpret_cast<int2 *>(&v);
        p.x = __builtin_amdgcn_ds_bpermute((lane ^ s) << 2, p.x);
        p.y = __builtin_amdgcn_ds_bpermute((lane ^ s) << 2, p.y);
        v += *reinterpret_cast<double *>(&p);
    }
    return v;
}

// out[a kb + b] = sum_j A[j lda + a] B[j ldb + b] (B == nullptr: 1), FP64,
// one workgroup per output in a fixed summation order.
__global__ __launch_bounds__(CM_BLOCK) void cross_kernel(const float *__restrict__ A, int lda,
                                                         const float *__restrict__ B, int ldb,
                                                         int n, int kb, double *__restrict__ out) {
    __shared__ double sh[CM_WAVES];
    const int a = blockIdx.x / kb, b = blockIdx.x - a * kb;
    double s = 0.0;
    for (int j = threadIdx.x; j < n; j += CM_BLOCK)
        s += (double)A[(size_t)j * lda + a] * (B ? (double)B[(size_t)j * ldb + b] : 1.0);
    s = wave_sum_d(s);
    if ((threadIdx.x & (WAVE - 1)) == 0) sh[threadIdx.x / WAVE] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < CM_WAVES; ++w) t += sh[w];
        out[blockIdx.x] = t;
    }
}

// out[j ldo + c] = sum_a (in[j ldi + a] - mu[a]) M[a ncol + c] (FP64 sums),
// for c < ncol; columns ncol <= c < ldo_pad of out are set to 0.
__global__ void apply_kernel(const float *__restrict__ in, int ldi, int nin,
                             const double *__restrict__ mu, const double *__restrict__ M,
                             int ncol, int n, float *__restrict__ out, int ldo, int ldo_pad) {
    const long tot = (long)n * ldo_pad;
    for (long q = blockIdx.x * (long)blockDim.x + threadIdx.x; q < tot;
         q += (long)gridDim.x * blockDim.x) {
        const long j = q / ldo_pad;
        const int c = (int)(q - j * ldo_pad);
        double v = 0.0;
        if (c < ncol)
            for (int a = 0; a < nin; ++a)
                v += ((double)in[j * ldi + a] - (mu ? mu[a] : 0.0)) * M[a * ncol + c];
        out[j * ldo + c] = (float)v;
    }
}

}  // namespace

hipError_t launch_sqprod(const DeltaPtrs &dp, int nsrc, float scale, int n, int K,
                         const float *V, float *W, hipStream_t s) {
    const unsigned nb = (unsigned)((n + CM_ROWS - 1) / CM_ROWS);
    switch (K) {
    case 4: sqprod_kernel<4><<<nb, CM_BLOCK, 0, s>>>(dp, nsrc, scale, n, V, W); break;
    case 8: sqprod_kernel<8><<<nb, CM_BLOCK, 0, s>>>(dp, nsrc, scale, n, V, W); break;
    case 12: sqprod_kernel<12><<<nb, CM_BLOCK, 0, s>>>(dp, nsrc, scale, n, V, W); break;
    case 16: sqprod_kernel<16><<<nb, CM_BLOCK, 0, s>>>(dp, nsrc, scale, n, V, W); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_cross(const float *A, int lda, int ka, const float *B, int ldb, int kb, int n,
                        double *out, hipStream_t s) {
    if (ka * kb == 0) return hipSuccess;
    cross_kernel<<<(unsigned)(ka * kb), CM_BLOCK, 0, s>>>(A, lda, B, ldb, n, kb, out);
    return hipGetLastError();
}

hipError_t launch_apply(const float *in, int ldi, int nin, const double *mu, const double *M,
                        int ncol, int n, float *out, int ldo, int ldo_pad, hipStream_t s) {
    const long tot = (long)n * ldo_pad;
    if (tot == 0) return hipSuccess;
    const unsigned nb = (unsigned)std::min<long>(8192, (tot + 255) / 256);
    apply_kernel<<<nb, 256, 0, s>>>(in, ldi, nin, mu, M, ncol, n, out, ldo, ldo_pad);
    return hipGetLastError();
}

}  // namespace fjofc
