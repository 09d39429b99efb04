// Kernels of the paper's initialisation (Algorithm 1 step 1, Algorithm 2's
// first lines): classical MDS of a dissimilarity matrix A (the mean of the
// Delta_i, or one Delta_i) needs the top eigenpairs of
//     P = -1/2 J (A o A) J,     J = I_n - 1 1^T / n,
// found here by subspace iteration on a block of K centred vectors V per
// problem: each step needs W = (A o A) V.  All m + 1 problems (the mean and
// every Delta_i) advance together, so one step streams every Delta_i once
// and forms all m + 1 products from the same reads (gram_kernel); J is
// applied on the K columns (the host folds the column means into the
// orthonormalisation).  Small K x K and d x d eigenproblems run on the host
// in FP64; these kernels provide the n-long products.
//
// (A o A) V is a dense n x n by n x K contraction, so it runs on the matrix
// cores: v_mfma_f32_16x16x4f32 with the squared entries as the A operand
// (16 rows x 4 columns of Delta per instruction) and V as the B operand
// (K padded to 16 columns).  FP32 products and sums, as on the vector path.
#include "fjofc_internal.h"
#include "wave_ops.h"

#include <algorithm>

namespace fjofc {
namespace {

typedef float f4v __attribute__((ext_vector_type(4)));

constexpr int GR_BLOCK = 256;
constexpr int GR_WAVES = GR_BLOCK / WAVE;

// Load 8 consecutive floats of a row from column l (l % 8 == 0); columns at
// or beyond n read as 0.  VEC: the row is 16-byte aligned and n % 4 == 0,
// so each half is either wholly inside or wholly outside.
template <bool VEC>
__device__ __forceinline__ void load8(const float *__restrict__ row, int l, int n, float (&v)[8]) {
    if (VEC) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            f4v q = {0.f, 0.f, 0.f, 0.f};
            if (l + 4 * h < n) q = *reinterpret_cast<const f4v *>(row + l + 4 * h);
            v[4 * h] = q.x;
            v[4 * h + 1] = q.y;
            v[4 * h + 2] = q.z;
            v[4 * h + 3] = q.w;
        }
    } else {
#pragma unroll
        for (int q = 0; q < 8; ++q) v[q] = (l + q < n) ? row[l + q] : 0.f;
    }
}

// One workgroup: GR_ROWS rows j0.. of every problem's (A o A) V over the
// columns [cbeg, cend) of its split, written to part.  Its four wavefronts
// take the split's 32-column steps in turn (wavefront w steps w, w + 4, ...),
// so together they read each row 512 contiguous bytes at a time, and their
// sums are added through LDS in a fixed order at the end.  Problems of the
// launch: the mean (MEAN) then modalities i0 .. i0 + G - 1.  With MEAN and
// G > 0 the launch holds all m modalities (nsrc == G) and the mean is formed
// from the same loaded values; with G == 0 the mean sums nsrc rows itself.
//
// MFMA operand layout (16 x 16 x 4, wave64): lane t supplies A[t % 16][t / 16]
// and B[t / 16][t % 16] and receives D[4 (t / 16) + r][t % 16] in register
// r.  The contraction index k of step q stands for column l0 + 8 (t / 16) + q
// in both operands, so each lane loads 8 consecutive columns of its row.
template <int G, bool MEAN, bool VEC>
__global__ __launch_bounds__(GR_BLOCK) void gram_kernel(GramArgs a) {
    constexpr int P = G + (MEAN ? 1 : 0);
    __shared__ f4v red[GR_RB * P][WAVE];
    const int lane = threadIdx.x & (WAVE - 1);
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / WAVE));
    const int split = blockIdx.x / a.nrowblk;
    const int rblk = blockIdx.x - split * a.nrowblk;
    const int j0 = rblk * GR_ROWS;
    const int cbeg = split * a.cpw;
    const int cend = min(a.n, cbeg + a.cpw);
    const int c = lane & 15, lq = 8 * (lane >> 4);
    f4v acc[GR_RB][P];
#pragma unroll
    for (int rb = 0; rb < GR_RB; ++rb)
#pragma unroll
        for (int p = 0; p < P; ++p) acc[rb][p] = f4v{0.f, 0.f, 0.f, 0.f};
    for (int l0 = cbeg + w * GR_CHUNK; l0 < cend; l0 += GR_WAVES * GR_CHUNK) {
        const int lb = l0 + lq;
        // B operands: V_p[lb + q][c] from the transposed copy (zero-padded
        // to 16 rows and npad columns)
        float vb[P][8];
#pragma unroll
        for (int p = 0; p < P; ++p) {
            const f4v *src = reinterpret_cast<const f4v *>(a.Vt[p] + (size_t)c * a.npad + lb);
            const f4v lo = src[0], hi = src[1];
            vb[p][0] = lo.x; vb[p][1] = lo.y; vb[p][2] = lo.z; vb[p][3] = lo.w;
            vb[p][4] = hi.x; vb[p][5] = hi.y; vb[p][6] = hi.z; vb[p][7] = hi.w;
        }
#pragma unroll
        for (int rb = 0; rb < GR_RB; ++rb) {
            const int j = j0 + rb * 16 + c;
            float sv[P][8];
            if (G > 0) {
                float av[G > 0 ? G : 1][8];
#pragma unroll
                for (int g = 0; g < G; ++g) {
                    if (j < a.n)
                        load8<VEC>(a.dp.p[a.i0 + g] + (size_t)j * a.n, lb, a.n, av[g]);
                    else
#pragma unroll
                        for (int q = 0; q < 8; ++q) av[g][q] = 0.f;
                }
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    if (MEAN) {
                        float s = 0.f;
#pragma unroll
                        for (int g = 0; g < G; ++g) s += av[g][q];
                        s *= a.scale;
                        sv[0][q] = s * s;
                    }
#pragma unroll
                    for (int g = 0; g < G; ++g) sv[P - G + g][q] = av[g][q] * av[g][q];
                }
            } else {
                float s[8];
#pragma unroll
                for (int q = 0; q < 8; ++q) s[q] = 0.f;
                if (j < a.n)
                    for (int src = 0; src < a.nsrc; ++src) {
                        float v[8];
                        load8<VEC>(a.dp.p[src] + (size_t)j * a.n, lb, a.n, v);
#pragma unroll
                        for (int q = 0; q < 8; ++q) s[q] += v[q];
                    }
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const float t = s[q] * a.scale;
                    sv[0][q] = t * t;
                }
            }
#pragma unroll
            for (int q = 0; q < 8; ++q)
#pragma unroll
                for (int p = 0; p < P; ++p)
                    acc[rb][p] = __builtin_amdgcn_mfma_f32_16x16x4f32(sv[p][q], vb[p][q],
                                                                      acc[rb][p], 0, 0, 0);
        }
    }
    // wavefront 0's sums + ((3's + 2's) + 1's), through LDS
    for (int src = GR_WAVES - 1; src >= 1; --src) {
        if (w == src) {
#pragma unroll
            for (int rb = 0; rb < GR_RB; ++rb)
#pragma unroll
                for (int p = 0; p < P; ++p)
                    red[rb * P + p][lane] = src == GR_WAVES - 1
                                                ? acc[rb][p]
                                                : red[rb * P + p][lane] + acc[rb][p];
        }
        __syncthreads();
    }
    if (w != 0) return;
    // partial results: part[split][pbase + p][row][16]
    const int rq = 4 * (lane >> 4);
#pragma unroll
    for (int rb = 0; rb < GR_RB; ++rb)
#pragma unroll
        for (int p = 0; p < P; ++p) {
            const f4v v = acc[rb][p] + red[rb * P + p][lane];
            float *dst = a.part + (((size_t)split * a.ptotal + a.pbase + p) * a.nrow_pad +
                                   j0 + rb * 16 + rq) * 16 + c;
#pragma unroll
            for (int r = 0; r < 4; ++r) dst[r * 16] = v[r];
        }
}

// W_p[j][c] = sum over splits (in order) of part[s][p][j][c], c < K.
__global__ void gram_combine_kernel(const float *__restrict__ part, int splits, int np,
                                    int nrow_pad, int n, int K, float *__restrict__ W,
                                    size_t wstride) {
    const long tot = (long)np * n * K;
    for (long q = blockIdx.x * (long)blockDim.x + threadIdx.x; q < tot;
         q += (long)gridDim.x * blockDim.x) {
        const int p = (int)(q / ((long)n * K));
        const long r = q - (long)p * n * K;
        const int j = (int)(r / K), cc = (int)(r - (long)j * K);
        float s = 0.f;
        for (int sp = 0; sp < splits; ++sp)
            s += part[(((size_t)sp * np + p) * nrow_pad + j) * 16 + cc];
        W[p * wstride + (size_t)j * K + cc] = s;
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

// For problem p = blockIdx.x / (ka kb): out_p[a kb + b] = sum_j A_p[j lda + a]
// B_p[j ldb + b] (B == nullptr: 1), FP64, one workgroup per output in a
// fixed summation order.
__global__ __launch_bounds__(GR_BLOCK) void cross_kernel(const float *__restrict__ A, int lda,
                                                         size_t sa, const float *__restrict__ B,
                                                         int ldb, size_t sb, int n, int ka,
                                                         int kb, double *__restrict__ out,
                                                         size_t so) {
    __shared__ double sh[GR_WAVES];
    const int per = ka * kb;
    const int p = blockIdx.x / per, o = blockIdx.x - p * per;
    const int ai = o / kb, bi = o - ai * kb;
    const float *Ap = A + p * sa;
    const float *Bp = B ? B + p * sb : nullptr;
    double s = 0.0;
    for (int j = threadIdx.x; j < n; j += GR_BLOCK)
        s += (double)Ap[(size_t)j * lda + ai] * (Bp ? (double)Bp[(size_t)j * ldb + bi] : 1.0);
    s = wave_sum_d(s);
    if ((threadIdx.x & (WAVE - 1)) == 0) sh[threadIdx.x / WAVE] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < GR_WAVES; ++w) t += sh[w];
        out[p * so + o] = t;
    }
}

// For problem p = blockIdx.y: out_p[j ldo + c] = sum_a (in_p[j ldi + a] -
// mu_p[a]) M_p[a ncol + c] (FP64 sums) for c < ncol, 0 for ncol <= c <
// ldo_pad; optionally also the transposed copy outT_p[c][j] (rows c < 16,
// columns j < npad, zero outside c < ncol, j < n).
__global__ void apply_kernel(ApplyArgs a) {
    const int p = blockIdx.y;
    const float *in = a.in + p * a.sin;
    const double *mu = a.mu ? a.mu + p * a.smu : nullptr;
    const double *M = a.M + p * a.sM;
    float *out = a.out + p * a.sout;
    float *outT = a.outT ? a.outT + p * a.soutT : nullptr;
    const long rows = outT ? (long)a.npad : (long)a.n;
    const int cols = outT ? 16 : a.ldo_pad;
    const long tot = rows * cols;
    for (long q = blockIdx.x * (long)blockDim.x + threadIdx.x; q < tot;
         q += (long)gridDim.x * blockDim.x) {
        const long j = q / cols;
        const int c = (int)(q - j * cols);
        double v = 0.0;
        if (j < a.n && c < a.ncol)
            for (int i = 0; i < a.nin; ++i)
                v += ((double)in[j * a.ldi + i] - (mu ? mu[i] : 0.0)) * M[i * a.ncol + c];
        if (j < a.n && c < a.ldo_pad) out[j * a.ldo + c] = (float)v;
        if (outT) outT[(size_t)c * a.npad + j] = (float)v;
    }
}

template <int G, bool MEAN>
hipError_t gram_go(const GramArgs &a, bool vec, unsigned nb, hipStream_t s) {
    if (vec)
        gram_kernel<G, MEAN, true><<<nb, GR_BLOCK, 0, s>>>(a);
    else
        gram_kernel<G, MEAN, false><<<nb, GR_BLOCK, 0, s>>>(a);
    return hipGetLastError();
}

}  // namespace

void gram_plan(int n, int &nrowblk, int &splits, int &cpw) {
    nrowblk = (n + GR_ROWS - 1) / GR_ROWS;
    const int chunks = (n + GR_CHUNK - 1) / GR_CHUNK;
    // enough workgroups to fill the chip, at least 4 column chunks per
    // wavefront
    int want = std::max(1, (1024 + nrowblk - 1) / nrowblk);
    want = std::min(want, std::max(1, chunks / (4 * GR_WAVES)));
    cpw = GR_CHUNK * ((chunks + want - 1) / want);
    splits = (n + cpw - 1) / cpw;
}

hipError_t launch_gram(const GramArgs &a, int G, bool mean, hipStream_t s) {
    const unsigned nb = (unsigned)((long)a.nrowblk * a.splits);
    bool vec = a.n % 4 == 0;
    for (int i = 0; i < a.nsrc && vec; ++i)
        vec = (reinterpret_cast<uintptr_t>(a.dp.p[i]) & 15) == 0;
    if (mean && G == 0) return gram_go<0, true>(a, vec, nb, s);
    if (mean && G != a.nsrc) return hipErrorInvalidValue;
    switch (G * 2 + (mean ? 1 : 0)) {
    case 3: return gram_go<1, true>(a, vec, nb, s);
    case 5: return gram_go<2, true>(a, vec, nb, s);
    case 7: return gram_go<3, true>(a, vec, nb, s);
    case 9: return gram_go<4, true>(a, vec, nb, s);
    case 2: return gram_go<1, false>(a, vec, nb, s);
    case 4: return gram_go<2, false>(a, vec, nb, s);
    case 6: return gram_go<3, false>(a, vec, nb, s);
    case 8: return gram_go<4, false>(a, vec, nb, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_gram_combine(const float *part, int splits, int np, int nrow_pad, int n, int K,
                               float *W, size_t wstride, hipStream_t s) {
    const long tot = (long)np * n * K;
    if (tot == 0) return hipSuccess;
    const unsigned nb = (unsigned)std::min<long>(8192, (tot + 255) / 256);
    gram_combine_kernel<<<nb, 256, 0, s>>>(part, splits, np, nrow_pad, n, K, W, wstride);
    return hipGetLastError();
}

hipError_t launch_cross(const float *A, int lda, size_t sa, int ka, const float *B, int ldb,
                        size_t sb, int kb, int n, double *out, size_t so, int np,
                        hipStream_t s) {
    if (ka * kb * np == 0) return hipSuccess;
    cross_kernel<<<(unsigned)(ka * kb * np), GR_BLOCK, 0, s>>>(A, lda, sa, B, ldb, sb, n, ka,
                                                               kb, out, so);
    return hipGetLastError();
}

hipError_t launch_apply(const ApplyArgs &a, int np, hipStream_t s) {
    const long rows = a.outT ? (long)a.npad : (long)a.n;
    const long tot = rows * (a.outT ? 16 : a.ldo_pad);
    if (tot == 0 || np == 0) return hipSuccess;
    const unsigned nb = (unsigned)std::min<long>(4096, (tot + 255) / 256);
    apply_kernel<<<dim3(nb, (unsigned)np), 256, 0, s>>>(a);
    return hipGetLastError();
}

}  // namespace fjofc
