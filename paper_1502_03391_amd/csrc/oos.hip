// Out-of-sample fast-JOFC kernel for gfx950 (Section 3).
//
// New objects carry no weight between one another, so the k out-of-sample
// problems are independent; one workgroup owns a block of OB objects and
// runs every Guttman transform of those objects itself (no grid-wide
// synchronisation).  Each transform needs, per object o and modality i,
//   r_j   = delta_oi(j) / ||X^(i)_j - y_oi||   (0 when the distance is 0)
//   psi_i = w_ii sum_j r_j,   xi_i = w_ii (sum_j X^(i)_j - sum_j r_j X^(i)_j)
// and then y_o <- L22^-1 (xi + diag(psi) y_o), L22 being the eq:modW matrix.
// Threads own in-sample columns j (coalesced delta reads); each X^(i)_j is
// loaded once per transform and reused for all OB objects of the block.
// The out-of-sample stress (eq:joos) of the current y is formed in the same
// pass, so the stop rules are tested on sigma(y_t) before y_{t+1} is made.
#include "fjofc_internal.h"
#include <float.h>

namespace fjofc {
namespace {

constexpr int OOS_BLOCK = 256;
constexpr int OOS_WAVES = OOS_BLOCK / WAVE;

__device__ __forceinline__ float wave_sum_f(float v) {
    const int lane = threadIdx.x & (WAVE - 1);
#pragma unroll
    for (int s = 32; s >= 1; s >>= 1)
        v += __int_as_float(__builtin_amdgcn_ds_bpermute((lane ^ s) << 2, __float_as_int(v)));
    return v;
}

template <int D, int OB>
__global__ __launch_bounds__(OOS_BLOCK) void oos_kernel(
    OOSArgs a, const double *__restrict__ colsum /* m x D */) {
    constexpr int NV = D + 2;  // per (object, modality): psi, sum r X (D), fidelity
    __shared__ float ys[OB][MAXM][D];
    __shared__ float ynew[OB][MAXM][D];
    __shared__ float red[OOS_WAVES][OB][NV];
    __shared__ double acc[OB][MAXM][NV];
    __shared__ int live[OB];
    __shared__ double prev[OB];
    __shared__ int any_live;

    const int tid = threadIdx.x, lane = tid & (WAVE - 1), wv = tid / WAVE;
    const int m = a.m, n = a.n, npad = a.npad;
    const int o0 = blockIdx.x * OB;

    for (int q = tid; q < OB * m * D; q += OOS_BLOCK) {
        const int o = q / (m * D), r = q - o * m * D, i = r / D, k = r - i * D;
        ys[o][i][k] = (o0 + o < a.k) ? a.Y[((size_t)(o0 + o) * m + i) * D + k] : 0.f;
    }
    if (tid < OB) {
        live[tid] = (o0 + tid < a.k) ? 1 : 0;
        prev[tid] = 0.0;
    }
    __syncthreads();

    for (int t = 0;; ++t) {
        // ---- stream pass at y_t ------------------------------------------
        for (int i = 0; i < m; ++i) {
            float s[OB][NV];
#pragma unroll
            for (int o = 0; o < OB; ++o)
#pragma unroll
                for (int v = 0; v < NV; ++v) s[o][v] = 0.f;
            float yv[OB][D];
            bool lv[OB];
#pragma unroll
            for (int o = 0; o < OB; ++o) {
                lv[o] = live[o] != 0;
#pragma unroll
                for (int k = 0; k < D; ++k) yv[o][k] = ys[o][i][k];
            }
            const float *Xi = a.Xs + (size_t)i * D * npad;
            for (int j = tid; j < n; j += OOS_BLOCK) {
                float x[D];
#pragma unroll
                for (int k = 0; k < D; ++k) x[k] = Xi[(size_t)k * npad + j];
                float dl[OB];
#pragma unroll
                for (int o = 0; o < OB; ++o)
                    dl[o] = lv[o] ? a.dnew[((size_t)(o0 + o) * m + i) * n + j] : 0.f;
#pragma unroll
                for (int o = 0; o < OB; ++o) {
                    if (!lv[o]) continue;
                    float d2 = 0.f;
#pragma unroll
                    for (int k = 0; k < D; ++k) {
                        const float df = x[k] - yv[o][k];
                        d2 = fmaf(df, df, d2);
                    }
                    const float rs = __builtin_amdgcn_rsqf(fmaxf(d2, FLT_MIN));
                    // eq:B's d = 0 rule for the new point
                    const float r = (d2 > 0.f) ? dl[o] * rs : 0.f;
                    s[o][0] += r;
#pragma unroll
                    for (int k = 0; k < D; ++k) s[o][1 + k] = fmaf(r, x[k], s[o][1 + k]);
                    const float e = dl[o] - d2 * rs;
                    s[o][NV - 1] = fmaf(e, e, s[o][NV - 1]);
                }
            }
#pragma unroll
            for (int o = 0; o < OB; ++o)
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    const float w = wave_sum_f(s[o][v]);
                    if (lane == 0) red[wv][o][v] = w;
                }
            __syncthreads();
            for (int q = tid; q < OB * NV; q += OOS_BLOCK) {
                const int o = q / NV, v = q - o * NV;
                double tot = 0.0;
                for (int w = 0; w < OOS_WAVES; ++w) tot += (double)red[w][o][v];
                acc[o][i][v] = tot;
            }
            __syncthreads();
        }
        // ---- per object: stress, stop rules, transform ------------------
        if (tid < OB) {
            const int o = tid;
            if (live[o]) {
                double sig = 0.0;
                for (int i = 0; i < m; ++i) sig += a.wmat[i * m + i] * acc[o][i][NV - 1];
                for (int i = 0; i < m; ++i)
                    for (int l = i + 1; l < m; ++l) {
                        double dd = 0.0;
                        for (int k = 0; k < D; ++k) {
                            const double df = (double)ys[o][i][k] - (double)ys[o][l][k];
                            dd += df * df;
                        }
                        sig += a.wmat[i * m + l] * dd;
                    }
                bool stop = false;
                if (a.target && sig <= a.target[o0 + o]) stop = true;
                else if (a.tol > 0.0 && t > 0 && prev[o] - sig < a.tol * prev[o]) stop = true;
                else if (t == a.iters) stop = true;
                if (stop) {
                    live[o] = 0;
                    if (a.stress_out) a.stress_out[o0 + o] = sig;
                    if (a.iters_out) a.iters_out[o0 + o] = t;
                }
                prev[o] = sig;
            }
        }
        __syncthreads();
        // y <- L22^-1 (xi + diag(psi) y), FP64 arithmetic; staged so that
        // every thread reads the old y before any is overwritten.
        for (int q = tid; q < OB * m * D; q += OOS_BLOCK) {
            const int o = q / (m * D), r = q - o * m * D, i = r / D, k = r - i * D;
            if (!live[o]) continue;
            double v = 0.0;
            for (int l = 0; l < m; ++l) {
                const double wl = a.wmat[l * m + l];
                const double xi = wl * (colsum[l * D + k] - acc[o][l][1 + k]);
                const double psi = wl * acc[o][l][0];
                v += a.Linv[i * m + l] * (xi + psi * (double)ys[o][l][k]);
            }
            ynew[o][i][k] = (float)v;
        }
        __syncthreads();
        for (int q = tid; q < OB * m * D; q += OOS_BLOCK) {
            const int o = q / (m * D), r = q - o * m * D, i = r / D, k = r - i * D;
            if (live[o]) ys[o][i][k] = ynew[o][i][k];
        }
        if (tid == 0) {
            int anyl = 0;
            for (int o = 0; o < OB; ++o) anyl |= live[o];
            any_live = anyl;
        }
        __syncthreads();
        if (!any_live) break;
    }
    for (int q = tid; q < OB * m * D; q += OOS_BLOCK) {
        const int o = q / (m * D), r = q - o * m * D, i = r / D, k = r - i * D;
        if (o0 + o < a.k) a.Y[((size_t)(o0 + o) * m + i) * D + k] = ys[o][i][k];
    }
}

__global__ void colsum_kernel(const float *__restrict__ Xs, int m, int n,
                              int npad, int D, double *__restrict__ out) {
    __shared__ double sh[OOS_WAVES];
    const int i = blockIdx.x / D, k = blockIdx.x - i * D;
    double s = 0.0;
    for (int j = threadIdx.x; j < n; j += OOS_BLOCK) s += (double)Xs[((size_t)i * D + k) * npad + j];
    const int lane = threadIdx.x & (WAVE - 1);
#pragma unroll
    for (int q = 32; q >= 1; q >>= 1) {
        int2 p = *reinterpret_cast<int2 *>(&s);
        p.x = __builtin_amdgcn_ds_bpermute((lane ^ q) << 2, p.x);
        p.y = __builtin_amdgcn_ds_bpermute((lane ^ q) << 2, p.y);
        s += *reinterpret_cast<double *>(&p);
    }
    if (lane == 0) sh[threadIdx.x / WAVE] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < OOS_WAVES; ++w) t += sh[w];
        out[blockIdx.x] = t;
    }
}

template <int D>
hipError_t launch_oos_d(const OOSArgs &a, const double *colsum, hipStream_t s) {
    constexpr int OB = 8;
    const unsigned nb = (unsigned)((a.k + OB - 1) / OB);
    oos_kernel<D, OB><<<nb, OOS_BLOCK, 0, s>>>(a, colsum);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_oos(const OOSArgs &a, double *colsum, hipStream_t s) {
    colsum_kernel<<<(unsigned)(a.m * a.D), OOS_BLOCK, 0, s>>>(a.Xs, a.m, a.n, a.npad, a.D, colsum);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (a.k == 0) return hipSuccess;
    switch (a.D) {
    case 1: return launch_oos_d<1>(a, colsum, s);
    case 2: return launch_oos_d<2>(a, colsum, s);
    case 3: return launch_oos_d<3>(a, colsum, s);
    case 4: return launch_oos_d<4>(a, colsum, s);
    case 5: return launch_oos_d<5>(a, colsum, s);
    case 6: return launch_oos_d<6>(a, colsum, s);
    case 7: return launch_oos_d<7>(a, colsum, s);
    case 8: return launch_oos_d<8>(a, colsum, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace fjofc
