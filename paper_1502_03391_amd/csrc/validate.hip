// Debug checks of dissimilarity inputs (the optional validation pass).
//
// The method takes each Delta_i to be a dissimilarity matrix in R_+^{n x n}
// (Section 1): finite, non-negative, symmetric, with a zero diagonal; the
// in-sample kernels read only its strict upper triangle and the fidelity
// term of the raw stress (Remark faststress) counts each pair once, so a
// matrix that breaks these rules gives a result that silently depends on
// which triangle was read.  These kernels find the first offending entry
// in row-major order; nothing here traps or faults on bad values.
#include "fjofc_internal.h"

namespace fjofc {
namespace {

constexpr int VT = 64;  // tile edge

// Offence codes, ordered by priority at one entry.
enum { V_NAN = 1, V_INF = 2, V_NEG = 3, V_ASYM = 4, V_DIAG = 5 };

__device__ __forceinline__ int value_offence(float v) {
    if (v != v) return V_NAN;
    if (__builtin_isinf(v)) return V_INF;
    if (v < 0.f) return V_NEG;
    return 0;
}

__device__ __forceinline__ void report(unsigned long long *first, long long idx, int kind) {
    atomicMin(first, ((unsigned long long)idx << 3) | (unsigned long long)kind);
}

__global__ void fill_u64_kernel(unsigned long long *p, unsigned long long v) { *p = v; }

// One workgroup per tile pair (I, J), I <= J (tile index q enumerates the
// upper triangle of tiles row by row).  A = Delta[I block, J block] and its
// mirror B = Delta[J block, I block] go through LDS; every entry of A is
// checked for its value, the diagonal rule and (above the diagonal)
// symmetry against B; every entry of B (below the diagonal) for its value.
__global__ __launch_bounds__(256) void square_kernel(const float *__restrict__ dl, int n,
                                                     int T, unsigned long long *first) {
    __shared__ float A[VT][VT + 1], Bm[VT][VT + 1];
    // tile pair from the linear index: row I holds T - I tiles
    long long q = blockIdx.x;
    int I = 0;
    while (q >= T - I) {
        q -= T - I;
        ++I;
    }
    const int J = I + (int)q;
    const int r0 = I * VT, c0 = J * VT;
    for (int e = threadIdx.x; e < VT * VT; e += blockDim.x) {
        const int r = e / VT, c = e - r * VT;
        A[r][c] = (r0 + r < n && c0 + c < n) ? dl[(size_t)(r0 + r) * n + c0 + c] : 0.f;
        if (I != J)
            Bm[r][c] = (c0 + r < n && r0 + c < n) ? dl[(size_t)(c0 + r) * n + r0 + c] : 0.f;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < VT * VT; e += blockDim.x) {
        const int r = e / VT, c = e - r * VT;
        const int i = r0 + r, j = c0 + c;
        if (i < n && j < n) {
            const float v = A[r][c];
            int k = value_offence(v);
            if (!k && i == j && v != 0.f) k = V_DIAG;
            if (!k && i < j) {
                const float u = I == J ? A[c][r] : Bm[c][r];
                if (u != v) k = V_ASYM;
            }
            if (k) report(first, (long long)i * n + j, k);
        }
        if (I != J) {
            const int i2 = c0 + r, j2 = r0 + c;
            if (i2 < n && j2 < n) {
                const int k = value_offence(Bm[r][c]);
                if (k) report(first, (long long)i2 * n + j2, k);
            }
        }
    }
}

// Rows of dissimilarities to new objects (no symmetry): finite and >= 0.
__global__ void rows_kernel(const float *__restrict__ d, long long count,
                            unsigned long long *first) {
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < count;
         q += (long long)gridDim.x * blockDim.x) {
        const int k = value_offence(d[q]);
        if (k) report(first, q, k);
    }
}

}  // namespace

hipError_t launch_validate_square(const float *delta, int n, unsigned long long *first,
                                  bool reset, hipStream_t s) {
    if (reset) fill_u64_kernel<<<1, 1, 0, s>>>(first, ~0ull);
    const int T = (n + VT - 1) / VT;
    const long long pairs = (long long)T * (T + 1) / 2;
    if (pairs > 0x7fffffffLL) return hipErrorInvalidValue;
    square_kernel<<<(unsigned)pairs, 256, 0, s>>>(delta, n, T, first);
    return hipGetLastError();
}

hipError_t launch_validate_rows(const float *d, long long count, unsigned long long *first,
                                bool reset, hipStream_t s) {
    if (reset) fill_u64_kernel<<<1, 1, 0, s>>>(first, ~0ull);
    if (count <= 0) return hipGetLastError();
    const unsigned nb = (unsigned)std::min<long long>(8192, (count + 255) / 256);
    rows_kernel<<<nb, 256, 0, s>>>(d, count, first);
    return hipGetLastError();
}

}  // namespace fjofc
