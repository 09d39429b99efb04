// In-sample fast-JOFC kernels for gfx950: the finalize, commensurability,
// reduce and per-instance set-up kernels, and the host-side launchers of
// every in-sample kernel.  The stream kernels and the persistent batched
// kernel are instantiated in stream_lo.hip, stream_hi.hip, batch5.hip and
// batch8.hip from the device code in stream_dev.h and batch_dev.h.
#include "stream_dev.h"

namespace fjofc {
namespace {

// TPR threads per (row j, component k).  With TPR = FIN_SLICES, thread
// slice s sums the slots congruent to s mod FIN_SLICES and slice 0 adds the
// slices in order; with TPR = 1 one thread forms the same slice sums one
// after the other and adds them in the same order, so both give the same
// bits.  The thread with slice 0 does the FP64 combine.
template <int MM, int TPR>
__global__ __launch_bounds__(FIN_ROWS *TPR) void finalize_kernel(
    const InstDesc *__restrict__ insts, const RowItem *__restrict__ rows, int cur,
    int want_com) {
    static_assert(TPR == 1 || TPR == FIN_SLICES, "one thread or one per slice");
    __shared__ double part[TPR][FIN_ROWS];
    __shared__ double sh[FIN_ROWS * TPR / WAVE];
    const RowItem ri = rows[blockIdx.x];
    const InstDesc &b = insts[ri.inst];
    if (b.st->done) return;
    const int k = ri.k, m = b.g.m;
    const int r = threadIdx.x % FIN_ROWS, sl = threadIdx.x / FIN_ROWS;
    const int j = ri.bx * FIN_ROWS + r;
    double bx[MM];
    for (int q = 0; q < m; ++q) {
        if constexpr (TPR == 1) {
            double t = fin_slice(b, q, k, j, 0);
            for (int e = 1; e < FIN_SLICES; ++e) t += fin_slice(b, q, k, j, e);
            bx[q] = b.wmat[q * m + q] * t;
        } else {
            part[sl][r] = fin_slice(b, q, k, j, sl);
            __syncthreads();
            if (sl == 0) {
                double t = part[0][r];
                for (int e = 1; e < FIN_SLICES; ++e) t += part[e][r];
                bx[q] = b.wmat[q * m + q] * t;
            }
            __syncthreads();
        }
    }
    const double com = sl == 0 ? fin_combine<MM>(b, k, j, cur, bx, want_com) : 0.0;
    if (want_com) {
        const double s = block_sum_d(com, sh);
        if (threadIdx.x == 0) b.comP[(size_t)k * (b.g.npad / FIN_ROWS) + ri.bx] = s;
    }
}

// Commensurability of X_0 (same partial layout as the finalize).
__global__ __launch_bounds__(FIN_ROWS) void com_kernel(
    const InstDesc *__restrict__ insts, const RowItem *__restrict__ rows) {
    __shared__ double sh[FIN_ROWS / WAVE];
    const RowItem ri = rows[blockIdx.x];
    const InstDesc &b = insts[ri.inst];
    const TriGeom &g = b.g;
    const int D = b.D, k = ri.k, m = g.m, npad = g.npad;
    const float *__restrict__ Xs = b.Xs[0];
    const int j = ri.bx * FIN_ROWS + threadIdx.x;
    double com = 0.0;
    if (j < g.n)
        for (int a = 0; a < m; ++a)
            for (int q = a + 1; q < m; ++q) {
                const double t = (double)Xs[((size_t)a * D + k) * npad + j] -
                                 (double)Xs[((size_t)q * D + k) * npad + j];
                com += b.wmat[a * m + q] * t * t;
            }
    const double s = block_sum_d(com, sh);
    if (threadIdx.x == 0) b.comP[(size_t)k * (npad / FIN_ROWS) + ri.bx] = s;
}

__global__ __launch_bounds__(RED_BLOCK) void reduce_kernel(
    const InstDesc *__restrict__ insts, int t, int check, int final_pass, int iters,
    double tol, int tol_mode) {
    reduce_body(insts[blockIdx.x], t, check, final_pass, iters, tol, tol_mode);
}

// Per instance: reset the loop state, fill the history with NaN, convert X0
// to SoA (padding rows 0) and zero the other buffer.  The finalize writes
// X_{t+1} only on rows below npad / FIN_ROWS * FIN_ROWS; when npad is not a
// multiple of FIN_ROWS (a tile height above the tile width) boundary tiles
// still read the rows above, with their terms masked to r = 0, so those
// rows must hold finite values (0) in both buffers.  One workgroup per
// instance.
__global__ void init_kernel(const InstDesc *__restrict__ insts, int nhist) {
    const InstDesc &b = insts[blockIdx.x];
    const TriGeom &g = b.g;
    const int D = b.D;
    if (threadIdx.x == 0) {
        EmbedState *st = b.st;
        st->done = 0;
        st->iters_run = 0;
        st->converged = 0;
        st->pad = 0;
        st->last = 0.0;
        st->sigma = st->fid = st->com = 0.0;
    }
    if (b.hist)
        for (int q = threadIdx.x; q < nhist; q += blockDim.x) b.hist[q] = __builtin_nan("");
    const int tot = g.m * g.npad;
    for (int q = threadIdx.x; q < tot; q += blockDim.x) {
        const int a = q / g.npad, j = q - a * g.npad;
        for (int k = 0; k < D; ++k) {
            b.Xs[0][((size_t)a * D + k) * g.npad + j] =
                (j < g.n) ? b.X[((size_t)a * g.n + j) * D + k] : 0.f;
            b.Xs[1][((size_t)a * D + k) * g.npad + j] = 0.f;
        }
    }
}

// Per instance: write the returned configuration X_{iters_run} back to the
// caller's AoS buffer.
__global__ void copy_out_kernel(const InstDesc *__restrict__ insts) {
    const InstDesc &b = insts[blockIdx.x];
    const TriGeom &g = b.g;
    const int D = b.D;
    const float *Xs = b.Xs[b.st->iters_run & 1];
    const int tot = g.m * g.n;
    for (int q = threadIdx.x; q < tot; q += blockDim.x) {
        const int a = q / g.n, j = q - a * g.n;
        for (int k = 0; k < D; ++k)
            b.X[((size_t)a * g.n + j) * D + k] = Xs[((size_t)a * D + k) * g.npad + j];
    }
}

__global__ void to_soa_kernel(TriGeom g, int D, const float *__restrict__ X,
                              float *__restrict__ Xs) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    const int a = idx / g.npad, j = idx - a * g.npad;
    if (a >= g.m) return;
    for (int k = 0; k < D; ++k)
        Xs[((size_t)a * D + k) * g.npad + j] =
            (j < g.n) ? X[((size_t)a * g.n + j) * D + k] : 0.f;
}

__global__ void batch_reset_kernel(BatchArgs a, int count) {
    for (int q = threadIdx.x; q < count; q += blockDim.x) {
        a.ctr[q].s_done = 0;
        a.ctr[q].r_done = 0;
        a.ctr[q].f_done = 0;
        a.ctr[q].pad = 0;
    }
    if (threadIdx.x == 0) {
        *reinterpret_cast<unsigned long long *>(a.head) = 0ull;
        *a.err = 0;
        *a.never = 0;
    }
}

}  // namespace

hipError_t launch_stream(int D, int variant, int vec4, const InstDesc *insts,
                         const StreamItem *items, int nitems, int cur, bool stress,
                         bool acc, size_t lds, hipStream_t s) {
    if (D >= 1 && D <= 4)
        return launch_stream_lo(D, variant, vec4, insts, items, nitems, cur, stress, acc, lds, s);
    return launch_stream_hi(D, variant, vec4, insts, items, nitems, cur, stress, acc, lds, s);
}

template <int TPR>
static void finalize_tpr(int maxm, const InstDesc *insts, const RowItem *rows, int nrows,
                         int cur, bool want_com, hipStream_t s) {
    const dim3 grid((unsigned)nrows), block(FIN_ROWS * TPR);
    if (maxm <= 4)
        finalize_kernel<4, TPR><<<grid, block, 0, s>>>(insts, rows, cur, want_com);
    else if (maxm <= 8)
        finalize_kernel<8, TPR><<<grid, block, 0, s>>>(insts, rows, cur, want_com);
    else
        finalize_kernel<MAXM, TPR><<<grid, block, 0, s>>>(insts, rows, cur, want_com);
}

hipError_t launch_finalize(int maxm, const InstDesc *insts, const RowItem *rows, int nrows,
                           int cur, bool want_com, bool one_thread, hipStream_t s) {
    if (nrows == 0) return hipSuccess;
    if (one_thread)
        finalize_tpr<1>(maxm, insts, rows, nrows, cur, want_com, s);
    else
        finalize_tpr<FIN_SLICES>(maxm, insts, rows, nrows, cur, want_com, s);
    return hipGetLastError();
}

hipError_t launch_com(const InstDesc *insts, const RowItem *rows, int nrows, hipStream_t s) {
    if (nrows == 0) return hipSuccess;
    com_kernel<<<dim3((unsigned)nrows), dim3(FIN_ROWS), 0, s>>>(insts, rows);
    return hipGetLastError();
}

hipError_t launch_reduce(const InstDesc *insts, int count, int t, int check, int final_pass,
                         int iters, double tol, int tol_mode, hipStream_t s) {
    reduce_kernel<<<(unsigned)count, RED_BLOCK, 0, s>>>(insts, t, check, final_pass, iters,
                                                        tol, tol_mode);
    return hipGetLastError();
}

hipError_t launch_init(const InstDesc *insts, int count, int nhist, hipStream_t s) {
    init_kernel<<<(unsigned)count, 256, 0, s>>>(insts, nhist);
    return hipGetLastError();
}

hipError_t launch_copy_out(const InstDesc *insts, int count, hipStream_t s) {
    copy_out_kernel<<<(unsigned)count, 256, 0, s>>>(insts);
    return hipGetLastError();
}

hipError_t launch_to_soa(const TriGeom &g, int D, const float *X, float *Xs,
                         hipStream_t s) {
    const size_t tot = (size_t)g.m * g.npad;
    to_soa_kernel<<<(unsigned)((tot + 255) / 256), 256, 0, s>>>(g, D, X, Xs);
    return hipGetLastError();
}

hipError_t launch_batch_reset(const BatchArgs &a, int count, hipStream_t s) {
    batch_reset_kernel<<<1, 256, 0, s>>>(a, count);
    return hipGetLastError();
}

hipError_t launch_batch_persistent(const BatchArgs &a, int maxd, int maxm, int grid, size_t lds,
                                   hipStream_t s) {
    (void)maxm;
    if (grid < 1) return hipErrorInvalidValue;
    return maxd <= 5 ? launch_batch_kernel5(a, grid, lds, s) : launch_batch_kernel8(a, grid, lds, s);
}

int batch_resident_blocks(int maxd, int maxm, size_t lds) {
    (void)maxm;
    int nb = 0;
    const void *k = maxd <= 5 ? batch_kernel5_address() : batch_kernel8_address();
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, BATCH_BLOCK, lds) != hipSuccess)
        return 0;
    return nb;
}

size_t batch_stream_lds(int D, int variant, size_t tile_lds) {
    // one-wavefront tiles: each of the four wavefronts its own [4 D][64]
    // reduction buffer; shared tiles: the tile's own layout
    return variant <= 1 ? (size_t)(BATCH_BLOCK / WAVE) * 4 * D * WAVE * sizeof(float) : tile_lds;
}

}  // namespace fjofc
