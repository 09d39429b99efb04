// Device code of the persistent batched launch (see BatchArgs), shared by
// batch5.hip and batch8.hip, which instantiate it for D <= 5 and D <= 8.
#pragma once
#include "stream_dev.h"

namespace fjofc {
namespace {

// ---------------------------------------------------------------------------
// Persistent batched launch (see BatchArgs): every transform of every
// problem in one launch, tasks taken from a queue in a fixed order, each
// waiting (bounded) on per-problem completion counters.
// ---------------------------------------------------------------------------

// One tile of a stream group: the same code as the lockstep kernel (results
// are bitwise equal), with the row points read coherently.  One-wavefront
// tiles (variant 1) run on the calling wavefront and its LDS slice, shared
// tiles (variants 4 and 5) on the whole workgroup.
template <int D, int VAR, bool VEC4, bool STRESS>
__device__ __forceinline__ void batch_tile(const InstDesc *__restrict__ insts,
                                           const StreamItem &it, int cur, lfloat *smem) {
    constexpr int R = VAR == 4 ? 4 : (VAR == 5 ? 2 : 1);
    constexpr int C = VAR == 5 ? 2 : 1;
    const InstDesc &b = insts[it.inst];
    const float *Xs = b.Xs[cur];
    const int I = it.tile >> 16, J = it.tile & 0xffff;
    if (it.ftile < b.g.nint)
        stream_tile<D, 4, 8, false, VEC4, false, STRESS, true, R, C, true>(
            b.g, b.dp, Xs, it.mod, I, J, it.ftile, b.P, b.F, smem);
    else
        stream_tile<D, 4, 8, false, VEC4, true, STRESS, true, R, C, true>(
            b.g, b.dp, Xs, it.mod, I, J, it.ftile, b.P, b.F, smem);
}

// A stream group: `count` tiles of one problem.  One-wavefront tiles:
// wavefront w takes tiles w, w + 4, ...  Shared tiles: the workgroup takes
// them in turn, with a barrier between two (the next tile reuses the LDS
// the last one's epilogue reads).
template <int D, int VAR, bool VEC4, bool STRESS>
__device__ __forceinline__ void batch_stream(const InstDesc *__restrict__ insts,
                                             const StreamItem *__restrict__ items, int count,
                                             int cur, lfloat *smem) {
    if constexpr (VAR == 1) {
        const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
        lfloat *ws = smem + (size_t)w * 4 * D * WAVE;
        for (int q = w; q < count; q += BATCH_BLOCK / WAVE)
            batch_tile<D, VAR, VEC4, STRESS>(insts, items[q], cur, ws);
    } else {
        for (int q = 0; q < count; ++q) {
            if (q > 0) __syncthreads();
            batch_tile<D, VAR, VEC4, STRESS>(insts, items[q], cur, smem);
        }
    }
}

template <int D>
__device__ __forceinline__ void batch_stream_d(int variant, int vec4, bool stress,
                                               const InstDesc *insts, const StreamItem *items,
                                               int count, int cur, lfloat *smem) {
#define FJOFC_BS(V, V4, S)                                                          \
    if (variant == V && (vec4 != 0) == V4 && stress == S)                           \
        return batch_stream<D, V, V4, S>(insts, items, count, cur, smem);
    FJOFC_BS(1, false, false) FJOFC_BS(1, false, true) FJOFC_BS(1, true, false)
    FJOFC_BS(1, true, true) FJOFC_BS(4, false, false) FJOFC_BS(4, false, true)
    FJOFC_BS(4, true, false) FJOFC_BS(4, true, true) FJOFC_BS(5, false, false)
    FJOFC_BS(5, false, true) FJOFC_BS(5, true, false) FJOFC_BS(5, true, true)
#undef FJOFC_BS
}

template <int MAXD>
__device__ __forceinline__ void batch_stream_any(int D, int variant, int vec4, bool stress,
                                                 const InstDesc *insts, const StreamItem *items,
                                                 int count, int cur, lfloat *smem) {
    switch (D) {
    case 1: if constexpr (MAXD >= 1) batch_stream_d<1>(variant, vec4, stress, insts, items, count, cur, smem); break;
    case 2: if constexpr (MAXD >= 2) batch_stream_d<2>(variant, vec4, stress, insts, items, count, cur, smem); break;
    case 3: if constexpr (MAXD >= 3) batch_stream_d<3>(variant, vec4, stress, insts, items, count, cur, smem); break;
    case 4: if constexpr (MAXD >= 4) batch_stream_d<4>(variant, vec4, stress, insts, items, count, cur, smem); break;
    case 5: if constexpr (MAXD >= 5) batch_stream_d<5>(variant, vec4, stress, insts, items, count, cur, smem); break;
    case 6: if constexpr (MAXD >= 6) batch_stream_d<6>(variant, vec4, stress, insts, items, count, cur, smem); break;
    case 7: if constexpr (MAXD >= 7) batch_stream_d<7>(variant, vec4, stress, insts, items, count, cur, smem); break;
    case 8: if constexpr (MAXD >= 8) batch_stream_d<8>(variant, vec4, stress, insts, items, count, cur, smem); break;
    default: break;
    }
}

// One finalize row item: rows [bx 256, bx 256 + 256) and component k, one
// row per thread, each thread summing both slot slices in the lockstep
// finalize's order, so the results are bitwise equal to it.
template <int MM>
__device__ __forceinline__ void batch_fin_row(const InstDesc &b, RowItem ri, int cur,
                                              int want_com, double *sh) {
    const int k = ri.k, m = b.g.m;
    const int j = ri.bx * FIN_ROWS + threadIdx.x;
    double bx[MM];
    for (int q = 0; q < m; ++q) {
        double t = fin_slice(b, q, k, j, 0);
        for (int e = 1; e < FIN_SLICES; ++e) t += fin_slice(b, q, k, j, e);
        bx[q] = b.wmat[q * m + q] * t;
    }
    const double com = fin_combine<MM>(b, k, j, cur, bx, want_com);
    if (want_com) {
        const double s = block_sum_d(com, sh);
        if (threadIdx.x == 0) b.comP[(size_t)k * (b.g.npad / FIN_ROWS) + ri.bx] = s;
    }
}

// A finalize group: `count` row items of one problem in turn (a barrier
// between two: the block sums reuse sh).
template <int MM>
__device__ __forceinline__ void batch_fin(const InstDesc &b, const RowItem *__restrict__ rows,
                                          int count, int cur, int want_com, double *sh) {
    for (int q = 0; q < count; ++q) {
        if (q > 0) __syncthreads();
        batch_fin_row<MM>(b, rows[q], cur, want_com, sh);
    }
}

// Bounded wait until *p >= need, run by a whole wavefront (every lane
// loads the same counter; the value is made wave-uniform, so the loop is
// uniform).  Gives up when another workgroup has flagged an error, or after
// a.timeout wall-clock ticks, flagging one itself: the launch then drains
// instead of hanging.
__device__ __forceinline__ int uniform_load(int *p) {
    return __builtin_amdgcn_readfirstlane(
        __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}

__device__ __forceinline__ bool batch_wait(const BatchArgs &a, int *p, int need) {
    if (uniform_load(p) >= need) return true;
    const long long t0 = (long long)wall_clock64();
    for (;;) {
        __builtin_amdgcn_s_sleep(2);
        if (uniform_load(p) >= need) return true;
        if (uniform_load(a.err)) return false;
        if ((long long)wall_clock64() - t0 > a.timeout) {
            __hip_atomic_store(a.err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
    }
}

// The reduce task (a noinline call keeps its per-thread branches out of the
// persistent loop's control flow).
__device__ __noinline__ void batch_red(const InstDesc *__restrict__ insts, int inst, int t,
                                       int check, int final_pass, int iters, double tol,
                                       int tol_mode) {
    reduce_body(insts[inst], t, check, final_pass, iters, tol, tol_mode);
}

// The task loop has no lane-divergent branch: the queue and the counters
// are handled by the whole of wavefront 0 (a wave-uniform branch), whose
// lanes all compute the same values; the atomics add 1 from lane 0 and 0
// from the others.  The values published through LDS are read back
// wave-uniform.  (With lane-divergent branches at the loop's head and tail
// the compiler may restructure it into nested loops in which the other
// lanes of wavefront 0 reach the next barrier before lane 0 has fetched
// the next task.)
template <int MAXD>
__global__ __launch_bounds__(BATCH_BLOCK)
__attribute__((amdgpu_waves_per_eu(MAXD <= 5 ? 4 : 2, 8))) void batch_kernel(BatchArgs a) {
    extern __shared__ float smem[];
    __shared__ long long sh_q;
    __shared__ int sh_state;
    __shared__ double sh_fin[BATCH_BLOCK / WAVE];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    const int one = (threadIdx.x & (WAVE - 1)) == 0 ? 1 : 0;
    for (;;) {
        if (wave == 0) {
            const unsigned long long o = atomicAdd(
                reinterpret_cast<unsigned long long *>(a.head), (unsigned long long)one);
            long long q = (long long)(((unsigned long long)(unsigned)__builtin_amdgcn_readfirstlane(
                                           (int)(o >> 32)) << 32) |
                                      (unsigned)__builtin_amdgcn_readfirstlane((int)o));
            if (uniform_load(a.err)) q = a.ntasks;
            sh_q = q;
        }
        __syncthreads();
        const long long q = (long long)(((unsigned long long)(unsigned)__builtin_amdgcn_readfirstlane(
                                              (int)((unsigned long long)sh_q >> 32)) << 32) |
                                        (unsigned)__builtin_amdgcn_readfirstlane((int)sh_q));
        if (q >= a.ntasks) break;
        int period, pos;
        batch_task_at(q, a.L, period, pos);
        const BatchTask tk = a.tmpl[pos];
        const int t = period - tk.lag;
        if (!batch_task_live(tk.kind, t, a.iters)) {
            // no such transform: nothing to wait for, run or count (the
            // barrier keeps wavefront 0 from overwriting sh_q before every
            // wavefront has read it)
            __syncthreads();
            continue;
        }
        const InstDesc &b = a.insts[tk.inst];
        int *c = &a.ctr[tk.inst].s_done;  // s_done, r_done, f_done
        const BatchDep dep = batch_dep(tk.kind, t, b.bnst, b.bnfin);
        int *wc = c + dep.wait, *dc = c + dep.done, need = dep.need;
        if (a.never_wait && q == 0) {
            wc = a.never;
            need = 1;
        }
        if (wave == 0) {
            const bool ok = batch_wait(a, wc, need);
            // acquire at agent scope: the producers' writes (released by
            // their workgroups, possibly on other XCDs) are visible
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            sh_state = !ok ? 0 : (uniform_load(&b.st->done) ? 1 : 2);
        }
        __syncthreads();
        const int state = __builtin_amdgcn_readfirstlane(sh_state);
        if (state == 0) break;
        const bool live = state == 2;
        const int cur = t & 1;
        if (tk.kind == BT_STREAM) {
            const bool stress = (t % a.every) == 0 || t == a.iters;
            if (live)
                batch_stream_any<MAXD>(b.D, b.g.variant, b.g.vec4, stress, a.insts,
                                       a.items + tk.first, tk.count, cur, to_lds(smem));
        } else if (tk.kind == BT_RED) {
            const bool fin = t == a.iters;
            if (fin || (t % a.every) == 0)
                batch_red(a.insts, tk.inst, t, fin ? ((a.iters % a.every) == 0 ? 1 : 0) : 1,
                          fin ? 1 : 0, a.iters, a.tol, a.tol_mode);
        } else if (live) {
            const int want_com = ((t + 1) % a.every) == 0 || (t + 1) == a.iters;
            const RowItem *rows = a.rows + tk.first;
            if (b.g.m <= 4)
                batch_fin<4>(b, rows, tk.count, cur, want_com, sh_fin);
            else if (b.g.m <= 8)
                batch_fin<8>(b, rows, tk.count, cur, want_com, sh_fin);
            else
                batch_fin<MAXM>(b, rows, tk.count, cur, want_com, sh_fin);
        }
        __syncthreads();
        if (wave == 0) {
            // release at agent scope: the workgroup's writes (ordered before
            // this point by the barrier) reach the device before the count
            // (the group's tiles, rows or one reduce)
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            atomicAdd(dc, one * tk.count);
        }
    }
}

}  // namespace
}  // namespace fjofc
