// In-sample fast-JOFC device code for gfx950 (shared by the stream,
// finalize and persistent translation units).
//
// One Guttman transform (Section 2.2, eq:update) is
//     X_t^(a) = sum_b [W^-1]_{ab} B_b(X^(b)) X^(b)
// where B_b(X) X has row j equal to sum_{l != j} r_jl (X_j - X_l) with
// r_jl = w_bb Delta_b[j,l] / d_jl and r_jl = 0 when d_jl = 0 (eq:B).
//
// Delta_b is symmetric, so every unordered pair {j,l} is read once, from the
// strict upper triangle: the pair's term t = r_jl (X_l - X_j) is added to the
// column accumulator of l and subtracted from the row accumulator of j.  The
// triangle is cut into th x tw tiles; a workgroup of R x C wavefronts streams
// one tile, each wavefront a slab of th / R rows and 64 lanes x CPL columns,
// walking its rows G at a time.  Each lane owns CPL columns (coalesced
// 16-byte loads of each row), keeps their column sums in registers for the
// whole slab, and keeps per-row partial sums for the current rows; every
// four rows those are summed across the 64 lanes through a small LDS buffer
// of the wavefront (each lane adds an eight-lane chunk of a few row
// components, then DPP adds the eight chunks) and each component is stored
// once.
// With several wavefronts the slabs' sums meet in LDS and are added in a
// fixed order at the end of the tile.  The configuration is held in SoA form
// [m][D][npad] so a group's row points are wave-uniform scalar loads and the
// column points are vector loads.  Tiles crossing the diagonal or the
// ragged edge run in a separate masked instance so the interior instance
// carries no per-element tests.
//
// Row and column sums of each tile go to a partial buffer (one slot per
// tile row / tile column), which the finalize kernel reduces in a fixed
// order (so results are bitwise reproducible), applies w_bb and W^-1 in
// FP64, and writes X_{t+1}.  The fidelity term of the raw stress
// (Remark faststress: it needs only the within-modality distances) is
// accumulated in the same stream when due: FP32 per lane and group, FP64
// per lane across groups, one FP64 value per tile.
#pragma once
#include "fjofc_internal.h"
#include <float.h>
#include <type_traits>

namespace fjofc {
namespace {

__device__ __forceinline__ double shfl_xor_d(double v, int mask) {
    const int lane = threadIdx.x & (WAVE - 1);
    int2 p = *reinterpret_cast<int2 *>(&v);
    p.x = __builtin_amdgcn_ds_bpermute((lane ^ mask) << 2, p.x);
    p.y = __builtin_amdgcn_ds_bpermute((lane ^ mask) << 2, p.y);
    return *reinterpret_cast<double *>(&p);
}

__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
    for (int s = 32; s >= 1; s >>= 1) v += shfl_xor_d(v, s);
    return v;
}

typedef float f4v __attribute__((ext_vector_type(4)));
// The configuration is never written while a stream kernel runs; reading it
// through the constant address space lets wave-uniform reads (a group's row
// points) compile to scalar loads.
typedef const __attribute__((address_space(4))) float cfloat;
// LDS pointers carry their address space explicitly, so that code taking
// them compiles to LDS instructions also where it is not inlined into the
// kernel that owns the LDS (the persistent batch calls its tile code; a
// generic pointer there would make every LDS access a flat instruction,
// which also waits for the outstanding global loads).
typedef __attribute__((address_space(3))) float lfloat;
typedef __attribute__((address_space(3))) double ldouble;
typedef __attribute__((address_space(3))) f4v lf4v;
__device__ __forceinline__ lfloat *to_lds(float *p) { return (lfloat *)p; }

// DPP controls (gfx9 encoding)
constexpr int DPP_QP_XOR1 = 0xB1;        // quad_perm [1,0,3,2]
constexpr int DPP_QP_XOR2 = 0x4E;        // quad_perm [2,3,0,1]
constexpr int DPP_ROW_HALF_MIRROR = 0x141;

template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}

// Column of the tile owned by `lane` for its q-th column (q < CPL).
// 16-byte path: runs of four consecutive columns, one run per 256 columns;
// otherwise one column per 64-lane stride.  Both give coalesced row reads.
template <bool VEC4>
__device__ __forceinline__ int lane_col(int lane, int q) {
    return VEC4 ? (q >> 2) * 256 + lane * 4 + (q & 3) : lane + WAVE * q;
}

// Orders this wavefront's LDS accesses (compiler and hardware): LDS
// operations of one wavefront complete in issue order, so a fence at
// wavefront scope is all that is needed.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Reduce the partial sums p[4][D] of four rows over the 64 lanes through
// this wavefront's LDS buffer red[4 D][64] and store each row component
// once.  Every lane writes its 4 D partials; lane (ob, c) = (lane / 8,
// lane % 8) then adds, for each of its T = ceil(4 D / 8) outputs ob T + t,
// the partials of lanes 8c .. 8c+7 (two 16-byte reads, taken in swapped
// order by odd ob so the two halves of a read fall in disjoint banks), and
// three DPP steps add the eight chunks, leaving the sum in all eight lanes
// of the group; lane c of the group stores output ob T + c.
template <int D, class SINK>
__device__ __forceinline__ void reduce4_lds(const float (&p)[4][D], lfloat *red, int lane,
                                            SINK *rsink, int rpitch, int rbase, int nvalid) {
    constexpr int V = 4 * D, T = (V + 7) / 8;
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int k = 0; k < D; ++k) red[(r * D + k) * WAVE + lane] = p[r][k];
    wave_sync();
    const int ob = lane >> 3, c = lane & 7;
    const int h0 = (ob & 1) * 4;
    float s[T];
#pragma unroll
    for (int t = 0; t < T; ++t) {
        const int o = min(ob * T + t, V - 1);
        const f4v a = *reinterpret_cast<const lf4v *>(red + o * WAVE + 8 * c + h0);
        const f4v b = *reinterpret_cast<const lf4v *>(red + o * WAVE + 8 * c + (4 - h0));
        s[t] = ((a.x + a.y) + (a.z + a.w)) + ((b.x + b.y) + (b.z + b.w));
    }
    wave_sync();
#pragma unroll
    for (int t = 0; t < T; ++t) {
        s[t] += dpp<DPP_QP_XOR1>(s[t]);
        s[t] += dpp<DPP_QP_XOR2>(s[t]);
        s[t] += dpp<DPP_ROW_HALF_MIRROR>(s[t]);
    }
    float v = s[0];
#pragma unroll
    for (int t = 1; t < T; ++t) v = c == t ? s[t] : v;
    const int o = ob * T + c, r = o / D, k = o - r * D;
    if (c < T && o < V && r < nvalid) rsink[(size_t)k * rpitch + rbase + r] = v;
}

template <int CPL, int G, bool VEC4, bool MASK>
__device__ __forceinline__ void load_rows(float (&dv)[G][CPL],
                                          const float *__restrict__ dl,
                                          int n, int j0, int c0, int lane,
                                          int nvalid) {
#pragma unroll
    for (int rr = 0; rr < G; ++rr) {
        const float *row = dl + (size_t)(j0 + rr) * n + c0;
        if (VEC4) {
#pragma unroll
            for (int h = 0; h < CPL / 4; ++h) {
                const int c = h * 256 + lane * 4;
                if (!MASK || (rr < nvalid && c0 + c < n)) {
                    const f4v v = __builtin_nontemporal_load(
                        reinterpret_cast<const f4v *>(row + c));
                    dv[rr][4 * h + 0] = v.x;
                    dv[rr][4 * h + 1] = v.y;
                    dv[rr][4 * h + 2] = v.z;
                    dv[rr][4 * h + 3] = v.w;
                } else {
#pragma unroll
                    for (int q = 0; q < 4; ++q) dv[rr][4 * h + q] = 0.f;
                }
            }
        } else {
#pragma unroll
            for (int q = 0; q < CPL; ++q) {
                const int c = lane_col<false>(lane, q);
                dv[rr][q] = (!MASK || (rr < nvalid && c0 + c < n))
                                ? __builtin_nontemporal_load(row + c) : 0.f;
            }
        }
    }
}

// Terms of G rows (given in dv) against the lane's CPL columns.  The G row
// sums go to rsink[k * rpitch + rbase + g0 + row], four rows at a time
// through the wavefront's LDS buffer red.
template <int D, int CPL, int G, bool VEC4, bool MASK, bool STRESS, bool ACC, bool COH,
          class SINK>
__device__ __forceinline__ void process_group(
    const float (&dv)[G][CPL], const float *__restrict__ X, int n, int npad,
    int r0, int c0, int g0, int nr, int lane, const float (&xc)[CPL][D],
    float (&cacc)[CPL][D], SINK *rsink, int rpitch, int rbase, lfloat *red, double &fid) {
    static_assert(G % 4 == 0, "rows are reduced four at a time");
    const int nv = MASK ? min(G, nr - g0) : G;
    // the group's row points (wave-uniform; padding rows are 0).  Within
    // one launch of the lockstep path the configuration is read-only, so
    // they are scalar loads through the constant address space.  In the
    // persistent batch (COH) the configuration is rewritten during the
    // launch, where the scalar cache would not see the new values: there
    // they are vector loads (after the task's acquire fence) made
    // wave-uniform with readfirstlane.
    float xr[G][D];
    if constexpr (COH) {
        // lane rr D + k loads X[k][row rr] once; readlane makes each uniform
        static_assert(G * D <= WAVE, "a group's row points fit one wavefront");
        float mine = 0.f;
        if (lane < G * D) {
            const int rr = lane / D, k = lane - rr * D;
            mine = __hip_atomic_load(X + (size_t)k * npad + r0 + g0 + rr, __ATOMIC_RELAXED,
                                     __HIP_MEMORY_SCOPE_WORKGROUP);
        }
#pragma unroll
        for (int k = 0; k < D; ++k)
#pragma unroll
            for (int rr = 0; rr < G; ++rr)
                xr[rr][k] = __int_as_float(
                    __builtin_amdgcn_readlane(__float_as_int(mine), rr * D + k));
    } else {
        cfloat *Xc = (cfloat *)X;
#pragma unroll
        for (int k = 0; k < D; ++k)
#pragma unroll
            for (int rr = 0; rr < G; ++rr) xr[rr][k] = Xc[(size_t)k * npad + r0 + g0 + rr];
    }
    float p[G][D];
#pragma unroll
    for (int rr = 0; rr < G; ++rr)
#pragma unroll
        for (int k = 0; k < D; ++k) p[rr][k] = 0.f;
    float fs = 0.f;
#pragma unroll
    for (int rr = 0; rr < G; ++rr) {
#pragma unroll
        for (int q = 0; q < CPL; ++q) {
            float diff[D];
#pragma unroll
            for (int k = 0; k < D; ++k) diff[k] = xc[q][k] - xr[rr][k];
            // Starting the squared distance at FLT_MIN keeps the reciprocal
            // finite for coincident points, whose diff is 0, so eq:B's
            // d = 0 => 0 rule holds with no extra test.
            float d2 = fmaf(diff[0], diff[0], FLT_MIN);
#pragma unroll
            for (int k = 1; k < D; ++k) d2 = fmaf(diff[k], diff[k], d2);
            const float rs = __builtin_amdgcn_rsqf(d2);
            float r = dv[rr][q] * rs;
            bool ok = true;
            if (MASK) {
                const int col = c0 + lane_col<VEC4>(lane, q);
                const int row = r0 + g0 + rr;
                ok = (col < n) && (row < n) && (col > row);
                r = ok ? r : 0.f;
            }
            if (ACC) {
#pragma unroll
                for (int k = 0; k < D; ++k) {
                    cacc[q][k] = fmaf(r, diff[k], cacc[q][k]);
                    p[rr][k] = fmaf(r, diff[k], p[rr][k]);
                }
            }
            if (STRESS) {
                const float e = dv[rr][q] - d2 * rs;
                fs = ok ? fmaf(e, e, fs) : fs;
            }
        }
        // Materialise the column sums row by row: otherwise the compiler
        // sinks their updates to the end of the group and keeps every
        // row's differences alive until then.
        if (ACC) {
#pragma unroll
            for (int q = 0; q < CPL; ++q)
#pragma unroll
                for (int k = 0; k < D; ++k) asm volatile("" : "+v"(cacc[q][k]));
        }
        if (STRESS) asm volatile("" : "+v"(fs));
        if (ACC && rr % 4 == 3)
            reduce4_lds<D>(*reinterpret_cast<float(*)[4][D]>(&p[rr - 3][0]), red, lane, rsink,
                           rpitch, rbase + g0 + rr - 3, nv - (rr - 3));
        __builtin_amdgcn_sched_barrier(0);
    }
    if (STRESS) fid += (double)fs;
}

// One workgroup of R x C wavefronts streams one tile of the strict upper
// triangle: wavefront (wr, wc) takes the tile's rows [wr th/R, (wr+1) th/R)
// and its columns [wc 64 CPL, (wc+1) 64 CPL).  With one wavefront the row and
// column sums go straight to the partial buffer.  With several, each
// wavefront leaves its sums in LDS and, after one barrier, the workgroup adds
// them in a fixed order (over wc for a row, over wr for a column) and writes
// each of the tile's rows and columns once, which divides the partial-sum
// traffic of a th x tw tile by the number of wavefronts sharing a row or
// column.  MASK is set for boundary tiles: those crossing the diagonal (only
// l > j counts) or the ragged edge (rows or columns >= n).
template <int D, int CPL, int G, bool DBUF, bool VEC4, bool MASK, bool STRESS, bool ACC, int R,
          int C, bool COH = false>
__device__ __forceinline__ void stream_tile(
    const TriGeom &g, const DeltaPtrs &dp, const float *__restrict__ Xs,
    int i, int I, int J, int ftile, float *__restrict__ P,
    double *__restrict__ F, lfloat *smem) {
    constexpr int NW = R * C, TWW = WAVE * CPL;
    const int lane = threadIdx.x & (WAVE - 1);
    const int w = NW == 1 ? 0 : __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    const int wr = w / C, wc = w - (w / C) * C;
    const int n = g.n, npad = g.npad;
    const int S = g.ntc + g.ntr;
    const float *__restrict__ dl = dp.p[i];
    const float *__restrict__ X = Xs + (size_t)i * D * npad;
    const int thw = g.th / R;
    const int ct0 = tile_col0(g, I, J), rt0 = I * g.th;   // the tile
    const int c0 = ct0 + wc * TWW, r0 = rt0 + wr * thw;   // this wavefront's part
    // rows to stream; none when the part holds no pair l > j inside n (its
    // columns start at or beyond n, or its rows are all >= its last column)
    const bool empty = MASK && (c0 >= n || r0 >= c0 + TWW - 1);
    const int nr = MASK ? (empty ? 0 : min(thw, n - r0)) : thw;

    float xc[CPL][D];
#pragma unroll
    for (int k = 0; k < D; ++k) {
        const float *xk = X + (size_t)k * npad + c0;
        if (VEC4) {
#pragma unroll
            for (int h = 0; h < CPL / 4; ++h) {
                const float4 v = *reinterpret_cast<const float4 *>(xk + h * 256 + lane * 4);
                xc[4 * h + 0][k] = v.x;
                xc[4 * h + 1][k] = v.y;
                xc[4 * h + 2][k] = v.z;
                xc[4 * h + 3][k] = v.w;
            }
        } else {
#pragma unroll
            for (int q = 0; q < CPL; ++q) xc[q][k] = xk[lane_col<false>(lane, q)];
        }
    }
    float cacc[CPL][D];
#pragma unroll
    for (int q = 0; q < CPL; ++q)
#pragma unroll
        for (int k = 0; k < D; ++k) cacc[q][k] = 0.f;
    double fid = 0.0;
    float *Pm = P + (size_t)i * S * D * npad;
    float *prow = Pm + (size_t)J * D * npad;
    float *pcol = Pm + (size_t)(g.ntc + I) * D * npad;
    // LDS layout (several wavefronts): row sums [C][D][th], column sums
    // [R][D][tw], then one double per wavefront for the fidelity.
    const int tw = C * TWW;
    lfloat *srow = smem, *scol = smem + (size_t)C * D * g.th;
    ldouble *sfid = reinterpret_cast<ldouble *>(scol + (size_t)R * D * tw);
    // row sums go to the partial buffer (global) with one wavefront, else
    // to LDS
    using RS = std::conditional_t<NW == 1, float, lfloat>;
    RS *rsink;
    if constexpr (NW == 1)
        rsink = prow;
    else
        rsink = srow + (size_t)wc * D * g.th;
    const int rpitch = NW == 1 ? npad : g.th;
    const int rbase = NW == 1 ? r0 : wr * thw;
    // this wavefront's row-reduction buffer [4 D][64]: the whole LDS with one
    // wavefront, else a slice of the column-sum region, which takes column
    // sums only after every wavefront's stream has finished
    static_assert(NW == 1 || CPL >= 4, "the reduction buffers fit the column region");
    lfloat *red = NW == 1 ? smem : scol + (size_t)w * 4 * D * WAVE;

    if (NW > 1 && ACC && empty) {
        // the workgroup still adds this wavefront's row sums for the rows
        // below n: they are zero
        for (int q = lane; q < D * thw; q += WAVE) {
            const int k = q / thw, r = q - k * thw;
            rsink[(size_t)k * rpitch + rbase + r] = 0.f;
        }
    }
    if (DBUF) {
        // Two row buffers used alternately (no register copies, so the
        // loads of the next group stay in flight while the current group
        // is computed).
        float da[G][CPL], db[G][CPL];
        load_rows<CPL, G, VEC4, MASK>(da, dl, n, r0, c0, lane, nr);
        for (int g0 = 0; g0 < nr; g0 += 2 * G) {
            if (g0 + G < nr)
                load_rows<CPL, G, VEC4, MASK>(db, dl, n, r0 + g0 + G, c0, lane, nr - g0 - G);
            process_group<D, CPL, G, VEC4, MASK, STRESS, ACC, COH, RS>(da, X, n, npad, r0, c0, g0, nr,
                                                              lane, xc, cacc, rsink, rpitch,
                                                              rbase, red, fid);
            if (g0 + G >= nr) break;
            if (g0 + 2 * G < nr)
                load_rows<CPL, G, VEC4, MASK>(da, dl, n, r0 + g0 + 2 * G, c0, lane,
                                              nr - g0 - 2 * G);
            process_group<D, CPL, G, VEC4, MASK, STRESS, ACC, COH, RS>(db, X, n, npad, r0, c0, g0 + G,
                                                              nr, lane, xc, cacc, rsink, rpitch,
                                                              rbase, red, fid);
        }
    } else {
        // One row buffer: other wavefronts on the SIMD cover the load latency.
        for (int g0 = 0; g0 < nr; g0 += G) {
            float da[G][CPL];
            load_rows<CPL, G, VEC4, MASK>(da, dl, n, r0 + g0, c0, lane, nr - g0);
            process_group<D, CPL, G, VEC4, MASK, STRESS, ACC, COH, RS>(da, X, n, npad, r0, c0, g0, nr,
                                                              lane, xc, cacc, rsink, rpitch,
                                                              rbase, red, fid);
        }
    }
    if constexpr (NW > 1) __syncthreads();
    if (ACC) {
        // this wavefront's column sums: to the partial buffer, or to LDS
        using CS = std::conditional_t<NW == 1, float, lfloat>;
        using CS4 = std::conditional_t<NW == 1, f4v, lf4v>;
        CS *csink;
        if constexpr (NW == 1)
            csink = pcol + c0;
        else
            csink = scol + (size_t)wr * D * tw + wc * TWW;
        const int cpitch = NW == 1 ? npad : tw;
#pragma unroll
        for (int k = 0; k < D; ++k) {
            if (VEC4) {
#pragma unroll
                for (int h = 0; h < CPL / 4; ++h)
                    *reinterpret_cast<CS4 *>(csink + (size_t)k * cpitch + h * 256 + lane * 4) =
                        f4v{cacc[4 * h][k], cacc[4 * h + 1][k], cacc[4 * h + 2][k],
                            cacc[4 * h + 3][k]};
            } else {
#pragma unroll
                for (int q = 0; q < CPL; ++q)
                    csink[(size_t)k * cpitch + lane_col<false>(lane, q)] = cacc[q][k];
            }
        }
    }
    if (STRESS) {
        fid = wave_sum_d(fid);
        if (NW == 1) {
            if (lane == 0) F[(size_t)i * (g.nint + g.nbnd) + ftile] = fid;
        } else if (lane == 0) {
            sfid[w] = fid;
        }
    }
    if constexpr (NW > 1) {
        __syncthreads();
        if (ACC) {
            // rows of the tile inside n, each summed over the C wavefronts
            // that share it
            const int th = g.th, nrows = MASK ? min(th, n - rt0) : th;
            for (int q = threadIdx.x; q < D * th; q += NW * WAVE) {
                const int k = q / th, r = q - k * th;
                if (r >= nrows) continue;
                float v = srow[(size_t)k * th + r];
#pragma unroll
                for (int c = 1; c < C; ++c) v += srow[((size_t)c * D + k) * th + r];
                prow[(size_t)k * npad + rt0 + r] = v;
            }
            // columns of the tile, each summed over the R wavefronts
            for (int q = threadIdx.x; q < D * tw; q += NW * WAVE) {
                const int k = q / tw, c = q - k * tw;
                float v = scol[(size_t)k * tw + c];
#pragma unroll
                for (int rr = 1; rr < R; ++rr) v += scol[((size_t)rr * D + k) * tw + c];
                pcol[(size_t)k * npad + ct0 + c] = v;
            }
        }
        if (STRESS && threadIdx.x == 0) {
            double t = sfid[0];
            for (int q = 1; q < NW; ++q) t += sfid[q];
            F[(size_t)i * (g.nint + g.nbnd) + ftile] = t;
        }
    }
}

// Stream kernel: one workgroup of R x C wavefronts per work item.  Items of
// interior tiles run the unmasked instance, boundary tiles (crossing the
// diagonal or the ragged edge) the masked instance.  With several
// wavefronts the launch supplies the LDS for their partial sums.
template <int D, int CPL, int G, bool DBUF, bool VEC4, bool STRESS, bool ACC, int R, int C>
__global__ __launch_bounds__(WAVE * R * C) void bx_kernel(
    const InstDesc *__restrict__ insts, const StreamItem *__restrict__ items, int cur) {
    extern __shared__ float smem[];
    const StreamItem it = items[blockIdx.x];
    const InstDesc &b = insts[it.inst];
    if (b.st->done) return;
    const float *Xs = b.Xs[cur];
    const int I = it.tile >> 16, J = it.tile & 0xffff;
    if (it.ftile < b.g.nint)
        stream_tile<D, CPL, G, DBUF, VEC4, false, STRESS, ACC, R, C>(b.g, b.dp, Xs, it.mod, I, J,
                                                                     it.ftile, b.P, b.F, to_lds(smem));
    else
        stream_tile<D, CPL, G, DBUF, VEC4, true, STRESS, ACC, R, C>(b.g, b.dp, Xs, it.mod, I, J,
                                                                    it.ftile, b.P, b.F, to_lds(smem));
}

// ---------------------------------------------------------------------------
// Finalize: reduce the partial slots of row j, apply w_bb (B_b's entries are
// -w_bb Delta/d), combine with W^-1 in FP64 (eq:update), store X_{t+1} and
// accumulate its commensurability sum_{a<b} w_ab ||X^(a)_j - X^(b)_j||^2
// from the stored FP32 values.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double block_sum_d(double v, double *sh) {
    v = wave_sum_d(v);
    const int wv = threadIdx.x / WAVE;
    if ((threadIdx.x & (WAVE - 1)) == 0) sh[wv] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int q = 0; q < (int)(blockDim.x / WAVE); ++q) s += sh[q];
    return s;
}

// Sum of the slots q0, q0 + step, ... below q1 of one partial column
// (stride `slot` floats), four independent FP64 accumulators so the loads
// overlap.
__device__ __forceinline__ double slot_sum(const float *__restrict__ p, size_t slot,
                                           int q0, int q1, int step) {
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    int q = q0;
    for (; q + 3 * step < q1; q += 4 * step) {
        a0 += (double)p[(size_t)q * slot];
        a1 += (double)p[(size_t)(q + step) * slot];
        a2 += (double)p[(size_t)(q + 2 * step) * slot];
        a3 += (double)p[(size_t)(q + 3 * step) * slot];
    }
    for (; q < q1; q += step) a0 += (double)p[(size_t)q * slot];
    return (a0 + a1) + (a2 + a3);
}

// Row j's partial sums of component k in modality q over the slots
// congruent to sl mod FIN_SLICES: its column sums (one tile of every row
// block I' <= j / th) minus its row sums (tiles (I, J), J < row_tiles(I)).
// A row block whose only row is n - 1 holds no pair and has no tiles.
constexpr int FIN_SLICES = 2;
__device__ __forceinline__ double fin_slice(const InstDesc &b, int q, int k, int j, int sl) {
    const TriGeom &g = b.g;
    if (j >= g.n) return 0.0;
    const int I = j / g.th;
    const bool live = g.n - 1 > I * g.th;
    const int jhi = live ? row_tiles(g, I) : 0;
    const int ihi = I + (live ? 1 : 0);
    const size_t slot = (size_t)b.D * g.npad;
    const int S = g.ntc + g.ntr;
    const float *Pb = b.P + (size_t)q * S * slot + (size_t)k * g.npad + j;
    return slot_sum(Pb, slot, g.ntc + sl, g.ntc + ihi, FIN_SLICES) -
           slot_sum(Pb, slot, sl, jhi, FIN_SLICES);
}

// eq:update for row j, component k from bx[q] = w_qq (B_q X^(q))_jk: writes
// X_{t+1} (relaxed when alpha != 1) and returns the row's weighted
// commensurability term when want_com; rows in [n, npad) get 0.
template <int MM>
__device__ __forceinline__ double fin_combine(const InstDesc &b, int k, int j, int cur,
                                              const double (&bx)[MM], int want_com) {
    const TriGeom &g = b.g;
    const int m = g.m, D = b.D, npad = g.npad;
    float *__restrict__ Xout = b.Xs[cur ^ 1];
    double com = 0.0;
    if (j < g.n) {
        float xn[MM];
        const double alpha = b.alpha;
        const float *__restrict__ Xin = b.Xs[cur];
        for (int a = 0; a < m; ++a) {
            double v = 0.0;
            for (int q = 0; q < m; ++q) v += b.Winv[a * m + q] * bx[q];
            if (alpha != 1.0) {
                // relaxed update: X_t + alpha (Gamma(X_t) - X_t)
                const double xt = (double)Xin[((size_t)a * D + k) * npad + j];
                v = xt + alpha * (v - xt);
            }
            xn[a] = (float)v;
            Xout[((size_t)a * D + k) * npad + j] = xn[a];
        }
        if (want_com)
            for (int a = 0; a < m; ++a)
                for (int q = a + 1; q < m; ++q) {
                    const double t = (double)xn[a] - (double)xn[q];
                    com += b.wmat[a * m + q] * t * t;
                }
    } else if (j < npad) {
        for (int a = 0; a < m; ++a) Xout[((size_t)a * D + k) * npad + j] = 0.f;
    }
    return com;
}

// Deterministic FP64 reduction of the per-tile fidelity partials (weighted
// by w_ii) and the commensurability partials, then Algorithm 2's stop test.
// One workgroup of RED_BLOCK threads per instance.  The loop state is read
// with atomic loads: in the persistent batch other workgroups rewrite it
// during the launch.
constexpr int RED_BLOCK = 256;
__device__ __forceinline__ void reduce_body(const InstDesc &b, int t, int check, int final_pass,
                                            int iters, double tol, int tol_mode) {
    __shared__ double shf[RED_BLOCK], shc[RED_BLOCK];
    EmbedState *st = b.st;
    if (__hip_atomic_load(&st->done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
    const int tid = threadIdx.x;
    const int m = b.g.m, ntiles = b.g.nint + b.g.nbnd;
    double f = 0.0, c = 0.0;
    for (int i = 0; i < m; ++i) {
        double fi = 0.0;
        for (int q = tid; q < ntiles; q += RED_BLOCK) fi += b.F[(size_t)i * ntiles + q];
        f += b.wmat[i * m + i] * fi;
    }
    for (int q = tid; q < b.ncom; q += RED_BLOCK) c += b.comP[q];
    shf[tid] = f;
    shc[tid] = c;
    __syncthreads();
    for (int s = RED_BLOCK / 2; s > 0; s >>= 1) {
        if (tid < s) {
            shf[tid] += shf[tid + s];
            shc[tid] += shc[tid + s];
        }
        __syncthreads();
    }
    if (tid == 0) {
        const double fid = shf[0], com = shc[0], sigma = fid + com;
        const double mn = (double)m * b.g.n;
        const double last = __hip_atomic_load(&st->last, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (b.hist) b.hist[t] = sigma;
        st->sigma = sigma;
        st->fid = fid;
        st->com = com;
        bool stopped = false;
        if (check && tol > 0.0) {
            bool stop;
            if (tol_mode == 3) {
                stop = sigma <= tol;  // stress target
            } else {
                const double thr = (tol_mode == 2) ? tol * 0.5 * mn * (mn - 1.0) : tol * last;
                stop = t > 0 && last - sigma < thr;
            }
            if (stop) {
                st->done = 1;
                st->converged = 1;
                st->iters_run = t;
                stopped = true;
            }
        }
        if (check) st->last = sigma;
        if (final_pass && !stopped) st->iters_run = iters;
    }
}

template <int D, int CPL, int G, bool DBUF, bool VEC4, int R, int C>
hipError_t launch_stream_t(const InstDesc *insts, const StreamItem *items, int nitems,
                           int cur, bool stress, bool acc, size_t lds, hipStream_t s) {
    if (nitems == 0) return hipSuccess;
    const dim3 grid((unsigned)nitems), block(WAVE * R * C);
    if (stress && acc)
        bx_kernel<D, CPL, G, DBUF, VEC4, true, true, R, C><<<grid, block, lds, s>>>(insts, items,
                                                                                 cur);
    else if (acc)
        bx_kernel<D, CPL, G, DBUF, VEC4, false, true, R, C><<<grid, block, lds, s>>>(insts, items,
                                                                                  cur);
    else
        bx_kernel<D, CPL, G, DBUF, VEC4, true, false, R, C><<<grid, block, lds, s>>>(insts, items,
                                                                                  cur);
    return hipGetLastError();
}

template <int D, int CPL, int G, bool DBUF, int R = 1, int C = 1>
hipError_t launch_stream_v(int vec4, const InstDesc *insts, const StreamItem *items,
                           int nitems, int cur, bool stress, bool acc, size_t lds,
                           hipStream_t s) {
    return vec4 ? launch_stream_t<D, CPL, G, DBUF, true, R, C>(insts, items, nitems, cur, stress,
                                                               acc, lds, s)
                : launch_stream_t<D, CPL, G, DBUF, false, R, C>(insts, items, nitems, cur, stress,
                                                                acc, lds, s);
}

// Kernel variants (columns per lane, rows per group, double-buffered rows,
// wavefronts per tile R x C); the numbering is shared with the host's
// variant table.
template <int D>
hipError_t launch_stream_d(int variant, int vec4, const InstDesc *insts,
                           const StreamItem *items, int nitems, int cur, bool stress,
                           bool acc, size_t lds, hipStream_t s) {
    switch (variant) {
    case 1: return launch_stream_v<D, 4, 8, false>(vec4, insts, items, nitems, cur, stress, acc, lds, s);
    case 2: return launch_stream_v<D, 8, 4, false>(vec4, insts, items, nitems, cur, stress, acc, lds, s);
    case 3: return launch_stream_v<D, 8, 8, false>(vec4, insts, items, nitems, cur, stress, acc, lds, s);
    case 4: return launch_stream_v<D, 4, 8, false, 4, 1>(vec4, insts, items, nitems, cur, stress, acc, lds, s);
    case 5: return launch_stream_v<D, 4, 8, false, 2, 2>(vec4, insts, items, nitems, cur, stress, acc, lds, s);
    default: return launch_stream_v<D, 4, 8, true>(vec4, insts, items, nitems, cur, stress, acc, lds, s);
    }
}

}  // namespace

// The D = 1..4 and D = 5..8 halves of launch_stream, each in a translation
// unit of its own (stream_lo.hip, stream_hi.hip) so that they compile in
// parallel.
hipError_t launch_stream_lo(int D, int variant, int vec4, const InstDesc *insts,
                            const StreamItem *items, int nitems, int cur, bool stress,
                            bool acc, size_t lds, hipStream_t s);
hipError_t launch_stream_hi(int D, int variant, int vec4, const InstDesc *insts,
                            const StreamItem *items, int nitems, int cur, bool stress,
                            bool acc, size_t lds, hipStream_t s);
// The persistent kernel for batches with D <= 5 (batch5.hip) and D <= 8
// (batch8.hip): launch, and the kernel's address for the occupancy query.
hipError_t launch_batch_kernel5(const BatchArgs &a, int grid, size_t lds, hipStream_t s);
hipError_t launch_batch_kernel8(const BatchArgs &a, int grid, size_t lds, hipStream_t s);
const void *batch_kernel5_address();
const void *batch_kernel8_address();

}  // namespace fjofc
