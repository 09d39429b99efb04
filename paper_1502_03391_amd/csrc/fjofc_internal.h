// Internal declarations shared by the fast-JOFC HIP kernels and the host
// library.  Not part of the public ABI (include/fjofc.h is).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

struct fjofc_ctx;

namespace fjofc {

constexpr int WAVE = 64;
constexpr int MAXM = 32;
constexpr int MAXD = 8;

struct DeltaPtrs {
    const float *p[MAXM];
};

// Device-resident state of one in-sample run (Algorithm 2's loop).
struct EmbedState {
    int done;       // stop rule fired: later kernels of the run do nothing
    int iters_run;  // transforms applied to X0
    int converged;
    int pad;
    double last;    // sigma at the previous checkpoint
    double sigma;   // sigma of the last evaluated configuration
    double fid;     // its weighted fidelity
    double com;     // its weighted commensurability
};

// Geometry of the tiled strict-upper-triangle stream of one n x n block.
// Tiles are th rows x tw columns (tw = 64 lanes x cpl columns per lane x
// the variant's column wavefronts).
// The tiling is staggered along the diagonal: row block I covers rows
// [I th, I th + th) and its tiles J = 0, 1, ... cover columns
// [c0, c0 + tw) with c0 = I th + J tw, so each row block's first tile
// starts on the diagonal (a diagonal tile wastes th^2 / 2 pairs instead of
// up to th tw / 2).  Tile (I, J) exists when it holds a pair j < l inside n.
struct TriGeom {
    int n;          // objects
    int m;          // modalities
    int npad;       // row pitch of SoA buffers (>= n + tw; multiple of max(th, tw))
    int th, tw;     // tile height and width
    int cpl;        // columns per lane (4 or 8)
    int variant;    // stream-kernel variant: (cpl, rows per group, buffering,
                    // wavefronts per tile)
    int ntr, ntc;   // row blocks / most tiles in a row block (that of block 0)
    int nint;       // interior tiles per modality (no masking needed)
    int nbnd;       // boundary tiles per modality (diagonal or ragged)
    int vec4;       // 1: rows are 16-byte aligned (n % 4 == 0)
};

__host__ __device__ inline int tile_col0(const TriGeom &g, int I, int J) {
    return I * g.th + J * g.tw;
}

__host__ __device__ inline bool tile_exists(const TriGeom &g, int I, int J) {
    const int c0 = tile_col0(g, I, J);
    return c0 < g.n && min(c0 + g.tw, g.n) - 1 > I * g.th;
}

// Tiles in row block I: ceil((n - I th) / tw).
__host__ __device__ inline int row_tiles(const TriGeom &g, int I) {
    const int rem = g.n - I * g.th;
    return rem > 0 ? (rem + g.tw - 1) / g.tw : 0;
}

// Partial sums produced by the stream, FP32, layout [m][S][D][npad] with
// S = ntc + ntr slots: slot J holds row sums of tile (I, J) for the rows of
// block I, slot ntc + I holds column sums of tile (I, J) for its columns
// (the tiles of one row block cover disjoint columns).
inline size_t partial_floats(const TriGeom &g, int D) {
    return (size_t)g.m * (g.ntc + g.ntr) * D * g.npad;
}

// One in-sample problem as the kernels see it (device-resident).
struct InstDesc {
    TriGeom g;
    int D;
    int ncom;           // commensurability partials (finalize blocks x D)
    DeltaPtrs dp;
    float *Xs[2];       // SoA [m][D][npad] configurations, double-buffered
    float *P;           // partial sums
    double *F;          // per-tile fidelity [m][nint + nbnd]
    double *comP;       // commensurability partials
    const double *Winv; // m x m
    const double *wmat; // m x m
    EmbedState *st;
    double *hist;       // optional: stress history (iters + 1)
    float *X;           // caller's (m n) x d configuration
    double alpha;       // relaxation: X_{t+1} = X_t + alpha (Gamma(X_t) - X_t)
    int bnst, bnfin;    // persistent batch: tiles and finalize row items per transform
};

// One wavefront's work: tile `tile` (I << 16 | J) of modality `mod` of
// instance `inst`; ftile is its index in the instance's tile list.
struct StreamItem {
    int inst, mod;
    uint32_t tile;
    int ftile;
};
// One finalize / commensurability workgroup: rows [bx 256, bx 256 + 256)
// and component k of instance `inst`.
struct RowItem {
    int inst, bx, k, pad;
};

// The finalize and commensurability kernels cover rows [0, npad / FIN_ROWS
// * FIN_ROWS), which holds every row below n because npad >= n + tw and
// tw >= FIN_ROWS; each writes one commensurability partial per block.
constexpr int FIN_ROWS = 256;
inline int commens_blocks(const TriGeom &g, int D) {
    return g.npad / FIN_ROWS * D;
}

// ---- in-sample launchers (insample.hip; kernels in stream_*.hip) -----
// Stream kernels for one (D, variant, vec4) group of items; `cur` selects
// the configuration buffer Xs[cur].
hipError_t launch_stream(int D, int variant, int vec4, const InstDesc *insts,
                         const StreamItem *items, int nitems, int cur,
                         bool stress, bool acc, size_t lds, hipStream_t s);
// one_thread: one thread per (row, component) forms the slice sums in turn
// (same bits as one thread per slice; fewer, fuller workgroups).
hipError_t launch_finalize(int maxm, const InstDesc *insts, const RowItem *rows,
                           int nrows, int cur, bool want_com, bool one_thread, hipStream_t s);
hipError_t launch_com(const InstDesc *insts, const RowItem *rows, int nrows,
                      hipStream_t s);
// One workgroup per instance [0, count).
hipError_t launch_reduce(const InstDesc *insts, int count, int t, int check,
                         int final_pass, int iters, double tol, int tol_mode,
                         hipStream_t s);
hipError_t launch_init(const InstDesc *insts, int count, int nhist,
                       hipStream_t s);
hipError_t launch_copy_out(const InstDesc *insts, int count, hipStream_t s);
// SoA conversion used by the out-of-sample path.
hipError_t launch_to_soa(const TriGeom &g, int D, const float *X, float *Xs,
                         hipStream_t s);

// ---- persistent batched launch (insample.hip, batch5.hip, batch8.hip) -
// One launch runs every transform of every problem of a batch.  Workgroups
// of BATCH_BLOCK threads take tasks from a queue in a fixed order (a task is
// a group of tiles, of finalize row items or one reduce, of one problem); a
// task waits (bounded) until the work it depends on, all earlier in the
// order, has completed, as counted per problem in tiles, row items and
// reduces:
//   stream (t): f_done >= t bnfin   (X_t complete)
//   reduce (t): s_done >= (t+1) bnst (every tile of transform t streamed)
//   finalize (t): r_done >= t + 1   (transform t's reduce, hence its streams)
// The queue repeats one template (`tmpl`, L tasks) per period.  The
// problems, largest first, are dealt into six groups (rank mod 6), and a
// period is, for g = 0..5, the streams of group g followed by the reduces
// and finalizes of group g - 3 (mod 6; one period late for g < 3).  So
// between a group's streams and its reduces and finalizes lie three other
// groups' stream blocks, and between those and the group's next streams
// two more: workgroups find ready work while a group's finalize waits for
// its last tiles.  A task's transform is the period minus its lag; the
// queue runs iters + 2 periods and skips the tasks of transforms that do not
// exist (batch_task_live).  Streams and reduces at t = iters give the stress
// of the returned configuration.  Every dependency of a task lies earlier
// in the order, so with all workgroups resident the earliest unfinished
// task can always run.
constexpr int BATCH_BLOCK = 256;
enum { BT_STREAM = 0, BT_RED = 1, BT_FIN = 2 };
struct BatchTask {
    int kind, inst;
    int first;   // stream: first item (tile) index; finalize: first row item
    int count;   // tiles or row items of the group (1 for a reduce)
    int lag;     // periods the task trails its period (its transform: period - lag)
};
struct BatchCtr {
    int s_done, r_done, f_done, pad;
};
// What a task of `kind` at transform t waits for and which counter its
// completion advances (by its count), for a problem with bnst tiles and
// bnfin finalize row items per transform: counter indices 0 = s_done,
// 1 = r_done, 2 = f_done.
struct BatchDep {
    int wait, need, done;
};
__host__ __device__ inline BatchDep batch_dep(int kind, int t, int bnst, int bnfin) {
    if (kind == BT_STREAM) return {2, t * bnfin, 0};   // X_t complete
    if (kind == BT_RED) return {0, (t + 1) * bnst, 1};  // transform t streamed
    return {1, t + 1, 2};                               // transform t reduced
}
// Task q of the sequence: period q / L, template position q % L.
__host__ __device__ inline void batch_task_at(long long q, int L, int &period, int &pos) {
    period = (int)(q / L);
    pos = (int)(q - (long long)period * L);
}
// Whether the task of `kind` at transform t exists: streams and reduces for
// t = 0..iters, finalizes for t < iters.
__host__ __device__ inline bool batch_task_live(int kind, int t, int iters) {
    return t >= 0 && t <= iters && !(kind == BT_FIN && t == iters);
}
// Periods of a run of `iters` transforms (the last one holds only the
// lagging group's reduces at t = iters).
inline long long batch_periods(int iters) { return (long long)iters + 2; }
// The template (host side): st[p] and fin[p] are problem p's stream and
// finalize tasks of one transform, `order` the problems largest first.
// On the uneven 512-problem batch (same box): 6 groups at distance 3 took
// 0.225 s, 8 at 4 0.225 s, 4 at 2 0.229 s, 5 at 2 0.229 s, 3 at 1 0.233 s,
// 6 at 2 0.237 s, 8 at 3 0.235 s.
constexpr int BATCH_GROUPS = 6, BATCH_GROUP_DIST = 3;
inline std::vector<BatchTask> batch_template(const std::vector<int> &order,
                                             const std::vector<std::vector<BatchTask>> &st,
                                             const std::vector<std::vector<BatchTask>> &fin) {
    constexpr int NG = BATCH_GROUPS, DIST = BATCH_GROUP_DIST;
    static_assert(DIST >= 1 && DIST < NG, "a group's closes follow its own streams");
    std::vector<BatchTask> out;
    auto streams = [&](int g) {
        for (size_t r = g; r < order.size(); r += NG)
            for (BatchTask tk : st[order[r]]) {
                tk.lag = 0;
                out.push_back(tk);
            }
    };
    auto closes = [&](int g, int lag) {
        for (size_t r = g; r < order.size(); r += NG) out.push_back({BT_RED, order[r], 0, 1, lag});
        for (size_t r = g; r < order.size(); r += NG)
            for (BatchTask tk : fin[order[r]]) {
                tk.lag = lag;
                out.push_back(tk);
            }
    };
    for (int g = 0; g < NG; ++g) {
        streams(g);
        closes((g - DIST + NG) % NG, g < DIST ? 1 : 0);
    }
    return out;
}
struct BatchArgs {
    const InstDesc *insts;
    const StreamItem *items;
    const RowItem *rows;
    const BatchTask *tmpl;
    int L, pad0;          // template length
    long long ntasks;     // batch_periods(iters) L
    BatchCtr *ctr;        // per problem
    int *head;            // next task
    int *err;             // non-zero: a wait timed out (the launch stops)
    int *never;           // a counter no task increments (host-forced wait test)
    int never_wait;       // 1: the first task waits on `never`
    long long timeout;    // wall-clock ticks a wait may last
    int iters, every, tol_mode, pad;
    double tol;
};
// Zeroes head, err and the count problems' counters.
hipError_t launch_batch_reset(const BatchArgs &a, int count, hipStream_t s);
// maxd, maxm: the largest D and m of the batch; grid at most the resident
// workgroups (batch_resident_blocks per CU times the CUs).
hipError_t launch_batch_persistent(const BatchArgs &a, int maxd, int maxm, int grid, size_t lds,
                                   hipStream_t s);
// Workgroups of the persistent kernel one CU holds at once (0 on error).
int batch_resident_blocks(int maxd, int maxm, size_t lds);
// Tiles per stream task: one-wavefront tiles, eight per wavefront; shared
// tiles, twelve in turn.  Finalize row items per task.  Every task ends in
// an agent-scope release and starts after an acquire, and a task that must
// wait holds its workgroup, so tasks are made coarse, but not so coarse
// that the last ones of a block run alone.  On the uneven 512-problem batch
// with the tile cache's tiles, in the three-group order, sweeps ranked
// (32, 12, 8) first at 0.250 s (same box: (32, 16, 12) 0.250 s, (40, 16, 8)
// 0.255 s, (32, 8, 8) 0.256 s, (32, 8, 16) 0.262 s, (16, 4, 8) 0.284 s,
// (32, 24, 8) 0.286 s).
constexpr int BATCH_TILES_1W = 32, BATCH_TILES_SHARED = 12, BATCH_ROWS = 8;
// Dynamic LDS one persistent workgroup needs for a problem's stream tasks.
size_t batch_stream_lds(int D, int variant, size_t tile_lds);
// Kernel variants the persistent kernel runs: one-wavefront 4 x 8 tiles
// (single-buffered) and 4 x 1 and 2 x 2 shared tiles.  The double-buffered
// and 8-column tiles need more registers than the kernel's other paths, and
// inlined into its one function they made it spill (1468 VGPRs with the
// double-buffered form; without it the launch was 7% faster).
inline bool batch_variant_ok(int variant) {
    return variant == 1 || variant == 4 || variant == 5;
}

// ---- launchers (oos.hip) ---------------------------------------------
struct OOSArgs {
    const float *Xs;      // in-sample configuration, SoA [m][D][npad_in]
    int m, n, npad, D;
    const float *dnew;    // k x m x n
    int k;
    float *Y;             // k x m x d (AoS, the ABI layout)
    const double *Linv;   // m x m
    const double *wmat;   // m x m
    const double *target; // optional k
    double *stress_out;   // optional k
    int *iters_out;       // optional k
    double tol;
    int iters;
    int ob;               // objects per workgroup, 1..4 (0: the default, four)
    int vec4;             // 1: n % 4 == 0 and dnew 16-byte aligned (16-byte loads)
};
// colsum: workspace of m * D doubles (sum_j X^(i)_j, computed first).
hipError_t launch_oos(const OOSArgs &a, double *colsum, hipStream_t s);
// Y[o][i] = X row i*n + argmin_j delta_new[o][i][j] (X in the ABI layout).
hipError_t launch_nearest(const float *X, int m, int n, int d, const float *dnew, int k,
                          float *Y, hipStream_t s);

// ---- classical MDS initialisation (cmds.hip) --------------------------
// (A o A) V for up to GR_MAXP problems of one launch: the mean of all m
// Delta_i and/or a group of modalities.  Each workgroup takes GR_ROWS rows
// and the cpw columns of one split (its wavefronts interleaving 32-column
// steps); results go to part[split][p][row][16]
// (nrow_pad = nrowblk GR_ROWS rows, 16 columns of which the first K are
// meaningful), summed over the splits by launch_gram_combine.
constexpr int GR_RB = 4;                // 16-row MFMA blocks per wavefront
constexpr int GR_ROWS = 16 * GR_RB;
constexpr int GR_CHUNK = 32;            // columns per step of a wavefront
constexpr int GR_MAXP = 5;
struct GramArgs {
    DeltaPtrs dp;                 // all m matrices (n x n row-major)
    int nsrc;                     // m: the mean's sources
    int i0;                       // first modality of the launch's group
    int n, npad;                  // npad: row length of Vt (multiple of 32, >= n)
    float scale;                  // 1 / m
    const float *Vt[GR_MAXP];     // per problem of the launch: V^T, [16][npad], zero-padded
    float *part;
    int pbase, ptotal;            // first global problem index; problems of the run
    int nrowblk, splits, cpw, nrow_pad;
};
// Workgroup grid of an n x n product: row blocks, column splits and
// columns per split (a multiple of GR_CHUNK).
void gram_plan(int n, int &nrowblk, int &splits, int &cpw);
// G modalities i0..i0+G-1 (G <= 4) and, with mean, the mean first (then
// G == 0, or G == nsrc: the launch holds every modality).
hipError_t launch_gram(const GramArgs &a, int G, bool mean, hipStream_t s);
// W_p (n x K row-major, p-th at W + p wstride) = sum over splits of part.
hipError_t launch_gram_combine(const float *part, int splits, int np, int nrow_pad, int n, int K,
                               float *W, size_t wstride, hipStream_t s);
// For each of np problems: out_p (ka x kb, FP64, at out + p so) = A_p^T B_p
// over n rows (A_p = A + p sa, B_p = B + p sb; B == nullptr: column sums).
hipError_t launch_cross(const float *A, int lda, size_t sa, int ka, const float *B, int ldb,
                        size_t sb, int kb, int n, double *out, size_t so, int np,
                        hipStream_t s);
// For each problem p: out_p[j][c] = sum_a (in_p[j][a] - mu_p[a]) M_p[a][c]
// for c < ncol, 0 for ncol <= c < ldo_pad (mu optional); with outT also
// its transpose, [16][npad], zero outside c < ncol, j < n.
struct ApplyArgs {
    const float *in;
    int ldi, nin;
    size_t sin;
    const double *mu;
    size_t smu;
    const double *M;
    size_t sM;
    int ncol, n;
    float *out;
    int ldo, ldo_pad;
    size_t sout;
    float *outT;
    size_t soutT;
    int npad;
};
hipError_t launch_apply(const ApplyArgs &a, int np, hipStream_t s);

// ---- warm-start network (mlp.hip) -------------------------------------
enum { GEMM_HIDDEN = 0, GEMM_LAST = 1, GEMM_BWD = 2, GEMM_STORE = 3 };
struct GemmEpi {
    const float *bias;  // HIDDEN, LAST
    float *outf;        // Z (HIDDEN), output (LAST), g (BWD), C (STORE); row-major, ldc
    uint16_t *outb;     // BF16 GELU(Z) (HIDDEN), BF16 g (BWD); row-major, ldc
    uint16_t *outbT;    // the same BF16 values transposed (column-major, ldt); optional
    const float *Z;     // pre-activations (BWD), row-major, ldc
    long ldc, ldt;
};
// C (M x N) = A (M x K) B (K x N) with both operands stored k-contiguous:
// A(m, k) = A[m lda + k], B(k, n) = Bt[n ldb + k].  BF16 in, FP32 accumulate.
hipError_t launch_gemm(int epi, int M, int N, int K, const uint16_t *A, long lda,
                       const uint16_t *Bt, long ldb, const GemmEpi &e, hipStream_t s);
// out (C x R, ld_out) = transpose of in (R x C, ld_in), BF16.
hipError_t launch_transpose16(const uint16_t *in, long ld_in, int R, int C, uint16_t *out,
                              long ld_out, hipStream_t s);
// GbT (optional): the BF16 gradient transposed (k x B, leading dimension ldt).
// scratch: at least 64 doubles.  accumulate: *loss += the MSE instead of =.
hipError_t launch_mse(const float *out, const float *y, int B, int k, float *G, uint16_t *Gb,
                      uint16_t *GbT, long ldt, double *loss, double *scratch, hipStream_t s,
                      bool accumulate = false);
// scratch: at least 16 N doubles.
hipError_t launch_colsum(const float *G, int B, int N, float *db, double *scratch,
                         hipStream_t s);
hipError_t launch_adam(float *p, const float *g, float *m, float *v, uint16_t *p16, long n,
                       float lr, float b1, float b2, float eps, float c1, float c2,
                       hipStream_t s);
hipError_t launch_to_bf16(const float *x, uint16_t *y, long n, hipStream_t s);
// Y (B x m x d) from the network output (B x P): P == d repeats the point
// for every modality, P == m d copies.
hipError_t launch_broadcast(const float *out, int B, int m, int d, int P, float *Y,
                            hipStream_t s);
hipError_t launch_features(const float *dnew, int k, int m, int n, const int *lm, int L,
                           const float *mu, const float *isd, uint16_t *x, hipStream_t s);

// Per-feature mean (mu) and 1 / max(sample SD, min_sd) (inv_sd) of an
// N x F FP32 matrix; scratch: colstats_scratch_doubles(F) doubles.
hipError_t launch_colstats(const float *raw, long N, int F, double min_sd, float *mu,
                           float *inv_sd, double *scratch, hipStream_t s);
size_t colstats_scratch_doubles(int F);
// out (k x d) = mean over the m points of each object in Y (k x m x d).
hipError_t launch_consensus(const float *Y, int k, int m, int d, float *out, hipStream_t s);

// ---- input validation (validate.hip) ----------------------------------
// Smallest ((row-major index) << 3 | offence) over the offending entries
// of an n x n dissimilarity matrix (offences: 1 NaN, 2 infinite, 3
// negative, 4 asymmetric (reported at the upper-triangle entry), 5 non-zero
// diagonal), atomically min-ed into *first (~0 when none; `reset` sets it
// to ~0 first).
hipError_t launch_validate_square(const float *delta, int n, unsigned long long *first,
                                  bool reset, hipStream_t s);
// The same over `count` consecutive dissimilarities (offences 1-3 only).
hipError_t launch_validate_rows(const float *d, long long count, unsigned long long *first,
                                bool reset, hipStream_t s);

// Records the calling thread's error message (host.cpp); returns `code`.
int set_error(int code, const char *fmt, ...);
// Kinds of timed work of the per-kernel profile (fjofc_profile_*).
enum ProfKind { K_STREAM = 0, K_EDGE, K_FIN, K_RED, K_OOS, K_BATCH, K_INIT, K_KINDS };
// Brackets what is enqueued on s during its lifetime with HIP events when
// the context's profiling is on (host.cpp).
struct Timed {
    fjofc_ctx *c;
    int kind;
    double bytes;
    hipStream_t s;
    hipEvent_t a = nullptr;
    Timed(fjofc_ctx *c_, int kind_, double bytes_, hipStream_t s_);
    ~Timed();
};
// Context services for entry points outside host.cpp: its device, its
// device workspace (grown to at least `bytes`; contents not preserved) and
// its pinned host staging buffer.
int ctx_device(const fjofc_ctx *ctx);
int ctx_workspace(fjofc_ctx *ctx, size_t bytes, void **ws);
int ctx_pinned(fjofc_ctx *ctx, size_t bytes, void **p);

}  // namespace fjofc
