// Internal declarations shared by the fast-JOFC HIP kernels and the host
// library.  Not part of the public ABI (include/fjofc.h is).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

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

// ---- launchers (insample.hip) ----------------------------------------
// Stream kernels for one (D, variant, vec4) group of items; `cur` selects
// the configuration buffer Xs[cur].
hipError_t launch_stream(int D, int variant, int vec4, const InstDesc *insts,
                         const StreamItem *items, int nitems, int cur,
                         bool stress, bool acc, size_t lds, hipStream_t s);
hipError_t launch_finalize(int maxm, const InstDesc *insts, const RowItem *rows,
                           int nrows, int cur, bool want_com, hipStream_t s);
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
// W (n x K) = (A o A) V with A = scale * sum of the nsrc matrices in dp
// (n x n row-major); V, W row-major with K in {4, 8, 12, 16} columns.
hipError_t launch_sqprod(const DeltaPtrs &dp, int nsrc, float scale, int n, int K,
                         const float *V, float *W, hipStream_t s);
// out (ka x kb, FP64) = A^T B over n rows (B == nullptr: column sums of A).
hipError_t launch_cross(const float *A, int lda, int ka, const float *B, int ldb, int kb, int n,
                        double *out, hipStream_t s);
// out[j][c] = sum_a (in[j][a] - mu[a]) M[a][c] for c < ncol, 0 for
// ncol <= c < ldo_pad; mu optional.
hipError_t launch_apply(const float *in, int ldi, int nin, const double *mu, const double *M,
                        int ncol, int n, float *out, int ldo, int ldo_pad, hipStream_t s);

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
// scratch: at least 64 doubles.
hipError_t launch_mse(const float *out, const float *y, int B, int k, float *G, uint16_t *Gb,
                      uint16_t *GbT, long ldt, double *loss, double *scratch, hipStream_t s);
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
// Context services for entry points outside host.cpp: its device, its
// device workspace (grown to at least `bytes`; contents not preserved) and
// its pinned host staging buffer.
int ctx_device(const fjofc_ctx *ctx);
int ctx_workspace(fjofc_ctx *ctx, size_t bytes, void **ws);
int ctx_pinned(fjofc_ctx *ctx, size_t bytes, void **p);

}  // namespace fjofc
