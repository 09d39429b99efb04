// Internal declarations shared by the fast-JOFC HIP kernels and the host
// library.  Not part of the public ABI (include/fjofc.h is).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

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
// Tiles are th rows x tw columns (tw = 64 lanes x cpl columns per lane);
// tile (I, J) covers rows [I th, I th + th) and columns [J tw, J tw + tw)
// and exists when it holds at least one pair j < l inside n.
struct TriGeom {
    int n;          // objects
    int m;          // modalities
    int npad;       // row pitch of SoA buffers (multiple of th and tw)
    int th, tw;     // tile height and width
    int cpl;        // columns per lane (4 or 8)
    int variant;    // stream-kernel variant: (cpl, rows per group, buffering)
    int ntr, ntc;   // row / column blocks
    int nint;       // interior tiles per modality (no masking needed)
    int nbnd;       // boundary tiles per modality (diagonal or ragged)
    int vec4;       // 1: rows are 16-byte aligned (n % 4 == 0)
};

__host__ __device__ inline bool tile_exists(const TriGeom &g, int I, int J) {
    const int cmax = min((J + 1) * g.tw, g.n) - 1;
    return cmax > I * g.th;
}

// Partial sums produced by the stream, FP32, layout [m][S][D][npad] with
// S = ntc + ntr slots: slot J holds row sums of tile (I, J) for the rows of
// block I, slot ntc + I holds column sums of tile (I, J) for the columns of
// block J.
inline size_t partial_floats(const TriGeom &g, int D) {
    return (size_t)g.m * (g.ntc + g.ntr) * D * g.npad;
}

// ---- launchers (insample.hip) ----------------------------------------
// tiles: nint interior tiles then nbnd boundary tiles (I << 16 | J);
// F: per-tile fidelity, [m][nint + nbnd].  One launch covers every tile.
hipError_t launch_bx(const TriGeom &g, int D, const DeltaPtrs &dp,
                     const float *Xs, const uint32_t *tiles, float *P,
                     double *F, const EmbedState *st, bool stress, bool acc,
                     hipStream_t s);
hipError_t launch_finalize(const TriGeom &g, int D, const float *P,
                           const double *Winv, const double *wmat,
                           float *Xout, double *comP, int ncomblk,
                           const EmbedState *st, bool want_com,
                           hipStream_t s);
int finalize_blocks(const TriGeom &g, int D);
hipError_t launch_com(const TriGeom &g, int D, const float *Xs,
                      const double *wmat, double *comP, int ncomblk,
                      hipStream_t s);
hipError_t launch_reduce(const TriGeom &g, const double *F,
                         const double *wmat, const double *comP, int ncomblk,
                         EmbedState *st, double *hist, int t, int check,
                         int final_pass, int iters, double tol, int tol_mode,
                         hipStream_t s);
hipError_t launch_init_state(EmbedState *st, double *hist, int nhist,
                             hipStream_t s);
hipError_t launch_to_soa(const TriGeom &g, int D, const float *X, float *Xs,
                         hipStream_t s);
hipError_t launch_from_soa(const TriGeom &g, int D, const float *Xa,
                           const float *Xb, const EmbedState *st, float *X,
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
};
// colsum: workspace of m * D doubles (sum_j X^(i)_j, computed first).
hipError_t launch_oos(const OOSArgs &a, double *colsum, hipStream_t s);

}  // namespace fjofc
