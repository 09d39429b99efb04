/*
 * fjofc.h — C ABI of the MI355X (gfx950) fast-JOFC library.
 *
 * Fast JOFC (Lyzinski, Park, Priebe, Trosset: "Fast Embedding for JOFC
 * Using the Raw Stress Criterion") embeds m matched n x n dissimilarity
 * matrices Delta_1..Delta_m in R^d by minimising the JOFC raw stress
 * (eq. stress) with successive Guttman transforms, applying the
 * pseudo-inverse of the omnibus Laplacian through its exact structured
 * form (Section 2.1 and Appendix A: L^dagger = W^-1 (x) I_n + Z (x) J_n,
 * whose J_n part drops out because 1^T B(X) = 0), so that one transform is
 *     X_t^(j) = sum_l [W^-1]_{jl} B_l(X^(l)) X^(l)        (eq:update)
 * with W the m x m matrix of eq:modW.  Out-of-sample embedding of new
 * objects against a fixed configuration (Section 3) is the second entry
 * point.
 *
 * Conventions for every call:
 *  - Integer return codes (FJOFC_OK = 0); nothing is thrown across the ABI.
 *    fjofc_last_error() gives a message for the calling thread's last
 *    failure.
 *  - "device" pointers are HIP device memory on the context's device,
 *    owned by the caller; the library never frees them.  "host" pointers
 *    are ordinary host memory.
 *  - All GPU work is enqueued on `stream` (a hipStream_t, NULL = default
 *    stream).  Calls that return host results synchronise that stream
 *    before returning.
 *  - Weights: `wmat` is the m x m FP64 row-major matrix of eq:W2:
 *    wmat[i*m+i] = w_ii > 0 is modality i's fidelity weight (Theorem 1
 *    needs w_ii > 0); wmat[i*m+k] = w_ik = w_ki >= 0 is the
 *    commensurability weight between modalities i and k.  The uniform case
 *    of eq:W is w_ii = 1, w_ik = w.  Arbitrary mn x mn weights are not
 *    accepted: the structured inverse needs the eq:W2 structure.
 *  - Dissimilarities are FP32, n x n row-major, symmetric with zero
 *    diagonal (the library reads only the strict upper triangle j < l).
 *  - Configurations are FP32 row-major: X is (m*n) x d, modality-major
 *    (rows i*n .. i*n+n-1 hold X^(i), Section 1.2.1).
 *
 * Tuning overrides (environment variables, read when a problem is planned
 * or launched; none changes what is computed beyond FP32 summation order):
 *  - FJOFC_TUNE_TABLE  path of the stream tile cache (default:
 *                      tune_cache.txt next to the library), read once per
 *                      process: lines "arch d n_max tile_height variant";
 *                      only the device architecture's rows apply, and a d
 *                      with no rows uses those of the nearest tabulated d;
 *  - FJOFC_TILE        "th:variant" forces the in-sample tile height and
 *                      kernel variant (the height is rounded up to whole
 *                      8-row groups per wavefront); a comma-separated list
 *                      of "d:n_lo:n_hi:th:variant" forces it only for the
 *                      problems of that d with n_lo <= n <= n_hi (the
 *                      autotuner's per-bucket candidates).  Variants: 0 one
 *                      wavefront, 4 columns per lane, 8-row groups,
 *                      double-buffered loads; 1 the same, single-buffered;
 *                      2 and 3 one wavefront, 8 columns per lane, 4- and
 *                      8-row groups; 4 and 5 variant 1's wavefronts 4 x 1
 *                      and 2 x 2 per tile (tile width 256, 256, 512, 512,
 *                      256 and 512 columns);
 *  - FJOFC_OOS_OB      1..4 objects per out-of-sample workgroup (default 4);
 *  - FJOFC_OOS_SCALAR  any value: the out-of-sample stream uses 4-byte
 *                      loads even when n % 4 == 0;
 *  - FJOFC_GEMM_WAVES  the form of the network's matrix products: "1" one
 *                      wavefront per 32 x 32 tile, "4" 2 x 2 wavefronts per
 *                      64 x 64 tile, "k" four wavefronts splitting K per
 *                      32 x 32 tile (default: by product size).
 * Debug switch:
 *  - FJOFC_VALIDATE    any value but "0": every in-sample call (fjofc_embed*,
 *                      fjofc_stress, fjofc_batch_create) first runs
 *                      fjofc_validate_delta on each Delta_i, and fjofc_oos
 *                      checks that delta_new is finite and non-negative;
 *                      an offending entry makes the call return
 *                      FJOFC_EINVAL (naming the entry) before any other work.
 */
#ifndef FJOFC_H
#define FJOFC_H

#ifdef __cplusplus
extern "C" {
#endif

enum {
    FJOFC_OK = 0,
    FJOFC_EINVAL = 1,   /* invalid argument (shape, weight, pointer)       */
    FJOFC_EHIP = 2,     /* a HIP runtime call failed                       */
    FJOFC_ENOMEM = 3,   /* device or host allocation failed                */
    FJOFC_ESINGULAR = 4 /* the eq:modW matrix is singular                   */
};

/* Stop-rule modes of fjofc_embed (Algorithm 2's loop; the printed loop test
 * has its sign reversed — the run continues while stress keeps decreasing):
 * every `stress_every` transforms the raw stress sigma(X_t) is compared with
 * the previous checkpoint's sigma_prev and the run stops, returning X_t,
 * when sigma_prev - sigma(X_t) < threshold.                                */
enum {
    FJOFC_TOL_NONE = 0, /* run exactly `iters` transforms                  */
    FJOFC_TOL_REL = 1,  /* threshold = tol * sigma_prev                    */
    FJOFC_TOL_PAPER = 2, /* threshold = tol * C(mn, 2): the normalised
                           stress sigma / C(mn,2) failed to decrease by
                           tol (the paper's experiments use tol = 1e-6)    */
    FJOFC_TOL_TARGET = 3 /* not a decrease test: stop at the first checkpoint
                           (t = 0 included) whose sigma(X_t) <= tol, for
                           measuring the time to reach a given stress      */
};

#define FJOFC_MAX_M 32  /* modalities per problem                        */
#define FJOFC_MAX_D 8   /* embedding dimension                           */

typedef struct fjofc_ctx fjofc_ctx;

typedef struct {
    int iters_run;       /* Guttman transforms applied to X0              */
    int converged;       /* 1 if the stop rule fired                      */
    double stress;       /* raw stress sigma of the returned X (FP64)     */
    double stress_norm;  /* sigma / C(mn, 2)                               */
    double fidelity;     /* sum_i w_ii sum_{j<l} (Delta_i[j,l] - d_jl)^2   */
    double commens;      /* sum_{i<k} w_ik sum_l ||X^(i)_l - X^(k)_l||^2   */
} fjofc_result;

/* Create a context bound to HIP device `device` (it owns the workspace,
 * kernel-tile tables and error state).  *out receives the handle.         */
int fjofc_create(fjofc_ctx **out, int device);
void fjofc_destroy(fjofc_ctx *ctx);

/* Thread-local message of the last failing call ("" if none).            */
const char *fjofc_last_error(void);
const char *fjofc_strerror(int code);

/*
 * In-sample fJOFC (Algorithm 2 from a given start; Sections 2.1-2.3).
 *   delta        host array of m device pointers, each an n x n FP32
 *                dissimilarity Delta_i (row-major, symmetric, zero diag).
 *   m, n, d      1 <= m <= FJOFC_MAX_M, n >= 2, 1 <= d <= FJOFC_MAX_D.
 *   wmat         host m x m FP64 eq:W2 weights (see conventions).
 *   X            device (m*n) x d FP32: X0 on entry, the returned X_t on
 *                exit.
 *   iters        maximum number of Guttman transforms (>= 0).
 *   tol,tol_mode stop rule (FJOFC_TOL_*); ignored when tol <= 0.
 *   stress_every stress is evaluated at t = 0, every stress_every
 *                transforms, and for the returned X (>= 1).
 *   stress_hist  optional host array of iters+1 doubles: sigma(X_t) where
 *                evaluated, NaN elsewhere.
 *   res          host result (required).
 * Each transform streams every Delta_i once (strict upper triangle only),
 * forming B_i(X^(i)) X^(i) from the pairwise distances (eq:B, with the
 * d_jl = 0 => 0 rule), then applies W^-1 (eq:update).  Returns after the
 * stream has been synchronised.                                           */
int fjofc_embed(fjofc_ctx *ctx, const float *const *delta, int m, int n,
                const double *wmat, int d, float *X, int iters, double tol,
                int tol_mode, int stress_every, double *stress_hist,
                fjofc_result *res, void *stream);

/*
 * Relaxed Guttman transforms, the acceleration of the linear convergence
 * that the Conclusion proposes (relaxed updates of iterative majorization):
 *     X_{t+1} = X_t + alpha (Gamma(X_t) - X_t),     0 < alpha < 2,
 * Gamma being the transform of fjofc_embed (eq:update).  For fixed X_t the
 * majorizing function of eq:major is a convex quadratic in X minimised at
 * Gamma(X_t); along this line it is symmetric about alpha = 1, so for every
 * alpha in (0, 2) it is at most its value at X_t, sigma(X_t), and the raw
 * stress still does not increase.  alpha = 1 is fjofc_embed exactly; other
 * arguments and results as for fjofc_embed.                               */
int fjofc_embed_relaxed(fjofc_ctx *ctx, const float *const *delta, int m,
                        int n, const double *wmat, int d, float *X, int iters,
                        double tol, int tol_mode, int stress_every,
                        double alpha, double *stress_hist, fjofc_result *res,
                        void *stream);

/*
 * The paper's initialisation X_0 for fjofc_embed (Algorithm 2's first
 * lines, with Algorithm 1 step 1's classical MDS):
 *   xi_0 = cMDS of the mean dissimilarity (sum_i Delta_i) / m,
 *   xi_i = cMDS of Delta_i,
 *   X^(i)_0 = xi_i Q_i, Q_i the orthogonal Procrustes rotation of xi_i onto
 *             xi_0 (Q_i maximises tr(Q^T xi_i^T xi_0): the polar factor of
 *             xi_i^T xi_0; the printed U V^T, from the SVD of xi_0^T xi_i,
 *             is its transpose).
 * cMDS of A: the d largest eigenpairs (lambda, u) of
 * P = -1/2 (I - J/n)(A o A)(I - J/n); X = [u_1..u_d] diag(max(lambda,0))^(1/2)
 * (centred).  They are computed by `iters` steps of subspace iteration on
 * a block of K >= max(2d, d + 3) vectors per matrix, then Rayleigh-Ritz.
 * The m + 1 iterations step together: for m <= 4 each step reads every
 * Delta_i once (full rows) and forms the mean's and all m per-matrix
 * products from those reads; for m > 4 the mean takes a pass of its own.
 *   delta, m, n, d  as for fjofc_embed (d <= FJOFC_MAX_D).
 *   X               device (m*n) x d FP32, written.
 *   iters           subspace-iteration steps per matrix, 1..10000.
 *   eigvals         optional host (m + 1) x d: the d largest Ritz values of
 *                   P for the mean, then for each Delta_i.
 * Synchronises `stream`.                                                  */
int fjofc_init_cmds(fjofc_ctx *ctx, const float *const *delta, int m, int n,
                    int d, float *X, int iters, double *eigvals, void *stream);

/* Uniform-weight form of fjofc_embed (eq:W: w_ii = 1, w_ik = w >= 0).     */
int fjofc_embed_w(fjofc_ctx *ctx, const float *const *delta, int m, int n,
                  double w, int d, float *X, int iters, double tol,
                  int tol_mode, int stress_every, double *stress_hist,
                  fjofc_result *res, void *stream);

/* Raw stress (eq. stress, eq:W2 weights) of a configuration X (device,
 * (m*n) x d), without changing it.  res->iters_run = 0.                   */
int fjofc_stress(fjofc_ctx *ctx, const float *const *delta, int m, int n,
                 const double *wmat, int d, const float *X,
                 fjofc_result *res, void *stream);

/*
 * Out-of-sample embedding (Section 3) of k new objects against a fixed
 * in-sample configuration.
 *   X_in       device (m*n) x d FP32 in-sample configuration (fixed).
 *   wmat       host m x m eq:W2 weights (as for fjofc_embed).
 *   delta_new  device k x m x n FP32: delta_new[(o*m + i)*n + j] is the
 *              dissimilarity of new object o to in-sample object j in
 *              modality i.
 *   Y          device k x m x d FP32: starts on entry (the paper starts
 *              from a random point), results on exit.  Object o's m points
 *              are rows o*m .. o*m+m-1.
 *   iters      maximum Guttman transforms per object.
 *   tol        per object, stop when its out-of-sample stress (eq:joos)
 *              decreased by less than tol * previous (tol <= 0: never).
 *   target     optional device k FP64: stop object o once its stress is
 *              <= target[o] (checked before every transform).
 *   stress_out optional device k FP64: eq:joos stress of the returned y.
 *   iters_out  optional device k int32: transforms applied per object.
 * New objects carry no weight between one another (their mutual
 * dissimilarities are unknown), so the k problems are independent and
 * share L22 = the eq:modW matrix (its inverse is the printed L22^dagger
 * for uniform weights).  Each transform is, per object and modality i,
 *   r_j = delta_i(j) / ||X^(i)_j - y_i|| (0 when the distance is 0),
 *   xi_i = w_ii sum_j (1 - r_j) X^(i)_j,  psi_i = w_ii sum_j r_j,
 *   y <- L22^-1 (xi + diag(psi) y).
 * The call does not synchronise the stream unless `sync` is non-zero.     */
int fjofc_oos(fjofc_ctx *ctx, const float *X_in, int m, int n, int d,
              const double *wmat, const float *delta_new, int k, float *Y,
              int iters, double tol, const double *target, double *stress_out,
              int *iters_out, int sync, void *stream);

/*
 * Allocation-free form of fjofc_oos, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Arguments, results and kernels are
 * those of fjofc_oos (the results are bitwise equal); the differences:
 *  - its working memory (the SoA copy of X_in, column sums, L22^-1 and the
 *    weights) is a 4 MiB array of device memory that the library holds per
 *    GPU from fjofc_create until the process ends; nothing is allocated,
 *    and m x m matrices reach the device as a kernel argument;
 *  - limits: m <= 8 and 4 (m d npad) + 8 (m d + 2 m^2) bytes (each piece
 *    rounded up to 256) <= 4 MiB, npad = n rounded up to 256 (e.g. m = 2,
 *    d = 5, n <= about 104000); larger problems return FJOFC_EINVAL;
 *  - every call on one GPU shares that GPU's array: calls that overlap in
 *    time on one GPU (other streams, other threads) race and must be
 *    serialised by the caller; each call rewrites all it reads;
 *  - no profiling records and no FJOFC_VALIDATE pass.
 */
int fjofc_oos_noalloc(fjofc_ctx *ctx, const float *X_in, int m, int n, int d,
                      const double *wmat, const float *delta_new, int k, float *Y,
                      int iters, double tol, const double *target, double *stress_out,
                      int *iters_out, int sync, void *stream);

/*
 * Nearest-in-sample start for fjofc_oos (a comparison start; the paper
 * starts from a random point): Y[o][i] = row i*n + j* of X_in, j* being the
 * smallest index minimising delta_new[o][i][j] over j.  Arrays as for
 * fjofc_oos; does not synchronise the stream.
 */
int fjofc_oos_nearest_start(fjofc_ctx *ctx, const float *X_in, int m, int n,
                            int d, const float *delta_new, int k, float *Y,
                            void *stream);

/*
 * Batched in-sample fJOFC: many independent problems of different m, n, d
 * advanced together (in lockstep launches, or in one persistent launch:
 * fjofc_batch_set_launch), the whole loop captured once into a HIP graph on
 * a library-owned stream and replayed.  Each problem keeps its own
 * stop rule (a stopped problem's tiles become no-ops).  Tile shapes come
 * from the autotuned table, per (d, n).
 */
typedef struct {
    int m, n, d;                /* as for fjofc_embed                        */
    const float *const *delta;  /* host array of m device pointers           */
    const double *wmat;         /* host m x m eq:W2 weights                  */
    float *X;                   /* device (m*n) x d: X0 in, result out       */
} fjofc_problem;

typedef struct fjofc_batch fjofc_batch;

/* Plan a batch: validate every problem, build tile lists and W^-1, allocate
 * the batch workspace (device memory owned by the plan).  The pointers in
 * probs must stay valid for the plan's lifetime; delta and wmat contents
 * are read at each run, wmat at creation.                                  */
int fjofc_batch_create(fjofc_ctx *ctx, const fjofc_problem *probs, int count,
                       fjofc_batch **out);
/* Run `iters` transforms of every problem (the first call with a given
 * (iters, tol, tol_mode, stress_every) captures the graph; later calls
 * replay it).  The run is ordered after prior work on `stream` and later
 * work on `stream` waits for it.  res (host, count results) is optional;
 * when given the call synchronises `stream`.                               */
int fjofc_batch_run(fjofc_batch *b, int iters, double tol, int tol_mode,
                    int stress_every, fjofc_result *res, void *stream);
/* The in-sample stream tile the library plans for an (n, d) problem on
 * ctx's device: tile height (rows, after rounding to whole row groups) and
 * kernel variant, from FJOFC_TILE, the tuning cache or the default.  Lets
 * a caller check which cache row applies.  FJOFC_EINVAL for n < 2 or d
 * outside [1, FJOFC_MAX_D] or NULL outputs.                                */
int fjofc_tile_choice(fjofc_ctx *ctx, int n, int d, int *tile_height, int *variant);

/* How fjofc_batch_run advances the batch (the paper's parallel structure,
 * Remarks rem:pargut and rem:parfjofc: the tiles of every problem and
 * transform are independent given the current configurations).
 *   FJOFC_LAUNCH_LOCKSTEP (the default): per transform one stream launch per
 *     kernel variant and one reduce/finalize launch per group, in one graph.
 *   FJOFC_LAUNCH_PERSISTENT: one persistent launch per run (in the graph),
 *     workgroups pulling (problem, transform, tile group / reduce /
 *     finalize group) tasks from a device queue and waiting, bounded, on
 *     per-problem progress counters; the grid is the co-resident workgroup
 *     count.  A wait that times out (5000 ms of wall clock by default,
 *     FJOFC_BATCH_TIMEOUT_MS) ends the launch and the run returns
 *     FJOFC_EHIP.  Both launches run the same tiles and sums: results are
 *     bitwise equal.
 * Returns FJOFC_EINVAL for an unknown value, or for the persistent launch
 * when a problem's tile has no persistent form (the persistent kernel runs
 * the single-buffered 4-column one-wavefront tile and the 4 x 1 and 2 x 2
 * shared tiles, variants 1, 4 and 5 of FJOFC_TILE; not the double-buffered
 * variant 0 or the 8-column variants 2 and 3).  A change of launch discards
 * the captured graph (the next run captures again).                       */
#define FJOFC_LAUNCH_LOCKSTEP 0
#define FJOFC_LAUNCH_PERSISTENT 1
int fjofc_batch_set_launch(fjofc_batch *b, int launch);
void fjofc_batch_destroy(fjofc_batch *b);
/* create + run + destroy.                                                  */
int fjofc_embed_batched(fjofc_ctx *ctx, const fjofc_problem *probs, int count,
                        int iters, double tol, int tol_mode, int stress_every,
                        fjofc_result *res, void *stream);

/*
 * Learned warm start for out-of-sample embedding: a multilayer perceptron
 * mapping a new object's dissimilarities to a fixed set of in-sample
 * landmark objects (all modalities) to a starting point for the Section 3
 * iteration, refined there by Guttman transforms (which also measure its
 * error).
 * Layers l = 0..L-1: z = h W_l + b_l (W_l is dims[l] x dims[l+1],
 * row-major), h' = GELU(z) = z Phi(z) after every layer but the last.
 * Products run on BF16 matrix cores with FP32 accumulation: FP32 master
 * weights with BF16 copies; activations and the backward gradients used as
 * product operands are BF16 (round to nearest even); everything else FP32.
 * Loss: mean squared error.  Optimiser: Adam with bias correction.
 * All array arguments are device memory; calls enqueue on `stream`.
 */
typedef struct fjofc_mlp fjofc_mlp;

/* dims: L + 1 widths; max_batch: rows per call.  On the current device.   */
int fjofc_mlp_create(fjofc_ctx *ctx, int L, const int *dims, int max_batch,
                     fjofc_mlp **out);
void fjofc_mlp_destroy(fjofc_mlp *net);
/* Copy FP32 parameters in (W[l], b[l] device arrays); resets Adam.         */
int fjofc_mlp_set_params(fjofc_mlp *net, const float *const *W,
                         const float *const *b, void *stream);
int fjofc_mlp_get_params(fjofc_mlp *net, float *const *W, float *const *b,
                         void *stream);
/* out (B x dims[L] FP32) = network(x), x: B x dims[0] BF16 (uint16 bits). */
int fjofc_mlp_forward(fjofc_mlp *net, const unsigned short *x, int B,
                      float *out, void *stream);
/* Warm start for fjofc_oos: Y is B x m x d FP32.  A network with
 * dims[L] == d gives one point that all m modalities start from; dims[L] ==
 * m*d gives one point per modality (row-major m x d).  Any other width is
 * FJOFC_EINVAL.                                                           */
int fjofc_mlp_predict_start(fjofc_mlp *net, const unsigned short *x, int B,
                            int m, int d, float *Y, void *stream);
/* Forward, MSE against y (B x dims[L] FP32), backward: the gradients are
 * kept in the network (fjofc_mlp_get_grads); loss (optional, FP64).      */
int fjofc_mlp_backward(fjofc_mlp *net, const unsigned short *x, const float *y,
                       int B, double *loss, void *stream);
int fjofc_mlp_get_grads(fjofc_mlp *net, float *const *dW, float *const *db,
                        void *stream);
/* One Adam step with the stored gradients (FP32 masters, BF16 refreshed). */
int fjofc_mlp_adam(fjofc_mlp *net, float lr, float beta1, float beta2,
                   float eps, void *stream);
/* `steps` training steps in one call: step q runs fjofc_mlp_backward on rows
 * [q B, (q + 1) B) of x (N x dims[0] BF16) and y (N x dims[L] FP32), then
 * fjofc_mlp_adam with learning rate lr[q] (host array of `steps` values)
 * and beta1, beta2, eps.  The same kernels in the same order as those calls,
 * so the parameters come out bitwise the same; each step's MSE is added to
 * *loss_sum (device FP64, optional).  FJOFC_EINVAL if steps B > N, B is
 * outside [1, max_batch], a learning rate is negative or NaN, or the Adam
 * constants are out of range.  Lets a training loop run without a host
 * call per step.                                                           */
int fjofc_mlp_train_steps(fjofc_mlp *net, const unsigned short *x, const float *y,
                          int N, int B, int steps, const float *lr, float beta1,
                          float beta2, float eps, double *loss_sum, void *stream);
/* Features of k new objects: x[o][i*L + l] = BF16((delta_new[o][i][lm[l]]
 * - mu[i*L + l]) * inv_sd[i*L + l]); delta_new is k x m x n FP32 (as for
 * fjofc_oos), landmarks L int32 indices in [0, n) (clamped).              */
int fjofc_mlp_features(fjofc_ctx *ctx, const float *delta_new, int k, int m,
                       int n, const int *landmarks, int L, const float *mu,
                       const float *inv_sd, unsigned short *x, void *stream);

/* Validation loss: out = network(x), *loss (device FP64) = mean squared
 * error against y (B x dims[L] FP32).  The parameter gradients are left
 * as they are.                                                             */
int fjofc_mlp_loss(fjofc_mlp *net, const unsigned short *x, const float *y, int B,
                   double *loss, void *stream);
/* Standardisation statistics of the network's inputs: for an N x F FP32
 * row-major matrix raw (device), mu[f] = mean of column f and inv_sd[f] =
 * 1 / max(sd_f, min_sd), sd_f the sample standard deviation (N - 1 in the
 * denominator; 0 when N = 1).  FP64 sums in a fixed order (two passes), so
 * results are reproducible.  mu, inv_sd: device F FP32.  Uses the context
 * workspace ((256 + 1) F doubles); does not synchronise.                  */
int fjofc_mlp_feature_stats(fjofc_ctx *ctx, const float *raw, int N, int F, double min_sd,
                            float *mu, float *inv_sd, void *stream);
/* Consensus point of each new object (the target of a network that
 * predicts one point for every modality): out[o][c] = (1/m) sum_i
 * Y[o][i][c], Y device k x m x d FP32 (as for fjofc_oos), out device k x d.
 */
int fjofc_oos_consensus(fjofc_ctx *ctx, const float *Y, int k, int m, int d, float *out,
                        void *stream);

/*
 * Validation pass over one dissimilarity matrix (a debug check; the
 * computing calls trust their inputs unless FJOFC_VALIDATE is set).  The
 * method takes Delta in R_+^{n x n} (Section 1) to be a dissimilarity: every
 * entry finite and >= 0, Delta symmetric with a zero diagonal.  The stream
 * reads only the strict upper triangle and the fidelity term of the raw
 * stress counts each pair once (Remark faststress), so a matrix breaking
 * these rules would give results that silently depend on the triangle read.
 *   delta  device n x n FP32 row-major (1 <= n <= 4194240).
 *   where  optional host: the row-major index i n + j of the first offending
 *          entry (the smallest such index; an asymmetric pair is reported at
 *          its upper-triangle entry), -1 when the matrix is valid.
 * Returns FJOFC_OK, or FJOFC_EINVAL with a message naming (i, j) and the
 * rule broken (NaN, infinite, negative, asymmetric, non-zero diagonal).
 * Reads the matrix once through LDS tiles; synchronises `stream`.  Bad
 * values are only compared, never used in arithmetic that could fault.    */
int fjofc_validate_delta(fjofc_ctx *ctx, const float *delta, int n, long long *where,
                         void *stream);

/*
 * Per-kernel timing (tracing aid).  While enabled, every kernel launch of
 * fjofc_embed / fjofc_stress / fjofc_oos (and each product pass of
 * fjofc_init_cmds) is bracketed by HIP events on the caller's stream; fjofc_profile_read synchronises and returns the summed
 * durations per kernel kind together with the algorithmic bytes the
 * in-sample stream launches read (4 bytes per unordered pair of every
 * dissimilarity block, i.e. one read of each strict-upper-triangle entry)
 * and that the out-of-sample launches read (4 bytes per
 * object x modality x in-sample object x transform).  Enabling resets the
 * counters.
 */
typedef struct {
    int stream_launches;     /* in-sample stream forming B(X)X (every tile) */
    double stream_ms;
    double stream_bytes;
    int edge_launches;       /* in-sample stress-only stream (returned X)  */
    double edge_ms;
    double edge_bytes;
    int finalize_launches;   /* W^-1 combine and new X                     */
    double finalize_ms;
    int reduce_launches;     /* FP64 stress reduction and stop test        */
    double reduce_ms;
    int oos_launches;        /* out-of-sample kernel                       */
    double oos_ms;
    double oos_bytes;
    int batch_launches;      /* whole batched graph replays                */
    double batch_ms;
    double batch_bytes;      /* 4 B per pair per transform, all problems   */
    int init_launches;       /* fjofc_init_cmds product passes             */
    double init_ms;
    double init_bytes;       /* 4 B per entry of every Delta_i read        */
} fjofc_profile;

int fjofc_profile_enable(fjofc_ctx *ctx, int on);
int fjofc_profile_read(fjofc_ctx *ctx, fjofc_profile *out);

#ifdef __cplusplus
}
#endif
#endif /* FJOFC_H */
