/*
 * Plain FP64 CPU oracle of fast JOFC (Lyzinski, Park, Priebe, Trosset,
 * "Fast Embedding for JOFC Using the Raw Stress Criterion").
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg may load this file's library.  It shares no
 * code with the GPU path and is deliberately simple: every quantity is
 * computed from its definition in the paper, in double precision, with no
 * blocking or fusion.  Dissimilarities arrive as FP32 (the same values the
 * GPU reads) and are promoted to FP64 when read.
 *
 * Notation (Section 1.2.1): m modalities, n objects, d dimensions.
 * X is (m n) x d, row-major, modality-major: block i holds X^(i) (n x d).
 * wmat is the m x m weight matrix of eq:W2 (w_ii fidelity, w_ij = w_ji
 * commensurability).  delta is m consecutive n x n row-major blocks.
 */
#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

/* Threads of the parallel loops below (for timing).  Only the fidelity
 * sum is an OpenMP reduction, so the thread count changes at most the
 * FP64 rounding of that sum. */
void orc_set_threads(int t) { omp_set_num_threads(t > 0 ? t : 1); }
int orc_get_threads(void) { return omp_get_max_threads(); }

#define IDX(i, j, ld) ((size_t)(i) * (size_t)(ld) + (size_t)(j))

/* ------------------------------------------------------------------ */
/* eq:modW: the m x m matrix whose inverse is the I_n part of L^dagger  */
/* diagonal n*w_ii + sum_{j!=i} w_ij, off-diagonal -w_ij.              */
/* ------------------------------------------------------------------ */
int orc_wmod(int m, int n, const double *wmat, double *W)
{
    for (int i = 0; i < m; ++i) {
        double off = 0.0;
        for (int j = 0; j < m; ++j)
            if (j != i) off += wmat[IDX(i, j, m)];
        for (int j = 0; j < m; ++j)
            W[IDX(i, j, m)] = (i == j) ? n * wmat[IDX(i, i, m)] + off
                                       : -wmat[IDX(i, j, m)];
    }
    return 0;
}

/* Gauss-Jordan inverse with partial pivoting.  Returns 1 if singular. */
int orc_inverse(int m, const double *A, double *Ainv)
{
    double *a = (double *)malloc(sizeof(double) * (size_t)m * 2 * m);
    if (!a) return 2;
    int w2 = 2 * m;
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < w2; ++j)
            a[IDX(i, j, w2)] = (j < m) ? A[IDX(i, j, m)] : (j - m == i ? 1.0 : 0.0);
    for (int c = 0; c < m; ++c) {
        int p = c;
        for (int r = c + 1; r < m; ++r)
            if (fabs(a[IDX(r, c, w2)]) > fabs(a[IDX(p, c, w2)])) p = r;
        if (a[IDX(p, c, w2)] == 0.0) { free(a); return 1; }
        if (p != c)
            for (int j = 0; j < w2; ++j) {
                double t = a[IDX(c, j, w2)];
                a[IDX(c, j, w2)] = a[IDX(p, j, w2)];
                a[IDX(p, j, w2)] = t;
            }
        double piv = a[IDX(c, c, w2)];
        for (int j = 0; j < w2; ++j) a[IDX(c, j, w2)] /= piv;
        for (int r = 0; r < m; ++r) {
            if (r == c) continue;
            double f = a[IDX(r, c, w2)];
            if (f == 0.0) continue;
            for (int j = 0; j < w2; ++j) a[IDX(r, j, w2)] -= f * a[IDX(c, j, w2)];
        }
    }
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < m; ++j) Ainv[IDX(i, j, m)] = a[IDX(i, j + m, w2)];
    free(a);
    return 0;
}

static double dist(const double *a, const double *b, int d)
{
    double s = 0.0;
    for (int k = 0; k < d; ++k) {
        double t = a[k] - b[k];
        s += t * t;
    }
    return sqrt(s);
}

/* ------------------------------------------------------------------ */
/* eq:B for one diagonal block B_i of B(X), multiplied by X^(i).        */
/* Off-diagonal entry b_jl = -w_ii Delta_jl / d_jl (0 when d_jl = 0);    */
/* diagonal b_jj = -sum_{l != j} b_jl.  Rows [row0, row1) only.          */
/* ------------------------------------------------------------------ */
void orc_block_bx(int n, int d, double wii, const float *delta,
                  const double *X, double *BX, int row0, int row1)
{
#pragma omp parallel for schedule(static)
    for (int j = row0; j < row1; ++j) {
        double *out = BX + IDX(j - row0, 0, d);
        for (int k = 0; k < d; ++k) out[k] = 0.0;
        double diag = 0.0;
        for (int l = 0; l < n; ++l) {
            if (l == j) continue;
            double djl = dist(X + IDX(j, 0, d), X + IDX(l, 0, d), d);
            double b = (djl != 0.0) ? -wii * (double)delta[IDX(j, l, n)] / djl : 0.0;
            diag -= b;
            for (int k = 0; k < d; ++k) out[k] += b * X[IDX(l, k, d)];
        }
        for (int k = 0; k < d; ++k) out[k] += diag * X[IDX(j, k, d)];
    }
}

/* ------------------------------------------------------------------ */
/* One Guttman transform X_t = L^dagger B(X) X through the structured    */
/* form (Section 2.2, eq:update):                                        */
/*   X_t^(j) = sum_l [W^-1]_{jl} B_l X^(l),                              */
/* the J_n part of L^dagger vanishing because 1^T B = 0.                 */
/* ------------------------------------------------------------------ */
int orc_guttman(int m, int n, int d, const float *delta, const double *wmat,
                const double *X, double *Xout)
{
    double *W = (double *)malloc(sizeof(double) * m * m);
    double *Wi = (double *)malloc(sizeof(double) * m * m);
    double *BX = (double *)malloc(sizeof(double) * (size_t)m * n * d);
    if (!W || !Wi || !BX) { free(W); free(Wi); free(BX); return 2; }
    orc_wmod(m, n, wmat, W);
    int rc = orc_inverse(m, W, Wi);
    if (rc == 0) {
        for (int i = 0; i < m; ++i)
            orc_block_bx(n, d, wmat[IDX(i, i, m)], delta + IDX(i, 0, (size_t)n * n),
                         X + IDX(i, 0, (size_t)n * d), BX + IDX(i, 0, (size_t)n * d), 0, n);
        for (int j = 0; j < m; ++j)
            for (int r = 0; r < n; ++r)
                for (int k = 0; k < d; ++k) {
                    double s = 0.0;
                    for (int l = 0; l < m; ++l)
                        s += Wi[IDX(j, l, m)] * BX[IDX((size_t)l * n + r, k, d)];
                    Xout[IDX((size_t)j * n + r, k, d)] = s;
                }
    }
    free(W); free(Wi); free(BX);
    return rc;
}

/* ------------------------------------------------------------------ */
/* Raw stress, eq. (stress) generalised to eq:W2 weights:                */
/*   sigma = sum_i w_ii sum_{j<l} (Delta_i[j,l] - d_jl(X^(i)))^2         */
/*         + sum_{i<k} w_ik sum_l ||X^(i)_l - X^(k)_l||^2                */
/* out[0] = sigma, out[1] = weighted fidelity, out[2] = weighted         */
/* commensurability.                                                     */
/* ------------------------------------------------------------------ */
double orc_fidelity_block(int n, int d, const float *delta, const double *X)
{
    double f = 0.0;
#pragma omp parallel for reduction(+ : f) schedule(dynamic, 16)
    for (int j = 0; j < n; ++j)
        for (int l = j + 1; l < n; ++l) {
            double e = (double)delta[IDX(j, l, n)] - dist(X + IDX(j, 0, d), X + IDX(l, 0, d), d);
            f += e * e;
        }
    return f;
}

double orc_commens_pair(int n, int d, const double *Xi, const double *Xk)
{
    double c = 0.0;
    for (int l = 0; l < n; ++l) {
        double t = dist(Xi + IDX(l, 0, d), Xk + IDX(l, 0, d), d);
        c += t * t;
    }
    return c;
}

int orc_stress(int m, int n, int d, const float *delta, const double *wmat,
               const double *X, double *out)
{
    double fid = 0.0, com = 0.0;
    for (int i = 0; i < m; ++i)
        fid += wmat[IDX(i, i, m)] *
               orc_fidelity_block(n, d, delta + IDX(i, 0, (size_t)n * n), X + IDX(i, 0, (size_t)n * d));
    for (int i = 0; i < m; ++i)
        for (int k = i + 1; k < m; ++k)
            com += wmat[IDX(i, k, m)] *
                   orc_commens_pair(n, d, X + IDX(i, 0, (size_t)n * d), X + IDX(k, 0, (size_t)n * d));
    out[0] = fid + com;
    out[1] = fid;
    out[2] = com;
    return 0;
}

/* ------------------------------------------------------------------ */
/* Algorithm 2's loop (from a given X0), with the stop rule read as:     */
/* every `stress_every` transforms compare sigma(X_t) with the sigma of  */
/* the previous checkpoint; stop (keeping X_t) when it has not decreased */
/* by at least the threshold.  tol_mode 1: threshold tol*sigma_prev      */
/* (relative); tol_mode 2: tol*C(mn,2) (normalised stress, Remark eps).  */
/* tol <= 0 runs exactly `iters` transforms.  hist (optional, iters+1)   */
/* receives sigma at every evaluated t, NaN elsewhere.                   */
/* stats: iters_run, converged, sigma, sigma/C(mn,2), fidelity, commens. */
/* ------------------------------------------------------------------ */
/* Algorithm 2's loop.  alpha = 1: the Guttman transform X <- Gamma(X).    */
/* Otherwise the relaxed update X <- X + alpha (Gamma(X) - X) that the      */
/* Conclusion proposes.  tol_mode 1: stop when sigma_prev - sigma <         */
/* tol sigma_prev; 2: ... < tol C(mn,2); 3: stop when sigma <= tol (a       */
/* stress target, tested at t = 0 too).  The tests run at t = 0, every     */
/* stress_every transforms and at t = iters.                                */
int orc_embed(int m, int n, int d, const float *delta, const double *wmat,
              double *X, int iters, double tol, int tol_mode, int stress_every,
              double alpha, double *hist, double *stats)
{
    size_t sz = (size_t)m * n * d;
    double *Xn = (double *)malloc(sizeof(double) * sz);
    if (!Xn) return 2;
    if (stress_every < 1) stress_every = 1;
    double pairs = 0.5 * (double)m * n * ((double)m * n - 1.0);
    double st[3];
    if (hist)
        for (int t = 0; t <= iters; ++t) hist[t] = NAN;
    orc_stress(m, n, d, delta, wmat, X, st);
    if (hist) hist[0] = st[0];
    double last_ck = st[0];
    int run = 0, conv = 0, rc = 0;
    if (tol_mode == 3 && tol > 0.0 && st[0] <= tol) conv = 1;
    for (int t = 1; t <= iters && !conv; ++t) {
        rc = orc_guttman(m, n, d, delta, wmat, X, Xn);
        if (rc) break;
        if (alpha == 1.0) {
            memcpy(X, Xn, sizeof(double) * sz);
        } else {
            for (size_t q = 0; q < sz; ++q) X[q] = X[q] + alpha * (Xn[q] - X[q]);
        }
        run = t;
        int ck = (t % stress_every) == 0;
        if (ck || t == iters) {
            orc_stress(m, n, d, delta, wmat, X, st);
            if (hist) hist[t] = st[0];
            if (ck && tol > 0.0) {
                if (tol_mode == 3) {
                    if (st[0] <= tol) { conv = 1; break; }
                } else {
                    double thr = (tol_mode == 2) ? tol * pairs : tol * last_ck;
                    if (last_ck - st[0] < thr) { conv = 1; break; }
                }
            }
            if (ck) last_ck = st[0];
        }
    }
    free(Xn);
    if (rc) return rc;
    if (run == 0) orc_stress(m, n, d, delta, wmat, X, st);
    stats[0] = run;
    stats[1] = conv;
    stats[2] = st[0];
    stats[3] = st[0] / pairs;
    stats[4] = st[1];
    stats[5] = st[2];
    return 0;
}

/* ------------------------------------------------------------------ */
/* Out-of-sample embedding (Section 3).  One new object: dissimilarities */
/* delta_i (n values per modality, m x n row-major) to the fixed         */
/* in-sample configuration X; its m points y (m x d).                    */
/*                                                                       */
/* Out-of-sample stress, eq:joos with eq:W2 weights:                     */
/*   sum_i w_ii sum_j (delta_i(j) - d(X^(i)_j, y_i))^2                   */
/*     + sum_{i<k} w_ik ||y_i - y_k||^2                                  */
/* ------------------------------------------------------------------ */
double orc_oos_stress(int m, int n, int d, const double *X, const double *wmat,
                      const float *dnew, const double *y)
{
    double s = 0.0;
    for (int i = 0; i < m; ++i) {
        double f = 0.0;
        for (int j = 0; j < n; ++j) {
            double e = (double)dnew[IDX(i, j, n)] -
                       dist(X + IDX((size_t)i * n + j, 0, d), y + IDX(i, 0, d), d);
            f += e * e;
        }
        s += wmat[IDX(i, i, m)] * f;
    }
    for (int i = 0; i < m; ++i)
        for (int k = i + 1; k < m; ++k) {
            double t = dist(y + IDX(i, 0, d), y + IDX(k, 0, d), d);
            s += wmat[IDX(i, k, m)] * t * t;
        }
    return s;
}

/* One out-of-sample Guttman transform, the closed form after
 * eq:joosupdate: with r_j = delta_i(j)/d(X^(i)_j, y_i) (0 when d = 0),
 *   xi_i  = w_ii sum_j (1 - r_j) X^(i)_j,   psi_i = w_ii sum_j r_j,
 *   y_new = L22^-1 (xi + diag(psi) y),   L22 = the eq:modW matrix.
 * Linv is L22^-1 (m x m).  For uniform weights L22^-1 is
 * I/(n+mw) + w J/(n(n+mw)), the form printed in Section 3. */
void orc_oos_step(int m, int n, int d, const double *X, const double *wmat,
                  const double *Linv, const float *dnew, const double *y,
                  double *ynew)
{
    double *xi = (double *)calloc((size_t)m * d, sizeof(double));
    double *psi = (double *)calloc((size_t)m, sizeof(double));
    for (int i = 0; i < m; ++i) {
        double wii = wmat[IDX(i, i, m)];
        for (int j = 0; j < n; ++j) {
            const double *xj = X + IDX((size_t)i * n + j, 0, d);
            double dj = dist(xj, y + IDX(i, 0, d), d);
            double r = dj != 0.0 ? (double)dnew[IDX(i, j, n)] / dj : 0.0;
            psi[i] += wii * r;
            for (int k = 0; k < d; ++k) xi[IDX(i, k, d)] += wii * (1.0 - r) * xj[k];
        }
    }
    for (int i = 0; i < m; ++i)
        for (int k = 0; k < d; ++k) {
            double s = 0.0;
            for (int l = 0; l < m; ++l)
                s += Linv[IDX(i, l, m)] * (xi[IDX(l, k, d)] + psi[l] * y[IDX(l, k, d)]);
            ynew[IDX(i, k, d)] = s;
        }
    free(xi);
    free(psi);
}

/* Out-of-sample embedding of k independent new objects (no weight between
 * new objects).  Y (k x m x d) holds the starts and receives the results.
 * Per object, for t = 0, 1, ...: with s_t = sigma_X(y_t),
 *   stop at t if target (optional) is given and s_t <= target[o];
 *   else stop at t if tol > 0, t > 0 and s_{t-1} - s_t < tol * s_{t-1};
 *   else, if t == iters stop, otherwise y_{t+1} = one transform of y_t.
 * stress_out[o] = s at the stop, iters_out[o] = t at the stop. */
int orc_oos(int m, int n, int d, const double *X, const double *wmat,
            const float *dnew, int k, double *Y, int iters, double tol,
            const double *target, double *stress_out, int *iters_out)
{
    double *W = (double *)malloc(sizeof(double) * m * m);
    double *Li = (double *)malloc(sizeof(double) * m * m);
    orc_wmod(m, n, wmat, W);
    int rc = orc_inverse(m, W, Li);
    free(W);
    if (rc) { free(Li); return rc; }
#pragma omp parallel for schedule(dynamic, 4)
    for (int o = 0; o < k; ++o) {
        const float *dn = dnew + IDX(o, 0, (size_t)m * n);
        double *y = Y + IDX(o, 0, (size_t)m * d);
        double *yn = (double *)malloc(sizeof(double) * m * d);
        double prev = 0.0, s = 0.0;
        int t = 0;
        for (;; ++t) {
            s = orc_oos_stress(m, n, d, X, wmat, dn, y);
            if (target && s <= target[o]) break;
            if (tol > 0.0 && t > 0 && prev - s < tol * prev) break;
            if (t == iters) break;
            orc_oos_step(m, n, d, X, wmat, Li, dn, y, yn);
            memcpy(y, yn, sizeof(double) * m * d);
            prev = s;
        }
        free(yn);
        if (stress_out) stress_out[o] = s;
        if (iters_out) iters_out[o] = t;
    }
    free(Li);
    return 0;
}
