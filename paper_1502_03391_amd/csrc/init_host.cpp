// The paper's initialisation of the in-sample iteration (Algorithm 2's
// first lines, with Algorithm 1 step 1's classical MDS):
//   xi_0 = cMDS of the mean dissimilarity (sum_i Delta_i) / m,
//   xi_i = cMDS of Delta_i, centred,
//   X^(i)_0 = orthogonal Procrustes fit of xi_i onto xi_0.
// cMDS of A: the d largest eigenpairs (lambda_k, u_k) of
// P = -1/2 J (A o A) J, X = [u_1 .. u_d] diag(lambda)^(1/2).  They come from
// subspace iteration on K >= d centred vectors: W = (A o A) V on the GPU,
// then on the host (FP64, K x K) the centred Gram W^T J W is diagonalised
// and V <- J W S diag(g)^(-1/2) is formed on the GPU; after the last step
// the Rayleigh-Ritz matrix V^T P V gives the Ritz pairs.  The m + 1
// problems (the mean and every Delta_i) take their steps together: one
// pass over the Delta_i per step forms all m + 1 products, and one host
// round trip per step serves every problem.  Procrustes: with
// M = xi_i^T xi_0, the rotation maximising tr(Q^T M) is the polar factor
// Q = M (M^T M)^(-1/2) (the printed xi_i U V^T with U S V^T = xi_0^T xi_i is
// its transpose; the fit uses Q).
#include "fjofc.h"
#include "fjofc_internal.h"

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

using namespace fjofc;

namespace {

#define INIT_TRY(expr)                                                             \
    do {                                                                           \
        hipError_t e_ = (expr);                                                    \
        if (e_ != hipSuccess)                                                      \
            return set_error(FJOFC_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

// Cyclic Jacobi eigen-decomposition of a symmetric k x k matrix (row-major,
// destroyed).  w: eigenvalues in descending order; V: eigenvectors as
// columns (row-major k x k).
void jacobi_eigh(int k, std::vector<double> A, std::vector<double> &w, std::vector<double> &V) {
    V.assign((size_t)k * k, 0.0);
    for (int i = 0; i < k; ++i) V[(size_t)i * k + i] = 1.0;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int i = 0; i < k; ++i)
            for (int j = 0; j < k; ++j) {
                const double a = A[(size_t)i * k + j];
                tot += a * a;
                if (i != j) off += a * a;
            }
        if (off <= 1e-30 * tot || off == 0.0) break;
        for (int p = 0; p < k - 1; ++p)
            for (int q = p + 1; q < k; ++q) {
                const double apq = A[(size_t)p * k + q];
                if (apq == 0.0) continue;
                const double app = A[(size_t)p * k + p], aqq = A[(size_t)q * k + q];
                const double theta = (aqq - app) / (2.0 * apq);
                const double t = (theta >= 0 ? 1.0 : -1.0) /
                                 (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
                for (int r = 0; r < k; ++r) {  // A <- A G (columns p, q)
                    const double arp = A[(size_t)r * k + p], arq = A[(size_t)r * k + q];
                    A[(size_t)r * k + p] = c * arp - s * arq;
                    A[(size_t)r * k + q] = s * arp + c * arq;
                }
                for (int r = 0; r < k; ++r) {  // A <- G^T A (rows p, q)
                    const double apr = A[(size_t)p * k + r], aqr = A[(size_t)q * k + r];
                    A[(size_t)p * k + r] = c * apr - s * aqr;
                    A[(size_t)q * k + r] = s * apr + c * aqr;
                }
                for (int r = 0; r < k; ++r) {
                    const double vrp = V[(size_t)r * k + p], vrq = V[(size_t)r * k + q];
                    V[(size_t)r * k + p] = c * vrp - s * vrq;
                    V[(size_t)r * k + q] = s * vrp + c * vrq;
                }
            }
    }
    std::vector<int> idx(k);
    for (int i = 0; i < k; ++i) idx[i] = i;
    std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) {
        return A[(size_t)a * k + a] > A[(size_t)b * k + b];
    });
    w.resize(k);
    std::vector<double> Vs((size_t)k * k);
    for (int c = 0; c < k; ++c) {
        w[c] = A[(size_t)idx[c] * k + idx[c]];
        for (int r = 0; r < k; ++r) Vs[(size_t)r * k + c] = V[(size_t)r * k + idx[c]];
    }
    V.swap(Vs);
}

uint64_t splitmix(uint64_t x) {
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

struct InitBufs {
    int P, K, n, d, npad;
    float *V, *W, *Vt, *part, *xi;  // per problem: n K, n K, 16 npad, -, n d
    double *stats, *small;          // per problem K K + K doubles each
    double *pin;                    // pinned host copy of stats / small
    int nrowblk, splits, cpw;
    size_t nK() const { return (size_t)n * K; }
    size_t kk() const { return (size_t)K * K + K; }
};

// Host step of one orthonormalisation: from the Gram G = W^T W and the
// column sums cs of W (n rows), the matrix M with V = (W - 1 cs^T / n) M
// orthonormal (columns of negligible weight become 0).
void ortho_matrix(int K, int n, const double *G, const double *cs, double *M, double *mu) {
    std::vector<double> Gc((size_t)K * K);
    for (int a = 0; a < K; ++a)
        for (int b = 0; b < K; ++b) Gc[(size_t)a * K + b] = G[a * K + b] - cs[a] * cs[b] / n;
    std::vector<double> w, S;
    jacobi_eigh(K, Gc, w, S);
    std::fill(M, M + (size_t)K * K, 0.0);
    const double top = std::max(w[0], 0.0);
    for (int c = 0; c < K; ++c) {
        if (!(w[c] > 1e-12 * top) || w[c] <= 0.0) continue;
        const double s = 1.0 / std::sqrt(w[c]);
        for (int a = 0; a < K; ++a) M[(size_t)a * K + c] = S[(size_t)a * K + c] * s;
    }
    for (int a = 0; a < K; ++a) mu[a] = cs[a] / n;
}

// W_p = (A_p o A_p) V_p for every problem: problem 0 the mean of the m
// matrices, problem 1 + i Delta_i.  m <= 4: one pass over the matrices;
// otherwise a pass for the mean and one per group of four modalities.
int products(fjofc_ctx *ctx, const DeltaPtrs &dp, int m, const InitBufs &b, hipStream_t s) {
    // every entry of every Delta_i once, and once more for the mean when
    // it takes a pass of its own
    const double rd = 4.0 * (double)b.n * b.n * (m <= 4 ? m : 2 * m);
    Timed tm(ctx, K_INIT, rd, s);
    GramArgs ga{};
    ga.dp = dp;
    ga.nsrc = m;
    ga.n = b.n;
    ga.npad = b.npad;
    ga.scale = (float)(1.0 / m);
    ga.part = b.part;
    ga.ptotal = b.P;
    ga.nrowblk = b.nrowblk;
    ga.splits = b.splits;
    ga.cpw = b.cpw;
    ga.nrow_pad = b.nrowblk * GR_ROWS;
    const size_t vts = (size_t)16 * b.npad;
    if (m <= 4) {
        for (int p = 0; p <= m; ++p) ga.Vt[p] = b.Vt + p * vts;
        INIT_TRY(launch_gram(ga, m, true, s));
    } else {
        ga.Vt[0] = b.Vt;
        INIT_TRY(launch_gram(ga, 0, true, s));
        for (int g0 = 0; g0 < m; g0 += 4) {
            const int G = std::min(4, m - g0);
            ga.i0 = g0;
            ga.pbase = 1 + g0;
            for (int q = 0; q < G; ++q) ga.Vt[q] = b.Vt + (1 + g0 + q) * vts;
            INIT_TRY(launch_gram(ga, G, false, s));
        }
    }
    INIT_TRY(launch_gram_combine(b.part, b.splits, b.P, ga.nrow_pad, b.n, b.K, b.W, b.nK(), s));
    return FJOFC_OK;
}

// V_p (and its transpose) = (in_p - 1 mu_p^T) M_p with M_p, mu_p from b.small.
int apply_all(const InitBufs &b, const float *in, hipStream_t s) {
    ApplyArgs aa{};
    aa.in = in;
    aa.ldi = b.K;
    aa.nin = b.K;
    aa.sin = b.nK();
    aa.mu = b.small + (size_t)b.K * b.K;
    aa.smu = b.kk();
    aa.M = b.small;
    aa.sM = b.kk();
    aa.ncol = b.K;
    aa.n = b.n;
    aa.out = b.V;
    aa.ldo = b.K;
    aa.ldo_pad = b.K;
    aa.sout = b.nK();
    aa.outT = b.Vt;
    aa.soutT = (size_t)16 * b.npad;
    aa.npad = b.npad;
    INIT_TRY(launch_apply(aa, b.P, s));
    return FJOFC_OK;
}

// cMDS of all P problems: xi_p (n x d, device, at b.xi + p n d) and the d
// largest Ritz values of each (eig + p d).
int cmds_all(fjofc_ctx *ctx, const DeltaPtrs &dp, int m, int iters, const InitBufs &b,
             double *eig, hipStream_t s) {
    const int K = b.K, P = b.P, d = b.d;
    const size_t KK = (size_t)K * K, kk = b.kk();
    // seeded starts in [-1, 1): the mean's stream 1, Delta_i's stream 2 + i
    {
        std::vector<float> R((size_t)P * b.nK());
        for (int p = 0; p < P; ++p) {
            const uint64_t seed = 1 + (uint64_t)p;
            float *r = R.data() + p * b.nK();
            for (size_t q = 0; q < b.nK(); ++q)
                r[q] = (float)((double)(splitmix(seed * 0x100000001B3ull + q) >> 11) * 0x1.0p-52 -
                               1.0);
        }
        INIT_TRY(hipMemcpyAsync(b.W, R.data(), sizeof(float) * R.size(), hipMemcpyHostToDevice, s));
        INIT_TRY(hipStreamSynchronize(s));
    }
    for (int it = 0; it <= iters; ++it) {
        if (it > 0) {
            const int rc = products(ctx, dp, m, b, s);
            if (rc) return rc;
        }
        INIT_TRY(launch_cross(b.W, K, b.nK(), K, b.W, K, b.nK(), K, b.n, b.stats, kk, P, s));
        INIT_TRY(launch_cross(b.W, K, b.nK(), K, nullptr, 0, 0, 1, b.n, b.stats + KK, kk, P, s));
        INIT_TRY(hipMemcpyAsync(b.pin, b.stats, sizeof(double) * kk * P, hipMemcpyDeviceToHost, s));
        INIT_TRY(hipStreamSynchronize(s));
        std::vector<double> out(kk * P);
        for (int p = 0; p < P; ++p)
            ortho_matrix(K, b.n, b.pin + p * kk, b.pin + p * kk + KK, out.data() + p * kk,
                         out.data() + p * kk + KK);
        std::memcpy(b.pin, out.data(), sizeof(double) * kk * P);
        INIT_TRY(hipMemcpyAsync(b.small, b.pin, sizeof(double) * kk * P, hipMemcpyHostToDevice, s));
        const int rc = apply_all(b, b.W, s);
        if (rc) return rc;
        INIT_TRY(hipStreamSynchronize(s));  // b.pin is reused next
    }
    // Rayleigh-Ritz: V^T P V = -1/2 V^T (A o A) V (V is centred)
    int rc = products(ctx, dp, m, b, s);
    if (rc) return rc;
    INIT_TRY(launch_cross(b.V, K, b.nK(), K, b.W, K, b.nK(), K, b.n, b.stats, kk, P, s));
    INIT_TRY(hipMemcpyAsync(b.pin, b.stats, sizeof(double) * kk * P, hipMemcpyDeviceToHost, s));
    INIT_TRY(hipStreamSynchronize(s));
    std::vector<double> M2(kk * P, 0.0);
    for (int p = 0; p < P; ++p) {
        const double *g = b.pin + p * kk;
        std::vector<double> H(KK);
        for (int a = 0; a < K; ++a)
            for (int c = 0; c < K; ++c)
                H[(size_t)a * K + c] = -0.25 * (g[a * K + c] + g[c * K + a]);
        std::vector<double> th, S;
        jacobi_eigh(K, H, th, S);
        double *Mp = M2.data() + p * kk;  // K x d
        for (int c = 0; c < d; ++c) {
            const double sc = std::sqrt(std::max(th[c], 0.0));
            for (int a = 0; a < K; ++a) Mp[(size_t)a * d + c] = S[(size_t)a * K + c] * sc;
            if (eig) eig[(size_t)p * d + c] = th[c];
        }
    }
    std::memcpy(b.pin, M2.data(), sizeof(double) * kk * P);
    INIT_TRY(hipMemcpyAsync(b.small, b.pin, sizeof(double) * kk * P, hipMemcpyHostToDevice, s));
    ApplyArgs aa{};
    aa.in = b.V;
    aa.ldi = K;
    aa.nin = K;
    aa.sin = b.nK();
    aa.M = b.small;
    aa.sM = kk;
    aa.ncol = d;
    aa.n = b.n;
    aa.out = b.xi;
    aa.ldo = d;
    aa.ldo_pad = d;
    aa.sout = (size_t)b.n * d;
    INIT_TRY(launch_apply(aa, P, s));
    INIT_TRY(hipStreamSynchronize(s));
    return FJOFC_OK;
}

}  // namespace

extern "C" int fjofc_init_cmds(fjofc_ctx *ctx, const float *const *delta, int m, int n, int d,
                               float *X, int iters, double *eigvals, void *stream) {
    if (!ctx) return set_error(FJOFC_EINVAL, "ctx is NULL");
    if (m < 1 || m > FJOFC_MAX_M) return set_error(FJOFC_EINVAL, "m=%d outside [1,%d]", m, FJOFC_MAX_M);
    if (n < 2) return set_error(FJOFC_EINVAL, "n=%d must be >= 2", n);
    if (d < 1 || d > FJOFC_MAX_D) return set_error(FJOFC_EINVAL, "d=%d outside [1,%d]", d, FJOFC_MAX_D);
    if (iters < 1 || iters > 10000) return set_error(FJOFC_EINVAL, "iters=%d outside [1,10000]", iters);
    if (!delta || !X) return set_error(FJOFC_EINVAL, "NULL array");
    for (int i = 0; i < m; ++i)
        if (!delta[i]) return set_error(FJOFC_EINVAL, "delta[%d] is NULL", i);
    const int need = std::max(2 * d, d + 3);
    const int K = need <= 4 ? 4 : need <= 8 ? 8 : need <= 12 ? 12 : 16;
    int prev = -1;
    (void)hipGetDevice(&prev);
    const int dev = ctx_device(ctx);
    if (prev != dev) (void)hipSetDevice(dev);
    struct Restore {
        int p, d;
        ~Restore() {
            if (p >= 0 && p != d) (void)hipSetDevice(p);
        }
    } restore{prev, dev};
    hipStream_t s = static_cast<hipStream_t>(stream);

    auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
    InitBufs b;
    b.P = m + 1;
    b.K = K;
    b.n = n;
    b.d = d;
    b.npad = (n + GR_CHUNK - 1) / GR_CHUNK * GR_CHUNK;
    gram_plan(n, b.nrowblk, b.splits, b.cpw);
    const size_t kk = b.kk(), P = (size_t)b.P;
    size_t off = 0;
    const size_t oV = off; off = al(off + sizeof(float) * P * b.nK());
    const size_t oW = off; off = al(off + sizeof(float) * P * b.nK());
    const size_t oVt = off; off = al(off + sizeof(float) * P * 16 * b.npad);
    const size_t oPt = off;
    off = al(off + sizeof(float) * (size_t)b.splits * P * b.nrowblk * GR_ROWS * 16);
    const size_t oXi = off; off = al(off + sizeof(float) * P * n * d);
    const size_t oSt = off; off = al(off + sizeof(double) * P * kk);
    const size_t oSm = off; off = al(off + sizeof(double) * P * kk);
    void *ws = nullptr, *pin = nullptr;
    int rc = ctx_workspace(ctx, off, &ws);
    if (rc) return rc;
    rc = ctx_pinned(ctx, sizeof(double) * P * kk, &pin);
    if (rc) return rc;
    char *base = static_cast<char *>(ws);
    b.V = reinterpret_cast<float *>(base + oV);
    b.W = reinterpret_cast<float *>(base + oW);
    b.Vt = reinterpret_cast<float *>(base + oVt);
    b.part = reinterpret_cast<float *>(base + oPt);
    b.xi = reinterpret_cast<float *>(base + oXi);
    b.stats = reinterpret_cast<double *>(base + oSt);
    b.small = reinterpret_cast<double *>(base + oSm);
    b.pin = static_cast<double *>(pin);
    INIT_TRY(hipStreamSynchronize(s));  // the workspace may have been in use

    DeltaPtrs all{};
    for (int i = 0; i < m; ++i) all.p[i] = delta[i];
    rc = cmds_all(ctx, all, m, iters, b, eigvals, s);
    if (rc) return rc;
    // Procrustes of every xi_i (problem 1 + i) onto xi_0:
    // M_i = xi_i^T xi_0, Q_i = M_i (M_i^T M_i)^(-1/2)
    const size_t dd = (size_t)d * d, nd = (size_t)n * d;
    INIT_TRY(launch_cross(b.xi + nd, d, nd, d, b.xi, d, 0, d, n, b.stats, dd, m, s));
    INIT_TRY(hipMemcpyAsync(b.pin, b.stats, sizeof(double) * dd * m, hipMemcpyDeviceToHost, s));
    INIT_TRY(hipStreamSynchronize(s));
    std::vector<double> Qall(dd * m);
    for (int i = 0; i < m; ++i) {
        const double *Mq = b.pin + i * dd;
        std::vector<double> MtM(dd, 0.0);
        for (int a = 0; a < d; ++a)
            for (int c = 0; c < d; ++c)
                for (int r = 0; r < d; ++r) MtM[(size_t)a * d + c] += Mq[(size_t)r * d + a] * Mq[(size_t)r * d + c];
        std::vector<double> w, S;
        jacobi_eigh(d, MtM, w, S);
        std::vector<double> Ris(dd, 0.0);  // (M^T M)^(-1/2)
        const double top = std::max(w[0], 0.0);
        for (int c = 0; c < d; ++c) {
            if (!(w[c] > 1e-24 * top) || w[c] <= 0.0) continue;
            const double sc = 1.0 / std::sqrt(w[c]);
            for (int a = 0; a < d; ++a)
                for (int e = 0; e < d; ++e)
                    Ris[(size_t)a * d + e] += S[(size_t)a * d + c] * sc * S[(size_t)e * d + c];
        }
        double *Q = Qall.data() + i * dd;
        for (int a = 0; a < d; ++a)
            for (int c = 0; c < d; ++c)
                for (int r = 0; r < d; ++r) Q[(size_t)a * d + c] += Mq[(size_t)a * d + r] * Ris[(size_t)r * d + c];
    }
    std::memcpy(b.pin, Qall.data(), sizeof(double) * dd * m);
    INIT_TRY(hipMemcpyAsync(b.small, b.pin, sizeof(double) * dd * m, hipMemcpyHostToDevice, s));
    ApplyArgs aa{};
    aa.in = b.xi + nd;
    aa.ldi = d;
    aa.nin = d;
    aa.sin = nd;
    aa.M = b.small;
    aa.sM = dd;
    aa.ncol = d;
    aa.n = n;
    aa.out = X;
    aa.ldo = d;
    aa.ldo_pad = d;
    aa.sout = nd;
    INIT_TRY(launch_apply(aa, m, s));
    INIT_TRY(hipStreamSynchronize(s));
    return FJOFC_OK;
}
