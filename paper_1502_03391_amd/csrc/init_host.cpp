// The paper's initialisation of the in-sample iteration (Algorithm 2's
// first lines, with Algorithm 1 step 1's classical MDS):
//   xi_0 = cMDS of the mean dissimilarity (sum_i Delta_i) / m,
//   xi_i = cMDS of Delta_i, centred,
//   X^(i)_0 = orthogonal Procrustes fit of xi_i onto xi_0.
// cMDS of A: the d largest eigenpairs (lambda_k, u_k) of
// P = -1/2 J (A o A) J, X = [u_1 .. u_d] diag(lambda)^(1/2).  They come from
// subspace iteration on K >= d centred vectors: W = (A o A) V on the GPU
// (one full stream of A), then on the host (FP64, K x K) the centred Gram
// W^T J W is diagonalised and V <- J W S diag(g)^(-1/2) is formed on the
// GPU; after the last step the Rayleigh-Ritz matrix V^T P V gives the Ritz
// pairs.  Procrustes: with M = xi_i^T xi_0, the rotation maximising
// tr(Q^T M) is the polar factor Q = M (M^T M)^(-1/2) (the printed
// xi_i U V^T with U S V^T = xi_0^T xi_i is its transpose; the fit uses Q).
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
    float *V, *W, *xi0, *xi;
    double *stats, *small;  // K*K + K doubles each
    double *pin;            // pinned host copy of stats / small
};

// Host step of one orthonormalisation: from the Gram G = W^T W and the
// column sums cs of W (n rows), the matrix M with V = (W - 1 cs^T / n) M
// orthonormal (columns of negligible weight become 0).
void ortho_matrix(int K, int n, const double *G, const double *cs, std::vector<double> &M,
                  std::vector<double> &mu) {
    std::vector<double> Gc((size_t)K * K);
    for (int a = 0; a < K; ++a)
        for (int b = 0; b < K; ++b) Gc[(size_t)a * K + b] = G[a * K + b] - cs[a] * cs[b] / n;
    std::vector<double> w, S;
    jacobi_eigh(K, Gc, w, S);
    M.assign((size_t)K * K, 0.0);
    const double top = std::max(w[0], 0.0);
    for (int c = 0; c < K; ++c) {
        if (!(w[c] > 1e-12 * top) || w[c] <= 0.0) continue;
        const double s = 1.0 / std::sqrt(w[c]);
        for (int a = 0; a < K; ++a) M[(size_t)a * K + c] = S[(size_t)a * K + c] * s;
    }
    mu.resize(K);
    for (int a = 0; a < K; ++a) mu[a] = cs[a] / n;
}

// cMDS of A = scale * sum of the nsrc matrices: xi (n x d, device) and the
// d largest Ritz values.
int cmds(const DeltaPtrs &dp, int nsrc, float scale, int n, int d, int K, int iters,
         uint64_t seed, const InitBufs &b, float *xi, double *eig, hipStream_t s) {
    const size_t KK = (size_t)K * K;
    // seeded start in [-1, 1)
    {
        std::vector<float> R((size_t)n * K);
        for (size_t q = 0; q < R.size(); ++q)
            R[q] = (float)((double)(splitmix(seed * 0x100000001B3ull + q) >> 11) * 0x1.0p-52 - 1.0);
        INIT_TRY(hipMemcpyAsync(b.W, R.data(), sizeof(float) * R.size(), hipMemcpyHostToDevice, s));
        INIT_TRY(hipStreamSynchronize(s));
    }
    std::vector<double> M, mu;
    for (int it = 0; it <= iters; ++it) {
        if (it > 0) INIT_TRY(launch_sqprod(dp, nsrc, scale, n, K, b.V, b.W, s));
        INIT_TRY(launch_cross(b.W, K, K, b.W, K, K, n, b.stats, s));
        INIT_TRY(launch_cross(b.W, K, K, nullptr, 0, 1, n, b.stats + KK, s));
        INIT_TRY(hipMemcpyAsync(b.pin, b.stats, sizeof(double) * (KK + K), hipMemcpyDeviceToHost, s));
        INIT_TRY(hipStreamSynchronize(s));
        ortho_matrix(K, n, b.pin, b.pin + KK, M, mu);
        std::memcpy(b.pin, M.data(), sizeof(double) * KK);
        std::memcpy(b.pin + KK, mu.data(), sizeof(double) * K);
        INIT_TRY(hipMemcpyAsync(b.small, b.pin, sizeof(double) * (KK + K), hipMemcpyHostToDevice, s));
        INIT_TRY(launch_apply(b.W, K, K, b.small + KK, b.small, K, n, b.V, K, K, s));
        INIT_TRY(hipStreamSynchronize(s));  // b.pin is reused next
    }
    // Rayleigh-Ritz: V^T P V = -1/2 V^T (A o A) V (V is centred)
    INIT_TRY(launch_sqprod(dp, nsrc, scale, n, K, b.V, b.W, s));
    INIT_TRY(launch_cross(b.V, K, K, b.W, K, K, n, b.stats, s));
    INIT_TRY(hipMemcpyAsync(b.pin, b.stats, sizeof(double) * KK, hipMemcpyDeviceToHost, s));
    INIT_TRY(hipStreamSynchronize(s));
    std::vector<double> H(KK);
    for (int a = 0; a < K; ++a)
        for (int c = 0; c < K; ++c)
            H[(size_t)a * K + c] = -0.25 * (b.pin[a * K + c] + b.pin[c * K + a]);
    std::vector<double> th, S;
    jacobi_eigh(K, H, th, S);
    std::vector<double> M2((size_t)K * d, 0.0);
    for (int c = 0; c < d; ++c) {
        const double sc = std::sqrt(std::max(th[c], 0.0));
        for (int a = 0; a < K; ++a) M2[(size_t)a * d + c] = S[(size_t)a * K + c] * sc;
        if (eig) eig[c] = th[c];
    }
    std::memcpy(b.pin, M2.data(), sizeof(double) * K * d);
    INIT_TRY(hipMemcpyAsync(b.small, b.pin, sizeof(double) * K * d, hipMemcpyHostToDevice, s));
    INIT_TRY(launch_apply(b.V, K, K, nullptr, b.small, d, n, xi, d, d, s));
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
    const size_t KK = (size_t)K * K;
    size_t off = 0;
    const size_t oV = off; off = al(off + sizeof(float) * n * K);
    const size_t oW = off; off = al(off + sizeof(float) * n * K);
    const size_t oX0 = off; off = al(off + sizeof(float) * n * d);
    const size_t oXi = off; off = al(off + sizeof(float) * n * d);
    const size_t oSt = off; off = al(off + sizeof(double) * (KK + K));
    const size_t oSm = off; off = al(off + sizeof(double) * (KK + K));
    void *ws = nullptr, *pin = nullptr;
    int rc = ctx_workspace(ctx, off, &ws);
    if (rc) return rc;
    rc = ctx_pinned(ctx, sizeof(double) * (KK + K), &pin);
    if (rc) return rc;
    char *base = static_cast<char *>(ws);
    InitBufs b;
    b.V = reinterpret_cast<float *>(base + oV);
    b.W = reinterpret_cast<float *>(base + oW);
    b.xi0 = reinterpret_cast<float *>(base + oX0);
    b.xi = reinterpret_cast<float *>(base + oXi);
    b.stats = reinterpret_cast<double *>(base + oSt);
    b.small = reinterpret_cast<double *>(base + oSm);
    b.pin = static_cast<double *>(pin);
    INIT_TRY(hipStreamSynchronize(s));  // the workspace may have been in use

    DeltaPtrs all{};
    for (int i = 0; i < m; ++i) all.p[i] = delta[i];
    rc = cmds(all, m, (float)(1.0 / m), n, d, K, iters, 1, b, b.xi0, eigvals, s);
    if (rc) return rc;
    for (int i = 0; i < m; ++i) {
        DeltaPtrs one{};
        one.p[0] = delta[i];
        rc = cmds(one, 1, 1.0f, n, d, K, iters, 2 + (uint64_t)i, b, b.xi,
                  eigvals ? eigvals + (size_t)(i + 1) * d : nullptr, s);
        if (rc) return rc;
        // Procrustes: M = xi_i^T xi_0, Q = M (M^T M)^(-1/2)
        INIT_TRY(launch_cross(b.xi, d, d, b.xi0, d, d, n, b.stats, s));
        INIT_TRY(hipMemcpyAsync(b.pin, b.stats, sizeof(double) * d * d, hipMemcpyDeviceToHost, s));
        INIT_TRY(hipStreamSynchronize(s));
        std::vector<double> Mq(b.pin, b.pin + (size_t)d * d), MtM((size_t)d * d, 0.0);
        for (int a = 0; a < d; ++a)
            for (int c = 0; c < d; ++c)
                for (int r = 0; r < d; ++r) MtM[(size_t)a * d + c] += Mq[(size_t)r * d + a] * Mq[(size_t)r * d + c];
        std::vector<double> w, S;
        jacobi_eigh(d, MtM, w, S);
        std::vector<double> Ris((size_t)d * d, 0.0);  // (M^T M)^(-1/2)
        const double top = std::max(w[0], 0.0);
        for (int c = 0; c < d; ++c) {
            if (!(w[c] > 1e-24 * top) || w[c] <= 0.0) continue;
            const double sc = 1.0 / std::sqrt(w[c]);
            for (int a = 0; a < d; ++a)
                for (int e = 0; e < d; ++e)
                    Ris[(size_t)a * d + e] += S[(size_t)a * d + c] * sc * S[(size_t)e * d + c];
        }
        std::vector<double> Q((size_t)d * d, 0.0);
        for (int a = 0; a < d; ++a)
            for (int c = 0; c < d; ++c)
                for (int r = 0; r < d; ++r) Q[(size_t)a * d + c] += Mq[(size_t)a * d + r] * Ris[(size_t)r * d + c];
        std::memcpy(b.pin, Q.data(), sizeof(double) * d * d);
        INIT_TRY(hipMemcpyAsync(b.small, b.pin, sizeof(double) * d * d, hipMemcpyHostToDevice, s));
        INIT_TRY(launch_apply(b.xi, d, d, nullptr, b.small, d, n, X + (size_t)i * n * d, d, d, s));
        INIT_TRY(hipStreamSynchronize(s));
    }
    return FJOFC_OK;
}
