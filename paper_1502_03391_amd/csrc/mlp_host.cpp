// Host side of the warm-start network ABI (include/fjofc.h, fjofc_mlp_*):
// parameter storage (FP32 masters, BF16 copies, Adam moments, gradients in
// flat arrays), activation buffers for up to max_batch rows, and the
// forward / backward / Adam sequences of kernel launches.
#include "fjofc.h"
#include "fjofc_internal.h"

#include <cmath>
#include <cstring>
#include <vector>

using namespace fjofc;

struct fjofc_mlp {
    int device = 0;
    int L = 0, maxb = 0, maxw = 0;
    long ldt = 0;  // leading dimension of the transposed (feature-major) buffers
    std::vector<int> dims;
    std::vector<size_t> offW, offb;  // offsets into the flat parameter arrays (multiples of 8)
    size_t nparam = 0;
    void *mem = nullptr;
    float *P = nullptr, *G = nullptr, *M1 = nullptr, *M2 = nullptr;
    uint16_t *P16 = nullptr;     // BF16 copies; W_l (dims[l] x dims[l+1]) at offW[l]
    std::vector<uint16_t *> WT;  // WT[l]: BF16 W_l transposed (dims[l+1] x dims[l])
    std::vector<uint16_t *> H;   // H[l], l = 1..L-1: BF16 activations (maxb x dims[l])
    std::vector<uint16_t *> HT;  // HT[l]: the same transposed (dims[l] x ldt); HT[0] = x^T
    std::vector<float *> Z;      // Z[l]: FP32 pre-activations feeding H[l]
    float *out = nullptr;        // maxb x dims[L]
    float *Gf[2] = {nullptr, nullptr};
    uint16_t *Gb[2] = {nullptr, nullptr};
    uint16_t *GbT[2] = {nullptr, nullptr};  // BF16 gradients transposed (width x ldt)
    double *scratch = nullptr;              // reduction partials (16 maxw + 64 doubles)
    int step = 0;
};

namespace {

#define HIP_CHECK(expr)                                                             \
    do {                                                                            \
        hipError_t e_ = (expr);                                                     \
        if (e_ != hipSuccess)                                                       \
            return set_error(FJOFC_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

struct Dev {
    int prev = -1;
    explicit Dev(int d) {
        if (hipGetDevice(&prev) == hipSuccess && prev != d) (void)hipSetDevice(d);
        else prev = -1;
    }
    ~Dev() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

size_t al(size_t x) { return (x + 255) & ~size_t(255); }

int check_batch(const fjofc_mlp *n, int B) {
    if (!n) return set_error(FJOFC_EINVAL, "mlp is NULL");
    if (B < 1 || B > n->maxb) return set_error(FJOFC_EINVAL, "batch %d outside [1,%d]", B, n->maxb);
    return FJOFC_OK;
}

size_t pad8(size_t x) { return (x + 7) & ~size_t(7); }

// Refresh the transposed BF16 weight copies from P16.
int refresh_wt(fjofc_mlp *n, hipStream_t s) {
    for (int l = 0; l < n->L; ++l)
        HIP_CHECK(launch_transpose16(n->P16 + n->offW[l], n->dims[l + 1], n->dims[l],
                                     n->dims[l + 1], n->WT[l], n->dims[l], s));
    return FJOFC_OK;
}

// Forward pass of B rows: H[l+1] = BF16(GELU(H[l] W_l + b_l)) (and its
// transpose for the weight gradients), out = last z.
int forward(fjofc_mlp *n, const uint16_t *x, int B, hipStream_t s) {
    const uint16_t *h = x;
    for (int l = 0; l < n->L; ++l) {
        const int in = n->dims[l], o = n->dims[l + 1];
        GemmEpi e{};
        e.bias = n->P + n->offb[l];
        e.ldc = o;
        e.ldt = n->ldt;
        const bool last = (l == n->L - 1);
        if (last) {
            e.outf = n->out;
        } else {
            e.outf = n->Z[l + 1];
            e.outb = n->H[l + 1];
            e.outbT = n->HT[l + 1];
        }
        HIP_CHECK(launch_gemm(last ? GEMM_LAST : GEMM_HIDDEN, B, o, in, h, in, n->WT[l], in, e, s));
        if (!last) h = n->H[l + 1];
    }
    return FJOFC_OK;
}

}  // namespace

extern "C" {

int fjofc_mlp_create(fjofc_ctx *ctx, int L, const int *dims, int max_batch, fjofc_mlp **out) {
    (void)ctx;
    if (!out || !dims) return set_error(FJOFC_EINVAL, "NULL argument");
    if (L < 1 || L > 16) return set_error(FJOFC_EINVAL, "layers %d outside [1,16]", L);
    if (max_batch < 1) return set_error(FJOFC_EINVAL, "max_batch must be >= 1");
    for (int l = 0; l <= L; ++l)
        if (dims[l] < 1 || dims[l] > 65536) return set_error(FJOFC_EINVAL, "bad width dims[%d]", l);
    fjofc_mlp *n = new fjofc_mlp();
    int dev = 0;
    (void)hipGetDevice(&dev);
    n->device = dev;
    n->L = L;
    n->maxb = max_batch;
    n->dims.assign(dims, dims + L + 1);
    for (int l = 0; l <= L; ++l) n->maxw = std::max(n->maxw, dims[l]);
    for (int l = 0; l < L; ++l) {
        n->offW.push_back(n->nparam);
        n->nparam = pad8(n->nparam + (size_t)dims[l] * dims[l + 1]);
        n->offb.push_back(n->nparam);
        n->nparam = pad8(n->nparam + dims[l + 1]);
    }
    n->ldt = (long)pad8(max_batch);
    // layout: P, G, M1, M2 (FP32), P16, WT, activations, gradients
    size_t off = 0;
    const size_t oP = off; off = al(off + 4 * n->nparam);
    const size_t oG = off; off = al(off + 4 * n->nparam);
    const size_t oM1 = off; off = al(off + 4 * n->nparam);
    const size_t oM2 = off; off = al(off + 4 * n->nparam);
    const size_t zero_end = off;
    const size_t oP16 = off; off = al(off + 2 * n->nparam);
    std::vector<size_t> oWT(L, 0);
    for (int l = 0; l < L; ++l) { oWT[l] = off; off = al(off + 2 * (size_t)dims[l] * dims[l + 1]); }
    std::vector<size_t> oH(L + 1, 0), oHT(L + 1, 0), oZ(L + 1, 0);
    for (int l = 0; l < L; ++l) {
        if (l > 0) {
            oH[l] = off; off = al(off + 2 * (size_t)max_batch * dims[l]);
            oZ[l] = off; off = al(off + 4 * (size_t)max_batch * dims[l]);
        }
        oHT[l] = off; off = al(off + 2 * (size_t)n->ldt * dims[l]);
    }
    const size_t oOut = off; off = al(off + 4 * (size_t)max_batch * dims[L]);
    size_t oGf[2], oGb[2], oGbT[2];
    for (int q = 0; q < 2; ++q) {
        oGf[q] = off; off = al(off + 4 * (size_t)max_batch * n->maxw);
        oGb[q] = off; off = al(off + 2 * (size_t)max_batch * n->maxw);
        oGbT[q] = off; off = al(off + 2 * (size_t)n->ldt * n->maxw);
    }
    const size_t oScr = off; off = al(off + 8 * (16 * (size_t)n->maxw + 64));
    if (hipMalloc(&n->mem, off) != hipSuccess) {
        delete n;
        return set_error(FJOFC_ENOMEM, "mlp workspace of %zu bytes", off);
    }
    // parameters, gradients and moments start at 0, so the padding between
    // layers stays 0 through Adam
    if (hipMemset(n->mem, 0, zero_end) != hipSuccess) {
        (void)hipFree(n->mem);
        delete n;
        return set_error(FJOFC_EHIP, "clearing the mlp workspace failed");
    }
    char *b = static_cast<char *>(n->mem);
    n->P = reinterpret_cast<float *>(b + oP);
    n->G = reinterpret_cast<float *>(b + oG);
    n->M1 = reinterpret_cast<float *>(b + oM1);
    n->M2 = reinterpret_cast<float *>(b + oM2);
    n->P16 = reinterpret_cast<uint16_t *>(b + oP16);
    n->WT.assign(L, nullptr);
    for (int l = 0; l < L; ++l) n->WT[l] = reinterpret_cast<uint16_t *>(b + oWT[l]);
    n->H.assign(L + 1, nullptr);
    n->HT.assign(L + 1, nullptr);
    n->Z.assign(L + 1, nullptr);
    for (int l = 0; l < L; ++l) {
        if (l > 0) {
            n->H[l] = reinterpret_cast<uint16_t *>(b + oH[l]);
            n->Z[l] = reinterpret_cast<float *>(b + oZ[l]);
        }
        n->HT[l] = reinterpret_cast<uint16_t *>(b + oHT[l]);
    }
    n->out = reinterpret_cast<float *>(b + oOut);
    for (int q = 0; q < 2; ++q) {
        n->Gf[q] = reinterpret_cast<float *>(b + oGf[q]);
        n->Gb[q] = reinterpret_cast<uint16_t *>(b + oGb[q]);
        n->GbT[q] = reinterpret_cast<uint16_t *>(b + oGbT[q]);
    }
    n->scratch = reinterpret_cast<double *>(b + oScr);
    *out = n;
    return FJOFC_OK;
}

void fjofc_mlp_destroy(fjofc_mlp *n) {
    if (!n) return;
    Dev dg(n->device);
    (void)hipDeviceSynchronize();
    if (n->mem) (void)hipFree(n->mem);
    delete n;
}

int fjofc_mlp_set_params(fjofc_mlp *n, const float *const *W, const float *const *b, void *stream) {
    if (!n || !W || !b) return set_error(FJOFC_EINVAL, "NULL argument");
    Dev dg(n->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    for (int l = 0; l < n->L; ++l) {
        HIP_CHECK(hipMemcpyAsync(n->P + n->offW[l], W[l],
                                 4 * (size_t)n->dims[l] * n->dims[l + 1],
                                 hipMemcpyDeviceToDevice, s));
        HIP_CHECK(hipMemcpyAsync(n->P + n->offb[l], b[l], 4 * (size_t)n->dims[l + 1],
                                 hipMemcpyDeviceToDevice, s));
    }
    HIP_CHECK(launch_to_bf16(n->P, n->P16, (long)n->nparam, s));
    int rc = refresh_wt(n, s);
    if (rc) return rc;
    // zero the Adam moments: 0 * finite stays 0 through the update form
    HIP_CHECK(hipMemsetAsync(n->M1, 0, 4 * n->nparam, s));
    HIP_CHECK(hipMemsetAsync(n->M2, 0, 4 * n->nparam, s));
    n->step = 0;
    return FJOFC_OK;
}

int fjofc_mlp_get_params(fjofc_mlp *n, float *const *W, float *const *b, void *stream) {
    if (!n || !W || !b) return set_error(FJOFC_EINVAL, "NULL argument");
    Dev dg(n->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    for (int l = 0; l < n->L; ++l) {
        HIP_CHECK(hipMemcpyAsync(W[l], n->P + n->offW[l], 4 * (size_t)n->dims[l] * n->dims[l + 1],
                                 hipMemcpyDeviceToDevice, s));
        HIP_CHECK(hipMemcpyAsync(b[l], n->P + n->offb[l], 4 * (size_t)n->dims[l + 1],
                                 hipMemcpyDeviceToDevice, s));
    }
    return FJOFC_OK;
}

int fjofc_mlp_forward(fjofc_mlp *n, const unsigned short *x, int B, float *out, void *stream) {
    int rc = check_batch(n, B);
    if (rc) return rc;
    if (!x || !out) return set_error(FJOFC_EINVAL, "NULL argument");
    Dev dg(n->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    rc = forward(n, x, B, s);
    if (rc) return rc;
    HIP_CHECK(hipMemcpyAsync(out, n->out, 4 * (size_t)B * n->dims[n->L], hipMemcpyDeviceToDevice, s));
    return FJOFC_OK;
}

int fjofc_mlp_predict_start(fjofc_mlp *n, const unsigned short *x, int B, int m, int d,
                            float *Y, void *stream) {
    int rc = check_batch(n, B);
    if (rc) return rc;
    if (!x || !Y || m < 1 || d < 1) return set_error(FJOFC_EINVAL, "bad argument");
    const int P = n->dims[n->L];
    if (P != d && P != m * d)
        return set_error(FJOFC_EINVAL, "network output width %d is neither d=%d nor m*d=%d", P,
                         d, m * d);
    Dev dg(n->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    rc = forward(n, x, B, s);
    if (rc) return rc;
    HIP_CHECK(launch_broadcast(n->out, B, m, d, P, Y, s));
    return FJOFC_OK;
}

namespace {

// Forward, MSE (written to *loss, or added to it with accumulate), backward.
int backward(fjofc_mlp *n, const unsigned short *x, const float *y, int B, double *loss,
             bool accumulate, hipStream_t s) {
    int rc = forward(n, x, B, s);
    if (rc) return rc;
    const int L = n->L;
    int cur = 0;
    HIP_CHECK(launch_transpose16(x, n->dims[0], B, n->dims[0], n->HT[0], n->ldt, s));
    HIP_CHECK(launch_mse(n->out, y, B, n->dims[L], n->Gf[cur], n->Gb[cur], n->GbT[cur], n->ldt,
                         loss, n->scratch, s, accumulate));
    for (int l = L - 1; l >= 0; --l) {
        const int in = n->dims[l], o = n->dims[l + 1];
        // dW_l = h^T g   (in x o), K = B: both operands feature-major
        GemmEpi e{};
        e.outf = n->G + n->offW[l];
        e.ldc = o;
        HIP_CHECK(launch_gemm(GEMM_STORE, in, o, B, n->HT[l], n->ldt, n->GbT[cur], n->ldt, e, s));
        HIP_CHECK(launch_colsum(n->Gf[cur], B, o, n->G + n->offb[l], n->scratch, s));
        if (l > 0) {
            // g' = (g W_l^T) * GELU'(z)   (B x in), K = o; W_l rows are k-contiguous
            GemmEpi eb{};
            eb.outf = n->Gf[cur ^ 1];
            eb.outb = n->Gb[cur ^ 1];
            eb.outbT = n->GbT[cur ^ 1];
            eb.Z = n->Z[l];
            eb.ldc = in;
            eb.ldt = n->ldt;
            HIP_CHECK(launch_gemm(GEMM_BWD, B, in, o, n->Gb[cur], o, n->P16 + n->offW[l], o, eb,
                                  s));
            cur ^= 1;
        }
    }
    return FJOFC_OK;
}

bool adam_args_ok(float lr, float beta1, float beta2, float eps) {
    return lr >= 0.f && beta1 >= 0.f && beta1 < 1.f && beta2 >= 0.f && beta2 < 1.f && eps > 0.f;
}

int adam(fjofc_mlp *n, float lr, float beta1, float beta2, float eps, hipStream_t s) {
    n->step += 1;
    const float c1 = (float)(1.0 - std::pow((double)beta1, n->step));
    const float c2 = (float)(1.0 - std::pow((double)beta2, n->step));
    HIP_CHECK(launch_adam(n->P, n->G, n->M1, n->M2, n->P16, (long)n->nparam, lr, beta1, beta2, eps,
                          c1, c2, s));
    return refresh_wt(n, s);
}

}  // namespace

int fjofc_mlp_backward(fjofc_mlp *n, const unsigned short *x, const float *y, int B, double *loss,
                       void *stream) {
    int rc = check_batch(n, B);
    if (rc) return rc;
    if (!x || !y) return set_error(FJOFC_EINVAL, "NULL argument");
    Dev dg(n->device);
    return backward(n, x, y, B, loss, false, static_cast<hipStream_t>(stream));
}

int fjofc_mlp_train_steps(fjofc_mlp *n, const unsigned short *x, const float *y, int N, int B,
                          int steps, const float *lr, float beta1, float beta2, float eps,
                          double *loss_sum, void *stream) {
    int rc = check_batch(n, B);
    if (rc) return rc;
    if (steps < 0 || N < 0 || (long long)steps * B > N)
        return set_error(FJOFC_EINVAL, "%d steps of %d rows need more than N = %d rows", steps, B,
                         N);
    if (steps == 0) return FJOFC_OK;
    if (!x || !y || !lr) return set_error(FJOFC_EINVAL, "NULL argument");
    if (!adam_args_ok(0.f, beta1, beta2, eps))
        return set_error(FJOFC_EINVAL, "bad Adam hyper-parameters");
    for (int q = 0; q < steps; ++q)
        if (!(lr[q] >= 0.f)) return set_error(FJOFC_EINVAL, "lr[%d] is not >= 0", q);
    Dev dg(n->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int L = n->L;
    for (int q = 0; q < steps; ++q) {
        rc = backward(n, x + (size_t)q * B * n->dims[0], y + (size_t)q * B * n->dims[L], B,
                      loss_sum, true, s);
        if (rc) return rc;
        rc = adam(n, lr[q], beta1, beta2, eps, s);
        if (rc) return rc;
    }
    return FJOFC_OK;
}

int fjofc_mlp_get_grads(fjofc_mlp *n, float *const *dW, float *const *db, void *stream) {
    if (!n || !dW || !db) return set_error(FJOFC_EINVAL, "NULL argument");
    Dev dg(n->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    for (int l = 0; l < n->L; ++l) {
        HIP_CHECK(hipMemcpyAsync(dW[l], n->G + n->offW[l], 4 * (size_t)n->dims[l] * n->dims[l + 1],
                                 hipMemcpyDeviceToDevice, s));
        HIP_CHECK(hipMemcpyAsync(db[l], n->G + n->offb[l], 4 * (size_t)n->dims[l + 1],
                                 hipMemcpyDeviceToDevice, s));
    }
    return FJOFC_OK;
}

int fjofc_mlp_adam(fjofc_mlp *n, float lr, float beta1, float beta2, float eps, void *stream) {
    if (!n) return set_error(FJOFC_EINVAL, "mlp is NULL");
    if (!adam_args_ok(lr, beta1, beta2, eps))
        return set_error(FJOFC_EINVAL, "bad Adam hyper-parameters");
    Dev dg(n->device);
    return adam(n, lr, beta1, beta2, eps, static_cast<hipStream_t>(stream));
}

int fjofc_mlp_features(fjofc_ctx *ctx, const float *delta_new, int k, int m, int n,
                       const int *landmarks, int L, const float *mu, const float *inv_sd,
                       unsigned short *x, void *stream) {
    (void)ctx;
    if (k < 0 || m < 1 || n < 1 || L < 1) return set_error(FJOFC_EINVAL, "bad sizes");
    if (k > 0 && (!delta_new || !landmarks || !mu || !inv_sd || !x))
        return set_error(FJOFC_EINVAL, "NULL argument");
    if (k == 0) return FJOFC_OK;
    HIP_CHECK(launch_features(delta_new, k, m, n, landmarks, L, mu, inv_sd, x,
                              static_cast<hipStream_t>(stream)));
    return FJOFC_OK;
}

int fjofc_mlp_loss(fjofc_mlp *n, const unsigned short *x, const float *y, int B, double *loss,
                   void *stream) {
    int rc = check_batch(n, B);
    if (rc) return rc;
    if (!x || !y || !loss) return set_error(FJOFC_EINVAL, "NULL argument");
    Dev dg(n->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    rc = forward(n, x, B, s);
    if (rc) return rc;
    // the output gradient lands in the network's own scratch buffers; the
    // parameter gradients are untouched
    HIP_CHECK(launch_mse(n->out, y, B, n->dims[n->L], n->Gf[0], n->Gb[0], n->GbT[0], n->ldt,
                         loss, n->scratch, s));
    return FJOFC_OK;
}

int fjofc_mlp_feature_stats(fjofc_ctx *ctx, const float *raw, int N, int F, double min_sd,
                            float *mu, float *inv_sd, void *stream) {
    if (!ctx) return set_error(FJOFC_EINVAL, "ctx is NULL");
    if (N < 1 || F < 1) return set_error(FJOFC_EINVAL, "bad sizes N=%d F=%d", N, F);
    if (!raw || !mu || !inv_sd) return set_error(FJOFC_EINVAL, "NULL argument");
    if (!(min_sd > 0.0) || !std::isfinite(min_sd))
        return set_error(FJOFC_EINVAL, "min_sd must be finite and > 0");
    Dev dg(ctx_device(ctx));
    void *ws = nullptr;
    int rc = ctx_workspace(ctx, sizeof(double) * colstats_scratch_doubles(F), &ws);
    if (rc) return rc;
    HIP_CHECK(launch_colstats(raw, N, F, min_sd, mu, inv_sd, static_cast<double *>(ws),
                              static_cast<hipStream_t>(stream)));
    return FJOFC_OK;
}

int fjofc_oos_consensus(fjofc_ctx *ctx, const float *Y, int k, int m, int d, float *out,
                        void *stream) {
    if (!ctx) return set_error(FJOFC_EINVAL, "ctx is NULL");
    if (k < 0 || m < 1 || d < 1) return set_error(FJOFC_EINVAL, "bad sizes");
    if (k == 0) return FJOFC_OK;
    if (!Y || !out) return set_error(FJOFC_EINVAL, "NULL argument");
    Dev dg(ctx_device(ctx));
    HIP_CHECK(launch_consensus(Y, k, m, d, out, static_cast<hipStream_t>(stream)));
    return FJOFC_OK;
}

}  // extern "C"
