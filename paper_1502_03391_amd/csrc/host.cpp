// Host side of the fast-JOFC C ABI (include/fjofc.h): argument checks, the
// m x m eq:modW matrix and its FP64 inverse (Section 2.1), workspace, and
// the enqueueing of Algorithm 2's loop on the caller's stream.
#include "fjofc.h"
#include "fjofc_internal.h"

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <cstdlib>
#include <map>
#include <tuple>
#include <string>
#include <vector>

using namespace fjofc;

struct fjofc_ctx {
    int device = 0;
    void *ws = nullptr;          // device workspace, grown on demand
    size_t ws_bytes = 0;
    void *pinned = nullptr;      // small pinned host staging buffer
    size_t pinned_bytes = 0;
    std::map<std::tuple<int, int, int>, uint32_t *> tiles;  // (n, th, tw) -> tile list
    // profiling: (kind, start, stop, bytes) per timed launch
    bool prof = false;
    struct Rec {
        int kind;
        hipEvent_t a, b;
        double bytes;
    };
    std::vector<Rec> recs;
    std::vector<hipEvent_t> pool;
};

enum { K_STREAM = 0, K_EDGE, K_FIN, K_RED, K_OOS, K_KINDS };

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIP_TRY(expr)                                                        \
    do {                                                                     \
        hipError_t e_ = (expr);                                              \
        if (e_ != hipSuccess)                                                \
            return fail(FJOFC_EHIP, "%s failed: %s", #expr,                  \
                        hipGetErrorString(e_));                              \
    } while (0)

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) == hipSuccess && prev != dev) (void)hipSetDevice(dev);
        else prev = -1;
    }
    ~DeviceGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

// Sub-allocator over the context workspace (256-byte aligned pieces).
struct Carve {
    size_t off = 0;
    template <class T> size_t take(size_t count) {
        off = (off + 255) & ~size_t(255);
        const size_t at = off;
        off += count * sizeof(T);
        return at;
    }
};

int ensure_ws(fjofc_ctx *c, size_t bytes) {
    if (bytes <= c->ws_bytes) return FJOFC_OK;
    if (c->ws) {
        HIP_TRY(hipDeviceSynchronize());
        HIP_TRY(hipFree(c->ws));
        c->ws = nullptr;
        c->ws_bytes = 0;
    }
    const size_t want = bytes + bytes / 8;
    if (hipMalloc(&c->ws, want) != hipSuccess) {
        c->ws = nullptr;
        return fail(FJOFC_ENOMEM, "workspace allocation of %zu bytes failed", want);
    }
    c->ws_bytes = want;
    return FJOFC_OK;
}

int ensure_pinned(fjofc_ctx *c, size_t bytes) {
    if (bytes <= c->pinned_bytes) return FJOFC_OK;
    if (c->pinned) (void)hipHostFree(c->pinned);
    c->pinned = nullptr;
    c->pinned_bytes = 0;
    if (hipHostMalloc(&c->pinned, bytes, hipHostMallocDefault) != hipSuccess)
        return fail(FJOFC_ENOMEM, "pinned host allocation of %zu bytes failed", bytes);
    c->pinned_bytes = bytes;
    return FJOFC_OK;
}

hipEvent_t take_event(fjofc_ctx *c) {
    if (!c->pool.empty()) {
        hipEvent_t e = c->pool.back();
        c->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Brackets one enqueued operation with events when profiling is on.
struct Timed {
    fjofc_ctx *c;
    int kind;
    double bytes;
    hipStream_t s;
    hipEvent_t a = nullptr;
    Timed(fjofc_ctx *c_, int kind_, double bytes_, hipStream_t s_)
        : c(c_), kind(kind_), bytes(bytes_), s(s_) {
        if (c->prof && (a = take_event(c))) (void)hipEventRecord(a, s);
    }
    ~Timed() {
        if (!a) return;
        hipEvent_t b = take_event(c);
        if (!b) return;
        (void)hipEventRecord(b, s);
        c->recs.push_back({kind, a, b, bytes});
    }
};

// Tile lists of the strict upper triangle: interior tiles (entirely above
// the diagonal and inside n) first, then boundary tiles (crossing the
// diagonal or the ragged edge), each in row-major order.
bool tile_interior(const TriGeom &g, int I, int J) {
    return (I + 1) * g.th <= g.n && (J + 1) * g.tw <= g.n && J * g.tw >= (I + 1) * g.th;
}

int get_tiles(fjofc_ctx *c, TriGeom &g, const uint32_t **out) {
    std::vector<uint32_t> in, bd;
    for (int I = 0; I < g.ntr; ++I)
        for (int J = 0; J < g.ntc; ++J) {
            if (!tile_exists(g, I, J)) continue;
            (tile_interior(g, I, J) ? in : bd).push_back(((uint32_t)I << 16) | (uint32_t)J);
        }
    g.nint = (int)in.size();
    g.nbnd = (int)bd.size();
    const auto key = std::make_tuple(g.n, g.th, g.tw);
    auto it = c->tiles.find(key);
    if (it != c->tiles.end()) {
        *out = it->second;
        return FJOFC_OK;
    }
    in.insert(in.end(), bd.begin(), bd.end());
    uint32_t *d = nullptr;
    HIP_TRY(hipMalloc(&d, std::max<size_t>(1, in.size()) * sizeof(uint32_t)));
    if (!in.empty())
        HIP_TRY(hipMemcpy(d, in.data(), in.size() * sizeof(uint32_t), hipMemcpyHostToDevice));
    c->tiles[key] = d;
    *out = d;
    return FJOFC_OK;
}

// Stream-kernel variants: columns per lane, rows reduced per group, and
// whether the row loads are double-buffered.
struct Variant {
    int cpl, g, dbuf;
};
constexpr Variant kVariants[] = {{4, 8, 1}, {4, 8, 0}, {4, 4, 1}, {8, 4, 1}, {8, 4, 0}, {8, 8, 0}};
constexpr int kNumVariants = sizeof(kVariants) / sizeof(kVariants[0]);

// Tile shape of the in-sample stream: th rows x (64 cpl) columns, and the
// kernel variant.  FJOFC_TILE ("th:variant", e.g. "256:0") overrides the
// default.
void choose_tiles(int n, int d, int &th, int &variant) {
    (void)n;
    (void)d;
    th = 256;
    variant = 5;  // 8 columns per lane, 8 rows per group, single-buffered
    if (const char *e = std::getenv("FJOFC_TILE")) {
        int a = 0, b = 0;
        if (std::sscanf(e, "%d:%d", &a, &b) == 2 && b >= 0 && b < kNumVariants && a >= 8 &&
            a <= 2048 && (a & (a - 1)) == 0) {
            th = a;
            variant = b;
        }
    }
}

// eq:modW: diagonal n w_ii + sum_{j != i} w_ij, off-diagonal -w_ij.
void wmod(int m, int n, const double *w, double *W) {
    for (int i = 0; i < m; ++i) {
        double off = 0.0;
        for (int j = 0; j < m; ++j)
            if (j != i) off += w[i * m + j];
        for (int j = 0; j < m; ++j)
            W[i * m + j] = (i == j) ? n * w[i * m + i] + off : -w[i * m + j];
    }
}

// FP64 inverse by LU-free Gauss-Jordan elimination with partial pivoting.
bool invert(int m, const double *A, double *Ai) {
    std::vector<double> a((size_t)m * 2 * m);
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < 2 * m; ++j)
            a[(size_t)i * 2 * m + j] = j < m ? A[i * m + j] : (j - m == i ? 1.0 : 0.0);
    for (int c = 0; c < m; ++c) {
        int p = c;
        for (int r = c + 1; r < m; ++r)
            if (std::fabs(a[(size_t)r * 2 * m + c]) > std::fabs(a[(size_t)p * 2 * m + c])) p = r;
        const double pv = a[(size_t)p * 2 * m + c];
        if (!(std::fabs(pv) > 0.0)) return false;
        if (p != c)
            for (int j = 0; j < 2 * m; ++j)
                std::swap(a[(size_t)p * 2 * m + j], a[(size_t)c * 2 * m + j]);
        for (int j = 0; j < 2 * m; ++j) a[(size_t)c * 2 * m + j] /= pv;
        for (int r = 0; r < m; ++r) {
            if (r == c) continue;
            const double f = a[(size_t)r * 2 * m + c];
            if (f == 0.0) continue;
            for (int j = 0; j < 2 * m; ++j) a[(size_t)r * 2 * m + j] -= f * a[(size_t)c * 2 * m + j];
        }
    }
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < m; ++j) Ai[i * m + j] = a[(size_t)i * 2 * m + m + j];
    return true;
}

int check_weights(int m, const double *wmat) {
    if (!wmat) return fail(FJOFC_EINVAL, "wmat is NULL");
    for (int i = 0; i < m; ++i) {
        if (!(wmat[i * m + i] > 0.0) || !std::isfinite(wmat[i * m + i]))
            return fail(FJOFC_EINVAL, "fidelity weight w_%d%d must be finite and > 0", i, i);
        for (int k = 0; k < m; ++k) {
            if (k == i) continue;
            const double a = wmat[i * m + k], b = wmat[k * m + i];
            if (!(a >= 0.0) || !std::isfinite(a))
                return fail(FJOFC_EINVAL, "commensurability weight w_%d%d must be finite and >= 0", i, k);
            if (a != b) return fail(FJOFC_EINVAL, "weights must be symmetric (w_%d%d != w_%d%d)", i, k, k, i);
        }
    }
    return FJOFC_OK;
}

TriGeom make_geom(int m, int n, int d, const float *const *delta) {
    TriGeom g;
    g.n = n;
    g.m = m;
    choose_tiles(n, d, g.th, g.variant);
    g.cpl = kVariants[g.variant].cpl;
    g.tw = WAVE * g.cpl;
    const int unit = std::max(g.th, g.tw);
    g.npad = (n + unit - 1) / unit * unit;
    g.ntr = (n + g.th - 1) / g.th;
    g.ntc = (n + g.tw - 1) / g.tw;
    g.nint = g.nbnd = 0;
    bool al = (n % 4) == 0;
    for (int i = 0; i < m; ++i)
        if ((reinterpret_cast<uintptr_t>(delta[i]) & 15) != 0) al = false;
    g.vec4 = al ? 1 : 0;
    return g;
}

struct InWork {
    float *Xs[2];
    float *P;
    double *F, *comP, *hist, *Winv, *wmat;
    EmbedState *st;
    int ncom;
};

int carve_insample(fjofc_ctx *c, const TriGeom &g, int D, int nhist, InWork &w) {
    Carve cv;
    const size_t xs = (size_t)g.m * D * g.npad;
    const int ncom = finalize_blocks(g, D);
    size_t oX0 = cv.take<float>(xs), oX1 = cv.take<float>(xs);
    size_t oP = cv.take<float>(partial_floats(g, D));
    size_t oF = cv.take<double>((size_t)g.m * (g.nint + g.nbnd));
    size_t oC = cv.take<double>(ncom);
    size_t oH = cv.take<double>(nhist);
    size_t oW = cv.take<double>((size_t)g.m * g.m);
    size_t oM = cv.take<double>((size_t)g.m * g.m);
    size_t oS = cv.take<EmbedState>(1);
    int rc = ensure_ws(c, cv.off);
    if (rc) return rc;
    char *b = static_cast<char *>(c->ws);
    w.Xs[0] = reinterpret_cast<float *>(b + oX0);
    w.Xs[1] = reinterpret_cast<float *>(b + oX1);
    w.P = reinterpret_cast<float *>(b + oP);
    w.F = reinterpret_cast<double *>(b + oF);
    w.comP = reinterpret_cast<double *>(b + oC);
    w.hist = reinterpret_cast<double *>(b + oH);
    w.Winv = reinterpret_cast<double *>(b + oW);
    w.wmat = reinterpret_cast<double *>(b + oM);
    w.st = reinterpret_cast<EmbedState *>(b + oS);
    w.ncom = ncom;
    return FJOFC_OK;
}

int check_insample_args(const float *const *delta, int m, int n, int d,
                        const void *X, fjofc_result *res) {
    if (m < 1 || m > FJOFC_MAX_M) return fail(FJOFC_EINVAL, "m=%d outside [1,%d]", m, FJOFC_MAX_M);
    if (n < 2 || n > (1 << 16) * 64) return fail(FJOFC_EINVAL, "n=%d out of range", n);
    if (d < 1 || d > FJOFC_MAX_D) return fail(FJOFC_EINVAL, "d=%d outside [1,%d]", d, FJOFC_MAX_D);
    if (!delta) return fail(FJOFC_EINVAL, "delta is NULL");
    for (int i = 0; i < m; ++i)
        if (!delta[i]) return fail(FJOFC_EINVAL, "delta[%d] is NULL", i);
    if (!X) return fail(FJOFC_EINVAL, "X is NULL");
    if (!res) return fail(FJOFC_EINVAL, "res is NULL");
    return FJOFC_OK;
}

// Runs `iters` transforms (or only the stress of X when iters < 0).
int run_insample(fjofc_ctx *ctx, const float *const *delta, int m, int n,
                 const double *wmat, int d, float *X, int iters, double tol,
                 int tol_mode, int stress_every, double *stress_hist,
                 fjofc_result *res, hipStream_t s) {
    const bool stress_only = iters < 0;
    if (stress_only) iters = 0;
    if (stress_every < 1) return fail(FJOFC_EINVAL, "stress_every must be >= 1");
    if (tol_mode < FJOFC_TOL_NONE || tol_mode > FJOFC_TOL_PAPER)
        return fail(FJOFC_EINVAL, "unknown tol_mode %d", tol_mode);
    if (tol_mode == FJOFC_TOL_NONE) tol = 0.0;
    int rc = check_weights(m, wmat);
    if (rc) return rc;

    std::vector<double> W((size_t)m * m), Wi((size_t)m * m);
    wmod(m, n, wmat, W.data());
    if (!invert(m, W.data(), Wi.data()))
        return fail(FJOFC_ESINGULAR, "eq:modW matrix is singular");

    TriGeom g = make_geom(m, n, d, delta);
    const int D = d;
    DeltaPtrs dp{};
    for (int i = 0; i < m; ++i) dp.p[i] = delta[i];
    const uint32_t *tiles = nullptr;
    rc = get_tiles(ctx, g, &tiles);
    if (rc) return rc;
    InWork w;
    rc = carve_insample(ctx, g, D, iters + 1, w);
    if (rc) return rc;
    rc = ensure_pinned(ctx, sizeof(EmbedState) + sizeof(double) * (size_t)(iters + 1) + 256);
    if (rc) return rc;

    HIP_TRY(hipMemcpyAsync(w.Winv, Wi.data(), sizeof(double) * m * m, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(w.wmat, wmat, sizeof(double) * m * m, hipMemcpyHostToDevice, s));
    HIP_TRY(launch_init_state(w.st, w.hist, iters + 1, s));
    HIP_TRY(launch_to_soa(g, D, X, w.Xs[0], s));
    HIP_TRY(launch_com(g, D, w.Xs[0], w.wmat, w.comP, w.ncom, s));

    // algorithmic bytes of a stream launch: one FP32 read of every
    // strict-upper-triangle entry of each block
    const double pairs_all = (double)g.m * 0.5 * n * (n - 1.0);
    auto stream_pass = [&](const float *Xcur, bool stress, bool acc) -> int {
        Timed tm(ctx, acc ? K_STREAM : K_EDGE, 4.0 * pairs_all, s);
        HIP_TRY(launch_bx(g, D, dp, Xcur, tiles, w.P, w.F, w.st, stress, acc, s));
        return FJOFC_OK;
    };
    for (int p = 0; p < iters; ++p) {
        const bool due = (p % stress_every) == 0;
        rc = stream_pass(w.Xs[p & 1], due, true);
        if (rc) return rc;
        if (due) {
            Timed tm(ctx, K_RED, 0.0, s);
            HIP_TRY(launch_reduce(g, w.F, w.wmat, w.comP, w.ncom, w.st, w.hist, p,
                                  /*check=*/1, /*final=*/0, iters, tol, tol_mode, s));
        }
        const bool next_due = ((p + 1) % stress_every) == 0 || (p + 1) == iters;
        Timed tm(ctx, K_FIN, 0.0, s);
        HIP_TRY(launch_finalize(g, D, w.P, w.Winv, w.wmat, w.Xs[(p + 1) & 1], w.comP,
                                w.ncom, w.st, next_due, s));
    }
    // stress of the returned configuration (and the checkpoint test at
    // t = iters) unless the stop rule already fired.
    rc = stream_pass(w.Xs[iters & 1], true, false);
    if (rc) return rc;
    {
        Timed tm(ctx, K_RED, 0.0, s);
        HIP_TRY(launch_reduce(g, w.F, w.wmat, w.comP, w.ncom, w.st, w.hist, iters,
                              (iters % stress_every) == 0 ? 1 : 0, 1, iters, tol, tol_mode, s));
    }
    if (!stress_only)
        HIP_TRY(launch_from_soa(g, D, w.Xs[0], w.Xs[1], w.st, X, s));

    char *pin = static_cast<char *>(ctx->pinned);
    HIP_TRY(hipMemcpyAsync(pin, w.st, sizeof(EmbedState), hipMemcpyDeviceToHost, s));
    if (stress_hist)
        HIP_TRY(hipMemcpyAsync(pin + 256, w.hist, sizeof(double) * (iters + 1),
                               hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    EmbedState st;
    std::memcpy(&st, pin, sizeof st);
    if (stress_hist) std::memcpy(stress_hist, pin + 256, sizeof(double) * (iters + 1));
    const double mn = (double)m * n;
    res->iters_run = st.iters_run;
    res->converged = st.converged;
    res->stress = st.sigma;
    res->stress_norm = st.sigma / (0.5 * mn * (mn - 1.0));
    res->fidelity = st.fid;
    res->commens = st.com;
    return FJOFC_OK;
}

}  // namespace

extern "C" {

const char *fjofc_last_error(void) { return g_err.c_str(); }

const char *fjofc_strerror(int code) {
    switch (code) {
    case FJOFC_OK: return "ok";
    case FJOFC_EINVAL: return "invalid argument";
    case FJOFC_EHIP: return "HIP runtime error";
    case FJOFC_ENOMEM: return "out of memory";
    case FJOFC_ESINGULAR: return "singular weight matrix";
    default: return "unknown error";
    }
}

int fjofc_create(fjofc_ctx **out, int device) {
    if (!out) return fail(FJOFC_EINVAL, "out is NULL");
    int ndev = 0;
    HIP_TRY(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev)
        return fail(FJOFC_EINVAL, "device %d not present (%d devices)", device, ndev);
    fjofc_ctx *c = new fjofc_ctx();
    c->device = device;
    *out = c;
    return FJOFC_OK;
}

void fjofc_destroy(fjofc_ctx *c) {
    if (!c) return;
    DeviceGuard dg(c->device);
    (void)hipDeviceSynchronize();
    if (c->ws) (void)hipFree(c->ws);
    if (c->pinned) (void)hipHostFree(c->pinned);
    for (auto &kv : c->tiles) (void)hipFree(kv.second);
    for (auto &r : c->recs) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    for (auto e : c->pool) (void)hipEventDestroy(e);
    delete c;
}

int fjofc_embed(fjofc_ctx *ctx, const float *const *delta, int m, int n,
                const double *wmat, int d, float *X, int iters, double tol,
                int tol_mode, int stress_every, double *stress_hist,
                fjofc_result *res, void *stream) {
    if (!ctx) return fail(FJOFC_EINVAL, "ctx is NULL");
    int rc = check_insample_args(delta, m, n, d, X, res);
    if (rc) return rc;
    if (iters < 0) return fail(FJOFC_EINVAL, "iters must be >= 0");
    DeviceGuard dg(ctx->device);
    return run_insample(ctx, delta, m, n, wmat, d, X, iters, tol, tol_mode,
                        stress_every, stress_hist, res,
                        static_cast<hipStream_t>(stream));
}

int fjofc_embed_w(fjofc_ctx *ctx, const float *const *delta, int m, int n,
                  double w, int d, float *X, int iters, double tol,
                  int tol_mode, int stress_every, double *stress_hist,
                  fjofc_result *res, void *stream) {
    if (m < 1 || m > FJOFC_MAX_M) return fail(FJOFC_EINVAL, "m=%d outside [1,%d]", m, FJOFC_MAX_M);
    std::vector<double> wm((size_t)m * m, w);
    for (int i = 0; i < m; ++i) wm[(size_t)i * m + i] = 1.0;
    return fjofc_embed(ctx, delta, m, n, wm.data(), d, X, iters, tol, tol_mode,
                       stress_every, stress_hist, res, stream);
}

int fjofc_stress(fjofc_ctx *ctx, const float *const *delta, int m, int n,
                 const double *wmat, int d, const float *X,
                 fjofc_result *res, void *stream) {
    if (!ctx) return fail(FJOFC_EINVAL, "ctx is NULL");
    int rc = check_insample_args(delta, m, n, d, X, res);
    if (rc) return rc;
    DeviceGuard dg(ctx->device);
    return run_insample(ctx, delta, m, n, wmat, d, const_cast<float *>(X), -1, 0.0,
                        FJOFC_TOL_NONE, 1, nullptr, res,
                        static_cast<hipStream_t>(stream));
}

int fjofc_oos(fjofc_ctx *ctx, const float *X_in, int m, int n, int d,
              const double *wmat, const float *delta_new, int k, float *Y,
              int iters, double tol, const double *target, double *stress_out,
              int *iters_out, int sync, void *stream) {
    if (!ctx) return fail(FJOFC_EINVAL, "ctx is NULL");
    if (m < 1 || m > FJOFC_MAX_M) return fail(FJOFC_EINVAL, "m=%d outside [1,%d]", m, FJOFC_MAX_M);
    if (n < 1) return fail(FJOFC_EINVAL, "n=%d must be >= 1", n);
    if (d < 1 || d > FJOFC_MAX_D) return fail(FJOFC_EINVAL, "d=%d outside [1,%d]", d, FJOFC_MAX_D);
    if (k < 0) return fail(FJOFC_EINVAL, "k=%d must be >= 0", k);
    if (iters < 0) return fail(FJOFC_EINVAL, "iters must be >= 0");
    if (!X_in || (k > 0 && (!delta_new || !Y))) return fail(FJOFC_EINVAL, "NULL array");
    int rc = check_weights(m, wmat);
    if (rc) return rc;
    DeviceGuard dg(ctx->device);
    hipStream_t s = static_cast<hipStream_t>(stream);

    std::vector<double> W((size_t)m * m), Li((size_t)m * m);
    wmod(m, n, wmat, W.data());
    if (!invert(m, W.data(), Li.data()))
        return fail(FJOFC_ESINGULAR, "eq:modW matrix is singular");

    TriGeom g{};
    g.n = n;
    g.m = m;
    g.npad = (n + 255) / 256 * 256;
    Carve cv;
    const size_t oX = cv.take<float>((size_t)m * d * g.npad);
    const size_t oC = cv.take<double>((size_t)m * d);
    const size_t oL = cv.take<double>((size_t)m * m);
    const size_t oW = cv.take<double>((size_t)m * m);
    rc = ensure_ws(ctx, cv.off);
    if (rc) return rc;
    char *b = static_cast<char *>(ctx->ws);
    float *Xs = reinterpret_cast<float *>(b + oX);
    double *colsum = reinterpret_cast<double *>(b + oC);
    double *dLi = reinterpret_cast<double *>(b + oL);
    double *dW = reinterpret_cast<double *>(b + oW);
    HIP_TRY(hipMemcpyAsync(dLi, Li.data(), sizeof(double) * m * m, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(dW, wmat, sizeof(double) * m * m, hipMemcpyHostToDevice, s));
    HIP_TRY(launch_to_soa(g, d, X_in, Xs, s));

    OOSArgs a;
    a.Xs = Xs;
    a.m = m;
    a.n = n;
    a.npad = g.npad;
    a.D = d;
    a.dnew = delta_new;
    a.k = k;
    a.Y = Y;
    a.Linv = dLi;
    a.wmat = dW;
    a.target = target;
    a.stress_out = stress_out;
    a.iters_out = iters_out;
    a.tol = tol;
    a.iters = iters;
    {
        Timed tm(ctx, K_OOS, 4.0 * (double)k * m * n * (iters + 1), s);
        HIP_TRY(launch_oos(a, colsum, s));
    }
    if (sync) HIP_TRY(hipStreamSynchronize(s));
    return FJOFC_OK;
}

int fjofc_profile_enable(fjofc_ctx *ctx, int on) {
    if (!ctx) return fail(FJOFC_EINVAL, "ctx is NULL");
    DeviceGuard dg(ctx->device);
    for (auto &r : ctx->recs) {
        ctx->pool.push_back(r.a);
        ctx->pool.push_back(r.b);
    }
    ctx->recs.clear();
    ctx->prof = on != 0;
    return FJOFC_OK;
}

int fjofc_profile_read(fjofc_ctx *ctx, fjofc_profile *out) {
    if (!ctx || !out) return fail(FJOFC_EINVAL, "NULL argument");
    DeviceGuard dg(ctx->device);
    HIP_TRY(hipDeviceSynchronize());
    int cnt[K_KINDS] = {0};
    double ms[K_KINDS] = {0}, by[K_KINDS] = {0};
    for (auto &r : ctx->recs) {
        float t = 0.f;
        HIP_TRY(hipEventElapsedTime(&t, r.a, r.b));
        cnt[r.kind] += 1;
        ms[r.kind] += t;
        by[r.kind] += r.bytes;
    }
    out->stream_launches = cnt[K_STREAM];
    out->stream_ms = ms[K_STREAM];
    out->stream_bytes = by[K_STREAM];
    out->edge_launches = cnt[K_EDGE];
    out->edge_ms = ms[K_EDGE];
    out->edge_bytes = by[K_EDGE];
    out->finalize_launches = cnt[K_FIN];
    out->finalize_ms = ms[K_FIN];
    out->reduce_launches = cnt[K_RED];
    out->reduce_ms = ms[K_RED];
    out->oos_launches = cnt[K_OOS];
    out->oos_ms = ms[K_OOS];
    out->oos_bytes = by[K_OOS];
    return FJOFC_OK;
}

}  // extern "C"
