// Host side of the fast-JOFC C ABI (include/fjofc.h): argument checks, the
// m x m eq:modW matrix and its FP64 inverse (Section 2.1), workspace, and
// the enqueueing of Algorithm 2's loop on the caller's stream.
#include "fjofc.h"
#include "fjofc_internal.h"
#include "tile_spec.h"

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <cstdlib>
#include <dlfcn.h>
#include <array>
#include <functional>
#include <map>
#include <mutex>
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
    unsigned long long *vslot = nullptr;  // device result of the validation pass
    hipEvent_t chunk_ev[2] = {nullptr, nullptr};  // chunked enqueue of stopping runs
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

// Tile lists of the strict upper triangle: interior tiles (entirely above
// the diagonal and inside n) first, then boundary tiles (crossing the
// diagonal or the ragged edge), each in row-major order.
// No masking needed: every row below n, every column below n, and every
// row below every column.
bool tile_interior(const TriGeom &g, int I, int J) {
    const int c0 = tile_col0(g, I, J);
    return (I + 1) * g.th <= g.n && c0 + g.tw <= g.n && c0 >= (I + 1) * g.th;
}

// Stream-kernel variants: columns per lane, rows reduced per group,
// whether the row loads are double-buffered, and the R x C wavefronts that
// share one tile (each takes th / R rows and 64 cpl columns, so tw =
// 64 cpl C).  Numbering shared with the kernels' dispatch.
struct Variant {
    int cpl, g, dbuf, r, c;
};
constexpr Variant kVariants[] = {{4, 8, 1, 1, 1}, {4, 8, 0, 1, 1}, {8, 4, 0, 1, 1},
                                 {8, 8, 0, 1, 1}, {4, 8, 0, 4, 1}, {4, 8, 0, 2, 2}};
constexpr int kNumVariants = sizeof(kVariants) / sizeof(kVariants[0]);
constexpr int kDefaultVariant = 5;

// Tile shape of the in-sample stream: th rows x (64 cpl) columns and the
// kernel variant.  Order of precedence: FJOFC_TILE, the autotuned cache
// (FJOFC_TUNE_TABLE, else tune_cache.txt next to the library) rows of the
// device's architecture, the built-in default.  The parsing and the row
// choice are in tile_spec.h.

// A tile height is a multiple of the 8-row group of every variant.
bool valid_th(int th) { return th >= 8 && th <= 2048 && th % 8 == 0; }
bool valid_tile(int th, int variant) {
    return valid_th(th) && variant >= 0 && variant < kNumVariants;
}

// The cache, read once per process.
std::vector<TuneRow> &tune_table() {
    static std::vector<TuneRow> rows;
    static std::once_flag once;
    std::call_once(once, [] {
        std::string path;
        if (const char *e = std::getenv("FJOFC_TUNE_TABLE")) {
            path = e;
        } else {
            Dl_info info;
            if (dladdr(reinterpret_cast<void *>(&tune_table), &info) && info.dli_fname) {
                path = info.dli_fname;
                const size_t sl = path.rfind('/');
                path = (sl == std::string::npos ? std::string(".") : path.substr(0, sl)) +
                       "/tune_cache.txt";
            }
        }
        if (FILE *f = path.empty() ? nullptr : std::fopen(path.c_str(), "r")) {
            char line[256];
            TuneRow r;
            while (std::fgets(line, sizeof line, f))
                if (parse_tune_line(line, valid_tile, r)) rows.push_back(r);
            std::fclose(f);
        }
    });
    return rows;
}

// The architecture name of the current device ("gfx950" of
// "gfx950:sramecc+:xnack-"), cached per device.
std::string device_arch() {
    static std::mutex mu;
    static std::map<int, std::string> cache;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return std::string();
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find(dev);
    if (it != cache.end()) return it->second;
    std::string a;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) {
        a = prop.gcnArchName;
        a = a.substr(0, a.find(':'));
    }
    cache[dev] = a;
    return a;
}

void choose_tiles(int n, int d, int &th, int &variant) {
    th = 256;
    variant = kDefaultVariant;
    if (!parse_tile_override(std::getenv("FJOFC_TILE"), n, d, valid_tile, th, variant))
        pick_tune_row(tune_table(), device_arch(), n, d, th, variant);
    // each of the variant's R row slabs holds whole 8-row groups
    const int unit = 8 * kVariants[variant].r;
    th = (th + unit - 1) / unit * unit;
}

// Dynamic LDS of one stream workgroup.  One wavefront: its row-reduction
// buffer [4 D][64].  Several: the row sums [C][D][th], column sums [R][D][tw]
// (which also hold the wavefronts' reduction buffers during the stream) and
// one double per wavefront.
size_t stream_lds(const TriGeom &g, int D) {
    const Variant &v = kVariants[g.variant];
    if (v.r * v.c == 1) return (size_t)4 * D * WAVE * sizeof(float);
    return ((size_t)v.c * g.th + (size_t)v.r * g.tw) * D * sizeof(float) +
           (size_t)v.r * v.c * sizeof(double);
}

int check_problem(const float *const *delta, int m, int n, int d, const void *X) {
    if (m < 1 || m > FJOFC_MAX_M) return fail(FJOFC_EINVAL, "m=%d outside [1,%d]", m, FJOFC_MAX_M);
    if (n < 2 || n > 65535 * 64) return fail(FJOFC_EINVAL, "n=%d out of range", n);
    if (d < 1 || d > FJOFC_MAX_D) return fail(FJOFC_EINVAL, "d=%d outside [1,%d]", d, FJOFC_MAX_D);
    if (!delta) return fail(FJOFC_EINVAL, "delta is NULL");
    for (int i = 0; i < m; ++i)
        if (!delta[i]) return fail(FJOFC_EINVAL, "delta[%d] is NULL", i);
    if (!X) return fail(FJOFC_EINVAL, "X is NULL");
    return FJOFC_OK;
}

// ---- optional validation of the dissimilarities ------------------------
// FJOFC_VALIDATE (any value but "0") runs the pass before every in-sample,
// batched and out-of-sample call.
bool validate_on() {
    const char *e = std::getenv("FJOFC_VALIDATE");
    return e && e[0] && !(e[0] == '0' && e[1] == 0);
}

const char *offence_name(int k) {
    switch (k) {
    case 1: return "is NaN";
    case 2: return "is infinite";
    case 3: return "is negative";
    case 4: return "differs from its mirror entry (Delta must be symmetric)";
    case 5: return "is a non-zero diagonal entry";
    default: return "is invalid";
    }
}

// Reads the validation slot (synchronises s); *code = ~0 when clean.
int read_vslot(fjofc_ctx *c, hipStream_t s, unsigned long long *code) {
    int rc = ensure_pinned(c, 256);
    if (rc) return rc;
    HIP_TRY(hipMemcpyAsync(c->pinned, c->vslot, sizeof(unsigned long long),
                           hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    std::memcpy(code, c->pinned, sizeof *code);
    return FJOFC_OK;
}

int ensure_vslot(fjofc_ctx *c) {
    if (c->vslot) return FJOFC_OK;
    if (hipMalloc(reinterpret_cast<void **>(&c->vslot), 256) != hipSuccess) {
        c->vslot = nullptr;
        return fail(FJOFC_ENOMEM, "validation slot allocation failed");
    }
    return FJOFC_OK;
}

// Checks one n x n matrix; `label` names it in the message.  *where (optional)
// receives the row-major index of the first offending entry, or -1.
int validate_square(fjofc_ctx *c, const float *delta, int n, const char *label,
                    long long *where, hipStream_t s) {
    if (where) *where = -1;
    int rc = ensure_vslot(c);
    if (rc) return rc;
    HIP_TRY(launch_validate_square(delta, n, c->vslot, true, s));
    unsigned long long code = 0;
    rc = read_vslot(c, s, &code);
    if (rc) return rc;
    if (code == ~0ull) return FJOFC_OK;
    const long long idx = (long long)(code >> 3);
    if (where) *where = idx;
    return fail(FJOFC_EINVAL, "%s: entry (%lld, %lld) %s", label, idx / n, idx % n,
                offence_name((int)(code & 7)));
}

int validate_problem(fjofc_ctx *c, const float *const *delta, int m, int n, hipStream_t s) {
    for (int i = 0; i < m; ++i) {
        char label[32];
        std::snprintf(label, sizeof label, "Delta_%d", i);
        const int rc = validate_square(c, delta[i], n, label, nullptr, s);
        if (rc) return rc;
    }
    return FJOFC_OK;
}

// Host-side plan of one in-sample problem: geometry, tile list, W^-1.
struct HostInst {
    TriGeom g{};
    int D = 0;
    DeltaPtrs dp{};
    std::vector<uint32_t> tiles;  // interior then boundary
    std::vector<double> Winv, wmat;
    float *X = nullptr;
    int nhist = 0;
    double alpha = 1.0;
};

int plan_instance(const float *const *delta, int m, int n, const double *wmat, int d,
                  float *X, int nhist, HostInst &h) {
    int rc = check_problem(delta, m, n, d, X);
    if (rc) return rc;
    rc = check_weights(m, wmat);
    if (rc) return rc;
    std::vector<double> W((size_t)m * m);
    h.Winv.assign((size_t)m * m, 0.0);
    h.wmat.assign(wmat, wmat + (size_t)m * m);
    wmod(m, n, wmat, W.data());
    if (!invert(m, W.data(), h.Winv.data()))
        return fail(FJOFC_ESINGULAR, "eq:modW matrix is singular");
    TriGeom &g = h.g;
    g.n = n;
    g.m = m;
    choose_tiles(n, d, g.th, g.variant);
    const Variant &var = kVariants[g.variant];
    g.cpl = var.cpl;
    g.tw = WAVE * var.cpl * var.c;
    // the workgroup's partial sums stay within 64 KB of LDS
    while (stream_lds(g, d) > 65536 && g.th > 8 * var.r) g.th -= 8 * var.r;
    // staggered tiles reach up to column n - 1 + tw; a multiple of th keeps
    // every row block's rows below npad
    const int unit = std::max(g.th, g.tw);
    g.npad = (n + g.tw + unit - 1) / unit * unit;
    if (g.tw < FIN_ROWS || g.npad / FIN_ROWS * FIN_ROWS < n)
        return fail(FJOFC_EINVAL, "internal: row padding %d does not cover n=%d", g.npad, n);
    g.ntr = (n + g.th - 1) / g.th;
    g.ntc = (n + g.tw - 1) / g.tw;
    // a stream item packs its tile as (I << 16) | J
    if (g.ntr > 65535 || g.ntc > 65535)
        return fail(FJOFC_EINVAL, "n=%d needs more than 65535 tile rows or columns of %d x %d",
                    n, g.th, g.tw);
    bool al = (n % 4) == 0;
    for (int i = 0; i < m; ++i)
        if ((reinterpret_cast<uintptr_t>(delta[i]) & 15) != 0) al = false;
    g.vec4 = al ? 1 : 0;
    std::vector<uint32_t> bd;
    h.tiles.clear();
    for (int I = 0; I < g.ntr; ++I)
        for (int J = 0; J < g.ntc; ++J) {
            if (!tile_exists(g, I, J)) continue;
            (tile_interior(g, I, J) ? h.tiles : bd).push_back(((uint32_t)I << 16) | (uint32_t)J);
        }
    g.nint = (int)h.tiles.size();
    g.nbnd = (int)bd.size();
    h.tiles.insert(h.tiles.end(), bd.begin(), bd.end());
    h.D = d;
    for (int i = 0; i < m; ++i) h.dp.p[i] = delta[i];
    h.X = X;
    h.nhist = nhist;
    return FJOFC_OK;
}

// Device buffers of one instance, carved from a workspace.
void carve_instance(Carve &cv, const HostInst &h, size_t offs[9]) {
    const TriGeom &g = h.g;
    const size_t xs = (size_t)g.m * h.D * g.npad;
    offs[0] = cv.take<float>(xs);
    offs[1] = cv.take<float>(xs);
    offs[2] = cv.take<float>(partial_floats(g, h.D));
    offs[3] = cv.take<double>((size_t)g.m * (g.nint + g.nbnd));
    offs[4] = cv.take<double>(commens_blocks(g, h.D));
    offs[5] = cv.take<double>((size_t)g.m * g.m);
    offs[6] = cv.take<double>((size_t)g.m * g.m);
    offs[7] = 0;  // loop states are carved contiguously by the caller
    offs[8] = cv.take<double>(std::max(1, h.nhist));
}

InstDesc make_desc(char *base, const HostInst &h, const size_t offs[9], EmbedState *st) {
    InstDesc d{};
    d.g = h.g;
    d.D = h.D;
    d.ncom = commens_blocks(h.g, h.D);
    d.dp = h.dp;
    d.Xs[0] = reinterpret_cast<float *>(base + offs[0]);
    d.Xs[1] = reinterpret_cast<float *>(base + offs[1]);
    d.P = reinterpret_cast<float *>(base + offs[2]);
    d.F = reinterpret_cast<double *>(base + offs[3]);
    d.comP = reinterpret_cast<double *>(base + offs[4]);
    d.Winv = reinterpret_cast<const double *>(base + offs[5]);
    d.wmat = reinterpret_cast<const double *>(base + offs[6]);
    d.st = st;
    d.hist = h.nhist > 0 ? reinterpret_cast<double *>(base + offs[8]) : nullptr;
    d.X = h.X;
    d.alpha = h.alpha;
    return d;
}

// Work items of one instance.  A boundary tile evaluates every pair of its
// th x tw block plus the masks, so it costs more than an interior tile; on
// its own an instance dispatches its boundary tiles first and lets the
// uniform interior tiles fill the tail of the launch (measured 1.5-4%
// shorter launches at n = 20000).  `bnd` receives the boundary items when
// given: a batch collects them from all its instances and appends them
// after all interior items (the order made no measurable difference there).
void append_items(int inst, const HostInst &h, std::vector<StreamItem> &items,
                  std::vector<StreamItem> *bnd = nullptr) {
    auto boundary = [&](std::vector<StreamItem> &out) {
        for (int i = 0; i < h.g.m; ++i)
            for (int t = h.g.nint; t < (int)h.tiles.size(); ++t)
                out.push_back({inst, i, h.tiles[t], t});
    };
    if (!bnd) boundary(items);
    for (int i = 0; i < h.g.m; ++i)
        for (int t = 0; t < h.g.nint; ++t) items.push_back({inst, i, h.tiles[t], t});
    if (bnd) boundary(*bnd);
}

void append_rows(int inst, const HostInst &h, std::vector<RowItem> &rows) {
    const int nbx = h.g.npad / FIN_ROWS;
    for (int k = 0; k < h.D; ++k)
        for (int bx = 0; bx < nbx; ++bx) rows.push_back({inst, bx, k, 0});
}

void fill_result(const EmbedState &st, int m, int n, fjofc_result *res) {
    const double mn = (double)m * n;
    res->iters_run = st.iters_run;
    res->converged = st.converged;
    res->stress = st.sigma;
    res->stress_norm = st.sigma / (0.5 * mn * (mn - 1.0));
    res->fidelity = st.fid;
    res->commens = st.com;
}

int check_loop_args(int iters, double &tol, int tol_mode, int stress_every) {
    if (iters < 0) return fail(FJOFC_EINVAL, "iters must be >= 0");
    if (stress_every < 1) return fail(FJOFC_EINVAL, "stress_every must be >= 1");
    if (tol_mode < FJOFC_TOL_NONE || tol_mode > FJOFC_TOL_TARGET)
        return fail(FJOFC_EINVAL, "unknown tol_mode %d", tol_mode);
    if (tol_mode == FJOFC_TOL_NONE) tol = 0.0;
    return FJOFC_OK;
}

// One stream launch of a transform: the items of one (D, variant, vec4)
// kernel instance.
struct StreamGroup {
    int D, variant, vec4;
    const StreamItem *items;
    int nitems;
    double bytes;  // algorithmic bytes of one launch
    size_t lds;    // dynamic LDS per workgroup (largest over the group's instances)
    // finalize work of the group's instances (a contiguous range of the
    // row items) and their largest m
    const RowItem *rows;
    int nrows, maxm;
};

// Side streams on which the stream launches of different groups run
// concurrently: group g > 0 runs on side[g - 1], forked from and joined back
// to the main stream with events.  Each instance belongs to one group and
// writes only its own partial sums, so the order of the groups does not
// change any result.
struct Fork {
    std::vector<hipStream_t> side;
    hipEvent_t fork = nullptr;
    std::vector<hipEvent_t> join;
};

// Transforms per enqueued chunk of a run that can stop early (eager runs
// with a stop rule): after every chunk the host reads the device's done
// flag of the chunk before, so at most one chunk is enqueued past a stop.
constexpr int kChunk = 32;

// Finalize launches: a launch of many row items (or one beside other groups'
// streams) takes one thread per row; one of few items (a single large
// problem) takes one thread per slice, which keeps more loads in flight.
// Both give the same bits.
constexpr int kFinOneThreadItems = 2048;

// Called after the transforms [0, p) are enqueued (p a multiple of kChunk,
// p < iters); sets `stop` when no more transforms need enqueueing.
using ChunkHook = std::function<int(int p, bool &stop)>;

// Enqueue Algorithm 2's loop for instances advancing in lockstep.  Used
// eagerly by fjofc_embed and under stream capture by the batched plan
// (which passes `fork` so that its groups become parallel graph branches).
// With `hook`, the loop asks after every kChunk transforms whether to go
// on; the closing stress pass and copy-out are enqueued in any case (they
// are no-ops for stopped instances).
int enqueue_loop(fjofc_ctx *ctx, const InstDesc *insts, int count, int maxm,
                 const std::vector<StreamGroup> &groups, const RowItem *rows, int nrows,
                 int iters, double tol, int tol_mode, int stress_every, int nhist,
                 bool stress_only, hipStream_t s, const Fork *fork = nullptr,
                 const ChunkHook *hook = nullptr) {
    HIP_TRY(launch_init(insts, count, nhist, s));
    HIP_TRY(launch_com(insts, rows, nrows, s));
    const bool forked = fork && groups.size() > 1 && fork->side.size() + 1 >= groups.size();
    // fin_com >= 0: each group's finalize (want_com = fin_com) follows its
    // stream launch on the group's branch
    auto stream_pass = [&](int cur, bool stress, bool acc, int fin_com) -> int {
        if (forked) HIP_TRY(hipEventRecord(fork->fork, s));
        for (size_t q = 0; q < groups.size(); ++q) {
            const StreamGroup &gr = groups[q];
            hipStream_t gs = (forked && q > 0) ? fork->side[q - 1] : s;
            if (gs != s) HIP_TRY(hipStreamWaitEvent(gs, fork->fork, 0));
            Timed tm(ctx, acc ? K_STREAM : K_EDGE, gr.bytes, gs);
            HIP_TRY(launch_stream(gr.D, gr.variant, gr.vec4, insts, gr.items, gr.nitems, cur,
                                  stress, acc, gr.lds, gs));
            if (fin_com >= 0) {
                Timed tf(ctx, K_FIN, 0.0, gs);
                HIP_TRY(launch_finalize(gr.maxm, insts, gr.rows, gr.nrows, cur, fin_com != 0,
                                        true, gs));
            }
        }
        if (forked)
            for (size_t q = 1; q < groups.size(); ++q) {
                HIP_TRY(hipEventRecord(fork->join[q - 1], fork->side[q - 1]));
                HIP_TRY(hipStreamWaitEvent(s, fork->join[q - 1], 0));
            }
        return FJOFC_OK;
    };
    for (int p = 0; p < iters; ++p) {
        const bool due = (p % stress_every) == 0;
        const bool next_due = ((p + 1) % stress_every) == 0 || (p + 1) == iters;
        // A transform without a stress test has nothing that needs every
        // group's stream before the finalize (no stop test can end an
        // instance), so with concurrent groups each group's finalize runs
        // on its own branch and overlaps the other groups' streams.  Rows
        // are independent, so the results do not change.
        const bool branch_fin = forked && !due;
        int rc = stream_pass(p & 1, due, true, branch_fin ? (next_due ? 1 : 0) : -1);
        if (rc) return rc;
        if (branch_fin) continue;
        if (due) {
            Timed tm(ctx, K_RED, 0.0, s);
            HIP_TRY(launch_reduce(insts, count, p, 1, 0, iters, tol, tol_mode, s));
        }
        {
            Timed tm(ctx, K_FIN, 0.0, s);
            HIP_TRY(launch_finalize(maxm, insts, rows, nrows, p & 1, next_due,
                                    nrows >= kFinOneThreadItems, s));
        }
        if (hook && (p + 1) % kChunk == 0 && p + 1 < iters) {
            bool stop = false;
            rc = (*hook)(p + 1, stop);
            if (rc) return rc;
            if (stop) break;
        }
    }
    // stress of the returned configuration (and the checkpoint test at
    // t = iters) unless the stop rule already fired.
    int rc = stream_pass(iters & 1, true, false, -1);
    if (rc) return rc;
    {
        Timed tm(ctx, K_RED, 0.0, s);
        HIP_TRY(launch_reduce(insts, count, iters, (iters % stress_every) == 0 ? 1 : 0, 1, iters,
                              tol, tol_mode, s));
    }
    if (!stress_only) HIP_TRY(launch_copy_out(insts, count, s));
    return FJOFC_OK;
}

// Runs `iters` transforms of one problem (or only the stress of X when
// iters < 0).
int run_insample(fjofc_ctx *ctx, const float *const *delta, int m, int n,
                 const double *wmat, int d, float *X, int iters, double tol,
                 int tol_mode, int stress_every, double alpha, double *stress_hist,
                 fjofc_result *res, hipStream_t s) {
    const bool stress_only = iters < 0;
    if (stress_only) iters = 0;
    int rc = check_loop_args(iters, tol, tol_mode, stress_every);
    if (rc) return rc;
    if (!res) return fail(FJOFC_EINVAL, "res is NULL");
    HostInst h;
    rc = plan_instance(delta, m, n, wmat, d, X, iters + 1, h);
    if (rc) return rc;
    if (validate_on() && (rc = validate_problem(ctx, delta, m, n, s))) return rc;
    h.alpha = alpha;
    std::vector<StreamItem> items;
    std::vector<RowItem> rows;
    append_items(0, h, items);
    append_rows(0, h, rows);

    Carve cv;
    const size_t o_desc = cv.take<InstDesc>(1);
    const size_t o_items = cv.take<StreamItem>(items.size());
    const size_t o_rows = cv.take<RowItem>(rows.size());
    const size_t o_st = cv.take<EmbedState>(1);
    size_t offs[9];
    carve_instance(cv, h, offs);
    rc = ensure_ws(ctx, cv.off);
    if (rc) return rc;
    rc = ensure_pinned(ctx, sizeof(EmbedState) + sizeof(double) * (size_t)(iters + 1) + 256);
    if (rc) return rc;
    char *base = static_cast<char *>(ctx->ws);
    const InstDesc desc = make_desc(base, h, offs, reinterpret_cast<EmbedState *>(base + o_st));
    InstDesc *d_desc = reinterpret_cast<InstDesc *>(base + o_desc);
    StreamItem *d_items = reinterpret_cast<StreamItem *>(base + o_items);
    RowItem *d_rows = reinterpret_cast<RowItem *>(base + o_rows);
    HIP_TRY(hipMemcpyAsync(d_desc, &desc, sizeof desc, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(d_items, items.data(), items.size() * sizeof(StreamItem),
                           hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(d_rows, rows.data(), rows.size() * sizeof(RowItem),
                           hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(const_cast<double *>(desc.Winv), h.Winv.data(),
                           sizeof(double) * m * m, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(const_cast<double *>(desc.wmat), wmat, sizeof(double) * m * m,
                           hipMemcpyHostToDevice, s));
    const double bytes = 4.0 * m * 0.5 * n * (n - 1.0);
    std::vector<StreamGroup> groups{{d, h.g.variant, h.g.vec4, d_items, (int)items.size(), bytes,
                                     stream_lds(h.g, d), d_rows, (int)rows.size(), m}};
    char *pin = static_cast<char *>(ctx->pinned);
    // A run that can stop early is enqueued chunk by chunk: after chunk c
    // the done flag is copied to pinned slot c % 2, and before enqueueing
    // chunk c + 1 the host reads the flag of chunk c - 1, so one chunk is
    // always queued ahead of the check.
    const bool can_stop = tol > 0.0 && tol_mode != FJOFC_TOL_NONE && iters > kChunk;
    int *flag[2] = {reinterpret_cast<int *>(pin + 128), reinterpret_cast<int *>(pin + 192)};
    ChunkHook hook = [&](int p, bool &stop) -> int {
        const int c = p / kChunk - 1;  // the chunk just enqueued
        HIP_TRY(hipMemcpyAsync(flag[c & 1], &desc.st->done, sizeof(int), hipMemcpyDeviceToHost,
                               s));
        HIP_TRY(hipEventRecord(ctx->chunk_ev[c & 1], s));
        if (c >= 1) {
            HIP_TRY(hipEventSynchronize(ctx->chunk_ev[(c - 1) & 1]));
            stop = *flag[(c - 1) & 1] != 0;
        }
        return FJOFC_OK;
    };
    if (can_stop)
        for (hipEvent_t &e : ctx->chunk_ev)
            if (!e) HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    rc = enqueue_loop(ctx, d_desc, 1, m, groups, d_rows, (int)rows.size(), iters, tol, tol_mode,
                      stress_every, iters + 1, stress_only, s, nullptr, can_stop ? &hook : nullptr);
    if (rc) return rc;

    HIP_TRY(hipMemcpyAsync(pin, desc.st, sizeof(EmbedState), hipMemcpyDeviceToHost, s));
    if (stress_hist)
        HIP_TRY(hipMemcpyAsync(pin + 256, desc.hist, sizeof(double) * (iters + 1),
                               hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    EmbedState st;
    std::memcpy(&st, pin, sizeof st);
    if (stress_hist) std::memcpy(stress_hist, pin + 256, sizeof(double) * (iters + 1));
    fill_result(st, m, n, res);
    return FJOFC_OK;
}

}  // namespace

fjofc::Timed::Timed(fjofc_ctx *c_, int kind_, double bytes_, hipStream_t s_)
    : c(c_), kind(kind_), bytes(bytes_), s(s_) {
    if (c->prof && (a = take_event(c))) (void)hipEventRecord(a, s);
}

fjofc::Timed::~Timed() {
    if (!a) return;
    hipEvent_t b = take_event(c);
    if (!b) return;
    (void)hipEventRecord(b, s);
    c->recs.push_back({kind, a, b, bytes});
}

int fjofc::ctx_device(const fjofc_ctx *ctx) { return ctx->device; }

int fjofc::ctx_workspace(fjofc_ctx *ctx, size_t bytes, void **ws) {
    const int rc = ensure_ws(ctx, bytes);
    if (rc) return rc;
    *ws = ctx->ws;
    return FJOFC_OK;
}

int fjofc::ctx_pinned(fjofc_ctx *ctx, size_t bytes, void **p) {
    const int rc = ensure_pinned(ctx, bytes);
    if (rc) return rc;
    *p = ctx->pinned;
    return FJOFC_OK;
}

int fjofc::set_error(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

// A batch of independent in-sample problems advanced in lockstep; the whole
// loop is captured once into a HIP graph on a library-owned stream and
// replayed by every fjofc_batch_run with the same loop parameters.
struct fjofc_batch {
    fjofc_ctx *ctx = nullptr;
    int count = 0, maxm = 0;
    std::vector<HostInst> hi;
    void *mem = nullptr;
    size_t bytes = 0;
    InstDesc *d_insts = nullptr;
    std::vector<StreamGroup> groups;
    RowItem *d_rows = nullptr;
    int nrows = 0;
    hipStream_t cs = nullptr;
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    Fork fork;  // side streams for the concurrent stream groups
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int key_iters = -1, key_every = -1, key_mode = -1;
    double key_tol = -1.0;
    EmbedState *pinned = nullptr;
    EmbedState *d_st = nullptr;
    // persistent launch: planned when every problem's tile variant is one the
    // persistent kernel runs (persist_ok); chosen with fjofc_batch_set_launch
    // (persist).  The default is the lockstep graph of per-group launches.
    bool persist_ok = false, persist = false;
    int maxd = 0, pgrid = 0;
    size_t plds = 0;
    BatchArgs pargs{};
    int *pin_err = nullptr;  // pinned copy of the error flag
};

namespace {

void batch_free(fjofc_batch *b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->ev_in) (void)hipEventDestroy(b->ev_in);
    if (b->ev_out) (void)hipEventDestroy(b->ev_out);
    if (b->cs) (void)hipStreamDestroy(b->cs);
    for (hipStream_t st : b->fork.side) (void)hipStreamDestroy(st);
    for (hipEvent_t ev : b->fork.join) (void)hipEventDestroy(ev);
    if (b->fork.fork) (void)hipEventDestroy(b->fork.fork);
    if (b->mem) (void)hipFree(b->mem);
    if (b->pinned) (void)hipHostFree(b->pinned);
    if (b->pin_err) (void)hipHostFree(b->pin_err);
    delete b;
}

}  // namespace

// ---- scratch of the allocation-free out-of-sample call ----------------
// A file-scope device array: each GPU the library runs on holds its own
// copy until the process ends.  Host code never uses the array's name as a
// device address; the address is taken once per device with
// hipGetSymbolAddress (fjofc_create, with that device current) and kept in
// g_scratch.  Every allocation-free call on a GPU shares that GPU's array,
// so such calls that overlap on one GPU race.
constexpr size_t kNoAllocBytes = size_t(4) << 20;
constexpr int kNoAllocMaxM = 8;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch[kMaxDevices] = {};

// Takes the scratch address of `dev`, which must be the current device.
int init_noalloc_scratch(int dev) {
    if (dev < 0 || dev >= kMaxDevices) return fail(FJOFC_EINVAL, "device %d out of range", dev);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch[dev]) return FJOFC_OK;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
        return fail(FJOFC_EHIP, "hipGetSymbolAddress(scratch) failed on device %d: %s", dev,
                    hipGetErrorString(e));
    g_scratch[dev] = p;
    return FJOFC_OK;
}

int noalloc_scratch(int dev, void **p) {
    if (dev < 0 || dev >= kMaxDevices) return fail(FJOFC_EINVAL, "device %d out of range", dev);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    *p = g_scratch[dev];
    if (!*p) return fail(FJOFC_EINVAL, "scratch of device %d not set up (fjofc_create)", dev);
    return FJOFC_OK;
}

// W^-1 and the weights of a problem with m <= kNoAllocMaxM, passed by value.
struct SmallMats {
    double a[kNoAllocMaxM * kNoAllocMaxM];
    double b[kNoAllocMaxM * kNoAllocMaxM];
    int count;
};

__global__ void noalloc_mats_kernel(SmallMats mats, double *__restrict__ a,
                                    double *__restrict__ b) {
    for (int q = threadIdx.x; q < mats.count; q += blockDim.x) {
        a[q] = mats.a[q];
        b[q] = mats.b[q];
    }
}

// fjofc_oos and its allocation-free variant.  With `noalloc` the SoA copy
// of X_in, the column sums and the two m x m matrices live in the
// module-scope scratch array (reached through its per-device address), the
// matrices travel as a kernel argument, and nothing is allocated, timed or
// validated.
int oos_run(fjofc_ctx *ctx, const float *X_in, int m, int n, int d, const double *wmat,
            const float *delta_new, int k, float *Y, int iters, double tol,
            const double *target, double *stress_out, int *iters_out, int sync, void *stream,
            bool noalloc) {
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
    if (noalloc && m > kNoAllocMaxM)
        return fail(FJOFC_EINVAL, "m=%d: the allocation-free call takes m <= %d", m,
                    kNoAllocMaxM);
    if (!noalloc && validate_on() && k > 0) {
        rc = ensure_vslot(ctx);
        if (rc) return rc;
        HIP_TRY(launch_validate_rows(delta_new, (long long)k * m * n, ctx->vslot, true, s));
        unsigned long long code = 0;
        rc = read_vslot(ctx, s, &code);
        if (rc) return rc;
        if (code != ~0ull) {
            const long long idx = (long long)(code >> 3), row = idx / n;
            return fail(FJOFC_EINVAL, "delta_new: object %lld, modality %lld, entry %lld %s",
                        row / m, row % m, idx % n, offence_name((int)(code & 7)));
        }
    }

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
    char *b = nullptr;
    if (noalloc) {
        if (cv.off > kNoAllocBytes)
            return fail(FJOFC_EINVAL,
                        "m=%d, n=%d, d=%d needs %zu bytes of scratch; the allocation-free call "
                        "has %zu (m d npad <= about %zu floats, npad = n rounded up to 256)",
                        m, n, d, cv.off, kNoAllocBytes, kNoAllocBytes / 4);
        void *sp = nullptr;
        rc = noalloc_scratch(ctx->device, &sp);
        if (rc) return rc;
        b = static_cast<char *>(sp);
    } else {
        rc = ensure_ws(ctx, cv.off);
        if (rc) return rc;
        b = static_cast<char *>(ctx->ws);
    }
    float *Xs = reinterpret_cast<float *>(b + oX);
    double *colsum = reinterpret_cast<double *>(b + oC);
    double *dLi = reinterpret_cast<double *>(b + oL);
    double *dW = reinterpret_cast<double *>(b + oW);
    if (noalloc) {
        SmallMats mats{};
        for (int q = 0; q < m * m; ++q) {
            mats.a[q] = Li[q];
            mats.b[q] = wmat[q];
        }
        mats.count = m * m;
        noalloc_mats_kernel<<<1, 64, 0, s>>>(mats, dLi, dW);
        HIP_TRY(hipGetLastError());
    } else {
        HIP_TRY(hipMemcpyAsync(dLi, Li.data(), sizeof(double) * m * m, hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(dW, wmat, sizeof(double) * m * m, hipMemcpyHostToDevice, s));
    }
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
    a.ob = 0;  // the default objects per workgroup
    a.vec4 = (n % 4 == 0 && (reinterpret_cast<uintptr_t>(delta_new) & 15) == 0 &&
              !std::getenv("FJOFC_OOS_SCALAR")) ? 1 : 0;
    if (noalloc) {
        HIP_TRY(launch_oos(a, colsum, s));
    } else {
        Timed tm(ctx, K_OOS, 4.0 * (double)k * m * n * (iters + 1), s);
        HIP_TRY(launch_oos(a, colsum, s));
    }
    if (sync) HIP_TRY(hipStreamSynchronize(s));
    return FJOFC_OK;
}

}  // namespace

namespace {

// The persistent batch as one captured sequence: X0 to SoA and the loop
// state (init), the commensurability of X0, the queue reset, the persistent
// launch, and the copy of the results back to the callers' layout.
int enqueue_persistent(fjofc_batch *b, int iters, double tol, int tol_mode, int stress_every) {
    hipStream_t s = b->cs;
    BatchArgs a = b->pargs;
    a.ntasks = batch_periods(iters) * a.L;
    a.iters = iters;
    a.every = stress_every;
    a.tol = tol;
    a.tol_mode = tol_mode;
    // wall-clock ticks a dependency wait may last (FJOFC_BATCH_TIMEOUT_MS,
    // default 5000 ms); FJOFC_BATCH_FORCE_WAIT makes the first task wait on
    // a counter no task increments (a test of the timeout path)
    int khz = 0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, b->ctx->device) != hipSuccess ||
        khz <= 0)
        khz = 100000;
    double ms = 5000.0;
    if (const char *e = std::getenv("FJOFC_BATCH_TIMEOUT_MS")) ms = std::max(0.0, std::atof(e));
    a.timeout = (long long)(ms * khz);
    const char *fw = std::getenv("FJOFC_BATCH_FORCE_WAIT");
    a.never_wait = (fw && fw[0] && fw[0] != '0') ? 1 : 0;
    HIP_TRY(launch_init(b->d_insts, b->count, 0, s));
    HIP_TRY(launch_com(b->d_insts, b->d_rows, b->nrows, s));
    HIP_TRY(launch_batch_reset(a, b->count, s));
    HIP_TRY(launch_batch_persistent(a, b->maxd, b->maxm, b->pgrid, b->plds, s));
    HIP_TRY(launch_copy_out(b->d_insts, b->count, s));
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
    {
        DeviceGuard dg(device);
        const int rc = init_noalloc_scratch(device);
        if (rc) return rc;
    }
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
    if (c->vslot) (void)hipFree(c->vslot);
    for (hipEvent_t e : c->chunk_ev)
        if (e) (void)hipEventDestroy(e);
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
    return fjofc_embed_relaxed(ctx, delta, m, n, wmat, d, X, iters, tol, tol_mode, stress_every,
                               1.0, stress_hist, res, stream);
}

int fjofc_embed_relaxed(fjofc_ctx *ctx, const float *const *delta, int m, int n,
                        const double *wmat, int d, float *X, int iters, double tol,
                        int tol_mode, int stress_every, double alpha, double *stress_hist,
                        fjofc_result *res, void *stream) {
    if (!ctx) return fail(FJOFC_EINVAL, "ctx is NULL");
    if (iters < 0) return fail(FJOFC_EINVAL, "iters must be >= 0");
    if (!(alpha > 0.0 && alpha < 2.0)) return fail(FJOFC_EINVAL, "alpha=%g outside (0, 2)", alpha);
    DeviceGuard dg(ctx->device);
    return run_insample(ctx, delta, m, n, wmat, d, X, iters, tol, tol_mode,
                        stress_every, alpha, stress_hist, res,
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
    DeviceGuard dg(ctx->device);
    return run_insample(ctx, delta, m, n, wmat, d, const_cast<float *>(X), -1, 0.0,
                        FJOFC_TOL_NONE, 1, 1.0, nullptr, res,
                        static_cast<hipStream_t>(stream));
}

int fjofc_oos(fjofc_ctx *ctx, const float *X_in, int m, int n, int d,
              const double *wmat, const float *delta_new, int k, float *Y,
              int iters, double tol, const double *target, double *stress_out,
              int *iters_out, int sync, void *stream) {
    return oos_run(ctx, X_in, m, n, d, wmat, delta_new, k, Y, iters, tol, target, stress_out,
                   iters_out, sync, stream, false);
}

int fjofc_oos_noalloc(fjofc_ctx *ctx, const float *X_in, int m, int n, int d,
                      const double *wmat, const float *delta_new, int k, float *Y,
                      int iters, double tol, const double *target, double *stress_out,
                      int *iters_out, int sync, void *stream) {
    return oos_run(ctx, X_in, m, n, d, wmat, delta_new, k, Y, iters, tol, target, stress_out,
                   iters_out, sync, stream, true);
}

int fjofc_oos_nearest_start(fjofc_ctx *ctx, const float *X_in, int m, int n, int d,
                            const float *delta_new, int k, float *Y, void *stream) {
    if (!ctx) return fail(FJOFC_EINVAL, "ctx is NULL");
    if (m < 1 || m > FJOFC_MAX_M) return fail(FJOFC_EINVAL, "m=%d outside [1,%d]", m, FJOFC_MAX_M);
    if (n < 1) return fail(FJOFC_EINVAL, "n=%d must be >= 1", n);
    if (d < 1 || d > FJOFC_MAX_D) return fail(FJOFC_EINVAL, "d=%d outside [1,%d]", d, FJOFC_MAX_D);
    if (k < 0) return fail(FJOFC_EINVAL, "k=%d must be >= 0", k);
    if (k > 0 && (!X_in || !delta_new || !Y)) return fail(FJOFC_EINVAL, "NULL array");
    DeviceGuard dg(ctx->device);
    HIP_TRY(launch_nearest(X_in, m, n, d, delta_new, k, Y, static_cast<hipStream_t>(stream)));
    return FJOFC_OK;
}

int fjofc_validate_delta(fjofc_ctx *ctx, const float *delta, int n, long long *where,
                         void *stream) {
    if (where) *where = -1;
    if (!ctx) return fail(FJOFC_EINVAL, "ctx is NULL");
    if (n < 1 || n > 65535 * 64) return fail(FJOFC_EINVAL, "n=%d out of range", n);
    if (!delta) return fail(FJOFC_EINVAL, "delta is NULL");
    DeviceGuard dg(ctx->device);
    return validate_square(ctx, delta, n, "Delta", where, static_cast<hipStream_t>(stream));
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
    out->batch_launches = cnt[K_BATCH];
    out->batch_ms = ms[K_BATCH];
    out->batch_bytes = by[K_BATCH];
    out->init_launches = cnt[K_INIT];
    out->init_ms = ms[K_INIT];
    out->init_bytes = by[K_INIT];
    return FJOFC_OK;
}


int fjofc_batch_create(fjofc_ctx *ctx, const fjofc_problem *probs, int count,
                       fjofc_batch **out) {
    if (!ctx || !probs || !out) return fail(FJOFC_EINVAL, "NULL argument");
    if (count < 1) return fail(FJOFC_EINVAL, "count must be >= 1");
    DeviceGuard dg(ctx->device);
    fjofc_batch *b = new fjofc_batch();
    b->ctx = ctx;
    b->count = count;
    b->hi.resize(count);
    for (int p = 0; p < count; ++p) {
        const fjofc_problem &q = probs[p];
        int rc = plan_instance(q.delta, q.m, q.n, q.wmat, q.d, q.X, 0, b->hi[p]);
        if (!rc && validate_on()) rc = validate_problem(ctx, q.delta, q.m, q.n, nullptr);
        if (rc) {
            batch_free(b);
            return fail(rc, "problem %d: %s", p, g_err.c_str());
        }
        b->maxm = std::max(b->maxm, q.m);
    }
    std::map<std::tuple<int, int, int>, std::vector<StreamItem>> gitems, gbnd;
    std::map<std::tuple<int, int, int>, double> gbytes;
    std::map<std::tuple<int, int, int>, size_t> glds;
    std::map<std::tuple<int, int, int>, std::vector<int>> ginst;
    std::vector<RowItem> rows;
    // largest problems first within each group: long items start early
    std::vector<int> order(count);
    for (int p = 0; p < count; ++p) order[p] = p;
    std::stable_sort(order.begin(), order.end(), [&](int a, int c) {
        return (double)b->hi[a].g.m * b->hi[a].g.n * b->hi[a].g.n >
               (double)b->hi[c].g.m * b->hi[c].g.n * b->hi[c].g.n;
    });
    for (int p : order) {
        const HostInst &h = b->hi[p];
        const auto key = std::make_tuple(h.D, h.g.variant, h.g.vec4);
        append_items(p, h, gitems[key], &gbnd[key]);
        gbytes[key] += 4.0 * h.g.m * 0.5 * h.g.n * (h.g.n - 1.0);
        glds[key] = std::max(glds[key], stream_lds(h.g, h.D));
        ginst[key].push_back(p);
    }
    for (auto &kv : gitems) kv.second.insert(kv.second.end(), gbnd[kv.first].begin(), gbnd[kv.first].end());
    // row items grouped like the stream items, so each group's finalize
    // work is one contiguous range
    std::map<std::tuple<int, int, int>, std::array<int, 3>> grows;  // offset, count, max m
    for (auto &kv : ginst) {
        std::sort(kv.second.begin(), kv.second.end());
        std::array<int, 3> r{(int)rows.size(), 0, 0};
        for (int p : kv.second) {
            append_rows(p, b->hi[p], rows);
            r[2] = std::max(r[2], b->hi[p].g.m);
        }
        r[1] = (int)rows.size() - r[0];
        grows[kv.first] = r;
    }
    // Persistent plan: per problem (largest first) its stream tasks (groups
    // of one-wavefront or shared tiles) and finalize tasks (groups of row
    // items), arranged by batch_template.
    b->persist_ok = true;
    for (int p = 0; p < count; ++p) {
        if (!batch_variant_ok(b->hi[p].g.variant)) b->persist_ok = false;
        b->maxd = std::max(b->maxd, b->hi[p].D);
    }
    std::vector<StreamItem> pitems;
    std::vector<RowItem> prows;
    std::vector<std::vector<BatchTask>> tstream(count), tfin(count);
    std::vector<int> nst(count, 0), nfin(count, 0);
    if (b->persist_ok) {
        for (int p : order) {
            const HostInst &h = b->hi[p];
            std::vector<StreamItem> its;
            append_items(p, h, its);
            const int per = h.g.variant <= 1 ? BATCH_TILES_1W : BATCH_TILES_SHARED;
            for (size_t q = 0; q < its.size(); q += per) {
                const int cnt = (int)std::min<size_t>(per, its.size() - q);
                tstream[p].push_back({BT_STREAM, p, (int)(pitems.size() + q), cnt, 0});
            }
            nst[p] = (int)its.size();
            pitems.insert(pitems.end(), its.begin(), its.end());
            std::vector<RowItem> rs;
            append_rows(p, h, rs);
            for (size_t q = 0; q < rs.size(); q += BATCH_ROWS) {
                const int cnt = (int)std::min<size_t>(BATCH_ROWS, rs.size() - q);
                tfin[p].push_back({BT_FIN, p, (int)(prows.size() + q), cnt, 0});
            }
            nfin[p] = (int)rs.size();
            prows.insert(prows.end(), rs.begin(), rs.end());
            b->plds = std::max(b->plds, batch_stream_lds(h.D, h.g.variant, stream_lds(h.g, h.D)));
        }
        int ncu = 0;
        if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, ctx->device) !=
            hipSuccess)
            ncu = 0;
        const int per_cu = batch_resident_blocks(b->maxd, b->maxm, b->plds);
        b->pgrid = per_cu * ncu;
        if (b->pgrid < 1) b->persist_ok = false;
    }
    const std::vector<BatchTask> tmpl =
        b->persist_ok ? batch_template(order, tstream, tfin) : std::vector<BatchTask>();

    Carve cv;
    const size_t o_insts = cv.take<InstDesc>(count);
    const size_t o_st = cv.take<EmbedState>(count);
    const size_t o_tmpl = cv.take<BatchTask>(std::max<size_t>(1, tmpl.size()));
    const size_t o_pitems = cv.take<StreamItem>(std::max<size_t>(1, pitems.size()));
    const size_t o_prows = cv.take<RowItem>(std::max<size_t>(1, prows.size()));
    const size_t o_ctr = cv.take<BatchCtr>(count);
    const size_t o_flags = cv.take<long long>(4);  // head, err, never
    std::vector<size_t> o_groups;
    for (auto &kv : gitems) o_groups.push_back(cv.take<StreamItem>(kv.second.size()));
    const size_t o_rows = cv.take<RowItem>(rows.size());
    std::vector<std::array<size_t, 9>> offs(count);
    for (int p = 0; p < count; ++p) carve_instance(cv, b->hi[p], offs[p].data());
    if (hipMalloc(&b->mem, cv.off) != hipSuccess) {
        b->mem = nullptr;
        batch_free(b);
        return fail(FJOFC_ENOMEM, "batch workspace of %zu bytes", cv.off);
    }
    b->bytes = cv.off;
    char *base = static_cast<char *>(b->mem);
    b->d_insts = reinterpret_cast<InstDesc *>(base + o_insts);
    EmbedState *d_st = reinterpret_cast<EmbedState *>(base + o_st);
    b->d_st = d_st;
    std::vector<InstDesc> descs(count);
    int rc = FJOFC_OK;
    auto copy = [&](void *dst, const void *src, size_t nb) {
        if (!rc && nb && hipMemcpy(dst, src, nb, hipMemcpyHostToDevice) != hipSuccess)
            rc = fail(FJOFC_EHIP, "batch descriptor upload failed");
    };
    for (int p = 0; p < count; ++p) {
        descs[p] = make_desc(base, b->hi[p], offs[p].data(), d_st + p);
        descs[p].bnst = nst[p];
        descs[p].bnfin = nfin[p];
        copy(const_cast<double *>(descs[p].Winv), b->hi[p].Winv.data(),
             sizeof(double) * b->hi[p].Winv.size());
        copy(const_cast<double *>(descs[p].wmat), b->hi[p].wmat.data(),
             sizeof(double) * b->hi[p].wmat.size());
    }
    copy(b->d_insts, descs.data(), sizeof(InstDesc) * count);
    b->d_rows = reinterpret_cast<RowItem *>(base + o_rows);
    size_t gi = 0;
    for (auto &kv : gitems) {
        StreamItem *d = reinterpret_cast<StreamItem *>(base + o_groups[gi++]);
        copy(d, kv.second.data(), kv.second.size() * sizeof(StreamItem));
        const std::array<int, 3> &r = grows[kv.first];
        b->groups.push_back({std::get<0>(kv.first), std::get<1>(kv.first), std::get<2>(kv.first),
                             d, (int)kv.second.size(), gbytes[kv.first], glds[kv.first],
                             b->d_rows + r[0], r[1], r[2]});
    }
    b->nrows = (int)rows.size();
    copy(b->d_rows, rows.data(), rows.size() * sizeof(RowItem));
    if (b->persist_ok) {
        BatchArgs &a = b->pargs;
        a.insts = b->d_insts;
        a.items = reinterpret_cast<const StreamItem *>(base + o_pitems);
        a.rows = reinterpret_cast<const RowItem *>(base + o_prows);
        a.tmpl = reinterpret_cast<const BatchTask *>(base + o_tmpl);
        a.L = (int)tmpl.size();
        a.ctr = reinterpret_cast<BatchCtr *>(base + o_ctr);
        long long *flags = reinterpret_cast<long long *>(base + o_flags);
        a.head = reinterpret_cast<int *>(flags);
        a.err = reinterpret_cast<int *>(flags + 1);
        a.never = reinterpret_cast<int *>(flags + 2);
        copy(base + o_tmpl, tmpl.data(), tmpl.size() * sizeof(BatchTask));
        copy(base + o_pitems, pitems.data(), pitems.size() * sizeof(StreamItem));
        copy(base + o_prows, prows.data(), prows.size() * sizeof(RowItem));
        if (!rc && hipHostMalloc(reinterpret_cast<void **>(&b->pin_err), 256,
                                 hipHostMallocDefault) != hipSuccess) {
            b->pin_err = nullptr;
            rc = fail(FJOFC_ENOMEM, "pinned batch flag");
        }
    }
    if (!rc && (hipStreamCreate(&b->cs) != hipSuccess ||
                hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming) != hipSuccess ||
                hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming) != hipSuccess))
        rc = fail(FJOFC_EHIP, "batch stream/event creation failed");
    // one side stream (default priority) and join event per extra group
    if (!rc && b->groups.size() > 1) {
        if (hipEventCreateWithFlags(&b->fork.fork, hipEventDisableTiming) != hipSuccess)
            rc = fail(FJOFC_EHIP, "batch event creation failed");
        for (size_t q = 1; !rc && q < b->groups.size(); ++q) {
            hipStream_t st = nullptr;
            hipEvent_t ev = nullptr;
            if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
                rc = fail(FJOFC_EHIP, "batch side stream creation failed");
                break;
            }
            b->fork.side.push_back(st);
            if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
                rc = fail(FJOFC_EHIP, "batch event creation failed");
                break;
            }
            b->fork.join.push_back(ev);
        }
    }
    if (!rc && hipHostMalloc(reinterpret_cast<void **>(&b->pinned), sizeof(EmbedState) * count,
                             hipHostMallocDefault) != hipSuccess) {
        b->pinned = nullptr;
        rc = fail(FJOFC_ENOMEM, "pinned batch results");
    }
    if (rc) {
        batch_free(b);
        return rc;
    }
    *out = b;
    return FJOFC_OK;
}

int fjofc_batch_run(fjofc_batch *b, int iters, double tol, int tol_mode, int stress_every,
                    fjofc_result *res, void *stream) {
    if (!b) return fail(FJOFC_EINVAL, "batch is NULL");
    int rc = check_loop_args(iters, tol, tol_mode, stress_every);
    if (rc) return rc;
    fjofc_ctx *ctx = b->ctx;
    DeviceGuard dg(ctx->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (!b->exec || b->key_iters != iters || b->key_every != stress_every ||
        b->key_mode != tol_mode || b->key_tol != tol) {
        if (b->exec) (void)hipGraphExecDestroy(b->exec);
        if (b->graph) (void)hipGraphDestroy(b->graph);
        b->exec = nullptr;
        b->graph = nullptr;
        const bool prof = ctx->prof;
        ctx->prof = false;  // no event records inside the captured graph
        HIP_TRY(hipStreamBeginCapture(b->cs, hipStreamCaptureModeThreadLocal));
        if (b->persist)
            rc = enqueue_persistent(b, iters, tol, tol_mode, stress_every);
        else
            rc = enqueue_loop(ctx, b->d_insts, b->count, b->maxm, b->groups, b->d_rows, b->nrows,
                              iters, tol, tol_mode, stress_every, 0, false, b->cs, &b->fork);
        const hipError_t ec = hipStreamEndCapture(b->cs, &b->graph);
        ctx->prof = prof;
        if (rc) return rc;
        if (ec != hipSuccess) return fail(FJOFC_EHIP, "graph capture failed: %s", hipGetErrorString(ec));
        HIP_TRY(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
        b->key_iters = iters;
        b->key_every = stress_every;
        b->key_mode = tol_mode;
        b->key_tol = tol;
    }
    HIP_TRY(hipEventRecord(b->ev_in, s));
    HIP_TRY(hipStreamWaitEvent(b->cs, b->ev_in, 0));
    {
        double bytes = 0.0;
        for (const StreamGroup &gr : b->groups) bytes += gr.bytes;
        Timed tm(ctx, K_BATCH, bytes * iters, b->cs);
        HIP_TRY(hipGraphLaunch(b->exec, b->cs));
    }
    HIP_TRY(hipEventRecord(b->ev_out, b->cs));
    HIP_TRY(hipStreamWaitEvent(s, b->ev_out, 0));
    if (b->persist) {
        // a dependency wait that timed out (workgroups not all resident, or
        // the host-forced wait test) ends the launch early: report it
        HIP_TRY(hipMemcpyAsync(b->pin_err, b->pargs.err, sizeof(int), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (*b->pin_err)
            return fail(FJOFC_EHIP,
                        "persistent batch: a dependency wait timed out (all %d workgroups must "
                        "be resident at once); the results are incomplete",
                        b->pgrid);
    }
    if (res) {
        HIP_TRY(hipMemcpyAsync(b->pinned, b->d_st, sizeof(EmbedState) * b->count,
                               hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        for (int p = 0; p < b->count; ++p)
            fill_result(b->pinned[p], b->hi[p].g.m, b->hi[p].g.n, res + p);
    }
    return FJOFC_OK;
}

int fjofc_embed_batched(fjofc_ctx *ctx, const fjofc_problem *probs, int count, int iters,
                        double tol, int tol_mode, int stress_every, fjofc_result *res,
                        void *stream) {
    fjofc_batch *b = nullptr;
    int rc = fjofc_batch_create(ctx, probs, count, &b);
    if (rc) return rc;
    rc = fjofc_batch_run(b, iters, tol, tol_mode, stress_every, res, stream);
    if (!res) (void)hipStreamSynchronize(static_cast<hipStream_t>(stream));
    fjofc_batch_destroy(b);
    return rc;
}

int fjofc_tile_choice(fjofc_ctx *ctx, int n, int d, int *tile_height, int *variant) {
    if (!ctx || !tile_height || !variant) return fail(FJOFC_EINVAL, "NULL argument");
    if (n < 2 || d < 1 || d > FJOFC_MAX_D) return fail(FJOFC_EINVAL, "n=%d, d=%d", n, d);
    DeviceGuard dg(ctx->device);
    choose_tiles(n, d, *tile_height, *variant);
    return FJOFC_OK;
}

int fjofc_batch_set_launch(fjofc_batch *b, int launch) {
    if (!b) return fail(FJOFC_EINVAL, "batch is NULL");
    if (launch != FJOFC_LAUNCH_LOCKSTEP && launch != FJOFC_LAUNCH_PERSISTENT)
        return fail(FJOFC_EINVAL, "unknown batch launch %d", launch);
    const bool want = launch == FJOFC_LAUNCH_PERSISTENT;
    if (want && !b->persist_ok)
        return fail(FJOFC_EINVAL,
                    "the persistent launch does not run this batch (a tile shape it has no "
                    "variant for, or no workgroup fits a CU)");
    if (want != b->persist) {
        // the captured graph belongs to the other launch: capture again
        DeviceGuard dg(b->ctx->device);
        (void)hipStreamSynchronize(b->cs);
        if (b->exec) (void)hipGraphExecDestroy(b->exec);
        if (b->graph) (void)hipGraphDestroy(b->graph);
        b->exec = nullptr;
        b->graph = nullptr;
        b->persist = want;
    }
    return FJOFC_OK;
}

void fjofc_batch_destroy(fjofc_batch *b) {
    if (!b) return;
    DeviceGuard dg(b->ctx->device);
    (void)hipStreamSynchronize(b->cs);
    batch_free(b);
}

}  // extern "C"
