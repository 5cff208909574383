// libgeninv C ABI: context, workspace and the orchestration of the method's
// steps on one HIP stream (declarations and contracts in include/geninv.h).
#include <algorithm>
#include <cmath>
#include <limits>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <string>
#include <mutex>
#include <numeric>
#include <vector>

#include "common.h"
#include "geninv.h"

using namespace geninv;

// Kernel classes for the optional event timers (geninv_prof_*).
enum ProfClass {
    PC_GRAM, PC_TOL, PC_FILL, PC_TRAILING, PC_PANEL_FACTOR, PC_LTL, PC_INV_PANEL, PC_INV_UPDATE,
    PC_MIRROR, PC_CHAIN_K, PC_CHAIN_P, PC_CHAIN_Y, PC_LSTSQ, PC_GEMM, PC_SLICE, PC_NS, PC_BATCHED, PC_COUNT
};
static const char *const kProfNames[PC_COUNT] = {
    "gram", "tol", "fill", "trailing_update", "panel_factor", "ltl", "inv_panel", "inv_update",
    "mirror", "chain_k", "chain_p", "chain_y", "lstsq_apply", "gemm", "slice", "newton_schulz", "batched"};

struct ProfState {
    unsigned mask = 0;
    struct Pending { int cls; hipEvent_t a, b; double flops; };
    std::vector<hipEvent_t> pool;
    std::vector<Pending> pending;
    double ms[PC_COUNT] = {};
    long cnt[PC_COUNT] = {};
    double fl[PC_COUNT] = {};
};

struct geninv_batch_plan;

namespace geninv {
// debug.hip
hipError_t launch_poison(void *p, size_t bytes, hipStream_t s);
// spdinv.hip: negate and mirror the lower triangle left by the sweeps
hipError_t launch_gj_finish(double *X, long ldx, Dim n, hipStream_t s);
// skinny.hip
int skinny_padded_width(int N);
hipError_t launch_skinny_gemm(const double *A, long lda, const double *B, long ldb, int transB, int M, int N, int K,
                              double alpha, double beta, double *C, long ldc, int kchunk, double *Bt, double *part,
                              hipStream_t s);
hipError_t launch_skinny_gemm_t(const double *A, long lda, const double *B, long ldb, int M, int N, int K,
                                double alpha, double beta, double *C, long ldc, int kchunk, double *part,
                                hipStream_t s);
}  // namespace geninv

// Fixed device scratch area of geninv_dlstsq_noalloc, for callers that
// cannot allocate.  Each device holds its own copy from module load until the
// process ends; host code reaches it only through the address
// hipGetSymbolAddress returns for the current device (kept per device in
// g_scratch and in each context), never through the array's name.
constexpr size_t NOALLOC_BYTES = size_t(256) << 20;
static __device__ __align__(256) char scratch[NOALLOC_BYTES];
constexpr int NOALLOC_MAX_DEVICES = 64;
static char *g_scratch[NOALLOC_MAX_DEVICES] = {};
static std::mutex g_scratch_mu;

struct geninv_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    // a second stream (default priority) for the Cholesky's trailing updates,
    // joined to `stream` by events within each call
    hipStream_t aux = nullptr;
    hipEvent_t ev_fact = nullptr, ev_rest[2] = {nullptr, nullptr}, ev_join = nullptr;
    char *ws = nullptr;
    size_t ws_bytes = 0;
    int *status = nullptr;     // device status word (separate from the workspace: survives regrowth)
    int host_sync = 1;         // read the rank back after the factorization (geninv_set_host_sync)
    int *hpin = nullptr;       // pinned host word for that read-back
    char *scratch = nullptr;   // this device's address of the fixed scratch area
    size_t ws_limit = 0;       // workspace cap in bytes, 0 = none (geninv_set_workspace_limit)
    int debug = 0;             // GENINV_DEBUG_POISON: NaN-fill every new workspace
    ProfState prof;
};

namespace {

constexpr int PART_S = 16;     // maximum split-K factor

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

#define HIPCHK(x)                                  \
    do {                                           \
        hipError_t e_ = (x);                       \
        if (e_ != hipSuccess) return GENINV_EHIP;  \
    } while (0)

#define CHK(x)                   \
    do {                         \
        int s_ = (x);            \
        if (s_ != GENINV_OK) return s_; \
    } while (0)

inline size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

// Records a pair of events on the context stream around the launches of one
// class when that class is enabled; the elapsed times are summed on read.
struct ProfScope {
    geninv_ctx *c;
    int cls;
    double flops;
    hipEvent_t a = nullptr;
    ProfScope(geninv_ctx *ctx, int k, double f) : c(ctx), cls(k), flops(f) {
        if (!((c->prof.mask >> cls) & 1u)) return;
        a = take();
        if (a) (void)hipEventRecord(a, c->stream);
    }
    ~ProfScope() {
        if (!a) return;
        hipEvent_t b = take();
        if (!b) return;
        (void)hipEventRecord(b, c->stream);
        c->prof.pending.push_back({cls, a, b, flops});
    }
    hipEvent_t take() {
        if (!c->prof.pool.empty()) {
            hipEvent_t e = c->prof.pool.back();
            c->prof.pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        return e;
    }
};

void prof_resolve(geninv_ctx *c) {
    for (auto &p : c->prof.pending) {
        float ms = 0.f;
        if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
            c->prof.ms[p.cls] += ms;
            c->prof.cnt[p.cls] += 1;
            c->prof.fl[p.cls] += p.flops;
        }
        c->prof.pool.push_back(p.a);
        c->prof.pool.push_back(p.b);
    }
    c->prof.pending.clear();
}

// Workspace carve-up for a problem whose factored dimension is nn (the
// smaller of m, n) with k right-hand sides.
struct Layout {
    size_t slotA, slotL, slotK, slotP, part, lpan, dbuf, rrow, ccol, dvals, tol, rank, piv, t0, t1, t2, gpart, total;
    int gram_splits;   // split-K factor of the float64 Gram matrix (partials in gpart)
    size_t split_elems;   // doubles in gpart: the Gram's partials, then those of the later products
    size_t part_elems;    // doubles in part
};

constexpr size_t GPART_MAX_BYTES = size_t(2) << 30;   // bound on the Gram's split-K partials

long lower_tiles128(int nn) {
    const long t = (nn + 127) / 128;
    return t * (t + 1) / 2;
}

// kdim: depth of the float64 Gram product (0 when the call forms none)
Layout make_layout(int nn, int k, int kdim = 0) {
    Layout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += align256(bytes);
        return o;
    };
    const size_t n2 = (size_t)nn * nn * sizeof(double);
    L.slotA = take(n2);
    L.slotL = take(n2);
    L.slotK = take(n2);
    L.slotP = take(n2);
    L.part_elems = (size_t)PART_S * nn * std::max(FR_NB, k);
    L.part = take(L.part_elems * sizeof(double));
    L.lpan = take((size_t)2 * nn * FR_NB * sizeof(double));   // two panels: see run_frchol
    L.dbuf = take((size_t)GJ_NB * GJ_NB * sizeof(double));
    L.rrow = take((size_t)GJ_NB * nn * sizeof(double));
    L.ccol = take((size_t)nn * GJ_NB * sizeof(double));
    L.dvals = take((size_t)nn * sizeof(double));
    L.tol = take(sizeof(double));
    L.rank = take((size_t)(nn / FR_NB + 2) * sizeof(int));
    L.piv = take((size_t)std::max(nn, 1) * sizeof(int));
    L.t0 = take((size_t)nn * std::max(k, 1) * sizeof(double));
    L.t1 = take((size_t)nn * std::max(k, 1) * sizeof(double));
    L.t2 = take((size_t)nn * std::max(k, 1) * sizeof(double));
    L.gram_splits = 1;
    L.gpart = 0;
    L.split_elems = 0;
    size_t gbytes = 0;
    if (kdim > 0 && nn > 0) {
        const int cap = (int)std::max<size_t>(1, std::min<size_t>(16, GPART_MAX_BYTES / n2));
        L.gram_splits = choose_splits(lower_tiles128(nn), kdim, cap);
        if (L.gram_splits > 1) gbytes = L.gram_splits * n2;
    }
    // the products after the factorization (L'L, L M, K K') reuse the area
    // for their own split-K partials, up to 8 n x n layers
    const size_t cbytes = nn >= 512 ? std::min<size_t>(GPART_MAX_BYTES, 8 * n2) : 0;
    if (std::max(gbytes, cbytes) > 0) {
        L.gpart = take(std::max(gbytes, cbytes));
        L.split_elems = std::max(gbytes, cbytes) / sizeof(double);
    }
    L.total = off;
    return L;
}

int ensure_ws(geninv_ctx *c, size_t bytes) {
    if (c->ws_limit && bytes > c->ws_limit) return GENINV_ENOMEM;
    if (bytes <= c->ws_bytes) return GENINV_OK;
    if (c->ws) {
        HIPCHK(hipStreamSynchronize(c->stream));
        HIPCHK(hipFree(c->ws));
        c->ws = nullptr;
        c->ws_bytes = 0;
    }
    void *p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return GENINV_ENOMEM;
    }
    c->ws = static_cast<char *>(p);
    c->ws_bytes = bytes;
    if (c->debug & GENINV_DEBUG_POISON) HIPCHK(launch_poison(c->ws, c->ws_bytes, c->stream));
    return GENINV_OK;
}

template <class T>
T *at(geninv_ctx *c, size_t off) { return reinterpret_cast<T *>(c->ws + off); }

GemmArgs gemm(const double *A, long lda, int tA, const double *B, long ldb, int tB, double *C, long ldc, Dim M,
              Dim N, Dim K, double alpha, double beta, int uplo = GEMM_FULL) {
    GemmArgs g{};
    g.A = A; g.lda = lda; g.transA = tA;
    g.B = B; g.ldb = ldb; g.transB = tB;
    g.C = C; g.ldc = ldc;
    g.M = M; g.N = N; g.K = K;
    g.alpha = alpha; g.beta = beta;
    g.uplo = uplo;
    g.splitk = 1;
    g.strideC = 0;
    g.onelevel = 0;
    return g;
}

// The chain's products (K = L M, P = K K', Y = P G'): their rounding is not
// amplified by a later inversion, so one running sum over K suffices (the
// Gram matrix and L'L keep the two-level sum).
GemmArgs chain(GemmArgs g) {
    g.onelevel = 1;
    return g;
}

// C (M x N) = op(A) op(B) with split-K through the partial buffer when the
// output has too few tiles to fill the chip.
int gemm_splitk(geninv_ctx *c, const Layout &lay, GemmArgs g, int min_tiles = 256) {
    const int tiles = ((g.M.host + 63) / 64) * ((g.N.host + 63) / 64);
    int S = 1;
    // about 1024 workgroups (several fit on a compute unit: these launches
    // are bound by load latency), at least 256 of K each, within `part`
    if (tiles < min_tiles && g.K.host >= 512) {
        S = (int)std::min<long>({64L, (1024 + tiles - 1) / tiles, (long)g.K.host / 256});
        while (S > 1 && (size_t)S * g.M.host * g.N.host > lay.part_elems) --S;
    }
    if (S <= 1) {
        HIPCHK(launch_dgemm(g, c->stream));
        return GENINV_OK;
    }
    double *part = at<double>(c, lay.part);
    const double alpha = g.alpha, beta = g.beta;
    double *C = g.C;
    const long ldc = g.ldc;
    GemmArgs p = g;
    p.C = part;
    p.ldc = g.M.host;
    p.splitk = S;
    p.strideC = (long)g.M.host * g.N.host;
    HIPCHK(launch_dgemm(p, c->stream));
    HIPCHK(launch_splitk_reduce(part, g.M.host, p.strideC, S, C, ldc, g.M, g.N, alpha, beta, g.uplo, c->stream));
    return GENINV_OK;
}

// C = op(A) op(B) for a product with host-known sizes after the
// factorization.  When its 128 x 128 tiles alone would leave compute units
// idle, K is split so that the 128 x 128 direct-to-LDS kernel runs full
// rounds; the partials go to gpart and are summed in a fixed order.
// Otherwise (or with a rank read from device memory) one launch.
int gemm_fill(geninv_ctx *c, const Layout &lay, GemmArgs g) {
    const long M = g.M.host, N = g.N.host;
    const int K = g.K.host;
    const bool host = !g.M.dev && !g.N.dev && !g.K.dev;
    if (!host || M <= 0 || N <= 0 || lay.split_elems == 0 || (g.uplo == GEMM_LOWER && M != N)) {
        HIPCHK(launch_dgemm(g, c->stream));
        return GENINV_OK;
    }
    const long tiles = g.uplo == GEMM_LOWER ? lower_tiles128((int)M) : ((M + 127) / 128) * ((N + 127) / 128);
    const int cap = (int)std::min<size_t>(64, lay.split_elems / (size_t)(M * N));
    // too few tiles for one round: the cheapest split that fills it; else a
    // split only where the cost model gains on the partly idle last round
    // (L'L of order 3072: 300 tiles run 2 rounds, the second one 17 % full)
    const int S = tiles >= 256 ? choose_splits(tiles, K, cap) : fill_splits(tiles, K, cap);
    if (S < 2) {
        HIPCHK(launch_dgemm(g, c->stream));
        return GENINV_OK;
    }
    double *part = at<double>(c, lay.gpart);
    GemmArgs p = g;
    p.C = part;
    p.ldc = M;
    p.splitk = S;
    p.strideC = M * N;
    HIPCHK(launch_dgemm(p, c->stream));
    HIPCHK(launch_splitk_reduce(part, M, M * N, S, g.C, g.ldc, g.M, g.N, g.alpha, g.beta, g.uplo, c->stream));
    return GENINV_OK;
}

// Step 1: lower triangle of A = op(G)' op(G) (nn x nn, ld nn) into slotA.
// The lower triangle has few 128 x 128 tiles for its depth (kdim = m), so K is
// split (choose_splits: whole rounds of 256 workgroups) with the partial
// Grams in gpart, then summed in a fixed order.
int run_gram(geninv_ctx *c, const Layout &lay, const double *G, long ldg, bool tr, int nn, int kdim) {
    double *A = at<double>(c, lay.slotA);
    GemmArgs g = tr ? gemm(G, ldg, 0, G, ldg, 1, A, nn, hdim(nn), hdim(nn), hdim(kdim), 1.0, 0.0, GEMM_LOWER)
                    : gemm(G, ldg, 1, G, ldg, 0, A, nn, hdim(nn), hdim(nn), hdim(kdim), 1.0, 0.0, GEMM_LOWER);
    ProfScope ps(c, PC_GRAM, (double)kdim * nn * (nn + 1.0));
    const int S = lay.gram_splits;
    if (S <= 1) {
        HIPCHK(launch_dgemm(g, c->stream));
        return GENINV_OK;
    }
    const long stride = (long)nn * nn;
    g.C = at<double>(c, lay.gpart);
    g.ldc = nn;
    g.splitk = S;
    g.strideC = stride;
    HIPCHK(launch_dgemm(g, c->stream));
    HIPCHK(launch_splitk_reduce(g.C, nn, stride, S, A, nn, hdim(nn), hdim(nn), 1.0, 0.0, GEMM_LOWER, c->stream));
    return GENINV_OK;
}

// Steps 2-3: tolerance and full-rank Cholesky of the lower triangle of A
// (nn x nn), right-looking: after panel p is factored, its new columns
// (uncompacted in lpan, zero where a column was dropped) are subtracted
// from the lower triangle of the trailing matrix in place,
//   A[k1:, k1:] -= Lp[k1:, :w] Lp[k1:, :w]'   (k1 = k0 + w),
// an MFMA product of depth w with host-known sizes, so that every later
// panel arrives fully updated.  The zero columns of dropped pivots add
// nothing.  L (nn x nn, ldl) is zeroed and receives the compacted factor.
int run_frchol(geninv_ctx *c, const Layout &lay, double *A, long lda, int nn, double user_tol, double *L,
               long ldl, int *piv, double *dvals) {
    double *tolp = at<double>(c, lay.tol);
    int *rank_buf = at<int>(c, lay.rank);
    double *Lp = at<double>(c, lay.lpan);
    const int np = (nn + FR_NB - 1) / FR_NB;
    {
        ProfScope ps(c, PC_TOL, 0.0);
        HIPCHK(launch_tol(A, lda, nn, user_tol, tolp, c->status, c->stream));
    }
    {
        ProfScope ps(c, PC_FILL, 0.0);
        HIPCHK(launch_fill(L, ldl, nn, nn, 0.0, c->stream));
        HIPCHK(launch_fill_int(rank_buf, np + 1, 0, c->stream));
    }
    // Without per-class timing (which records events on the call's stream
    // only) and outside stream capture, the trailing update of panel p runs on the second stream, beside
    // the next panel's own column update and factorization: panel p's
    // contribution to the next panel's columns goes first on the call's
    // stream, and the rest of the trailing matrix (columns from the panel
    // after next) on the second stream, which the following column update
    // waits for (both write those columns).  The two streams touch disjoint
    // columns meanwhile; the panel buffers alternate, so a factorization does
    // not overwrite the panel that an update in flight still reads.
    // (a stream being captured into a graph keeps the single-stream form)
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (c->stream && hipStreamIsCapturing(c->stream, &cap) != hipSuccess) {
        (void)hipGetLastError();
        cap = hipStreamCaptureStatusActive;
    }
    const bool overlap = c->aux && c->prof.mask == 0 && np > 2 && cap == hipStreamCaptureStatusNone;
    for (int p = 0; p < np; ++p) {
        const int k0 = p * FR_NB;
        const int w = std::min(FR_NB, nn - k0);
        double *panel = A + k0 + (long)k0 * lda;
        double *Lpp = overlap ? Lp + (long)(p & 1) * nn * FR_NB : Lp;
        {
            ProfScope ps(c, PC_PANEL_FACTOR, 0.0);
            HIPCHK(launch_frchol_panel(panel, lda, L, ldl, rank_buf, p, k0, w, nn, tolp, piv, dvals, Lpp, nn,
                                       c->stream));
        }
        const int k1 = k0 + w;
        const int rows = nn - k1;
        if (rows <= 0) continue;
        if (!overlap) {
            ProfScope ps(c, PC_TRAILING, 2.0 * rows * (rows + 1.0) / 2.0 * w);
            HIPCHK(launch_dgemm(gemm(Lpp + k1, nn, 0, Lpp + k1, nn, 1, A + k1 + (long)k1 * lda, lda, hdim(rows),
                                     hdim(rows), hdim(w), -1.0, 1.0, GEMM_LOWER),
                                c->stream));
            continue;
        }
        const int w2 = std::min(FR_NB, rows), k2 = k1 + w2, rest = nn - k2;
        if (rest > 0) {
            HIPCHK(hipEventRecord(c->ev_fact, c->stream));
            HIPCHK(hipStreamWaitEvent(c->aux, c->ev_fact, 0));
            HIPCHK(launch_dgemm(gemm(Lpp + k2, nn, 0, Lpp + k2, nn, 1, A + k2 + (long)k2 * lda, lda, hdim(rest),
                                     hdim(rest), hdim(w), -1.0, 1.0, GEMM_LOWER),
                                c->aux));
            HIPCHK(hipEventRecord(c->ev_rest[p & 1], c->aux));
        }
        // the previous panel's rest update also wrote these columns
        if (p > 0) HIPCHK(hipStreamWaitEvent(c->stream, c->ev_rest[(p - 1) & 1], 0));
        HIPCHK(launch_dgemm(gemm(Lpp + k1, nn, 0, Lpp + k1, nn, 1, A + k1 + (long)k1 * lda, lda, hdim(rows),
                                 hdim(w2), hdim(w), -1.0, 1.0, GEMM_FULL),
                            c->stream));
    }
    if (overlap) {
        HIPCHK(hipEventRecord(c->ev_join, c->aux));
        HIPCHK(hipStreamWaitEvent(c->stream, c->ev_join, 0));
    }
    return GENINV_OK;
}

// M = B^-1 in place (B r x r symmetric, ldb; the sweeps read the lower block
// triangle and the diagonal blocks in full), r on device (bound rb).
int run_spdinv(geninv_ctx *c, const Layout &lay, double *B, long ldb, Dim r) {
    double *D = at<double>(c, lay.dbuf);
    double *R = at<double>(c, lay.rrow);
    double *Cc = at<double>(c, lay.ccol);
    const int nbk = (r.host + GJ_NB - 1) / GJ_NB;
    for (int b = 0; b < nbk; ++b) {
        {
            ProfScope ps(c, PC_INV_PANEL, 0.0);
            HIPCHK(launch_gj_panel(B, ldb, r, b, D, R, Cc, c->status, c->stream));
        }
        ProfScope ps(c, PC_INV_UPDATE, 0.0);
        HIPCHK(launch_gj_update(B, ldb, r, b, D, R, Cc, c->stream));
    }
    ProfScope ps(c, PC_MIRROR, 0.0);
    HIPCHK(launch_gj_finish(B, ldb, r, c->stream));
    return GENINV_OK;
}

// B = L'L (r x r, full) into dst; then M = B^-1 in place.
int run_factor_inverse(geninv_ctx *c, const Layout &lay, const double *L, long ldl, int nn, Dim r, double *dst,
                       long ldd) {
    GemmArgs g = gemm(L, ldl, 1, L, ldl, 0, dst, ldd, r, r, hdim(nn), 1.0, 0.0, GEMM_LOWER);
    {
        ProfScope ps(c, PC_LTL, 0.0);
        CHK(gemm_fill(c, lay, g));
    }
    {
        ProfScope ps(c, PC_MIRROR, 0.0);
        HIPCHK(launch_mirror_lower(dst, ldd, r, c->stream));
    }
    return run_spdinv(c, lay, dst, ldd, r);
}

// The rank after the factorization as a launch dimension.  With host
// synchronization on (the default) it is copied to the host, one stream
// synchronization, and every later launch is sized for it exactly: no
// Gauss-Jordan step, tile or GEMM block past r is launched.  With it off the
// later kernels are launched for the bound nn and read r from device memory
// (no host synchronization inside the call, e.g. for stream capture).
int rank_dim(geninv_ctx *c, int nn, const int *rdev, Dim *out) {
    if (!c->host_sync) {
        *out = ddim(nn, rdev);
        return GENINV_OK;
    }
    HIPCHK(hipMemcpyAsync(c->hpin, rdev, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    const int r = *c->hpin;
    if (r < 0 || r > nn) return GENINV_EHIP;
    *out = hdim(r);
    return GENINV_OK;
}

int finish_rank(geninv_ctx *c, const int *rdev, int *rank) {
    if (!rank) return GENINV_OK;
    int st = 0;
    HIPCHK(hipMemcpyAsync(rank, rdev, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipMemcpyAsync(&st, c->status, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    if (st != 0) {
        int zero = 0;
        HIPCHK(hipMemcpy(c->status, &zero, sizeof(int), hipMemcpyHostToDevice));
    }
    return st;
}

bool bad_ld(long ld, int rows) { return ld < std::max(1, rows); }

// Step 5's last product for a rank under half the order (rank known on the
// host): Y = K (K' G'), or (G' K) K' in the transpose branch, 4 nn r m flops
// instead of the nn(nn+1) r + 2 nn^2 m of forming P = K K' first; equal to
// L M M L' G' in exact arithmetic (Theorem 1).  The r-row intermediate goes
// through the P slot (nn x nn elements) in blocks of Y's columns (rows in the
// transpose branch).
bool lowrank_chain(int nn, Dim r) { return !r.dev && r.host > 0 && 2 * r.host < nn; }

int run_chain_lowrank(geninv_ctx *c, const Layout &lay, const double *K, long ld, int nn, int r, const double *G,
                      long ldg, bool tr, int n, int m, double *Y, long ldy) {
    double *Z = at<double>(c, lay.slotP);
    const long cap = (long)nn * nn;
    const int other = tr ? n : m;            // Y's long dimension
    long blk = std::min<long>(other, cap / r);
    if (blk > 128) blk -= blk % 128;
    for (long j0 = 0; j0 < other; j0 += blk) {
        const int w = (int)std::min<long>(blk, other - j0);
        if (!tr) {
            // Z (r x w) = K' G(j0:j0+w, :)', then Y(:, j0:j0+w) = K Z
            CHK(gemm_fill(c, lay, chain(gemm(K, ld, 1, G + j0, ldg, 1, Z, r, hdim(r), hdim(w), hdim(nn), 1.0, 0.0))));
            CHK(gemm_fill(c, lay,
                          chain(gemm(K, ld, 0, Z, r, 0, Y + j0 * ldy, ldy, hdim(nn), hdim(w), hdim(r), 1.0, 0.0))));
        } else {
            // Z (w x r) = G(:, j0:j0+w)' K, then Y(j0:j0+w, :) = Z K'
            CHK(gemm_fill(c, lay,
                          chain(gemm(G + j0 * ldg, ldg, 1, K, ld, 0, Z, w, hdim(w), hdim(r), hdim(nn), 1.0, 0.0))));
            CHK(gemm_fill(c, lay, chain(gemm(Z, w, 0, K, ld, 1, Y + j0, ldy, hdim(w), hdim(nn), hdim(r), 1.0, 0.0))));
        }
    }
    return GENINV_OK;
}

// ---- mixed precision (sliced bfloat16 products) --------------------------

inline long pad64(long x) { return (x + 63) / 64 * 64; }

struct MixedLayout {
    size_t gc, gt, pc, ecg, erg, ep, gram, gpart, total;
    size_t gpart_elems;
};

SlicedGemmArgs sliced(const __bf16 *A, long lda, long sa, const __bf16 *B, long ldb, long sb, int S, const int *ea,
                      const int *eb, double *C, long ldc, int M, int N, int Kpad, int lower);
int sliced_splits(const SlicedGemmArgs &g, int maxS);

// extra workspace of the mixed form, placed after the float64 layout
MixedLayout make_mixed_layout(size_t base, int m, int n, int s, int sy, bool keep_gram) {
    MixedLayout L{};
    size_t off = base;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += align256(bytes);
        return o;
    };
    L.gc = take((size_t)s * pad64(m) * n * sizeof(__bf16));
    L.gt = take((size_t)sy * pad64(n) * m * sizeof(__bf16));
    L.pc = take((size_t)sy * pad64(n) * n * sizeof(__bf16));
    L.ecg = take((size_t)n * sizeof(int));
    L.erg = take((size_t)m * sizeof(int));
    L.ep = take((size_t)n * sizeof(int));
    L.gram = keep_gram ? take((size_t)n * n * sizeof(double)) : 0;
    // split-K partials of the sliced Gram matrix
    {
        SlicedGemmArgs g = sliced(nullptr, 0, 0, nullptr, 0, 0, s, nullptr, nullptr, nullptr, 0, n, n,
                                  (int)pad64(m), 1);
        const size_t n2 = (size_t)n * n;
        const int cap = (int)std::max<size_t>(1, std::min<size_t>(16, GPART_MAX_BYTES / (n2 * sizeof(double))));
        const int S = sliced_splits(g, cap);
        L.gpart_elems = S > 1 ? S * n2 : 0;
        L.gpart = S > 1 ? take(L.gpart_elems * sizeof(double)) : 0;
    }
    L.total = off;
    return L;
}

SlicedGemmArgs sliced(const __bf16 *A, long lda, long sa, const __bf16 *B, long ldb, long sb, int S, const int *ea,
                      const int *eb, double *C, long ldc, int M, int N, int Kpad, int lower) {
    SlicedGemmArgs g{};
    g.A = A; g.lda = lda; g.sa = sa;
    g.B = B; g.ldb = ldb; g.sb = sb;
    g.ea = ea; g.eb = eb;
    g.C = C; g.ldc = ldc;
    g.M = M; g.N = N; g.Kpad = Kpad;
    g.S = S;
    g.nclass = 2 * S - 1;
    g.lower = lower;
    g.beta = 0.0;
    g.splitk = 1;
    g.strideC = 0;
    return g;
}

// Split-K factor of a sliced product (one 128 x 64 workgroup per compute unit
// at a time; 32-deep stages of about 0.6 us at 4 slices).
int sliced_splits(const SlicedGemmArgs &g, int maxS) {
    const long tiles = sliced_tiles(g.M, g.N, g.lower);
    const int S = choose_splits(tiles, g.Kpad, maxS);   // rounds of 256 workgroups
    return std::max(1, S);
}

// C = sliced product, split over K into `part` (S partial results of M x N,
// scaled) and summed when that fills the compute units better.
int run_sliced(geninv_ctx *c, SlicedGemmArgs g, double *part, size_t part_elems) {
    const size_t mn = (size_t)g.M * g.N;
    const int cap = (int)std::max<size_t>(1, std::min<size_t>(16, part ? part_elems / std::max<size_t>(mn, 1) : 1));
    const int S = g.beta == 0.0 ? sliced_splits(g, cap) : 1;
    if (S <= 1) {
        HIPCHK(launch_sliced_gemm(g, c->stream));
        return GENINV_OK;
    }
    double *C = g.C;
    const long ldc = g.ldc;
    g.C = part;
    g.ldc = g.M;
    g.splitk = S;
    g.strideC = (long)mn;
    HIPCHK(launch_sliced_gemm(g, c->stream));
    HIPCHK(launch_splitk_reduce(part, g.M, (long)mn, S, C, ldc, hdim(g.M), hdim(g.N), 1.0, 0.0,
                                g.lower ? GEMM_LOWER : GEMM_FULL, c->stream));
    return GENINV_OK;
}

// ---- int8 modular engine ---------------------------------------------------

// Workspace and launch shape of one engine product C = op(A) op(B) (M x N,
// depth K): int8 residue planes of both operands (shared for a Gram matrix),
// their exponents, and the residue planes of the result.
struct ModPlan {
    int M = 0, N = 0, K = 0, Kpad = 0, beta = -1, splitk = 1, lower = 0, cfg = 0;
    bool same = false;
    long sa = 0, sb = 0, strideR = 0;
    size_t pa = 0, pb = 0, ea = 0, eb = 0, res = 0, total = 0;
};

ModPlan mod_plan(size_t base, int M, int N, int K, const ModConsts &mc, bool same, int lower) {
    ModPlan P;
    P.M = M;
    P.N = N;
    P.K = K;
    P.lower = lower;
    P.same = same;
    P.Kpad = (int)pad64(std::max(K, 1));
    P.beta = mod_beta(mc, K);
    // 256 x 256 tiles (one workgroup per compute unit) when they give every
    // compute unit at least two rounds, else 128 x 128 (three per compute
    // unit); K split when the tiles of all moduli still leave the compute
    // units short, keeping at least 16 stages per slice
    const int nst = P.Kpad / 64;
    const int S0 = mod_min_splits(P.Kpad);
    P.cfg = mod_tiles(M, N, lower, 1) * mc.n * S0 >= 512 ? 1 : 0;
    const long tiles = mod_tiles(M, N, lower, P.cfg);
    const long target = P.cfg ? 512 : 768;
    int S = S0;
    while (S < 16 && tiles * mc.n * S < target && nst / (S + 1) >= 16) ++S;
    P.splitk = S;
    size_t off = base;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += align256(bytes);
        return o;
    };
    // planes hold whole 16-row groups (the GEMM loads 16 rows at a time)
    P.sa = (long)P.Kpad * ((M + 15) / 16 * 16);
    P.pa = take((size_t)mc.n * P.sa);
    P.sb = same ? P.sa : (long)P.Kpad * ((N + 15) / 16 * 16);
    P.pb = same ? P.pa : take((size_t)mc.n * P.sb);
    P.ea = take((size_t)std::max(M, 1) * sizeof(int));
    P.eb = same ? P.ea : take((size_t)std::max(N, 1) * sizeof(int));
    P.strideR = (long)mod_residue_bytes(M, N, lower, P.cfg);
    P.res = take((size_t)mc.n * S * P.strideR);
    P.total = off;
    return P;
}

// C = op(A) op(B) through the engine: op(A)(i, k) = A(k, i) when transA
// (columns of A, column exponents), A(i, k) otherwise (rows of A through the
// transposing slicer); op(B)(k, j) = B(k, j) unless transB.  With P.same the
// operands are one matrix (A = B, transA, !transB) sliced once.
int run_mod_product(geninv_ctx *c, const ModPlan &P, const ModConsts &mc, int transA, const double *A, long lda,
                    int transB, const double *B, long ldb, double *C, long ldc) {
    if (P.M <= 0 || P.N <= 0) return GENINV_OK;
    if (P.beta < 0) return GENINV_EINVAL;
    int8_t *pa = at<int8_t>(c, P.pa), *pb = at<int8_t>(c, P.pb);
    int *ea = at<int>(c, P.ea), *eb = at<int>(c, P.eb);
    if (transA) {
        HIPCHK(launch_col_exponents(A, lda, P.K, P.M, ea, c->stream));
        HIPCHK(launch_mod_slice_cols(A, lda, P.K, P.M, ea, P.beta, mc, pa, P.Kpad, P.sa, c->stream));
    } else {
        HIPCHK(launch_row_exponents(A, lda, P.M, P.K, ea, c->stream));
        HIPCHK(launch_mod_slice_rows_t(A, lda, P.M, P.K, ea, P.beta, mc, pa, P.Kpad, P.sa, c->stream));
    }
    if (!P.same) {
        if (!transB) {
            HIPCHK(launch_col_exponents(B, ldb, P.K, P.N, eb, c->stream));
            HIPCHK(launch_mod_slice_cols(B, ldb, P.K, P.N, eb, P.beta, mc, pb, P.Kpad, P.sb, c->stream));
        } else {
            HIPCHK(launch_row_exponents(B, ldb, P.N, P.K, eb, c->stream));
            HIPCHK(launch_mod_slice_rows_t(B, ldb, P.N, P.K, eb, P.beta, mc, pb, P.Kpad, P.sb, c->stream));
        }
    }
    int8_t *res = at<int8_t>(c, P.res);
    ModGemmArgs g{};
    g.A = pa; g.lda = P.Kpad; g.sa = P.sa;
    g.B = pb; g.ldb = P.Kpad; g.sb = P.sb;
    g.M = P.M; g.N = P.N; g.Kpad = P.Kpad;
    g.lower = P.lower;
    g.cfg = P.cfg;
    g.splitk = P.splitk;
    g.R = res; g.strideR = P.strideR;
    g.mc = mc;
    HIPCHK(launch_mod_gemm(g, c->stream));
    ModRecArgs r{};
    r.R = res; r.strideR = P.strideR;
    r.M = P.M; r.N = P.N; r.lower = P.lower; r.cfg = P.cfg; r.splitk = P.splitk; r.beta = P.beta;
    r.ea = ea; r.eb = P.same ? ea : eb;
    r.C = C; r.ldc = ldc;
    r.mc = mc;
    HIPCHK(launch_mod_reconstruct(r, c->stream));
    return GENINV_OK;
}

// ---- the mixed form's workspace ---------------------------------------------

constexpr int PROBES = 16;   // random sign vectors of the error estimate
constexpr long PROBE_PART = 1024L * 256;   // rows x K chunks of a probe product's partial sums at most

// After the float64 layout of the factored dimension nn: the engine's
// operands (bf16 slice planes, or the int8 plans of the Gram matrix and of
// the chain, which run at different times and share one region) and the
// error estimate's probe blocks, sums and Gram diagonal.
struct MixedPlan {
    int precision = 0, gd = 0, cd = 0, ns = 0;
    MixedLayout bf{};
    ModConsts mg{}, mch{};
    ModPlan pg{}, pch{};
    size_t probe = 0, norms = 0, skin = 0, total = 0;
    long pld = 0;   // rows of each probe block
};

int make_mixed_plan(size_t base, int m, int n, int precision, int gd, int cd, int ns, MixedPlan &P) {
    const bool tr = m < n;
    const int nn = tr ? m : n, mm = tr ? n : m;
    P.precision = precision;
    P.gd = gd;
    P.cd = cd;
    P.ns = ns;
    size_t off = base;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += align256(bytes);
        return o;
    };
    if (precision == GENINV_MIXED_BF16) {
        P.bf = make_mixed_layout(off, mm, nn, gd, cd, false);
        off = P.bf.total;
    } else {
        if (!mod_consts(gd, P.mg)) return GENINV_EINVAL;
        P.pg = mod_plan(off, nn, nn, mm, P.mg, true, 1);
        if (P.pg.beta < 0) return GENINV_EINVAL;
        size_t end = P.pg.total;
        if (cd > 0) {
            if (!mod_consts(cd, P.mch)) return GENINV_EINVAL;
            // Y (n x m) = P G' or G' P: depth nn
            P.pch = mod_plan(off, n, m, nn, P.mch, false, 0);
            if (P.pch.beta < 0) return GENINV_EINVAL;
            end = std::max(end, P.pch.total);
        }
        off = end;
    }
    P.pld = std::max(m, n);
    P.probe = take((size_t)8 * P.pld * PROBES * sizeof(double));
    P.norms = take((size_t)(8 + nn) * sizeof(double));   // sums, then the Gram diagonal
    // the probe products' K-chunk partial sums and transposed right factor
    P.skin = take((size_t)(std::max(PROBE_PART, P.pld) + P.pld) * PROBES * sizeof(double));
    P.total = off;
    return GENINV_OK;
}

}  // namespace

extern "C" {

int geninv_version(void) { return 200; }

int geninv_prof_classes(void) { return PC_COUNT; }

const char *geninv_prof_name(int cls) { return (cls >= 0 && cls < PC_COUNT) ? kProfNames[cls] : "unknown"; }

int geninv_prof_enable(geninv_ctx *c, unsigned mask) {
    if (!c) return GENINV_EINVAL;
    DeviceGuard g(c->device);
    prof_resolve(c);
    c->prof.mask = mask;
    std::fill(std::begin(c->prof.ms), std::end(c->prof.ms), 0.0);
    std::fill(std::begin(c->prof.cnt), std::end(c->prof.cnt), 0L);
    std::fill(std::begin(c->prof.fl), std::end(c->prof.fl), 0.0);
    return GENINV_OK;
}

int geninv_prof_read(geninv_ctx *c, int cls, double *total_ms, long *launches, double *flops) {
    if (!c || cls < 0 || cls >= PC_COUNT) return GENINV_EINVAL;
    DeviceGuard g(c->device);
    prof_resolve(c);
    if (total_ms) *total_ms = c->prof.ms[cls];
    if (launches) *launches = c->prof.cnt[cls];
    if (flops) *flops = c->prof.fl[cls];
    return GENINV_OK;
}

const char *geninv_strerror(int s) {
    switch (s) {
        case GENINV_OK: return "success";
        case GENINV_EINVAL: return "invalid argument";
        case GENINV_ENOMEM: return "device workspace allocation failed";
        case GENINV_EHIP: return "HIP runtime error";
        case GENINV_ENONFINITE: return "input holds Inf or NaN (or its Gram matrix overflows)";
        case GENINV_ENOTSPD: return "L'L is not positive definite in floating point";
        case GENINV_ENOTSUP: return "not supported by the library";
        case GENINV_EACCURACY: return "result written, but its error estimate exceeds the requested accuracy";
        case GENINV_ESCRATCH: return "problem needs more device memory than the fixed scratch area holds";
        default: return "unknown status";
    }
}

int geninv_create(geninv_ctx **ctx, int device, void *hip_stream) {
    if (!ctx) return GENINV_EINVAL;
    *ctx = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess) return GENINV_EHIP;
    if (device < 0 || device >= ndev) return GENINV_EINVAL;
    DeviceGuard g(device);
    geninv_ctx *c = new geninv_ctx();
    c->device = device;
    c->stream = static_cast<hipStream_t>(hip_stream);
    void *p = nullptr;
    if (hipMalloc(&p, 256) != hipSuccess) {
        delete c;
        return GENINV_ENOMEM;
    }
    c->status = static_cast<int *>(p);
    if (hipMemset(c->status, 0, 256) != hipSuccess) {
        (void)hipFree(p);
        delete c;
        return GENINV_EHIP;
    }
    void *h = nullptr;
    if (hipHostMalloc(&h, 64, hipHostMallocDefault) != hipSuccess) {
        (void)hipFree(p);
        delete c;
        return GENINV_ENOMEM;
    }
    c->hpin = static_cast<int *>(h);
    bool aux_ok = hipStreamCreateWithFlags(&c->aux, hipStreamNonBlocking) == hipSuccess;
    for (hipEvent_t *e : {&c->ev_fact, &c->ev_rest[0], &c->ev_rest[1], &c->ev_join})
        aux_ok = aux_ok && hipEventCreateWithFlags(e, hipEventDisableTiming) == hipSuccess;
    if (!aux_ok) {
        (void)hipGetLastError();
        for (hipEvent_t e : {c->ev_fact, c->ev_rest[0], c->ev_rest[1], c->ev_join})
            if (e) (void)hipEventDestroy(e);
        if (c->aux) (void)hipStreamDestroy(c->aux);
        (void)hipHostFree(h);
        (void)hipFree(p);
        delete c;
        return GENINV_EHIP;
    }
    if (device < NOALLOC_MAX_DEVICES) {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        if (!g_scratch[device]) {
            void *sp = nullptr;
            if (hipGetSymbolAddress(&sp, HIP_SYMBOL(scratch)) != hipSuccess || !sp) {
                (void)hipGetLastError();
                for (hipEvent_t e : {c->ev_fact, c->ev_rest[0], c->ev_rest[1], c->ev_join}) (void)hipEventDestroy(e);
                (void)hipStreamDestroy(c->aux);
                (void)hipHostFree(h);
                (void)hipFree(p);
                delete c;
                return GENINV_EHIP;
            }
            g_scratch[device] = static_cast<char *>(sp);
        }
        c->scratch = g_scratch[device];
    }
    if (const char *e = getenv("GENINV_DEBUG")) c->debug = atoi(e);
    if (const char *e = getenv("GENINV_WORKSPACE_LIMIT")) c->ws_limit = strtoull(e, nullptr, 10);
    *ctx = c;
    return GENINV_OK;
}

int geninv_destroy(geninv_ctx *c) {
    if (!c) return GENINV_OK;
    DeviceGuard g(c->device);
    (void)hipStreamSynchronize(c->stream);
    prof_resolve(c);
    for (hipEvent_t e : c->prof.pool) (void)hipEventDestroy(e);
    if (c->aux) (void)hipStreamSynchronize(c->aux);
    for (hipEvent_t e : {c->ev_fact, c->ev_rest[0], c->ev_rest[1], c->ev_join})
        if (e) (void)hipEventDestroy(e);
    if (c->aux) (void)hipStreamDestroy(c->aux);
    if (c->ws) (void)hipFree(c->ws);
    if (c->status) (void)hipFree(c->status);
    if (c->hpin) (void)hipHostFree(c->hpin);
    delete c;
    return GENINV_OK;
}

int geninv_set_host_sync(geninv_ctx *c, int enable) {
    if (!c) return GENINV_EINVAL;
    c->host_sync = enable ? 1 : 0;
    return GENINV_OK;
}

int geninv_set_workspace_limit(geninv_ctx *c, size_t bytes) {
    if (!c) return GENINV_EINVAL;
    c->ws_limit = bytes;
    return GENINV_OK;
}

int geninv_set_debug(geninv_ctx *c, int flags) {
    if (!c || (flags & ~GENINV_DEBUG_POISON)) return GENINV_EINVAL;
    c->debug = flags;
    return GENINV_OK;
}

int geninv_debug_poison(geninv_ctx *c) {
    if (!c) return GENINV_EINVAL;
    if (!c->ws) return GENINV_OK;
    DeviceGuard g(c->device);
    HIPCHK(launch_poison(c->ws, c->ws_bytes, c->stream));
    return GENINV_OK;
}

int geninv_set_stream(geninv_ctx *c, void *hip_stream) {
    if (!c) return GENINV_EINVAL;
    c->stream = static_cast<hipStream_t>(hip_stream);
    return GENINV_OK;
}

int geninv_sync_status(geninv_ctx *c) {
    if (!c) return GENINV_EINVAL;
    DeviceGuard g(c->device);
    int st = 0;
    HIPCHK(hipMemcpyAsync(&st, c->status, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    if (st != 0) {
        int zero = 0;
        HIPCHK(hipMemcpy(c->status, &zero, sizeof(int), hipMemcpyHostToDevice));
    }
    return st;
}

size_t geninv_workspace_bytes(int m, int n, int k, int precision, int gram_digits, int chain_digits, int ns_steps) {
    if (m <= 0 || n <= 0 || k < 0) return 0;
    if (precision == GENINV_FP64) return make_layout(std::min(m, n), k, std::max(m, n)).total;
    const int dmax = precision == GENINV_MIXED_BF16 ? SG_MAX_S : (precision == GENINV_MIXED_INT8 ? MOD_MAX : 0);
    if (gram_digits < 1 || gram_digits > dmax || chain_digits < 0 || chain_digits > dmax || ns_steps < 0) return 0;
    const Layout lay = make_layout(std::min(m, n), PROBES);
    MixedPlan mp;
    if (make_mixed_plan(lay.total, m, n, precision, gram_digits, chain_digits, ns_steps, mp) != GENINV_OK) return 0;
    return mp.total;
}

int geninv_dgemm(geninv_ctx *c, int transA, int transB, int M, int N, int K, double alpha, const double *A,
                 int lda, const double *B, int ldb, double beta, double *C, int ldc) {
    if (!c || M < 0 || N < 0 || K < 0) return GENINV_EINVAL;
    if (M == 0 || N == 0) return GENINV_OK;
    if (!C || bad_ld(ldc, M)) return GENINV_EINVAL;
    if (K > 0 && (!A || !B || bad_ld(lda, transA ? K : M) || bad_ld(ldb, transB ? N : K))) return GENINV_EINVAL;
    DeviceGuard g(c->device);
    GemmArgs a = gemm(A, lda, transA ? 1 : 0, B, ldb, transB ? 1 : 0, C, ldc, hdim(M), hdim(N), hdim(K), alpha,
                      beta);
    ProfScope ps(c, PC_GEMM, 2.0 * M * N * K);
    // at most 16 output columns, A not transposed, long K: bound by reading A
    // once (skinny.hip), split into up to 64 chunks of at least 128 of K
    if (!transA && N <= 16 && K >= 1024) {
        const long rowblocks = (M + 255) / 256;
        const int S = (int)std::max<long>(1, std::min<long>({64L, (1024 + rowblocks - 1) / rowblocks, (long)K / 128}));
        const int kchunk = (K + S - 1) / S;
        const int Sx = (K + kchunk - 1) / kchunk;
        const size_t pelems = (size_t)Sx * M * N;
        CHK(ensure_ws(c, (pelems + (size_t)K * skinny_padded_width(N)) * sizeof(double)));
        double *part = at<double>(c, 0);
        HIPCHK(launch_skinny_gemm(A, lda, B, ldb, transB ? 1 : 0, M, N, K, alpha, beta, C, ldc, kchunk, part + pelems,
                                  part, c->stream));
        return GENINV_OK;
    }
    // the same with A transposed (op(A) = A', A K x M, B not transposed): a
    // wavefront walks rows of A for four of its columns (skinny.hip)
    if (transA && !transB && N <= 16 && K >= 1024) {
        const long colblocks = (M + 15) / 16;
        const int S = (int)std::max<long>(1, std::min<long>({64L, (1024 + colblocks - 1) / colblocks, (long)K / 256}));
        const int kchunk = (K + S - 1) / S;
        const int Sx = (K + kchunk - 1) / kchunk;
        CHK(ensure_ws(c, (size_t)Sx * M * N * sizeof(double)));
        HIPCHK(launch_skinny_gemm_t(A, lda, B, ldb, M, N, K, alpha, beta, C, ldc, kchunk, at<double>(c, 0),
                                    c->stream));
        return GENINV_OK;
    }
    // a skinny product (few output tiles, long K) is split over K: about 1024
    // workgroups (several fit on a compute unit; these launches are bound by
    // load latency), at least 256 of K each
    const long tiles = gemm_tiles(a, 64);
    if (tiles < 256 && K >= 1024) {
        const int S = (int)std::min<long>({64L, (1024 + tiles - 1) / tiles, (long)K / 256});
        if (S > 1) {
            CHK(ensure_ws(c, (size_t)S * M * N * sizeof(double)));
            GemmArgs p = a;
            p.C = at<double>(c, 0);
            p.ldc = M;
            p.splitk = S;
            p.strideC = (long)M * N;
            HIPCHK(launch_dgemm(p, c->stream));
            HIPCHK(launch_splitk_reduce(p.C, M, p.strideC, S, C, ldc, hdim(M), hdim(N), alpha, beta, GEMM_FULL,
                                        c->stream));
            return GENINV_OK;
        }
    }
    HIPCHK(launch_dgemm(a, c->stream));
    return GENINV_OK;
}

int geninv_dgram(geninv_ctx *c, int m, int n, const double *G, int ldg, double *A, int lda, int full) {
    if (!c || m < 0 || n < 0) return GENINV_EINVAL;
    if (n == 0) return GENINV_OK;
    if (!A || bad_ld(lda, n) || (m > 0 && (!G || bad_ld(ldg, m)))) return GENINV_EINVAL;
    DeviceGuard g(c->device);
    GemmArgs a = gemm(G, ldg, 1, G, ldg, 0, A, lda, hdim(n), hdim(n), hdim(m), 1.0, 0.0,
                      full ? GEMM_FULL : GEMM_LOWER);
    HIPCHK(launch_dgemm(a, c->stream));
    return GENINV_OK;
}

int geninv_dfrchol(geninv_ctx *c, int n, const double *A, int lda, double tol, double *L, int ldl, int *piv,
                   double *d, double *tol_used, int *rank) {
    if (!c || n < 0) return GENINV_EINVAL;
    if (n == 0) {
        if (rank) *rank = 0;
        return GENINV_OK;
    }
    if (!A || !L || bad_ld(lda, n) || bad_ld(ldl, n)) return GENINV_EINVAL;
    DeviceGuard g(c->device);
    const Layout lay = make_layout(n, 0);
    CHK(ensure_ws(c, lay.total));
    int *pv = piv ? piv : at<int>(c, lay.piv);
    double *dv = d ? d : at<double>(c, lay.dvals);
    double *Aw = at<double>(c, lay.slotA);
    HIPCHK(launch_copy(A, lda, Aw, n, hdim(n), hdim(n), c->stream));
    CHK(run_frchol(c, lay, Aw, n, n, tol, L, ldl, pv, dv));
    const int np = (n + FR_NB - 1) / FR_NB;
    if (tol_used) HIPCHK(launch_copy(at<double>(c, lay.tol), 1, tol_used, 1, hdim(1), hdim(1), c->stream));
    return finish_rank(c, at<int>(c, lay.rank) + np, rank);
}

int geninv_dspdinv(geninv_ctx *c, int r, const double *B, int ldb, double *M, int ldm) {
    if (!c || r < 0) return GENINV_EINVAL;
    if (r == 0) return GENINV_OK;
    if (!B || !M || bad_ld(ldb, r) || bad_ld(ldm, r)) return GENINV_EINVAL;
    DeviceGuard g(c->device);
    const Layout lay = make_layout(r, 0);
    CHK(ensure_ws(c, lay.total));
    HIPCHK(launch_copy(B, ldb, M, ldm, hdim(r), hdim(r), c->stream));
    return run_spdinv(c, lay, M, ldm, hdim(r));
}

}  // extern "C"

namespace geninv {
hipError_t launch_ns_scaled_eye(double *X, long ldx, int n, double a, hipStream_t s);
hipError_t launch_ns_two_minus(double *T, long ldt, int n, double *sum2, hipStream_t s);
hipError_t launch_fro2(const double *B, long ldb, int n, double *sum2, hipStream_t s);
}  // namespace geninv

extern "C" {

int geninv_dspdinv_ns(geninv_ctx *c, int r, const double *B, int ldb, double *M, int ldm, int max_iter, int *iters,
                      double *resid) {
    if (!c || r < 0 || max_iter < 1) return GENINV_EINVAL;
    if (iters) *iters = 0;
    if (resid) *resid = 0.0;
    if (r == 0) return GENINV_OK;
    if (!B || !M || bad_ld(ldb, r) || bad_ld(ldm, r)) return GENINV_EINVAL;
    DeviceGuard g(c->device);
    const Layout lay = make_layout(r, 0);
    CHK(ensure_ws(c, lay.total + 256));
    double *X = at<double>(c, lay.slotA), *T = at<double>(c, lay.slotL), *Xn = at<double>(c, lay.slotK);
    double *sum2 = at<double>(c, lay.total);   // one device scalar after the layout
    const long ld = r;
    auto read_sum = [&](double *host) -> int {
        HIPCHK(hipMemcpyAsync(host, sum2, sizeof(double), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        return GENINV_OK;
    };
    double nb2 = 0.0;
    HIPCHK(launch_fill(sum2, 1, 1, 1, 0.0, c->stream));
    HIPCHK(launch_fro2(B, ldb, r, sum2, c->stream));
    CHK(read_sum(&nb2));
    if (!(nb2 > 0.0) || !std::isfinite(nb2)) return nb2 > 0.0 ? GENINV_ENONFINITE : GENINV_ENOTSPD;
    // X_0 = I / ||B||_F: the eigenvalues of I - B X_0 lie in [0, 1) for SPD B
    HIPCHK(launch_ns_scaled_eye(X, ld, r, 1.0 / std::sqrt(nb2), c->stream));
    // Each step evaluates the residual of the current X first; once it stops
    // falling (the rounding floor, about cond(B) u), the previous iterate,
    // still in Xn, is the result.
    double prev = std::numeric_limits<double>::infinity();
    const double *result = X;
    int evals = 0;
    for (int it = 0; it < max_iter; ++it) {
        // T = B X, then T := 2I - T with the residual ||I - B X||_F of this X
        HIPCHK(launch_dgemm(gemm(B, ldb, 0, X, ld, 0, T, ld, hdim(r), hdim(r), hdim(r), 1.0, 0.0), c->stream));
        double s2 = 0.0;
        HIPCHK(launch_fill(sum2, 1, 1, 1, 0.0, c->stream));
        HIPCHK(launch_ns_two_minus(T, ld, r, sum2, c->stream));
        CHK(read_sum(&s2));
        ++evals;
        const double rho = std::sqrt(s2 / r);
        if (!std::isfinite(rho)) return GENINV_ENONFINITE;
        if (rho >= prev) {
            result = Xn;   // X_{k-1}
            break;
        }
        prev = rho;
        result = X;
        if (rho < 1e-15) break;
        // X <- X (2I - B X)
        HIPCHK(launch_dgemm(gemm(X, ld, 0, T, ld, 0, Xn, ld, hdim(r), hdim(r), hdim(r), 1.0, 0.0), c->stream));
        std::swap(X, Xn);
        result = X;   // not yet evaluated; kept if the iteration count runs out
    }
    HIPCHK(launch_copy(result, ld, M, ldm, hdim(r), hdim(r), c->stream));
    if (iters) *iters = evals;
    if (resid) *resid = prev;
    return GENINV_OK;
}

int geninv_dchain(geninv_ctx *c, int m, int n, int r, const double *L, int ldl, const double *M, int ldm,
                  const double *G, int ldg, double *Y, int ldy) {
    if (!c || m < 0 || n < 0 || r < 0 || r > n) return GENINV_EINVAL;
    if (m == 0 || n == 0) return GENINV_OK;
    if (!G || !Y || bad_ld(ldg, m) || bad_ld(ldy, n)) return GENINV_EINVAL;
    if (r > 0 && (!L || !M || bad_ld(ldl, n) || bad_ld(ldm, r))) return GENINV_EINVAL;
    DeviceGuard g(c->device);
    const Layout lay = make_layout(n, 0);
    CHK(ensure_ws(c, lay.total));
    double *K = at<double>(c, lay.slotK);
    double *P = at<double>(c, lay.slotP);
    CHK(gemm_fill(c, lay, chain(gemm(L, ldl, 0, M, ldm, 0, K, n, hdim(n), hdim(r), hdim(r), 1.0, 0.0))));
    if (lowrank_chain(n, hdim(r))) return run_chain_lowrank(c, lay, K, n, n, r, G, ldg, false, n, m, Y, ldy);
    CHK(gemm_fill(c, lay, chain(gemm(K, n, 0, K, n, 1, P, n, hdim(n), hdim(n), hdim(r), 1.0, 0.0, GEMM_LOWER))));
    HIPCHK(launch_mirror_lower(P, n, hdim(n), c->stream));
    HIPCHK(launch_dgemm(chain(gemm(P, n, 0, G, ldg, 1, Y, ldy, hdim(n), hdim(m), hdim(n), 1.0, 0.0)), c->stream));
    return GENINV_OK;
}

int geninv_dgeninv(geninv_ctx *c, int m, int n, const double *G, int ldg, double tol, double *Y, int ldy,
                   int *rank, int *piv) {
    if (!c || m < 0 || n < 0) return GENINV_EINVAL;
    if (m == 0 || n == 0) {
        if (rank) *rank = 0;
        return GENINV_OK;
    }
    if (!G || !Y || bad_ld(ldg, m) || bad_ld(ldy, n)) return GENINV_EINVAL;
    DeviceGuard g(c->device);
    const bool tr = m < n;              // Appendix: factor G G' when m < n
    const int nn = tr ? m : n;
    const Layout lay = make_layout(nn, 0, tr ? n : m);
    CHK(ensure_ws(c, lay.total));
    double *A = at<double>(c, lay.slotA);
    double *L = at<double>(c, lay.slotL);
    double *K = at<double>(c, lay.slotK);
    double *P = at<double>(c, lay.slotP);
    int *pv = piv ? piv : at<int>(c, lay.piv);
    const long ld = nn;

    // 1. Gram matrix, lower triangle: A = G'G, or G G' in the transpose branch
    CHK(run_gram(c, lay, G, ldg, tr, nn, tr ? n : m));
    // 2-3. tolerance and full-rank Cholesky
    CHK(run_frchol(c, lay, A, ld, nn, tol, L, ld, pv, at<double>(c, lay.dvals)));
    const int *rdev = at<int>(c, lay.rank) + (nn + FR_NB - 1) / FR_NB;
    Dim r;
    CHK(rank_dim(c, nn, rdev, &r));
    // 4. M = (L'L)^-1 into the Gram's slot
    CHK(run_factor_inverse(c, lay, L, ld, nn, r, A, ld));
    // 5. K = L M, P = K K' (= (G'G)^+), then Y = P G' or Y = G' P; for a rank
    //    under half the order Y = K (K' G') or (G' K) K' instead
    {
        ProfScope ps(c, PC_CHAIN_K, 0.0);
        CHK(gemm_fill(c, lay, chain(gemm(L, ld, 0, A, ld, 0, K, ld, hdim(nn), r, r, 1.0, 0.0))));
    }
    if (lowrank_chain(nn, r)) {
        ProfScope ps(c, PC_CHAIN_Y, 4.0 * n * m * r.host);
        CHK(run_chain_lowrank(c, lay, K, ld, nn, r.host, G, ldg, tr, n, m, Y, ldy));
        return finish_rank(c, rdev, rank);
    }
    {
        ProfScope ps(c, PC_CHAIN_P, 0.0);
        CHK(gemm_fill(c, lay, chain(gemm(K, ld, 0, K, ld, 1, P, ld, hdim(nn), hdim(nn), r, 1.0, 0.0, GEMM_LOWER))));
    }
    {
        ProfScope ps(c, PC_MIRROR, 0.0);
        HIPCHK(launch_mirror_lower(P, ld, hdim(nn), c->stream));
    }
    {
        ProfScope ps(c, PC_CHAIN_Y, 2.0 * n * m * nn);
        if (!tr) HIPCHK(launch_dgemm(chain(gemm(P, ld, 0, G, ldg, 1, Y, ldy, hdim(n), hdim(m), hdim(n), 1.0, 0.0)),
                                     c->stream));
        else HIPCHK(launch_dgemm(chain(gemm(G, ldg, 1, P, ld, 0, Y, ldy, hdim(n), hdim(m), hdim(m), 1.0, 0.0)),
                                 c->stream));
    }
    return finish_rank(c, rdev, rank);
}

}  // extern "C"

namespace {

// Points the context's workspace at the fixed scratch area (and switches
// the event timers off, which would create events) for one call.
struct ScratchWorkspace {
    geninv_ctx *c;
    char *ws;
    size_t bytes;
    unsigned mask;
    explicit ScratchWorkspace(geninv_ctx *ctx) : c(ctx), ws(ctx->ws), bytes(ctx->ws_bytes), mask(ctx->prof.mask) {
        c->ws = c->scratch;
        c->ws_bytes = NOALLOC_BYTES;
        c->prof.mask = 0;
    }
    ~ScratchWorkspace() {
        c->ws = ws;
        c->ws_bytes = bytes;
        c->prof.mask = mask;
    }
};

int dlstsq_run(geninv_ctx *c, int m, int n, int k, const double *G, int ldg, const double *F, int ldf, double tol,
               double *W, int ldw, int *rank, bool noalloc) {
    if (!c || m < 0 || n < 0 || k < 0) return GENINV_EINVAL;
    if (n == 0 || m == 0) {
        // G^+ is n x 0 or 0 x m: W = 0 (n x k)
        if (n > 0 && k > 0) {
            if (!W || bad_ld(ldw, n)) return GENINV_EINVAL;
            DeviceGuard g(c->device);
            HIPCHK(launch_fill(W, ldw, n, k, 0.0, c->stream));
        }
        if (rank) *rank = 0;
        return GENINV_OK;
    }
    if (!G || !F || !W || bad_ld(ldg, m) || bad_ld(ldf, m) || bad_ld(ldw, n)) return GENINV_EINVAL;
    if (k > 4096) return GENINV_ENOTSUP;
    DeviceGuard g(c->device);
    const bool tr = m < n;              // Appendix: factor G G' when m < n
    const int nn = tr ? m : n;
    const Layout lay = make_layout(nn, k, tr ? n : m);
    if (noalloc) {
        if (!c->scratch) return GENINV_EHIP;
        if (lay.total > NOALLOC_BYTES) return GENINV_ESCRATCH;
    } else {
        CHK(ensure_ws(c, lay.total));
    }
    double *A = at<double>(c, lay.slotA);
    double *L = at<double>(c, lay.slotL);
    double *T0 = at<double>(c, lay.t0);
    double *T1 = at<double>(c, lay.t1);
    double *T2 = at<double>(c, lay.t2);
    const long ld = nn;

    CHK(run_gram(c, lay, G, ldg, tr, nn, tr ? n : m));
    CHK(run_frchol(c, lay, A, ld, nn, tol, L, ld, at<int>(c, lay.piv), at<double>(c, lay.dvals)));
    const int *rdev = at<int>(c, lay.rank) + (nn + FR_NB - 1) / FR_NB;
    Dim r;
    CHK(rank_dim(c, nn, rdev, &r));
    CHK(run_factor_inverse(c, lay, L, ld, nn, r, A, ld));
    if (k > 0 && !tr) {
        // W = L (M (M (L' (G' F))))
        ProfScope ps(c, PC_LSTSQ, 0.0);
        CHK(gemm_splitk(c, lay, gemm(G, ldg, 1, F, ldf, 0, T0, ld, hdim(nn), hdim(k), hdim(m), 1.0, 0.0)));
        HIPCHK(launch_dgemm(gemm(L, ld, 1, T0, ld, 0, T1, ld, r, hdim(k), hdim(nn), 1.0, 0.0), c->stream));
        HIPCHK(launch_dgemm(gemm(A, ld, 0, T1, ld, 0, T2, ld, r, hdim(k), r, 1.0, 0.0), c->stream));
        HIPCHK(launch_dgemm(gemm(A, ld, 0, T2, ld, 0, T1, ld, r, hdim(k), r, 1.0, 0.0), c->stream));
        HIPCHK(launch_dgemm(gemm(L, ld, 0, T1, ld, 0, W, ldw, hdim(nn), hdim(k), r, 1.0, 0.0), c->stream));
    } else if (k > 0) {
        // transpose branch, Y = G' L M M L': W = G' (L (M (M (L' F))))
        ProfScope ps(c, PC_LSTSQ, 0.0);
        HIPCHK(launch_dgemm(gemm(L, ld, 1, F, ldf, 0, T1, ld, r, hdim(k), hdim(nn), 1.0, 0.0), c->stream));
        HIPCHK(launch_dgemm(gemm(A, ld, 0, T1, ld, 0, T2, ld, r, hdim(k), r, 1.0, 0.0), c->stream));
        HIPCHK(launch_dgemm(gemm(A, ld, 0, T2, ld, 0, T1, ld, r, hdim(k), r, 1.0, 0.0), c->stream));
        HIPCHK(launch_dgemm(gemm(L, ld, 0, T1, ld, 0, T0, ld, hdim(nn), hdim(k), r, 1.0, 0.0), c->stream));
        CHK(gemm_splitk(c, lay, gemm(G, ldg, 1, T0, ld, 0, W, ldw, hdim(n), hdim(k), hdim(m), 1.0, 0.0)));
    }
    return finish_rank(c, rdev, rank);
}

}  // namespace

extern "C" {

int geninv_dlstsq(geninv_ctx *c, int m, int n, int k, const double *G, int ldg, const double *F, int ldf,
                  double tol, double *W, int ldw, int *rank) {
    return dlstsq_run(c, m, n, k, G, ldg, F, ldf, tol, W, ldw, rank, false);
}

size_t geninv_noalloc_capacity(void) { return NOALLOC_BYTES; }

int geninv_dlstsq_noalloc(geninv_ctx *c, int m, int n, int k, const double *G, int ldg, const double *F, int ldf,
                          double tol, double *W, int ldw, int *rank) {
    if (!c) return GENINV_EINVAL;
    ScratchWorkspace sw(c);
    return dlstsq_run(c, m, n, k, G, ldg, F, ldf, tol, W, ldw, rank, true);
}



// C (M x N, ldc) = op(A) op(B) split over K into `part` when the output is
// too small to fill the compute units (S partial results, then a reduction)
static int rows_gemm(geninv_ctx *c, GemmArgs g, double *part, size_t part_elems) {
    const long tiles = (long)((g.M.host + 63) / 64) * ((g.N.host + 63) / 64);
    const size_t mn = (size_t)g.M.host * g.N.host;
    int S = (int)std::min<long>({16L, (256 + tiles - 1) / tiles, (long)g.K.host / 256});
    while (S > 1 && (size_t)S * mn > part_elems) --S;
    if (S <= 1) {
        HIPCHK(launch_dgemm(g, c->stream));
        return GENINV_OK;
    }
    double *C = g.C;
    const long ldc = g.ldc;
    g.C = part;
    g.ldc = g.M.host;
    g.splitk = S;
    g.strideC = (long)mn;
    HIPCHK(launch_dgemm(g, c->stream));
    HIPCHK(launch_splitk_reduce(part, g.M.host, (long)mn, S, C, ldc, g.M, g.N, 1.0, 0.0, GEMM_FULL, c->stream));
    return GENINV_OK;
}

int geninv_inc_gram(geninv_ctx *c, int m, int n_old, int p, int k, const double *G, int ldg, const double *F,
                    int ldf, double *A, int lda, double *B, int ldb) {
    if (!c || m < 0 || n_old < 0 || p < 0 || k < 0) return GENINV_EINVAL;
    const int n_new = n_old + p;
    if (p == 0) return GENINV_OK;
    if (!A || bad_ld(lda, n_new) || (k > 0 && (!B || bad_ld(ldb, n_new)))) return GENINV_EINVAL;
    DeviceGuard g(c->device);
    if (m == 0) {
        HIPCHK(launch_fill(A + n_old, lda, p, n_new, 0.0, c->stream));
        if (k > 0) HIPCHK(launch_fill(B + n_old, ldb, p, k, 0.0, c->stream));
        return GENINV_OK;
    }
    if (!G || bad_ld(ldg, m) || (k > 0 && (!F || bad_ld(ldf, m)))) return GENINV_EINVAL;
    // split-K partials: up to 16 copies of the larger of the two row blocks
    const size_t part_elems = (size_t)16 * p * std::max(n_new, k);
    CHK(ensure_ws(c, part_elems * sizeof(double)));
    double *part = at<double>(c, 0);
    const double *Gn = G + (long)n_old * ldg;   // the p new columns
    ProfScope ps(c, PC_GRAM, 2.0 * m * (double)p * n_new);
    // A[n_old + i, j] = G(:, n_old + i)' G(:, j), all j < n_new (the part above
    // the diagonal of the new block is its symmetric copy)
    CHK(rows_gemm(c, gemm(Gn, ldg, 1, G, ldg, 0, A + n_old, lda, hdim(p), hdim(n_new), hdim(m), 1.0, 0.0), part,
                  part_elems));
    if (k > 0)
        CHK(rows_gemm(c, gemm(Gn, ldg, 1, F, ldf, 0, B + n_old, ldb, hdim(p), hdim(k), hdim(m), 1.0, 0.0), part,
                      part_elems));
    return GENINV_OK;
}

}  // extern "C"

namespace geninv {
hipError_t launch_ns_scaled_eye(double *X, long ldx, int n, double a, hipStream_t s);
}

namespace {

Layout shift_layout(Layout L, size_t base) {
    for (size_t *f : {&L.slotA, &L.slotL, &L.slotK, &L.slotP, &L.part, &L.lpan, &L.dbuf, &L.rrow, &L.ccol, &L.dvals,
                      &L.tol, &L.rank, &L.piv, &L.t0, &L.t1, &L.t2, &L.gpart, &L.total})
        *f += base;
    return L;
}

// Full factorization of the Gram matrix A (n x n) for geninv_inc_factor:
// L, piv, dvals, M = (L'L)^-1, rank and tol_used.
int inc_full(geninv_ctx *c, int n, const double *A, long lda, double tol, double *L, long ldl, int *piv,
             double *dvals, double *M, long ldm, int *rank, double *tol_io) {
    const Layout lay = make_layout(n, 0);
    CHK(ensure_ws(c, lay.total));
    double *Aw = at<double>(c, lay.slotA);
    HIPCHK(launch_copy(A, lda, Aw, n, hdim(n), hdim(n), c->stream));
    CHK(run_frchol(c, lay, Aw, n, n, tol, L, ldl, piv, dvals));
    const int *rdev = at<int>(c, lay.rank) + (n + FR_NB - 1) / FR_NB;
    int r = 0;
    double t = 0.0;
    HIPCHK(hipMemcpyAsync(c->hpin, rdev, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipMemcpyAsync(&t, at<double>(c, lay.tol), sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    r = *c->hpin;
    if (r < 0 || r > n) return GENINV_EHIP;
    if (r > 0) CHK(run_factor_inverse(c, lay, L, ldl, n, hdim(r), M, ldm));
    *rank = r;
    *tol_io = t;
    return GENINV_OK;
}

}  // namespace

extern "C" {

int geninv_inc_factor(geninv_ctx *c, int n_old, int p, const double *A, int lda, double tol, double *L, int ldl,
                      int *piv, double *dvals, double *M, int ldm, int *rank_io, double *tol_io) {
    if (!c || n_old < 0 || p < 0 || !rank_io || !tol_io) return GENINV_EINVAL;
    const int n = n_old + p;
    if (n == 0) {
        *rank_io = 0;
        return GENINV_OK;
    }
    if (!A || !L || !piv || !dvals || !M || bad_ld(lda, n) || bad_ld(ldl, n) || bad_ld(ldm, n)) return GENINV_EINVAL;
    const int r0 = n_old > 0 ? *rank_io : 0;
    if (r0 < 0 || r0 > n_old) return GENINV_EINVAL;
    DeviceGuard g(c->device);
    if (p == 0) return GENINV_OK;
    if (n_old == 0 || r0 == 0) return inc_full(c, n, A, lda, tol, L, ldl, piv, dvals, M, ldm, rank_io, tol_io);

    // the threshold for all n columns (the paper's default follows the
    // smallest positive diagonal); the earlier decisions stand unless a
    // dropped pivot lies between the new threshold and the old one
    const Layout full = make_layout(n, 0);
    CHK(ensure_ws(c, full.total));
    double tol_new = tol;
    {
        double *tp = at<double>(c, full.tol);
        HIPCHK(launch_tol(A, lda, n, tol, tp, c->status, c->stream));
        HIPCHK(hipMemcpyAsync(&tol_new, tp, sizeof(double), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
    }
    if (tol_new != *tol_io) {
        std::vector<double> dv(n_old);
        std::vector<int> pv(r0);
        HIPCHK(hipMemcpy(dv.data(), dvals, sizeof(double) * n_old, hipMemcpyDeviceToHost));
        HIPCHK(hipMemcpy(pv.data(), piv, sizeof(int) * r0, hipMemcpyDeviceToHost));
        std::vector<char> kept(n_old, 0);
        for (int q : pv) kept[q] = 1;
        bool flips = false;
        for (int k = 0; k < n_old; ++k) {
            const bool keep_new = dv[k] > tol_new, keep_old = kept[k] != 0;
            flips = flips || keep_new != keep_old;
        }
        if (flips) return inc_full(c, n, A, lda, tol, L, ldl, piv, dvals, M, ldm, rank_io, tol_io);
    }

    // workspace: the incremental step's blocks, then a layout for the p x p
    // Schur complement
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += align256(bytes);
        return o;
    };
    const int nbk = (r0 + 63) / 64;
    const size_t oLp = take(sizeof(double) * r0 * (size_t)r0), oBw = take(sizeof(double) * r0 * (size_t)p),
                 oX = take(sizeof(double) * r0 * (size_t)p), oDi = take(sizeof(double) * 4096 * (size_t)nbk),
                 oS = take(sizeof(double) * p * (size_t)p), oLS = take(sizeof(double) * p * (size_t)p),
                 oPs = take(sizeof(int) * (size_t)p), oDs = take(sizeof(double) * 2 * (size_t)p),
                 oZ = take(sizeof(double) * r0 * (size_t)p), oH = take(sizeof(double) * p * (size_t)p),
                 oQ = take(sizeof(double) * r0 * (size_t)p), oB12 = take(sizeof(double) * r0 * (size_t)p),
                 oU = take(sizeof(double) * r0 * (size_t)p), oV = take(sizeof(double) * r0 * (size_t)p),
                 oT = take(sizeof(double) * p * (size_t)p);
    const Layout sub = shift_layout(make_layout(p, 0), off);
    CHK(ensure_ws(c, sub.total));
    double *Lp = at<double>(c, oLp), *Bw = at<double>(c, oBw), *X = at<double>(c, oX), *Di = at<double>(c, oDi);
    double *S = at<double>(c, oS), *LS = at<double>(c, oLS), *ds = at<double>(c, oDs);
    int *ps = at<int>(c, oPs);
    double *Z = at<double>(c, oZ), *H = at<double>(c, oH), *Q = at<double>(c, oQ), *B12 = at<double>(c, oB12);
    double *U = at<double>(c, oU), *V = at<double>(c, oV), *T = at<double>(c, oT);
    auto mm = [&](const double *Am, long la, int ta, const double *Bm, long lb, int tb, double *Cm, long lc, int Mr,
                  int Nc, int Kd, double al, double be, int uplo = GEMM_FULL) -> int {
        if (Mr <= 0 || Nc <= 0) return GENINV_OK;
        HIPCHK(launch_dgemm(gemm(Am, la, ta, Bm, lb, tb, Cm, lc, hdim(Mr), hdim(Nc), hdim(Kd), al, be, uplo),
                            c->stream));
        return GENINV_OK;
    };

    // new rows of L: L_P X = B_P, blocked by 64 with inverted diagonal blocks
    HIPCHK(launch_gather_rows(L, ldl, piv, r0, r0, Lp, r0, c->stream));
    HIPCHK(launch_gather_cols_t(A, lda, n_old, piv, r0, p, Bw, r0, c->stream));
    HIPCHK(launch_trinv64(Lp, r0, r0, Di, c->stream));
    for (int b = 0; b < nbk; ++b) {
        const int k0 = b * 64, bs = std::min(64, r0 - k0), rest = r0 - k0 - bs;
        CHK(mm(Di + (long)b * 4096, 64, 0, Bw + k0, r0, 0, X + k0, r0, bs, p, bs, 1.0, 0.0));
        CHK(mm(Lp + (k0 + bs) + (long)k0 * r0, r0, 0, X + k0, r0, 0, Bw + k0 + bs, r0, rest, p, bs, -1.0, 1.0));
    }
    // the new columns' Schur complement and its full-rank Cholesky
    HIPCHK(launch_copy(A + n_old + (long)n_old * lda, lda, S, p, hdim(p), hdim(p), c->stream));
    CHK(mm(X, r0, 1, X, r0, 0, S, p, p, p, r0, -1.0, 1.0, GEMM_LOWER));
    HIPCHK(launch_fill(L + (long)r0 * ldl, ldl, n_old, p, 0.0, c->stream));   // zeros above the new pivots
    CHK(run_frchol(c, sub, S, p, p, tol_new, LS, p, ps, ds));
    // Woodbury's H = I + X' M0 X (Z = M0 X), read back with the new rank
    CHK(mm(M, ldm, 0, X, r0, 0, Z, r0, r0, p, r0, 1.0, 0.0));
    HIPCHK(launch_ns_scaled_eye(H, p, p, 1.0, c->stream));
    CHK(mm(X, r0, 1, Z, r0, 0, H, p, p, p, r0, 1.0, 1.0));
    std::vector<double> hdiag(p);
    HIPCHK(launch_copy(H, p + 1, ds + p, 1, hdim(1), hdim(p), c->stream));   // diag(H) behind ds
    HIPCHK(hipMemcpyAsync(hdiag.data(), ds + p, sizeof(double) * p, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipMemcpyAsync(c->hpin, at<int>(c, sub.rank) + (p + FR_NB - 1) / FR_NB, sizeof(int), hipMemcpyDeviceToHost,
                          c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    const int rs = *c->hpin;
    if (rs < 0 || rs > p) return GENINV_EHIP;
    double htrace = 0.0;
    for (double v : hdiag) htrace += v;
    HIPCHK(launch_transpose(X, r0, L + n_old, ldl, r0, p, c->stream));
    if (rs > 0) {
        HIPCHK(launch_copy(LS, p, L + n_old + (long)r0 * ldl, ldl, hdim(p), hdim(rs), c->stream));
        HIPCHK(launch_offset_int(ps, rs, n_old, piv + r0, c->stream));
    }
    HIPCHK(launch_copy(ds, 1, dvals + n_old, 1, hdim(1), hdim(p), c->stream));

    // M = (L'L)^-1 for the extended L = [L_old 0; X' LS]:
    //   L'L = [B11 B12; B12' LS'LS] with B11 = L_old'L_old + X X', B12 = X LS;
    //   B11^-1 = M0 - Z (I + X'Z)^-1 Z'  (Z = M0 X, Woodbury);
    //   with U = B11^-1 B12 and T = LS'LS - B12' U (Schur complement):
    //   M = [B11^-1 + U T^-1 U', -U T^-1; -T^-1 U', T^-1].
    // Woodbury's subtraction loses about u ||H|| relative: when the new rows
    // dominate (trace(H) above 2 p + 64, e.g. appended columns that are
    // combinations of many earlier ones), M is formed from the extended L
    // directly instead (L'L on the matrix cores and its Gauss-Jordan
    // inverse, O(r^3)).
    if (htrace > 2.0 * p + 64.0) {
        const int r = r0 + rs;
        CHK(run_factor_inverse(c, full, L, ldl, n, hdim(r), M, ldm));
        *rank_io = r;
        *tol_io = tol_new;
        return geninv_sync_status(c);
    }
    CHK(run_spdinv(c, sub, H, p, hdim(p)));
    CHK(mm(Z, r0, 0, H, p, 0, Q, r0, r0, p, p, 1.0, 0.0));
    CHK(mm(Q, r0, 0, Z, r0, 1, M, ldm, r0, r0, p, -1.0, 1.0));
    if (rs > 0) {
        CHK(mm(X, r0, 0, LS, p, 0, B12, r0, r0, rs, p, 1.0, 0.0));
        CHK(mm(M, ldm, 0, B12, r0, 0, U, r0, r0, rs, r0, 1.0, 0.0));
        CHK(mm(LS, p, 1, LS, p, 0, T, p, rs, rs, p, 1.0, 0.0));
        CHK(mm(B12, r0, 1, U, r0, 0, T, p, rs, rs, r0, -1.0, 1.0));
        CHK(run_spdinv(c, sub, T, p, hdim(rs)));
        CHK(mm(U, r0, 0, T, p, 0, V, r0, r0, rs, rs, 1.0, 0.0));
        CHK(mm(V, r0, 0, U, r0, 1, M, ldm, r0, r0, rs, 1.0, 1.0));                     // + U T^-1 U'
        CHK(mm(U, r0, 0, T, p, 0, M + (long)r0 * ldm, ldm, r0, rs, rs, -1.0, 0.0));   // -U T^-1
        CHK(mm(T, p, 0, U, r0, 1, M + r0, ldm, rs, r0, rs, -1.0, 0.0));               // -T^-1 U'
        HIPCHK(launch_copy(T, p, M + r0 + (long)r0 * ldm, ldm, hdim(rs), hdim(rs), c->stream));
    }
    *rank_io = r0 + rs;
    *tol_io = tol_new;
    int st = 0;
    HIPCHK(hipMemcpyAsync(&st, c->status, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    if (st != 0) {
        int zero = 0;
        HIPCHK(hipMemcpy(c->status, &zero, sizeof(int), hipMemcpyHostToDevice));
    }
    return st;
}

int geninv_factored_lstsq(geninv_ctx *c, int n, int r, int k, const double *L, int ldl, const double *M, int ldm,
                          const double *B, int ldb, double *W, int ldw) {
    if (!c || n < 0 || r < 0 || r > n || k < 0) return GENINV_EINVAL;
    if (n == 0 || k == 0) return GENINV_OK;
    if (!W || !B || bad_ld(ldw, n) || bad_ld(ldb, n)) return GENINV_EINVAL;
    DeviceGuard g(c->device);
    if (r == 0) {
        HIPCHK(launch_fill(W, ldw, n, k, 0.0, c->stream));
        return GENINV_OK;
    }
    if (!L || !M || bad_ld(ldl, n) || bad_ld(ldm, r)) return GENINV_EINVAL;
    size_t off = 0;
    const size_t o1 = off;
    off += align256(sizeof(double) * r * (size_t)k);
    const size_t o2 = off;
    off += align256(sizeof(double) * r * (size_t)k);
    CHK(ensure_ws(c, off));
    double *T1 = at<double>(c, o1), *T2 = at<double>(c, o2);
    // W = L (M (M (L' B)))
    HIPCHK(launch_dgemm(gemm(L, ldl, 1, B, ldb, 0, T1, r, hdim(r), hdim(k), hdim(n), 1.0, 0.0), c->stream));
    HIPCHK(launch_dgemm(gemm(M, ldm, 0, T1, r, 0, T2, r, hdim(r), hdim(k), hdim(r), 1.0, 0.0), c->stream));
    HIPCHK(launch_dgemm(gemm(M, ldm, 0, T2, r, 0, T1, r, hdim(r), hdim(k), hdim(r), 1.0, 0.0), c->stream));
    HIPCHK(launch_dgemm(gemm(L, ldl, 0, T1, r, 0, W, ldw, hdim(n), hdim(k), hdim(r), 1.0, 0.0), c->stream));
    return GENINV_OK;
}

int geninv_dlstsq_gram(geninv_ctx *c, int n, int k, const double *A, int lda, const double *B, int ldb, double tol,
                       double *W, int ldw, int *rank) {
    if (!c || n < 0 || k < 0) return GENINV_EINVAL;
    if (n == 0) {
        if (rank) *rank = 0;
        return GENINV_OK;
    }
    if (!A || bad_ld(lda, n) || (k > 0 && (!B || !W || bad_ld(ldb, n) || bad_ld(ldw, n)))) return GENINV_EINVAL;
    if (k > 4096) return GENINV_ENOTSUP;
    DeviceGuard g(c->device);
    const int nn = n;
    const Layout lay = make_layout(nn, k, 0);
    CHK(ensure_ws(c, lay.total));
    double *Aw = at<double>(c, lay.slotA);
    double *L = at<double>(c, lay.slotL);
    double *T1 = at<double>(c, lay.t1);
    double *T2 = at<double>(c, lay.t2);
    const long ld = nn;
    // the factorization overwrites its Gram matrix: work on a copy
    HIPCHK(launch_copy(A, lda, Aw, ld, hdim(nn), hdim(nn), c->stream));
    CHK(run_frchol(c, lay, Aw, ld, nn, tol, L, ld, at<int>(c, lay.piv), at<double>(c, lay.dvals)));
    const int *rdev = at<int>(c, lay.rank) + (nn + FR_NB - 1) / FR_NB;
    Dim r;
    CHK(rank_dim(c, nn, rdev, &r));
    CHK(run_factor_inverse(c, lay, L, ld, nn, r, Aw, ld));
    if (k > 0) {
        // W = L (M (M (L' B)))
        ProfScope ps(c, PC_LSTSQ, 0.0);
        HIPCHK(launch_dgemm(gemm(L, ld, 1, B, ldb, 0, T1, ld, r, hdim(k), hdim(nn), 1.0, 0.0), c->stream));
        HIPCHK(launch_dgemm(gemm(Aw, ld, 0, T1, ld, 0, T2, ld, r, hdim(k), r, 1.0, 0.0), c->stream));
        HIPCHK(launch_dgemm(gemm(Aw, ld, 0, T2, ld, 0, T1, ld, r, hdim(k), r, 1.0, 0.0), c->stream));
        HIPCHK(launch_dgemm(gemm(L, ld, 0, T1, ld, 0, W, ldw, hdim(nn), hdim(k), r, 1.0, 0.0), c->stream));
    }
    return finish_rank(c, rdev, rank);
}

int geninv_bslice(geninv_ctx *c, int rows, int cols, const double *X, int ldx, int slices, int transposed,
                  void *planes, int ldp, int *e) {
    if (!c || rows < 0 || cols < 0 || slices < 1 || slices > 6) return GENINV_EINVAL;
    if (rows == 0 || cols == 0) return GENINV_OK;
    if (!X || !planes || !e || bad_ld(ldx, rows)) return GENINV_EINVAL;
    if (bad_ld(ldp, transposed ? cols : rows) || ldp % 8 != 0 || (reinterpret_cast<uintptr_t>(planes) & 15))
        return GENINV_EINVAL;
    DeviceGuard g(c->device);
    __bf16 *P = static_cast<__bf16 *>(planes);
    if (!transposed) {
        HIPCHK(launch_col_exponents(X, ldx, rows, cols, e, c->stream));
        HIPCHK(launch_slice_cols(X, ldx, rows, cols, e, slices, P, ldp, (long)ldp * cols, c->stream));
    } else {
        HIPCHK(launch_row_exponents(X, ldx, rows, cols, e, c->stream));
        HIPCHK(launch_slice_rows_t(X, ldx, rows, cols, e, slices, P, ldp, (long)ldp * rows, c->stream));
    }
    return GENINV_OK;
}

int geninv_bgram(geninv_ctx *c, int m, int n, const double *G, int ldg, int slices, double *A, int lda) {
    if (!c || m < 0 || n < 0 || slices < 1 || slices > SG_MAX_S) return GENINV_EINVAL;
    if (n == 0) return GENINV_OK;
    if (!A || bad_ld(lda, n) || (m > 0 && (!G || bad_ld(ldg, m)))) return GENINV_EINVAL;
    DeviceGuard g(c->device);
    const MixedLayout ml = make_mixed_layout(0, std::max(m, 1), n, slices, 0, false);
    CHK(ensure_ws(c, ml.total));
    __bf16 *Gc = at<__bf16>(c, ml.gc);
    int *ecg = at<int>(c, ml.ecg);
    const long mp = pad64(std::max(m, 1));
    if (m == 0) {
        HIPCHK(launch_fill(A, lda, n, n, 0.0, c->stream));
        return GENINV_OK;
    }
    HIPCHK(launch_col_exponents(G, ldg, m, n, ecg, c->stream));
    HIPCHK(launch_slice_cols(G, ldg, m, n, ecg, slices, Gc, mp, mp * n, c->stream));
    ProfScope ps(c, PC_GRAM, 0.5 * slices * (slices + 1) * (double)m * n * (n + 1.0));
    return run_sliced(c, sliced(Gc, mp, mp * n, Gc, mp, mp * n, slices, ecg, ecg, A, lda, n, n, (int)mp, 1),
                      ml.gpart ? at<double>(c, ml.gpart) : nullptr, ml.gpart_elems);
}

int geninv_bchain(geninv_ctx *c, int n, int m, int k, const double *P, int ldp, const double *G, int ldg, int slices,
                  double *Y, int ldy) {
    if (!c || n < 0 || m < 0 || k < 0 || slices < 1 || slices > SG_MAX_S) return GENINV_EINVAL;
    if (n == 0 || m == 0) return GENINV_OK;
    if (!Y || bad_ld(ldy, n) || (k > 0 && (!P || !G || bad_ld(ldp, n) || bad_ld(ldg, m)))) return GENINV_EINVAL;
    DeviceGuard g(c->device);
    if (k == 0) {
        HIPCHK(launch_fill(Y, ldy, n, m, 0.0, c->stream));
        return GENINV_OK;
    }
    const long kp = pad64(k);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += align256(bytes);
        return o;
    };
    const size_t opa = take((size_t)slices * kp * n * sizeof(__bf16));
    const size_t opb = take((size_t)slices * kp * m * sizeof(__bf16));
    const size_t oea = take((size_t)n * sizeof(int));
    const size_t oeb = take((size_t)m * sizeof(int));
    CHK(ensure_ws(c, off));
    __bf16 *Pa = at<__bf16>(c, opa), *Gb = at<__bf16>(c, opb);
    int *ea = at<int>(c, oea), *eb = at<int>(c, oeb);
    HIPCHK(launch_row_exponents(P, ldp, n, k, ea, c->stream));
    HIPCHK(launch_slice_rows_t(P, ldp, n, k, ea, slices, Pa, kp, kp * n, c->stream));
    HIPCHK(launch_row_exponents(G, ldg, m, k, eb, c->stream));
    HIPCHK(launch_slice_rows_t(G, ldg, m, k, eb, slices, Gb, kp, kp * m, c->stream));
    SlicedGemmArgs sg = sliced(Pa, kp, kp * n, Gb, kp, kp * m, slices, ea, eb, Y, ldy, n, m, (int)kp, 0);
    sg.nclass = sliced_chain_classes(slices);
    return run_sliced(c, sg, nullptr, 0);
}

// The error estimate of a mixed result (geninv_mixed), from PROBES random
// sign vectors and float64 products with the caller's G:
//   resA = ||A_e V - G'(G V)|| / ||G'(G V)||, the engine's Gram matrix A_e
//          against float64 products (its representation error, measured);
//   kappa = max_k A_kk / (smallest accepted pivot), the factorization's
//          amplification of a relative Gram perturbation into P;
//   resY = ||Y V' - P (G' V')|| / ||P (G' V')||, the engine's chain product
//          against float64 products on the same P (measured).
// err_est = kappa resA + resY: a first-order estimate of the relative change
// the engine makes to Y against the float64 form on the same G (Frobenius
// norms estimated from the probes, relative spread about 1 / sqrt(2 PROBES)).
struct MixedProbe {
    double *blk, *nrm;
    long L;
    double *skin;   // (max(PROBE_PART, L) + L) PROBES doubles of scratch for probe_mm
    double *col(int i) const { return blk + (long)i * L * PROBES; }
};

// C (M x PROBES, leading dimension pr.L) = op(X) B, B K x PROBES (ldb): a
// product with 16 columns and a long K reads X once and is bound by HBM, so
// it runs on the bandwidth kernels of skinny.hip (X in place, or X' through
// the transposed form), split into chunks of K so that about a thousand
// workgroups stream X (at most PROBE_PART / M chunks: the partial sums' room).
int probe_mm(geninv_ctx *c, const MixedProbe &pr, const double *X, long ldx, int tX, const double *B, long ldb,
             double *C, int M, int K) {
    const int p = PROBES;
    if (M <= 0) return GENINV_OK;
    if (K <= 0) {
        HIPCHK(launch_fill(C, pr.L, M, p, 0.0, c->stream));
        return GENINV_OK;
    }
    double *part = pr.skin, *Bt = pr.skin + std::max(PROBE_PART, pr.L) * p;
    const long blocks = tX ? (M + 15) / 16 : (M + 255) / 256;   // workgroups per chunk of K
    const int S = (int)std::max<long>(1, std::min<long>({64L, (1024 + blocks - 1) / blocks, (long)K / 256,
                                                         PROBE_PART / M}));
    const int kchunk = (K + S - 1) / S;
    if (!tX)
        HIPCHK(launch_skinny_gemm(X, ldx, B, ldb, 0, M, p, K, 1.0, 0.0, C, pr.L, kchunk, Bt, part, c->stream));
    else
        HIPCHK(launch_skinny_gemm_t(X, ldx, B, ldb, M, p, K, 1.0, 0.0, C, pr.L, kchunk, part, c->stream));
    return GENINV_OK;
}

// resA terms (nrm[0], nrm[1]) right after the Gram matrix, mirrored to full
// in A (the factorization reads only the lower triangle), and its diagonal
// into nrm + 8 ..
int probe_gram(geninv_ctx *c, const Layout &lay, const MixedProbe &pr, int m, int n, const double *G, long ldg,
               const double *A, long lda, double *diag) {
    const bool tr = m < n;
    const int nn = tr ? m : n;
    const int p = PROBES;
    const long L = pr.L;
    double *V = pr.col(0), *W1 = pr.col(1), *W2 = pr.col(2), *U = pr.col(3);
    auto mm_ = [&](const double *X, long ldx, int tX, const double *Bm, long ldb, double *Cm, int M, int K) {
        return probe_mm(c, pr, X, ldx, tX, Bm, ldb, Cm, M, K);
    };
    HIPCHK(launch_fill(pr.nrm, 8, 8, 1, 0.0, c->stream));
    HIPCHK(launch_copy(A, lda + 1, diag, 1, hdim(1), hdim(nn), c->stream));
    HIPCHK(launch_probe_fill(V, L, nn, p, 0x5eed0001ULL, c->stream));
    CHK(mm_(A, lda, 0, V, L, U, nn, nn));
    if (!tr) {
        CHK(mm_(G, ldg, 0, V, L, W1, m, n));     // G V   (m x p)
        CHK(mm_(G, ldg, 1, W1, L, W2, n, m));    // G' W1 (n x p)
    } else {
        CHK(mm_(G, ldg, 1, V, L, W1, n, m));     // G' V  (n x p)
        CHK(mm_(G, ldg, 0, W1, L, W2, m, n));    // G W1  (m x p)
    }
    HIPCHK(launch_diff_fro2(U, L, W2, L, nn, p, pr.nrm, c->stream));
    return GENINV_OK;
}

// resY terms (nrm[2], nrm[3]) and kappa (nrm[4]) after the chain; one host
// synchronization for all of them.
int probe_finish(geninv_ctx *c, const Layout &lay, const MixedProbe &pr, int m, int n, const double *G, long ldg,
                 const double *P, long ldp, const double *Y, long ldy, const double *diag, const int *rdev,
                 const int *pv, double *est) {
    const bool tr = m < n;
    const int nn = tr ? m : n;
    const int p = PROBES;
    const long L = pr.L;
    double *Oy = pr.col(4), *T = pr.col(5), *Yr = pr.col(6), *Yo = pr.col(7);
    auto mm_ = [&](const double *X, long ldx, int tX, const double *Bm, long ldb, double *Cm, int M, int K) {
        return probe_mm(c, pr, X, ldx, tX, Bm, ldb, Cm, M, K);
    };
    HIPCHK(launch_probe_fill(Oy, L, m, p, 0x5eed0002ULL, c->stream));
    CHK(mm_(Y, ldy, 0, Oy, L, Yo, n, m));
    if (!tr) {
        CHK(mm_(G, ldg, 1, Oy, L, T, n, m));     // G' V'
        CHK(mm_(P, ldp, 0, T, L, Yr, n, n));     // P (G' V')
    } else {
        CHK(mm_(P, ldp, 0, Oy, L, T, m, m));     // P V'
        CHK(mm_(G, ldg, 1, T, L, Yr, n, m));     // G' (P V')
    }
    HIPCHK(launch_diff_fro2(Yo, L, Yr, L, n, p, pr.nrm + 2, c->stream));
    HIPCHK(launch_kappa(diag, at<double>(c, lay.dvals), pv, rdev, nn, pr.nrm + 4, c->stream));
    double h[5] = {0, 0, 0, 0, 0};
    HIPCHK(hipMemcpyAsync(h, pr.nrm, sizeof(h), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    const double resA = h[1] > 0.0 ? std::sqrt(h[0] / h[1]) : 0.0;
    const double resY = h[3] > 0.0 ? std::sqrt(h[2] / h[3]) : 0.0;
    *est = h[4] * resA + resY;
    if (!std::isfinite(*est)) *est = std::numeric_limits<double>::infinity();
    return GENINV_OK;
}

int geninv_mixed(geninv_ctx *c, int m, int n, const double *G, int ldg, double tol, int precision, int gram_digits,
                 int chain_digits, int ns_steps, double target, double *Y, int ldy, int *rank, int *piv,
                 double *err_est) {
    if (!c || m < 0 || n < 0 || ns_steps < 0 || ns_steps > 16) return GENINV_EINVAL;
    if (precision == GENINV_MIXED_BF16) {
        if (gram_digits < 1 || gram_digits > SG_MAX_S || chain_digits < 0 || chain_digits > SG_MAX_S)
            return GENINV_EINVAL;
    } else if (precision == GENINV_MIXED_INT8) {
        if (gram_digits < 1 || gram_digits > MOD_MAX || chain_digits < 0 || chain_digits > MOD_MAX)
            return GENINV_EINVAL;
    } else {
        return GENINV_EINVAL;
    }
    if (err_est) *err_est = 0.0;
    if (m == 0 || n == 0) {
        if (rank) *rank = 0;
        return GENINV_OK;
    }
    if (!G || !Y || bad_ld(ldg, m) || bad_ld(ldy, n)) return GENINV_EINVAL;
    DeviceGuard g(c->device);
    const bool tr = m < n;                 // Appendix: factor G G' when m < n
    const int nn = tr ? m : n, mm = tr ? n : m;
    const Layout lay = make_layout(nn, PROBES);
    MixedPlan mp;
    CHK(make_mixed_plan(lay.total, m, n, precision, gram_digits, chain_digits, ns_steps, mp));
    CHK(ensure_ws(c, mp.total));
    double *A = at<double>(c, lay.slotA);
    double *L = at<double>(c, lay.slotL);
    double *K = at<double>(c, lay.slotK);
    double *P = at<double>(c, lay.slotP);
    int *pv = piv ? piv : at<int>(c, lay.piv);
    const long ld = nn;

    // 1. Gram matrix (lower triangle) on the engine: G'G, or G G' when m < n
    if (precision == GENINV_MIXED_BF16) {
        const int s = gram_digits;
        __bf16 *Gc = at<__bf16>(c, mp.bf.gc);
        int *eg = at<int>(c, mp.bf.ecg);
        const long kp = pad64(mm);
        {
            ProfScope ps(c, PC_SLICE, 0.0);
            if (!tr) {
                HIPCHK(launch_col_exponents(G, ldg, m, n, eg, c->stream));
                HIPCHK(launch_slice_cols(G, ldg, m, n, eg, s, Gc, kp, kp * nn, c->stream));
            } else {
                HIPCHK(launch_row_exponents(G, ldg, m, n, eg, c->stream));
                HIPCHK(launch_slice_rows_t(G, ldg, m, n, eg, s, Gc, kp, kp * nn, c->stream));
            }
        }
        ProfScope ps(c, PC_GRAM, (double)mm * nn * (nn + 1.0));
        CHK(run_sliced(c, sliced(Gc, kp, kp * nn, Gc, kp, kp * nn, s, eg, eg, A, ld, nn, nn, (int)kp, 1),
                       mp.bf.gpart ? at<double>(c, mp.bf.gpart) : nullptr, mp.bf.gpart_elems));
    } else {
        ProfScope ps(c, PC_GRAM, (double)mm * nn * (nn + 1.0));
        CHK(run_mod_product(c, mp.pg, mp.mg, tr ? 0 : 1, G, ldg, tr ? 1 : 0, G, ldg, A, ld));
    }
    const bool estimate = err_est || target > 0.0;
    const MixedProbe pr{at<double>(c, mp.probe), at<double>(c, mp.norms), mp.pld, at<double>(c, mp.skin)};
    double *diag = pr.nrm + 8;
    if (estimate) {
        HIPCHK(launch_mirror_lower(A, ld, hdim(nn), c->stream));
        CHK(probe_gram(c, lay, pr, m, n, G, ldg, A, ld, diag));
    }
    // 2-4. tolerance, full-rank Cholesky, (L'L)^-1 in float64
    CHK(run_frchol(c, lay, A, ld, nn, tol, L, ld, pv, at<double>(c, lay.dvals)));
    const int *rdev = at<int>(c, lay.rank) + (nn + FR_NB - 1) / FR_NB;
    Dim r;
    CHK(rank_dim(c, nn, rdev, &r));
    CHK(run_factor_inverse(c, lay, L, ld, nn, r, A, ld));
    // 5. K = L M, P = K K' (float64)
    {
        ProfScope ps(c, PC_CHAIN_K, 0.0);
        CHK(gemm_fill(c, lay, chain(gemm(L, ld, 0, A, ld, 0, K, ld, hdim(nn), r, r, 1.0, 0.0))));
    }
    {
        ProfScope ps(c, PC_CHAIN_P, 0.0);
        CHK(gemm_fill(c, lay, chain(gemm(K, ld, 0, K, ld, 1, P, ld, hdim(nn), hdim(nn), r, 1.0, 0.0, GEMM_LOWER))));
        HIPCHK(launch_mirror_lower(P, ld, hdim(nn), c->stream));
    }
    // 6. Newton-Schulz steps X <- X (2I - G_r X) in the factored form on P
    //    (X = P G'): P <- 2P - P (L L') P, float64 products.  L L' is the
    //    Gram matrix of the columns the factorization kept; P = (L L')^+ is
    //    the method's own fixed point, so the steps correct the rounding of
    //    (L'L)^-1, K and P.  (Against the full Gram matrix A the step would
    //    not converge on rank-deficient inputs: A - L L' holds the dropped
    //    pivots, up to tol, and P (A - L L') P is of the order of P itself
    //    once accepted pivots come near tol.)  A step is taken only while
    //    its correction ||P L L' P - P||_F / ||P||_F keeps falling.
    double prev = std::numeric_limits<double>::infinity();
    for (int it = 0; it < ns_steps; ++it) {
        ProfScope ps(c, PC_NS, 3.0 * nn * (double)nn * r.host);
        double *T = A;   // M is no longer needed: T = P L (nn x r)
        CHK(gemm_fill(c, lay, gemm(P, ld, 0, L, ld, 0, T, ld, hdim(nn), r, hdim(nn), 1.0, 0.0)));
        CHK(gemm_fill(c, lay, gemm(T, ld, 0, T, ld, 1, K, ld, hdim(nn), hdim(nn), r, 1.0, 0.0, GEMM_LOWER)));
        HIPCHK(launch_mirror_lower(K, ld, hdim(nn), c->stream));
        HIPCHK(launch_fill(pr.nrm + 6, 2, 2, 1, 0.0, c->stream));
        HIPCHK(launch_diff_fro2(K, ld, P, ld, nn, nn, pr.nrm + 6, c->stream));
        double h[2] = {0, 0};
        HIPCHK(hipMemcpyAsync(h, pr.nrm + 6, sizeof(h), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        const double corr = h[1] > 0.0 ? std::sqrt(h[0] / h[1]) : 0.0;
        if (!(corr < prev)) break;
        prev = corr;
        // K = P L L' P;  P <- 2P - K (both exactly symmetric)
        HIPCHK(launch_axpby(K, ld, P, ld, hdim(nn), hdim(nn), -1.0, 2.0, c->stream));
    }
    // 7. Y = P G' (G' P in the transpose branch)
    if (chain_digits == 0) {
        ProfScope ps(c, PC_CHAIN_Y, 2.0 * n * m * (double)nn);
        if (!tr) HIPCHK(launch_dgemm(chain(gemm(P, ld, 0, G, ldg, 1, Y, ldy, hdim(n), hdim(m), hdim(n), 1.0, 0.0)),
                                     c->stream));
        else HIPCHK(launch_dgemm(chain(gemm(G, ldg, 1, P, ld, 0, Y, ldy, hdim(n), hdim(m), hdim(m), 1.0, 0.0)),
                                 c->stream));
    } else if (precision == GENINV_MIXED_BF16) {
        const int s = chain_digits;
        __bf16 *Gt = at<__bf16>(c, mp.bf.gt);
        __bf16 *Pc = at<__bf16>(c, mp.bf.pc);
        int *eg = at<int>(c, mp.bf.erg);
        int *ep = at<int>(c, mp.bf.ep);
        const long np = pad64(nn);
        {
            ProfScope ps(c, PC_SLICE, 0.0);
            // P is symmetric: its column slices are its row slices
            HIPCHK(launch_col_exponents(P, ld, nn, nn, ep, c->stream));
            HIPCHK(launch_slice_cols(P, ld, nn, nn, ep, s, Pc, np, np * nn, c->stream));
            if (!tr) {   // rows of G (columns of G')
                HIPCHK(launch_row_exponents(G, ldg, m, n, eg, c->stream));
                HIPCHK(launch_slice_rows_t(G, ldg, m, n, eg, s, Gt, np, np * m, c->stream));
            } else {     // columns of G (rows of G')
                HIPCHK(launch_col_exponents(G, ldg, m, n, eg, c->stream));
                HIPCHK(launch_slice_cols(G, ldg, m, n, eg, s, Gt, np, np * n, c->stream));
            }
        }
        ProfScope ps(c, PC_CHAIN_Y, 2.0 * n * m * (double)nn);
        SlicedGemmArgs sg = !tr ? sliced(Pc, np, np * nn, Gt, np, np * m, s, ep, eg, Y, ldy, n, m, (int)np, 0)
                                : sliced(Gt, np, np * n, Pc, np, np * nn, s, eg, ep, Y, ldy, n, m, (int)np, 0);
        sg.nclass = sliced_chain_classes(s);
        CHK(run_sliced(c, sg, nullptr, 0));
    } else {
        ProfScope ps(c, PC_CHAIN_Y, 2.0 * n * m * (double)nn);
        // P symmetric: op(P) = P' through the column slicer
        if (!tr) CHK(run_mod_product(c, mp.pch, mp.mch, 1, P, ld, 1, G, ldg, Y, ldy));
        else CHK(run_mod_product(c, mp.pch, mp.mch, 1, G, ldg, 0, P, ld, Y, ldy));
    }
    // 8. error estimate against float64 products with the caller's G
    double est = 0.0;
    if (estimate) {
        CHK(probe_finish(c, lay, pr, m, n, G, ldg, P, ld, Y, ldy, diag, rdev, pv, &est));
        if (err_est) *err_est = est;
    }
    const int st = finish_rank(c, rdev, rank);
    if (st != GENINV_OK) return st;
    if (target > 0.0 && !(est <= target)) return GENINV_EACCURACY;
    return GENINV_OK;
}

// C = op(A) op(B) (M x N, ldc) on the int8 engine with `moduli` moduli,
// exactly as geninv_mixed forms its products; lower != 0 writes the lower
// triangle of a square product only.
int geninv_mgemm(geninv_ctx *c, int transA, int transB, int M, int N, int K, const double *A, int lda,
                 const double *B, int ldb, int moduli, int lower, double *C, int ldc) {
    if (!c || M < 0 || N < 0 || K < 0 || moduli < 1 || moduli > MOD_MAX) return GENINV_EINVAL;
    if (M == 0 || N == 0) return GENINV_OK;
    if (!C || bad_ld(ldc, M) || (lower && M != N)) return GENINV_EINVAL;
    DeviceGuard g(c->device);
    if (K == 0) {
        HIPCHK(launch_fill(C, ldc, M, N, 0.0, c->stream));
        return GENINV_OK;
    }
    if (!A || !B || bad_ld(lda, transA ? K : M) || bad_ld(ldb, transB ? N : K)) return GENINV_EINVAL;
    ModConsts mc{};
    if (!mod_consts(moduli, mc)) return GENINV_EINVAL;
    const bool same = A == B && lda == ldb && transA && !transB && M == N;
    const ModPlan P = mod_plan(0, M, N, K, mc, same, lower ? 1 : 0);
    if (P.beta < 0) return GENINV_EINVAL;
    CHK(ensure_ws(c, P.total));
    ProfScope ps(c, PC_GEMM, 2.0 * M * N * (double)K);
    return run_mod_product(c, P, mc, transA ? 1 : 0, A, lda, transB ? 1 : 0, B, ldb, C, ldc);
}

}  // extern "C"

// ---- batched least squares ----------------------------------------------

struct geninv_batch_plan {
    geninv_ctx *c = nullptr;
    int batch = 0, k = 0, nmax = 0;
    double tol = 0.0;
    void *desc = nullptr;        // device BatchDesc[batch]
    int *order = nullptr;        // device int[batch], largest problem first
    int *queue = nullptr;        // device work counter
    double *slabs = nullptr;     // device per-workgroup slabs
    int max_grid = 0;
    int *rank = nullptr;         // caller's device int[batch]
    int nl = 0, grid = 0;        // LDS threshold and workgroups (autotuned)
    int ntall = 0;               // order[0 .. ntall): tall problems (m >= n); the rest wide (m < n)
    unsigned long long shape_hash = 0;   // FNV-1a of k and every (m_b, n_b): the autotune cache key
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t graph_stream = nullptr;
    int graph_fallbacks = 0;     // runs that asked for the graph and launched directly
};

namespace {

void plan_drop_graph(geninv_batch_plan *p) {
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    p->exec = nullptr;
    p->graph = nullptr;
    p->graph_stream = nullptr;
}

// tall problems, then (same slabs, same stream) the wide ones; each launch
// has its own queue counter
int plan_launch(geninv_batch_plan *p, hipStream_t s) {
    if (p->ntall > 0)
        HIPCHK(launch_batched(p->desc, p->order, p->ntall, p->k, p->tol, p->nl, p->queue, p->slabs, p->grid, p->nmax,
                              p->rank, p->c->status, s));
    if (p->batch > p->ntall)
        HIPCHK(launch_batched_wide(p->desc, p->order + p->ntall, p->batch - p->ntall, p->k, p->tol, p->nl,
                                   p->queue + 16, p->slabs, p->grid, p->nmax, p->rank, p->c->status, s));
    return GENINV_OK;
}

// LDS threshold -> workgroups per compute unit that fit 160 KB of LDS
int wgs_per_cu(int nl, int nmax, int k) {
    const size_t lds = batched_lds_bytes(nl, nmax, k);
    int w = (int)(160 * 1024 / lds);
    return std::max(1, std::min(w, 4));
}

}  // namespace

extern "C" {

int geninv_batch_plan_destroy(geninv_batch_plan *p);

int geninv_batch_plan_create(geninv_ctx *c, geninv_batch_plan **plan, int batch, const int *m, const int *n, int k,
                             const float *const *G, const int *ldg, const float *const *F, const int *ldf,
                             double *const *W, const int *ldw, double tol, int *rank) {
    if (!c || !plan || batch < 0 || k < 1 || k > BATCH_KMAX) return GENINV_EINVAL;
    *plan = nullptr;
    if (batch > 0 && (!m || !n || !G || !ldg || !F || !ldf || !W || !ldw || !rank)) return GENINV_EINVAL;
    int nmax = 1;
    for (int b = 0; b < batch; ++b) {
        const int nn = std::min(m[b], n[b]);   // order of the factored matrix (G'G, or G G' when m < n)
        if (nn < 1 || nn > BATCH_NMAX || !G[b] || !F[b] || !W[b]) return GENINV_EINVAL;
        if (ldg[b] < m[b] || ldf[b] < m[b] || ldw[b] < n[b]) return GENINV_EINVAL;
        nmax = std::max(nmax, nn);
    }
    DeviceGuard g(c->device);
    geninv_batch_plan *p = new geninv_batch_plan();
    p->c = c;
    p->batch = batch;
    p->k = k;
    p->nmax = nmax;
    p->tol = tol;
    p->rank = rank;
    {
        unsigned long long h = 1469598103934665603ull;
        auto mix = [&](unsigned v) {
            for (int q = 0; q < 4; ++q) {
                h ^= (v >> (8 * q)) & 0xffu;
                h *= 1099511628211ull;
            }
        };
        mix((unsigned)k);
        for (int b = 0; b < batch; ++b) {
            mix((unsigned)m[b]);
            mix((unsigned)n[b]);
        }
        p->shape_hash = h;
    }
    // the tall problems, then the wide ones (two launches), each largest
    // first: estimated work max(m, n) nn^2 + nn^3 with nn = min(m, n) (Gram,
    // then factorization and inverse)
    std::vector<int> order(batch);
    std::iota(order.begin(), order.end(), 0);
    auto work = [&](int q) {
        const double a = std::max(m[q], n[q]), o = std::min(m[q], n[q]);
        return a * o * o + o * o * o;
    };
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        const bool ta = m[a] >= n[a], tb = m[b] >= n[b];
        return ta != tb ? ta : work(a) > work(b);
    });
    p->ntall = 0;
    for (int b = 0; b < batch; ++b) p->ntall += m[b] >= n[b] ? 1 : 0;
    std::vector<char> desc(batched_desc_bytes() * std::max(batch, 1));
    for (int b = 0; b < batch; ++b)
        batched_fill_desc(desc.data() + b * batched_desc_bytes(), G[b], F[b], W[b], m[b], n[b], ldg[b], ldf[b], ldw[b]);
    // default LDS threshold: the largest candidate whose LDS fits a compute unit
    p->nl = 0;
    for (int nl : {128, 96, 64, 48, 32}) {
        const int nlc = std::min(nl, nmax);
        if (batched_lds_bytes(nlc, nmax, k) <= 160 * 1024) {
            p->nl = nlc;
            break;
        }
    }
    p->grid = 256 * wgs_per_cu(p->nl, nmax, k);
    p->max_grid = 256 * 4;
    const size_t slab_bytes = batched_slab_doubles(nmax, k) * sizeof(double) * p->max_grid;
    bool ok = hipMalloc(&p->desc, desc.size()) == hipSuccess &&
              hipMalloc((void **)&p->order, sizeof(int) * std::max(batch, 1)) == hipSuccess &&
              hipMalloc((void **)&p->queue, 256) == hipSuccess &&
              hipMalloc((void **)&p->slabs, slab_bytes) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        geninv_batch_plan_destroy(p);
        return GENINV_ENOMEM;
    }
    if (hipMemcpy(p->desc, desc.data(), desc.size(), hipMemcpyHostToDevice) != hipSuccess ||
        (batch > 0 && hipMemcpy(p->order, order.data(), sizeof(int) * batch, hipMemcpyHostToDevice) != hipSuccess)) {
        geninv_batch_plan_destroy(p);
        return GENINV_EHIP;
    }
    *plan = p;
    return GENINV_OK;
}

int geninv_batch_plan_destroy(geninv_batch_plan *p) {
    if (!p) return GENINV_OK;
    DeviceGuard g(p->c->device);
    (void)hipStreamSynchronize(p->c->stream);
    plan_drop_graph(p);
    if (p->desc) (void)hipFree(p->desc);
    if (p->order) (void)hipFree(p->order);
    if (p->queue) (void)hipFree(p->queue);
    if (p->slabs) (void)hipFree(p->slabs);
    delete p;
    return GENINV_OK;
}

int geninv_lstsq_batched(geninv_ctx *c, int batch, const int *m, const int *n, int k, const float *const *G,
                         const int *ldg, const float *const *F, const int *ldf, double tol, double *const *W,
                         const int *ldw, int *rank, int *status) {
    geninv_batch_plan *p = nullptr;
    CHK(geninv_batch_plan_create(c, &p, batch, m, n, k, G, ldg, F, ldf, W, ldw, tol, rank));
    const int st = geninv_batch_plan_run(p, 0);
    (void)geninv_batch_plan_destroy(p);   // synchronizes the context stream
    if (st != GENINV_OK) return st;
    if (status) *status = geninv_sync_status(c);
    return GENINV_OK;
}

int geninv_batch_plan_set_pivots(geninv_batch_plan *p, int *const *piv) {
    if (!p) return GENINV_EINVAL;
    if (p->batch == 0) return GENINV_OK;
    DeviceGuard g(p->c->device);
    std::vector<char> desc(batched_desc_bytes() * p->batch);
    HIPCHK(hipStreamSynchronize(p->c->stream));
    HIPCHK(hipMemcpy(desc.data(), p->desc, desc.size(), hipMemcpyDeviceToHost));
    for (int b = 0; b < p->batch; ++b) batched_set_piv(desc.data(), b, piv ? piv[b] : nullptr);
    HIPCHK(hipMemcpy(p->desc, desc.data(), desc.size(), hipMemcpyHostToDevice));
    return GENINV_OK;
}

int geninv_batch_plan_config(geninv_batch_plan *p, int nl, int grid) {
    if (!p || nl < 0 || grid < 1 || grid > p->max_grid) return GENINV_EINVAL;
    if (batched_lds_bytes(nl, p->nmax, p->k) > 160 * 1024) return GENINV_EINVAL;
    if (nl != p->nl || grid != p->grid) plan_drop_graph(p);
    p->nl = nl;
    p->grid = grid;
    return GENINV_OK;
}

int geninv_batch_plan_get_config(geninv_batch_plan *p, int *nl, int *grid) {
    if (!p) return GENINV_EINVAL;
    if (nl) *nl = p->nl;
    if (grid) *grid = p->grid;
    return GENINV_OK;
}

int geninv_batch_plan_run(geninv_batch_plan *p, int use_graph) {
    if (!p) return GENINV_EINVAL;
    if (p->batch == 0) return GENINV_OK;
    geninv_ctx *c = p->c;
    DeviceGuard g(c->device);
    ProfScope ps(c, PC_BATCHED, 0.0);
    if (!use_graph || c->stream == nullptr) return plan_launch(p, c->stream);
    // A stream that the caller is already capturing gets the direct launches
    // (they become part of the caller's graph); so does any run whose own
    // capture or instantiation fails.  Either way the run's work is the
    // same, and graph_fallbacks counts it.
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    HIPCHK(hipStreamIsCapturing(c->stream, &cs));
    if (cs != hipStreamCaptureStatusNone) {
        ++p->graph_fallbacks;
        return plan_launch(p, c->stream);
    }
    if (p->exec && p->graph_stream != c->stream) plan_drop_graph(p);
    if (!p->exec) {
        bool ok = hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal) == hipSuccess;
        if (ok) {
            const int st = plan_launch(p, c->stream);
            hipGraph_t graph = nullptr;
            const hipError_t e = hipStreamEndCapture(c->stream, &graph);
            if (st != GENINV_OK || e != hipSuccess) {
                if (graph) (void)hipGraphDestroy(graph);
                if (st != GENINV_OK) return st;   // an argument or launch error, not a capture failure
                ok = false;
            } else {
                p->graph = graph;
                ok = hipGraphInstantiate(&p->exec, graph, nullptr, nullptr, 0) == hipSuccess;
                if (!ok) plan_drop_graph(p);
            }
        }
        if (!ok) {
            (void)hipGetLastError();
            ++p->graph_fallbacks;
            return plan_launch(p, c->stream);
        }
        p->graph_stream = c->stream;
    }
    HIPCHK(hipGraphLaunch(p->exec, c->stream));
    return GENINV_OK;
}

int geninv_batch_plan_graph_fallbacks(const geninv_batch_plan *p) { return p ? p->graph_fallbacks : GENINV_EINVAL; }

}  // extern "C"

// The autotune cache: a text file of lines "key nl grid ms", the key
// naming the library version, the device (architecture and compute units)
// and the batch's shapes (k and every (m_b, n_b), hashed).  Lines that do not
// parse, or whose configuration this plan cannot launch, are ignored; a
// missing or unreadable file means "not cached".
namespace {

std::string cache_key(const geninv_batch_plan *p) {
    hipDeviceProp_t prop{};
    const bool ok = hipGetDeviceProperties(&prop, p->c->device) == hipSuccess;
    char buf[256];
    std::snprintf(buf, sizeof buf, "geninv%d:%s:%dcu:k%d:b%d:%016llx", geninv_version(), ok ? prop.gcnArchName : "?",
                  ok ? prop.multiProcessorCount : 0, p->k, p->batch, p->shape_hash);
    for (char *q = buf; *q; ++q)
        if (*q == ' ' || *q == '\n') *q = '_';
    return buf;
}

bool plan_config_ok(const geninv_batch_plan *p, int nl, int grid) {
    return nl >= 0 && grid >= 1 && grid <= p->max_grid && (nl == 0 || nl <= p->nmax) &&
           batched_lds_bytes(nl, p->nmax, p->k) <= 160 * 1024;
}

// the cached entry for key, if any (the last valid one wins)
// one cache line "key nl grid ms" (exactly four fields)
bool cache_parse(const char *line, char *kbuf, int *nl, int *grid, double *ms) {
    int pos = -1;
    if (std::sscanf(line, "%299s %d %d %lf %n", kbuf, nl, grid, ms, &pos) != 4 || pos < 0) return false;
    return line[pos] == '\0';
}

bool cache_lookup(const char *path, const std::string &key, const geninv_batch_plan *p, int *nl, int *grid,
                  double *ms) {
    FILE *f = std::fopen(path, "r");
    if (!f) return false;
    char line[512], kbuf[300];
    bool found = false;
    while (std::fgets(line, sizeof line, f)) {
        int a = 0, b = 0;
        double x = 0.0;
        if (!cache_parse(line, kbuf, &a, &b, &x)) continue;
        if (key != kbuf || !plan_config_ok(p, a, b) || !(x > 0.0)) continue;
        *nl = a;
        *grid = b;
        *ms = x;
        found = true;
    }
    std::fclose(f);
    return found;
}

// rewrite the file with every other parsable line kept and this key's entry
// replaced; through a temporary file and a rename, so readers never see a
// half-written cache.  Failure to write is not an error of the tuning.
void cache_store(const char *path, const std::string &key, int nl, int grid, double ms) {
    std::vector<std::string> keep;
    if (FILE *f = std::fopen(path, "r")) {
        char line[512], kbuf[300];
        while (std::fgets(line, sizeof line, f)) {
            int a = 0, b = 0;
            double x = 0.0;
            if (!cache_parse(line, kbuf, &a, &b, &x) || key == kbuf) continue;
            std::string l(line);
            if (l.empty() || l.back() != '\n') l += '\n';
            keep.push_back(l);
        }
        std::fclose(f);
    }
    const std::string tmp = std::string(path) + ".tmp";
    FILE *f = std::fopen(tmp.c_str(), "w");
    if (!f) return;
    bool ok = true;
    for (const auto &l : keep) ok = ok && std::fputs(l.c_str(), f) >= 0;
    ok = ok && std::fprintf(f, "%s %d %d %.6f\n", key.c_str(), nl, grid, ms) > 0;
    ok = (std::fclose(f) == 0) && ok;
    if (!ok || std::rename(tmp.c_str(), path) != 0) std::remove(tmp.c_str());
}

}  // namespace

extern "C" {

// Times every (LDS threshold, workgroups per CU) candidate `reps`
// times with events on the context stream and keeps the fastest; with a
// cache path, a cached entry for this batch is taken instead of timing, and
// a new result is stored.
int geninv_batch_plan_autotune(geninv_batch_plan *p, int reps, const char *cache_path, int *best_nl, int *best_grid,
                               double *best_ms, int *from_cache) {
    if (!p || reps < 1) return GENINV_EINVAL;
    geninv_ctx *c = p->c;
    DeviceGuard g(c->device);
    if (from_cache) *from_cache = 0;
    std::string key;
    if (cache_path) {
        key = cache_key(p);
        int nl = 0, grid = 0;
        double ms = 0.0;
        if (cache_lookup(cache_path, key, p, &nl, &grid, &ms)) {
            CHK(geninv_batch_plan_config(p, nl, grid));
            if (best_nl) *best_nl = nl;
            if (best_grid) *best_grid = grid;
            if (best_ms) *best_ms = ms;
            if (from_cache) *from_cache = 1;
            return GENINV_OK;
        }
    }
    const int cand_nl[] = {128, 96, 64, 48, 32, 0};
    hipEvent_t a = nullptr, b = nullptr;
    HIPCHK(hipEventCreate(&a));
    HIPCHK(hipEventCreate(&b));
    double best = 1e300;
    int bnl = p->nl, bgrid = p->grid;
    for (int nl : cand_nl) {
        if (nl > p->nmax && nl != 128) continue;
        const int nlc = std::min(nl, p->nmax);
        if (batched_lds_bytes(nlc, p->nmax, p->k) > 160 * 1024) continue;
        const int w = wgs_per_cu(nlc, p->nmax, p->k);
        for (int ww = 1; ww <= w; ww *= 2) {
            const int grid = 256 * ww;
            plan_drop_graph(p);
            p->nl = nlc;
            p->grid = grid;
            CHK(plan_launch(p, c->stream));   // warm-up
            std::vector<float> t;
            for (int r = 0; r < reps; ++r) {
                HIPCHK(hipEventRecord(a, c->stream));
                CHK(plan_launch(p, c->stream));
                HIPCHK(hipEventRecord(b, c->stream));
                HIPCHK(hipEventSynchronize(b));
                float ms = 0.f;
                HIPCHK(hipEventElapsedTime(&ms, a, b));
                t.push_back(ms);
            }
            std::sort(t.begin(), t.end());
            const double med = t[t.size() / 2];
            if (med < best) {
                best = med;
                bnl = nlc;
                bgrid = grid;
            }
        }
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    plan_drop_graph(p);
    p->nl = bnl;
    p->grid = bgrid;
    if (cache_path) cache_store(cache_path, key, bnl, bgrid, best);
    if (best_nl) *best_nl = bnl;
    if (best_grid) *best_grid = bgrid;
    if (best_ms) *best_ms = best;
    return GENINV_OK;
}

}  // extern "C"
