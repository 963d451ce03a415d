// C-ABI entry points: argument validation, scratch management and the
// orchestration of the kernels for SpAMM products and Newton-Schulz solves.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "internal.h"
#include "spamm.h"

using namespace spk;

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIPCHK(x)                                                                                 \
    do {                                                                                          \
        hipError_t e_ = (x);                                                                      \
        if (e_ != hipSuccess) return fail(SPAMM_EHIP, "%s failed: %s", #x, hipGetErrorString(e_)); \
    } while (0)

#define TRY(x)                     \
    do {                           \
        int s_ = (x);              \
        if (s_ < 0) return s_;     \
    } while (0)

bool valid_leaf(int b) { return b == 16 || b == 32 || b == 64; }
bool valid_prec(int p) { return p == SPAMM_F64 || p == SPAMM_F32 || p == SPAMM_BF16X3; }
size_t elt_size(int prec) { return prec == SPAMM_F64 ? 8 : 4; }

// Named scratch slots owned by a context.
enum Slot {
    S_T0, S_T1, S_T2, S_T3, S_T4,      // tiles
    S_Q0, S_Q1, S_Q2, S_Q3, S_Q4,      // squared-norm pyramids
    S_N0, S_N1, S_N2, S_N3, S_N4,      // leaf norms
    S_CNT0, S_CNT1, S_CNT2,            // per-tile retained counts
    S_KIDX0, S_KIDX1, S_KIDX2,         // per-tile retained-k lists
    S_PART,                            // per-tile NS partial sums
    S_CHECK,                           // input-check partials / column sums
    S_SCAL,                            // device scalars
    S_HIST_R, S_HIST_T, S_HIST_NR,     // per-iteration records
    S_OFFS,                            // triple export offsets
    S_ORDER,                           // Morton order of output tiles
    S_WORK,                            // longest-first work list of one launch
    S_COUNT
};

}  // namespace

struct ProfRec {
    int kind;
    hipEvent_t a, b;
};

struct spamm_ctx {
    int device = 0;
    void *buf[S_COUNT] = {};
    size_t cap[S_COUNT] = {};
    double *pinned = nullptr;  // 64 doubles of pinned host memory
    int order_nb = -1;         // nb for which S_ORDER holds the tile order
    std::vector<double> hist_r, hist_t;
    std::vector<int64_t> hist_nR;
    // launch timing
    bool prof = false;
    std::vector<hipEvent_t> pool;
    size_t pool_used = 0;
    std::vector<ProfRec> recs;
};

namespace {

int ensure(spamm_ctx *ctx, int slot, size_t bytes) {
    if (bytes == 0) bytes = 256;
    if (ctx->cap[slot] >= bytes) return SPAMM_OK;
    if (ctx->buf[slot]) {
        HIPCHK(hipFree(ctx->buf[slot]));
        ctx->buf[slot] = nullptr;
        ctx->cap[slot] = 0;
    }
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(SPAMM_ENOMEM, "hipMalloc(%zu bytes) failed: %s", bytes, hipGetErrorString(e));
    }
    ctx->buf[slot] = p;
    ctx->cap[slot] = bytes;
    return SPAMM_OK;
}

template <typename P>
P *slot_ptr(spamm_ctx *ctx, int slot) {
    return reinterpret_cast<P *>(ctx->buf[slot]);
}

int enter(spamm_ctx *ctx) {
    if (!ctx) return fail(SPAMM_EINVAL, "NULL context");
    HIPCHK(hipSetDevice(ctx->device));
    return SPAMM_OK;
}

// Scratch for `nmat` operands (tiles, pyramids, leaf norms) and `nlist` task lists.
int ensure_mats(spamm_ctx *ctx, const Geom &g, int prec, int nmat, int nlist) {
    const size_t tiles = (size_t)g.nb * g.nb * g.b * g.b * elt_size(prec);
    const size_t pyr = (size_t)pyr_len(g.P) * sizeof(double);
    const size_t nrm = (size_t)g.nb * g.nb * sizeof(double);
    for (int m = 0; m < nmat; ++m) {
        TRY(ensure(ctx, S_T0 + m, tiles));
        TRY(ensure(ctx, S_Q0 + m, pyr));
        TRY(ensure(ctx, S_N0 + m, nrm));
    }
    const size_t cnt = (size_t)g.nb * g.nb * sizeof(int32_t);
    const size_t kidx = (size_t)g.nb * g.nb * g.nb * sizeof(int32_t);
    for (int l = 0; l < nlist; ++l) {
        TRY(ensure(ctx, S_CNT0 + l, cnt));
        TRY(ensure(ctx, S_KIDX0 + l, kidx));
    }
    TRY(ensure(ctx, S_SCAL, 64 * sizeof(double)));
    if (ctx->order_nb != g.nb) {
        TRY(ensure(ctx, S_ORDER, (size_t)g.nb * g.nb * sizeof(int32_t)));
        std::vector<int32_t> order((size_t)g.nb * g.nb);
        tile_order(g.nb, order.data());
        HIPCHK(hipMemcpy(ctx->buf[S_ORDER], order.data(), order.size() * sizeof(int32_t), hipMemcpyHostToDevice));
        ctx->order_nb = g.nb;
    }
    TRY(ensure(ctx, S_WORK, (size_t)2 * g.nb * g.nb * sizeof(int32_t)));
    return SPAMM_OK;
}

enum { K_GEMM = 0, K_CULL = 1, K_PYR = 2, K_NKINDS = 3 };
constexpr size_t PROF_POOL = 16384;

// Records the opening event of a timed launch; returns nullptr when not timing.
hipEvent_t prof_begin(spamm_ctx *ctx, hipStream_t st) {
    if (!ctx->prof || ctx->pool_used + 2 > ctx->pool.size()) return nullptr;
    hipEvent_t a = ctx->pool[ctx->pool_used++];
    if (hipEventRecord(a, st) != hipSuccess) return nullptr;
    return a;
}

void prof_end(spamm_ctx *ctx, hipStream_t st, int kind, hipEvent_t a) {
    if (!a) return;
    hipEvent_t b = ctx->pool[ctx->pool_used++];
    if (hipEventRecord(b, st) != hipSuccess) return;
    ctx->recs.push_back(ProfRec{kind, a, b});
}

#define TIMED(kind, call)                              \
    do {                                               \
        hipEvent_t ev_ = prof_begin(ctx, st);          \
        HIPCHK(call);                                  \
        prof_end(ctx, st, kind, ev_);                  \
    } while (0)

const int32_t *order_of(spamm_ctx *ctx) { return slot_ptr<int32_t>(ctx, S_ORDER); }

// Longest-first work list for the products whose counts are in `probs`.
hipError_t plan_gemm(spamm_ctx *ctx, const Geom &g, const GemmProb *probs, int nprob, hipStream_t st) {
    return launch_lpt_order(g, probs[0].cnt, nprob > 1 ? probs[1].cnt : probs[0].cnt, nprob, order_of(ctx),
                            slot_ptr<int32_t>(ctx, S_WORK), st);
}
const int32_t *work_of(spamm_ctx *ctx) { return slot_ptr<int32_t>(ctx, S_WORK); }

Mat mat_of(spamm_ctx *ctx, int m) {
    Mat x;
    x.tiles = ctx->buf[S_T0 + m];
    x.q = slot_ptr<double>(ctx, S_Q0 + m);
    x.nrm = slot_ptr<double>(ctx, S_N0 + m);
    return x;
}

const double *root_q(const Geom &g, const Mat &m) { return m.q + level_off(g.P, 1); }

// Virtual blocks of the padded tree (index >= nb on the leaf level) are never
// written by any kernel; they must read as zero norm.
hipError_t zero_leaf_levels(spamm_ctx *ctx, const Geom &g, int nmat, hipStream_t st) {
    for (int m = 0; m < nmat; ++m) {
        hipError_t e = hipMemsetAsync(ctx->buf[S_Q0 + m], 0, (size_t)g.P * g.P * sizeof(double), st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

CullProb cull_prob(const Geom &g, const Mat &a, const Mat &b, double tau, spamm_ctx *ctx, int list) {
    CullProb p;
    p.nrmA = a.nrm;
    p.nrmB = b.nrm;
    p.rootA = root_q(g, a);
    p.rootB = root_q(g, b);
    p.tau = tau;
    p.cnt = slot_ptr<int32_t>(ctx, S_CNT0 + list);
    p.kidx = slot_ptr<int32_t>(ctx, S_KIDX0 + list);
    return p;
}

GemmProb gemm_prob(const Mat &a, const Mat &b, const Mat &c, spamm_ctx *ctx, int list, double *part) {
    GemmProb p;
    p.A = a.tiles;
    p.B = b.tiles;
    p.C = c.tiles;
    p.cnt = slot_ptr<int32_t>(ctx, S_CNT0 + list);
    p.kidx = slot_ptr<int32_t>(ctx, S_KIDX0 + list);
    p.qC = c.q;
    p.part = part;
    return p;
}

int kernel_prec(int prec) { return prec == SPAMM_F64 ? P_F64 : P_F32; }

int validate_common(spamm_ctx *ctx, const void *A, int64_t n, int64_t ld, int leaf) {
    if (!ctx) return fail(SPAMM_EINVAL, "NULL context");
    if (!A) return fail(SPAMM_EINVAL, "NULL matrix pointer");
    if (n <= 0) return fail(SPAMM_EINVAL, "n must be positive (got %lld)", (long long)n);
    if (ld < n) return fail(SPAMM_EINVAL, "ld (%lld) < n (%lld)", (long long)ld, (long long)n);
    if (!valid_leaf(leaf)) return fail(SPAMM_EINVAL, "leaf must be 16, 32 or 64 (got %d)", leaf);
    const int64_t nb = (n + leaf - 1) / leaf;
    if (nb > 2048) return fail(SPAMM_EINVAL, "n/leaf too large (%lld blocks per side)", (long long)nb);
    return SPAMM_OK;
}

}  // namespace

extern "C" {

const char *spamm_last_error(void) { return g_err.c_str(); }

int spamm_create(spamm_ctx **out, int device) {
    if (!out) return fail(SPAMM_EINVAL, "NULL output handle");
    *out = nullptr;
    int count = 0;
    HIPCHK(hipGetDeviceCount(&count));
    if (device < 0 || device >= count) return fail(SPAMM_EINVAL, "device %d out of range [0,%d)", device, count);
    HIPCHK(hipSetDevice(device));
    spamm_ctx *ctx = new spamm_ctx();
    ctx->device = device;
    hipError_t e = hipHostMalloc((void **)&ctx->pinned, 64 * sizeof(double), hipHostMallocDefault);
    if (e != hipSuccess) {
        delete ctx;
        return fail(SPAMM_ENOMEM, "hipHostMalloc failed: %s", hipGetErrorString(e));
    }
    *out = ctx;
    return SPAMM_OK;
}

int spamm_destroy(spamm_ctx *ctx) {
    if (!ctx) return SPAMM_OK;
    HIPCHK(hipSetDevice(ctx->device));
    HIPCHK(hipDeviceSynchronize());
    for (hipEvent_t e : ctx->pool) HIPCHK(hipEventDestroy(e));
    for (int s = 0; s < S_COUNT; ++s)
        if (ctx->buf[s]) HIPCHK(hipFree(ctx->buf[s]));
    if (ctx->pinned) HIPCHK(hipHostFree(ctx->pinned));
    delete ctx;
    return SPAMM_OK;
}

int64_t spamm_pyramid_len(int64_t n, int leaf) {
    if (n <= 0 || !valid_leaf(leaf)) return -1;
    const Geom g = make_geom(n, leaf);
    return pyr_len(g.P);
}

int spamm_norms(spamm_ctx *ctx, const double *A, int64_t n, int64_t ld, int leaf, double *pyramid,
                double *root_norm_host, void *stream) {
    TRY(validate_common(ctx, A, n, ld, leaf));
    if (!pyramid) return fail(SPAMM_EINVAL, "NULL pyramid output");
    TRY(enter(ctx));
    hipStream_t st = (hipStream_t)stream;
    const Geom g = make_geom(n, leaf);
    TRY(ensure_mats(ctx, g, SPAMM_F64, 1, 0));
    HIPCHK(zero_leaf_levels(ctx, g, 1, st));
    Mat a = mat_of(ctx, 0);
    HIPCHK(launch_ingest(P_F64, A, ld, 0.0, 1.0, g, a, st));
    TIMED(K_PYR, launch_pyramid(g, a, st));
    HIPCHK(launch_norms_out(g, a.q, pyramid, st));
    if (root_norm_host) {
        HIPCHK(hipMemcpyAsync(ctx->pinned, root_q(g, a), sizeof(double), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        *root_norm_host = std::sqrt(ctx->pinned[0]);
    }
    return SPAMM_OK;
}

int spamm_multiply(spamm_ctx *ctx, const double *A, const double *B, double *C, int64_t n, int64_t ld,
                   double tau, int leaf, int prec, int32_t *triples, int64_t cap, spamm_stats *stats,
                   void *stream) {
    TRY(validate_common(ctx, A, n, ld, leaf));
    if (!B || !C) return fail(SPAMM_EINVAL, "NULL matrix pointer");
    if (!(tau >= 0.0) || std::isinf(tau)) return fail(SPAMM_EINVAL, "tau must be finite and >= 0");
    if (!valid_prec(prec)) return fail(SPAMM_EINVAL, "unknown precision %d", prec);
    if (prec == SPAMM_BF16X3) return fail(SPAMM_EINVAL, "BF16x3 leaves are not available in this build");
    if (triples && cap < 0) return fail(SPAMM_EINVAL, "negative triple capacity");
    TRY(enter(ctx));
    hipStream_t st = (hipStream_t)stream;
    const Geom g = make_geom(n, leaf);
    const int kp = kernel_prec(prec);
    TRY(ensure_mats(ctx, g, prec, 3, 1));
    HIPCHK(zero_leaf_levels(ctx, g, 3, st));
    Mat a = mat_of(ctx, 0), b = mat_of(ctx, 1), c = mat_of(ctx, 2);
    HIPCHK(launch_ingest(kp, A, ld, 0.0, 1.0, g, a, st));
    HIPCHK(launch_ingest(kp, B, ld, 0.0, 1.0, g, b, st));
    TIMED(K_PYR, launch_pyramid2(g, a, b, st));
    CullProb cp = cull_prob(g, a, b, tau, ctx, 0);
    TIMED(K_CULL, launch_cull(g, &cp, 1, st));
    GemmProb gp = gemm_prob(a, b, c, ctx, 0, nullptr);
    HIPCHK(plan_gemm(ctx, g, &gp, 1, st));
    TIMED(K_GEMM, launch_gemm(kp, MODE_PLAIN, g, work_of(ctx), &gp, 1, st));
    HIPCHK(launch_egress(kp, g, c.tiles, C, ld, 1.0, 0, st));
    int status = SPAMM_OK;
    if (stats || triples) {
        TRY(ensure(ctx, S_OFFS, (size_t)g.nb * g.nb * sizeof(int64_t)));
        int64_t *offs = slot_ptr<int64_t>(ctx, S_OFFS);
        int64_t *total = reinterpret_cast<int64_t *>(slot_ptr<double>(ctx, S_SCAL) + 8);
        HIPCHK(launch_count_triples(g, cp.cnt, offs, total, st));
        HIPCHK(hipMemcpyAsync(ctx->pinned, total, sizeof(int64_t), hipMemcpyDeviceToHost, st));
        HIPCHK(hipMemcpyAsync(ctx->pinned + 1, cp.rootA, sizeof(double), hipMemcpyDeviceToHost, st));
        HIPCHK(hipMemcpyAsync(ctx->pinned + 2, cp.rootB, sizeof(double), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        int64_t retained;
        std::memcpy(&retained, ctx->pinned, sizeof(int64_t));
        if (triples) {
            if (retained > cap)
                status = fail(SPAMM_ECAPACITY, "|R| = %lld exceeds triple capacity %lld", (long long)retained,
                              (long long)cap);
            else {
                HIPCHK(launch_write_triples(g, cp.cnt, cp.kidx, offs, triples, st));
                HIPCHK(hipStreamSynchronize(st));
            }
        }
        if (stats) {
            stats->retained = retained;
            stats->possible = (int64_t)g.nb * g.nb * g.nb;
            stats->thr = tau * (std::sqrt(ctx->pinned[1]) * std::sqrt(ctx->pinned[2]));
            stats->flops = 2.0 * (double)leaf * leaf * leaf * (double)retained;
        }
    }
    return status;
}

int ns_sqrt(spamm_ctx *ctx, const double *s, double *Y, double *Z, int64_t n, int64_t ld, double tau,
            double tol, int maxit, const spamm_ns_opts *opts, spamm_ns_result *res, void *stream) {
    spamm_ns_opts o;
    o.leaf = 32;
    o.prec = SPAMM_F64;
    o.tau_s = -1.0;
    o.mu_rel = 0.0;
    o.stagnation_stop = 0;
    if (opts) {
        o = *opts;
        if (o.leaf == 0) o.leaf = 32;
    }
    TRY(validate_common(ctx, s, n, ld, o.leaf));
    if (!Y || !Z) return fail(SPAMM_EINVAL, "NULL output pointer");
    if (!(tau >= 0.0) || std::isinf(tau)) return fail(SPAMM_EINVAL, "tau must be finite and >= 0");
    if (!(tol > 0.0)) return fail(SPAMM_EINVAL, "tol must be > 0");
    if (maxit < 0) return fail(SPAMM_EINVAL, "maxit must be >= 0");
    if (!valid_prec(o.prec)) return fail(SPAMM_EINVAL, "unknown precision %d", o.prec);
    if (o.prec == SPAMM_BF16X3) return fail(SPAMM_EINVAL, "BF16x3 leaves are not available in this build");
    if (!(o.mu_rel >= 0.0) || std::isinf(o.mu_rel)) return fail(SPAMM_EINVAL, "mu_rel must be finite and >= 0");
    if (std::isnan(o.tau_s) || std::isinf(o.tau_s)) return fail(SPAMM_EINVAL, "tau_s must be finite");
    const double tau_s = o.tau_s < 0.0 ? tau : o.tau_s;
    TRY(enter(ctx));
    hipStream_t st = (hipStream_t)stream;
    const Geom g = make_geom(n, o.leaf);
    const int kp = kernel_prec(o.prec);

    // operands: 0,1 = y (ping-pong), 2,3 = z (ping-pong), 4 = h; lists: 0 = x, 1 = y, 2 = z
    TRY(ensure_mats(ctx, g, o.prec, 5, 3));
    const int64_t nbk = (n + 31) / 32;
    TRY(ensure(ctx, S_CHECK, (size_t)std::max<int64_t>(3 * nbk * nbk, n) * sizeof(double)));
    TRY(ensure(ctx, S_PART, (size_t)2 * g.nb * g.nb * sizeof(double)));
    TRY(ensure(ctx, S_HIST_R, (size_t)(maxit + 1) * sizeof(double)));
    TRY(ensure(ctx, S_HIST_T, (size_t)(maxit + 1) * sizeof(double)));
    TRY(ensure(ctx, S_HIST_NR, (size_t)3 * (maxit + 1) * sizeof(int64_t)));
    double *scal = slot_ptr<double>(ctx, S_SCAL);
    double *check = slot_ptr<double>(ctx, S_CHECK);
    double *part = slot_ptr<double>(ctx, S_PART);
    double *hist_r = slot_ptr<double>(ctx, S_HIST_R);
    double *hist_t = slot_ptr<double>(ctx, S_HIST_T);
    int64_t *hist_nR = slot_ptr<int64_t>(ctx, S_HIST_NR);
    double *pin = ctx->pinned;

    // input checks and the Gershgorin scale
    HIPCHK(launch_check_input(s, n, ld, check, scal, st));
    HIPCHK(launch_colsum_max(s, n, ld, 0.0, check, scal + 3, st));
    HIPCHK(hipMemcpyAsync(pin, scal, 4 * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (pin[2] != 0.0) return fail(SPAMM_EINVAL, "s has a NaN or infinite entry");
    if (pin[0] > 1e-14 * pin[1])
        return fail(SPAMM_EINVAL, "s is not symmetric: max|s - s^T| = %g, max|s| = %g", pin[0], pin[1]);
    double mu = 0.0, c = pin[3];
    if (o.mu_rel > 0.0) {
        mu = o.mu_rel * c;
        HIPCHK(launch_colsum_max(s, n, ld, mu, check, scal + 3, st));
        HIPCHK(hipMemcpyAsync(pin, scal + 3, sizeof(double), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        c = pin[0];
    }
    if (!(c > 0.0)) return fail(SPAMM_EINVAL, "s has a zero Gershgorin bound");

    HIPCHK(hipMemsetAsync(hist_nR, 0, (size_t)3 * (maxit + 1) * sizeof(int64_t), st));
    HIPCHK(zero_leaf_levels(ctx, g, 5, st));
    int yi = 0, zi = 2;
    Mat h = mat_of(ctx, 4);
    HIPCHK(launch_ingest(kp, s, ld, mu, c, g, mat_of(ctx, yi), st));
    HIPCHK(launch_identity(kp, g, mat_of(ctx, zi), st));
    TIMED(K_PYR, launch_pyramid2(g, mat_of(ctx, yi), mat_of(ctx, zi), st));

    int status = SPAMM_NOT_CONVERGED;
    int k = 0;
    double r0 = 0.0, r_prev = 0.0, r = 0.0, tk = 0.0;
    int nondecrease = 0;
    for (k = 0;; ++k) {
        Mat y = mat_of(ctx, yi), z = mat_of(ctx, zi);
        CullProb cx = cull_prob(g, y, z, tau, ctx, 0);
        TIMED(K_CULL, launch_cull(g, &cx, 1, st));
        GemmProb gx = gemm_prob(y, z, h, ctx, 0, part);
        HIPCHK(plan_gemm(ctx, g, &gx, 1, st));
        TIMED(K_GEMM, launch_gemm(kp, MODE_NSX, g, work_of(ctx), &gx, 1, st));
        HIPCHK(launch_ns_reduce(g, part, cx.cnt, slot_ptr<int32_t>(ctx, S_CNT1), slot_ptr<int32_t>(ctx, S_CNT2), k,
                                hist_r, hist_t, hist_nR, scal + 8, st));
        TIMED(K_PYR, launch_pyramid(g, h, st));
        HIPCHK(hipMemcpyAsync(pin, scal + 8, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        r = pin[0];
        tk = pin[1];
        if (k == 0) r0 = r;
        if (r < tol) {
            status = SPAMM_OK;
            break;
        }
        if (!std::isfinite(r) || r > 10.0 * std::fmax(r0, std::sqrt((double)n))) {
            status = fail(SPAMM_EDIVERGED, "iteration diverged at k = %d (r = %g)", k, r);
            break;
        }
        if (o.stagnation_stop && k > 0) {
            nondecrease = (r >= 0.99 * r_prev) ? nondecrease + 1 : 0;
            if (nondecrease >= 2) {
                status = SPAMM_STAGNATED;
                break;
            }
        }
        r_prev = r;
        if (k == maxit) {
            status = SPAMM_NOT_CONVERGED;
            break;
        }
        const int yn = yi ^ 1, zn = zi ^ 1;
        Mat ynm = mat_of(ctx, yn), znm = mat_of(ctx, zn);
        CullProb cu[2] = {cull_prob(g, h, y, tau_s, ctx, 1), cull_prob(g, z, h, tau, ctx, 2)};
        TIMED(K_CULL, launch_cull(g, cu, 2, st));
        GemmProb gu[2] = {gemm_prob(h, y, ynm, ctx, 1, nullptr), gemm_prob(z, h, znm, ctx, 2, nullptr)};
        HIPCHK(plan_gemm(ctx, g, gu, 2, st));
        TIMED(K_GEMM, launch_gemm(kp, MODE_PLAIN, g, work_of(ctx), gu, 2, st));
        TIMED(K_PYR, launch_pyramid2(g, ynm, znm, st));
        yi = yn;
        zi = zn;
    }
    const double sc = std::sqrt(c);
    HIPCHK(launch_egress(kp, g, mat_of(ctx, yi).tiles, Y, ld, sc, 0, st));
    HIPCHK(launch_egress(kp, g, mat_of(ctx, zi).tiles, Z, ld, sc, 1, st));
    ctx->hist_r.assign(k + 1, 0.0);
    ctx->hist_t.assign(k + 1, 0.0);
    ctx->hist_nR.assign(3 * (size_t)(k + 1), 0);
    HIPCHK(hipMemcpyAsync(ctx->hist_r.data(), hist_r, (k + 1) * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(ctx->hist_t.data(), hist_t, (k + 1) * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(ctx->hist_nR.data(), hist_nR, 3 * (k + 1) * sizeof(int64_t), hipMemcpyDeviceToHost,
                          st));
    HIPCHK(hipStreamSynchronize(st));
    if (res) {
        res->iterations = k;
        res->resid = r;
        res->trace_err = tk;
        res->scale = c;
        int64_t tot = 0;
        for (int64_t v : ctx->hist_nR) tot += v;
        res->triples_total = tot;
        res->flops_total = 2.0 * (double)o.leaf * o.leaf * o.leaf * (double)tot;
    }
    return status;
}

int spamm_ns_history(spamm_ctx *ctx, double *r, double *t, int64_t *nR, int cap) {
    if (!ctx) return fail(SPAMM_EINVAL, "NULL context");
    if (cap < 0) return fail(SPAMM_EINVAL, "negative capacity");
    const int m = (int)ctx->hist_r.size();
    const int c = m < cap ? m : cap;
    if (r) std::memcpy(r, ctx->hist_r.data(), c * sizeof(double));
    if (t) std::memcpy(t, ctx->hist_t.data(), c * sizeof(double));
    if (nR) std::memcpy(nR, ctx->hist_nR.data(), 3 * (size_t)c * sizeof(int64_t));
    return m;
}

int spamm_profile_enable(spamm_ctx *ctx, int enable) {
    TRY(enter(ctx));
    ctx->recs.clear();
    ctx->pool_used = 0;
    ctx->prof = enable != 0;
    if (ctx->prof && ctx->pool.empty()) {
        ctx->pool.resize(PROF_POOL);
        for (size_t i = 0; i < PROF_POOL; ++i) HIPCHK(hipEventCreate(&ctx->pool[i]));
    }
    return SPAMM_OK;
}

int spamm_profile_reset(spamm_ctx *ctx) {
    if (!ctx) return fail(SPAMM_EINVAL, "NULL context");
    ctx->recs.clear();
    ctx->pool_used = 0;
    return SPAMM_OK;
}

int spamm_profile_read(spamm_ctx *ctx, int kind, double *ms, int cap) {
    TRY(enter(ctx));
    if (kind < 0 || kind >= K_NKINDS) return fail(SPAMM_EINVAL, "unknown launch kind %d", kind);
    if (cap < 0 || (cap > 0 && !ms)) return fail(SPAMM_EINVAL, "bad output buffer");
    int m = 0;
    for (const ProfRec &r : ctx->recs) {
        if (r.kind != kind) continue;
        if (m < cap) {
            float t = 0.f;
            HIPCHK(hipEventElapsedTime(&t, r.a, r.b));
            ms[m] = (double)t;
        }
        ++m;
    }
    return m;
}

}  // extern "C"
