// C-ABI entry points and the Newton-Schulz solve engine.
//
// A solve owns one device arena (its iterates, norm pyramids, task lists,
// records and its device-side state).  Solves are advanced in steps: every
// iteration of every solve of a step is enqueued as a fixed sequence of
// batched launches over product tables (cull, longest-first plan, leaf
// products, stop decision, pyramid; the same for the (y, z) update), and the
// stop decision is taken on the device, so the host synchronises once per
// step, not once per product.  ns_sqrt is begin + steps + finish.
//
// Device memory of the solve engine is recycled, not freed: solve arenas,
// plan tables and pinned read-back buffers return to pools of the context
// when a solve finishes or a plan is dropped, and are taken from them again
// (best fit).  spamm_solve_begin reserves what the solve's group will need,
// so once a context is warm, steps and finishes allocate and free nothing
// (hipFree would also synchronise the whole device, stalling other streams).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "internal.h"
#include "spamm.h"

using namespace spk;

// Static scratch of the allocation-free product (spamm_multiply_noalloc).
// Every GPU the library runs on holds its own copy until the process ends.
// In host code the name is only a stand-in for the symbol: each device's copy
// is located once, with that device current, by hipGetSymbolAddress when a
// context is created on it, and only that address is passed to kernels.
static __device__ __align__(256) char scratch[SPAMM_NOALLOC_BYTES];

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

#define TRY(x)                 \
    do {                       \
        int s_ = (x);          \
        if (s_ < 0) return s_; \
    } while (0)

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_dev[MAX_DEVICES] = {};

// Locates the current device's copy of `scratch` (once per device).
int scratch_setup(int device, void **out) {
    if (device < 0 || device >= MAX_DEVICES) return fail(SPAMM_EINVAL, "device %d beyond %d", device, MAX_DEVICES);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[device]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(SPAMM_EHIP, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
        g_scratch_dev[device] = ptr;
    }
    *out = g_scratch_dev[device];
    return SPAMM_OK;
}

bool valid_leaf(int b) { return b == 16 || b == 32 || b == 64; }
bool valid_prec(int p) { return p == SPAMM_F64 || p == SPAMM_F32 || p == SPAMM_BF16X3 || p == SPAMM_BF16X6; }
bool split_bf16(int p) { return p == SPAMM_BF16X3 || p == SPAMM_BF16X6; }
size_t elt_size(int prec) { return prec == SPAMM_F64 ? 8 : 4; }
// storage type of the tiles: the split-bf16 modes keep FP32 operands and split them inside the leaf product
int kernel_prec(int prec) { return prec == SPAMM_F64 ? P_F64 : P_F32; }
int gemm_prec(int prec) {
    return prec == SPAMM_F64 ? P_F64 : (prec == SPAMM_BF16X3 ? P_BF16X3 : (prec == SPAMM_BF16X6 ? P_BF16X6 : P_F32));
}
constexpr int MAX_NB = 1024;  // the pyramid's two passes cover P <= 1024
static_assert(MAX_NB <= QUAD_NB_MAX, "the quad kernel's k union covers every supported nb");

int64_t round_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

// Bump allocator over one device allocation (256-byte aligned pieces).
struct Carve {
    char *base;
    size_t off;
    template <typename T>
    T *take(size_t count) {
        T *p = reinterpret_cast<T *>(base ? base + off : nullptr);
        off += (size_t)round_up((int64_t)(count * sizeof(T)), 256);
        return p;
    }
};

// Scratch slots of a context (spamm_norms / spamm_multiply / solve set-up).
enum Slot {
    S_T0, S_T1, S_T2,          // tiles
    S_Q0, S_Q1, S_Q2,          // squared-norm pyramids
    S_N0, S_N1, S_N2,          // leaf norms
    S_CNT, S_KIDX,             // task list of the product
    S_CHECK, S_SCAL, S_OFFS,   // input checks, device scalars, triple offsets
    S_TAB,                     // product table of a multiply
    S_COUNT
};

}  // namespace

struct ProfRec {
    int kind;
    hipEvent_t a, b;
};

// A device (or pinned host) allocation kept in a context's pool.
struct Block {
    char *p = nullptr;
    size_t cap = 0;
};

// Device tables for one ordered set of solves of one (precision, leaf).
struct Plan {
    std::vector<unsigned long long> ids;
    int prec = 0, leaf = 0;
    bool damped = false;  // some solve of the set uses the damped map
    bool single = false;  // single-channel solves (a plan holds one instance)
    char *mem = nullptr;
    size_t cap = 0;
    ProdTable tx{}, tyz{};      // dual: x products; the y and z updates
    ProdTable tt{}, ty{}, tz{}; // single: transposes z^T; y = s' z; z updates (x products in tx)
    SolveDesc *solves = nullptr;
    SolveState *gather = nullptr;
    SolveState *gather_host = nullptr;  // pinned
    size_t pin_cap = 0;
    std::vector<char> image;            // host image of the tables (source of their upload)
    int uses = 0;                       // steps that have run this plan
    int nsolve = 0;
    unsigned long long last_use = 0;
    hipGraph_t graph = nullptr;         // one captured iteration of this set
    hipGraphExec_t graph_exec = nullptr;
};

struct spamm_ctx {
    int device = 0;
    void *buf[S_COUNT] = {};
    size_t cap[S_COUNT] = {};
    double *pinned = nullptr;            // 64 doubles of pinned host memory
    std::vector<double> hist_r, hist_t;  // records of the last finished solve
    std::vector<int64_t> hist_nR;
    bool prof = false;
    std::vector<hipEvent_t> pool;
    size_t pool_used = 0;
    std::vector<ProfRec> recs;
    std::vector<Plan *> plans;
    unsigned long long next_id = 1, use_clock = 0;
    bool graphs = true;                   // replay captured iterations when not timing launches
    hipStream_t gstream = nullptr;        // stream the graphs are captured on and replayed on
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    // further replay streams (default priority), one per plan of a step beyond
    // the first, so that the plans of one step run concurrently
    std::vector<hipStream_t> xstream;
    std::vector<hipEvent_t> xdone;
    void *scratch = nullptr;              // this device's copy of the static scratch
    // recycled memory of the solve engine, and the solves begun and not finished
    std::vector<Block> free_arena, free_table, free_pin;
    std::vector<spamm_solve *> live;
    int64_t allocs = 0;                   // device and pinned allocations made so far
    size_t pool_limit = SIZE_MAX;         // device bytes kept in free_arena + free_table at most
};

struct spamm_solve {
    spamm_ctx *ctx;
    unsigned long long id;
    Geom g;
    int prec;
    double tau, tau_s, tol, mu, c;
    int maxit, stagnation, damped, single;
    char *mem;
    size_t bytes;
    // dual: y[parity], z[parity], h.  single: y[0] = s', y[1] = y_k, z[parity],
    // zt = z_k^T, h.
    void *y[2], *z[2], *h, *zt;
    double *qy[2], *qz[2], *qh, *ny[2], *nz[2], *nh, *qzt, *nzt;
    int32_t *cnt[3], *kidx[3];
    double *part, *hist_r, *hist_t;
    int64_t *hist_nR;
    SolveState *state;
    SolveState host_state;
};

namespace {

// ---- pooled memory of the solve engine -------------------------------------
// Takes the smallest pooled block of at least `bytes` (for solve arenas at
// most a quarter more, so a solve holds about its footprint); allocates only
// when none fits.
int pool_take(spamm_ctx *ctx, std::vector<Block> &pool, size_t bytes, bool pinned, Block *out) {
    if (bytes == 0) bytes = 256;
    const bool bounded = &pool == &ctx->free_arena;
    auto best = pool.end();
    for (auto it = pool.begin(); it != pool.end(); ++it)
        if (it->cap >= bytes && (!bounded || it->cap <= bytes + bytes / 4 + (16u << 20)) &&
            (best == pool.end() || it->cap < best->cap))
            best = it;
    if (best != pool.end()) {
        *out = *best;
        pool.erase(best);
        return SPAMM_OK;
    }
    void *p = nullptr;
    const hipError_t e = pinned ? hipHostMalloc(&p, bytes, hipHostMallocDefault) : hipMalloc(&p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(SPAMM_ENOMEM, "%s of %zu bytes failed: %s", pinned ? "hipHostMalloc" : "hipMalloc", bytes,
                    hipGetErrorString(e));
    }
    ++ctx->allocs;
    *out = Block{(char *)p, bytes};
    return SPAMM_OK;
}

size_t pooled_device_bytes(const spamm_ctx *ctx) {
    size_t t = 0;
    for (const Block &b : ctx->free_arena) t += b.cap;
    for (const Block &b : ctx->free_table) t += b.cap;
    return t;
}

void pool_give(std::vector<Block> &pool, Block b) {
    if (b.p) pool.push_back(b);
}

// Device memory returned by a finished solve or a dropped plan: pooled, or
// freed when pooling it would exceed the context's limit (hipFree then
// synchronises the device).
void pool_return(spamm_ctx *ctx, std::vector<Block> &pool, Block b) {
    if (!b.p) return;
    if (pooled_device_bytes(ctx) + b.cap > ctx->pool_limit) {
        (void)hipFree(b.p);
        return;
    }
    pool.push_back(b);
}

// Frees pooled device blocks, largest first, until at most `limit` bytes stay.
void pool_trim(spamm_ctx *ctx, size_t limit) {
    while (pooled_device_bytes(ctx) > limit) {
        std::vector<Block> *from = nullptr;
        size_t at = 0, best = 0;
        for (std::vector<Block> *pl : {&ctx->free_arena, &ctx->free_table})
            for (size_t i = 0; i < pl->size(); ++i)
                if ((*pl)[i].cap >= best) {
                    best = (*pl)[i].cap;
                    from = pl;
                    at = i;
                }
        if (!from) return;
        (void)hipFree((*from)[at].p);
        from->erase(from->begin() + at);
    }
}

// Frees every block of a pool (context teardown, or before retrying an
// allocation that ran out of memory); synchronises the device.
void pool_drain(std::vector<Block> &pool, bool pinned) {
    for (const Block &b : pool) {
        if (pinned)
            (void)hipHostFree(b.p);
        else
            (void)hipFree(b.p);
    }
    pool.clear();
}

// ---- measurement hooks -----------------------------------------------------
enum { K_GEMM = 0, K_CULL = 1, K_PYR = 2, K_NKINDS = 3 };
constexpr size_t PROF_POOL = 16384;

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

#define TIMED(kind, call)                     \
    do {                                      \
        hipEvent_t ev_ = prof_begin(ctx, st); \
        HIPCHK(call);                         \
        prof_end(ctx, st, kind, ev_);         \
    } while (0)

// ---- context scratch -------------------------------------------------------
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
    ++ctx->allocs;
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

int validate_common(spamm_ctx *ctx, const void *A, int64_t n, int64_t ld, int leaf) {
    if (!ctx) return fail(SPAMM_EINVAL, "NULL context");
    if (!A) return fail(SPAMM_EINVAL, "NULL matrix pointer");
    if (n <= 0) return fail(SPAMM_EINVAL, "n must be positive (got %lld)", (long long)n);
    if (ld < n) return fail(SPAMM_EINVAL, "ld (%lld) < n (%lld)", (long long)ld, (long long)n);
    if (!valid_leaf(leaf)) return fail(SPAMM_EINVAL, "leaf must be 16, 32 or 64 (got %d)", leaf);
    const int64_t nb = (n + leaf - 1) / leaf;
    if (nb > MAX_NB)
        return fail(SPAMM_EINVAL, "n/leaf too large (%lld blocks per side, at most %d)", (long long)nb, MAX_NB);
    return SPAMM_OK;
}

// ---- product tables ----------------------------------------------------------
struct TableSizes {
    int nprod, total_cull, total_cullb, total_tiles, total_pyr, total_pyr2, total_quads, max_nb, hist_blocks;
};

TableSizes table_sizes(const ProdDesc *prods, int nprod) {
    TableSizes z{nprod, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int p = 0; p < nprod; ++p) {
        const ProdDesc &d = prods[p];
        z.total_cull += cull_blocks(d.nb);
        z.total_cullb += cull_blk_blocks(d.nb);
        z.total_tiles += d.nb * d.nb;
        z.total_quads += ((d.nb + 1) / 2) * ((d.nb + 1) / 2);
        z.total_pyr += d.P <= 32 ? 1 : (d.P / 32) * (d.P / 32);
        z.total_pyr2 += d.P > 32 ? 1 : 0;
        z.max_nb = std::max(z.max_nb, d.nb);
    }
    const int per_block = 256 * PLAN_HIST_ITEMS;
    z.hist_blocks = z.total_tiles <= PLAN_SMALL_MAX ? 0 : std::min(1024, (z.total_tiles + per_block - 1) / per_block);
    return z;
}

// Lays out one table in `c` (device addresses) and, when `host` is non-null,
// writes its contents into the host staging image at the same offsets.
ProdTable layout_table(Carve &c, const ProdDesc *prods, int nprod, std::vector<char> *host) {
    const TableSizes z = table_sizes(prods, nprod);
    ProdTable t{};
    const size_t o_prods = c.off;
    t.prods = c.take<ProdDesc>(z.nprod);
    const size_t o_cull = c.off;
    t.cull_pre = c.take<int32_t>(z.nprod + 1);
    const size_t o_cullb = c.off;
    t.cullb_pre = c.take<int32_t>(z.nprod + 1);
    const size_t o_tile = c.off;
    t.tile_pre = c.take<int32_t>(z.nprod + 1);
    const size_t o_pyr = c.off;
    t.pyr_pre = c.take<int32_t>(z.nprod + 1);
    const size_t o_pyr2 = c.off;
    t.pyr2_pre = c.take<int32_t>(z.nprod + 1);
    const size_t o_mort = c.off;
    t.morton = c.take<int32_t>(z.total_tiles);
    t.work = c.take<int32_t>(z.total_tiles);
    t.jobs = c.take<Job>(4 * (size_t)z.total_quads);  // >= total_tiles
    t.work_count = c.take<int32_t>(1);
    t.hist = c.take<int32_t>((size_t)NBUCKET * std::max(z.hist_blocks, 1));
    t.nprod = z.nprod;
    t.hist_blocks = z.hist_blocks;
    t.total_cull = z.total_cull;
    t.total_cullb = z.total_cullb;
    t.total_tiles = z.total_tiles;
    t.total_quads = z.total_quads;
    t.total_pyr = z.total_pyr;
    t.total_pyr2 = z.total_pyr2;
    t.max_nb = z.max_nb;
    if (host) {
        if (host->size() < c.off) host->resize(c.off);
        char *h = host->data();
        std::memcpy(h + o_prods, prods, (size_t)nprod * sizeof(ProdDesc));
        int32_t *cull = (int32_t *)(h + o_cull), *cullb = (int32_t *)(h + o_cullb), *tile = (int32_t *)(h + o_tile);
        int32_t *pyr = (int32_t *)(h + o_pyr), *pyr2 = (int32_t *)(h + o_pyr2);
        int32_t *mort = (int32_t *)(h + o_mort);
        cull[0] = cullb[0] = tile[0] = pyr[0] = pyr2[0] = 0;
        for (int p = 0; p < z.nprod; ++p) {
            const ProdDesc &d = prods[p];
            cull[p + 1] = cull[p] + cull_blocks(d.nb);
            cullb[p + 1] = cullb[p] + cull_blk_blocks(d.nb);
            tile[p + 1] = tile[p] + d.nb * d.nb;
            pyr[p + 1] = pyr[p] + (d.P <= 32 ? 1 : (d.P / 32) * (d.P / 32));
            pyr2[p + 1] = pyr2[p] + (d.P > 32 ? 1 : 0);
            tile_order(d.nb, mort + tile[p]);
        }
    }
    return t;
}

const double *root_of(const double *q, int P) { return q + level_off(P, 1); }

// x = y (x)_tau z (dual), or x = z^T (x)_tau y_k (single)
ProdDesc x_product(const spamm_solve *s) {
    ProdDesc d{};
    d.n = s->g.n;
    d.nb = s->g.nb;
    d.P = s->g.P;
    d.tau = s->tau;
    for (int q = 0; q < 2; ++q) {
        if (s->single) {
            d.A[q] = s->zt;
            d.B[q] = s->y[1];
            d.nrmA[q] = s->nzt;
            d.nrmB[q] = s->ny[1];
            d.rootA[q] = root_of(s->qzt, s->g.P);
            d.rootB[q] = root_of(s->qy[1], s->g.P);
        } else {
            d.A[q] = s->y[q];
            d.B[q] = s->z[q];
            d.nrmA[q] = s->ny[q];
            d.nrmB[q] = s->nz[q];
            d.rootA[q] = root_of(s->qy[q], s->g.P);
            d.rootB[q] = root_of(s->qz[q], s->g.P);
        }
        d.C[q] = s->h;
        d.qC[q] = s->qh;
        d.nrmC[q] = s->nh;
    }
    d.cnt = s->cnt[0];
    d.kidx = s->kidx[0];
    d.part = s->part;
    d.fused_map = s->damped ? 0 : 1;
    d.state = s->state;
    return d;
}

// y' = h (x)_{tau_s} y  (which = 0)  or  z' = z (x)_tau h  (which = 1)
ProdDesc update_product(const spamm_solve *s, int which) {
    ProdDesc d{};
    d.n = s->g.n;
    d.nb = s->g.nb;
    d.P = s->g.P;
    const double *rh = root_of(s->qh, s->g.P);
    for (int q = 0; q < 2; ++q) {
        if (which == 0) {
            d.A[q] = s->h;
            d.B[q] = s->y[q];
            d.C[q] = s->y[q ^ 1];
            d.nrmA[q] = s->nh;
            d.nrmB[q] = s->ny[q];
            d.rootA[q] = rh;
            d.rootB[q] = root_of(s->qy[q], s->g.P);
            d.qC[q] = s->qy[q ^ 1];
            d.nrmC[q] = s->ny[q ^ 1];
        } else {
            d.A[q] = s->z[q];
            d.B[q] = s->h;
            d.C[q] = s->z[q ^ 1];
            d.nrmA[q] = s->nz[q];
            d.nrmB[q] = s->nh;
            d.rootA[q] = root_of(s->qz[q], s->g.P);
            d.rootB[q] = rh;
            d.qC[q] = s->qz[q ^ 1];
            d.nrmC[q] = s->nz[q ^ 1];
        }
    }
    d.tau = which == 0 ? s->tau_s : s->tau;
    d.cnt = s->cnt[1 + which];
    d.kidx = s->kidx[1 + which];
    d.part = nullptr;
    d.state = s->state;
    return d;
}

// Single instance: y_k = s' (x)_{tau_s} z_k.
ProdDesc single_y_product(const spamm_solve *s) {
    ProdDesc d{};
    d.n = s->g.n;
    d.nb = s->g.nb;
    d.P = s->g.P;
    d.tau = s->tau_s;
    for (int q = 0; q < 2; ++q) {
        d.A[q] = s->y[0];
        d.B[q] = s->z[q];
        d.C[q] = s->y[1];
        d.nrmA[q] = s->ny[0];
        d.nrmB[q] = s->nz[q];
        d.rootA[q] = root_of(s->qy[0], s->g.P);
        d.rootB[q] = root_of(s->qz[q], s->g.P);
        d.qC[q] = s->qy[1];
        d.nrmC[q] = s->ny[1];
    }
    d.cnt = s->cnt[1];
    d.kidx = s->kidx[1];
    d.state = s->state;
    return d;
}

// Single instance: z_{k+1} = z_k (x)_tau h_k.
ProdDesc single_z_product(const spamm_solve *s) {
    ProdDesc d = update_product(s, 1);
    return d;
}

// Single instance: zt = z_k^T (a transpose, not a product; the table entry
// carries the source in A and the destination in C).
ProdDesc transpose_desc(const spamm_solve *s) {
    ProdDesc d{};
    d.n = s->g.n;
    d.nb = s->g.nb;
    d.P = s->g.P;
    for (int q = 0; q < 2; ++q) {
        d.A[q] = s->z[q];
        d.C[q] = s->zt;
        d.qC[q] = s->qzt;
        d.nrmC[q] = s->nzt;
    }
    d.state = s->state;
    return d;
}

SolveDesc solve_desc(const spamm_solve *s) {
    SolveDesc d{};
    d.state = s->state;
    d.n = s->g.n;
    d.nb = s->g.nb;
    d.maxit = s->maxit;
    d.stagnation_stop = s->stagnation;
    d.damped = s->damped;
    d.single = s->single;
    d.tol = s->tol;
    d.part = s->part;
    d.cnt_x = s->cnt[0];
    d.cnt_y = s->cnt[1];
    d.cnt_z = s->cnt[2];
    d.hist_r = s->hist_r;
    d.hist_t = s->hist_t;
    d.hist_nR = s->hist_nR;
    return d;
}

// Drops a plan; its device tables and pinned read-back buffer return to the
// context's pools (every step synchronises before it returns, so no work on
// them is pending).
void free_plan(spamm_ctx *ctx, Plan *p) {
    if (!p) return;
    if (p->graph_exec) (void)hipGraphExecDestroy(p->graph_exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    pool_return(ctx, ctx->free_table, Block{p->mem, p->cap});
    pool_give(ctx->free_pin, Block{(char *)p->gather_host, p->pin_cap});
    delete p;
}

// Drop cached tables that mention a solve (called when it finishes).
void forget_solve(spamm_ctx *ctx, unsigned long long id) {
    for (size_t i = 0; i < ctx->plans.size();) {
        Plan *p = ctx->plans[i];
        if (std::find(p->ids.begin(), p->ids.end(), id) != p->ids.end()) {
            free_plan(ctx, p);
            ctx->plans.erase(ctx->plans.begin() + i);
        } else {
            ++i;
        }
    }
}

bool same_group(const spamm_solve *a, const spamm_solve *b) {
    return a->prec == b->prec && a->g.b == b->g.b && a->single == b->single;
}

// Device bytes of the tables of a plan over `group` (all of one group).
size_t plan_bytes(const std::vector<spamm_solve *> &group);

// Product and solve descriptors of the tables of a plan over `group`.
struct PlanDescs {
    bool single = false;
    std::vector<ProdDesc> px, pyz, pt, py, pz;
    std::vector<SolveDesc> sd;
};

PlanDescs plan_descs(const std::vector<spamm_solve *> &group) {
    PlanDescs d;
    d.single = group[0]->single != 0;
    for (spamm_solve *s : group) {
        d.px.push_back(x_product(s));
        if (d.single) {
            d.pt.push_back(transpose_desc(s));
            d.py.push_back(single_y_product(s));
            d.pz.push_back(single_z_product(s));
        } else {
            d.pyz.push_back(update_product(s, 0));
            d.pyz.push_back(update_product(s, 1));
        }
        d.sd.push_back(solve_desc(s));
    }
    return d;
}

// Lays out (c.base null: sizes only) the tables of a plan in c.
void plan_layout(Carve &c, const PlanDescs &d, Plan *p, std::vector<char> *image) {
    const ProdTable tx = layout_table(c, d.px.data(), (int)d.px.size(), image);
    ProdTable tt{}, ty{}, tz{}, tyz{};
    if (d.single) {
        tt = layout_table(c, d.pt.data(), (int)d.pt.size(), image);
        ty = layout_table(c, d.py.data(), (int)d.py.size(), image);
        tz = layout_table(c, d.pz.data(), (int)d.pz.size(), image);
    } else {
        tyz = layout_table(c, d.pyz.data(), (int)d.pyz.size(), image);
    }
    const size_t o_sd = c.off;
    SolveDesc *solves = c.take<SolveDesc>(d.sd.size());
    SolveState *gather = c.take<SolveState>(d.sd.size());
    if (image) {
        image->resize(c.off);
        std::memcpy(image->data() + o_sd, d.sd.data(), d.sd.size() * sizeof(SolveDesc));
    }
    if (p) {
        p->tx = tx;
        p->tt = tt;
        p->ty = ty;
        p->tz = tz;
        p->tyz = tyz;
        p->solves = solves;
        p->gather = gather;
    }
}

size_t plan_bytes(const std::vector<spamm_solve *> &group) {
    Carve sizing{nullptr, 0};
    plan_layout(sizing, plan_descs(group), nullptr, nullptr);
    return sizing.off;
}

// Tables for an ordered group of solves sharing (precision, leaf, channel).
// Plans with last_use > keep_after are in use by the current step and are
// never dropped (the step holds their pointers until it has synchronised).
// A new plan replaces the cached plans of its group that the step does not
// use (a group's set changes as solves join and leave), and the cache holds
// at most 8 plans besides those of the current step.  The tables come from
// the context's pool and are uploaded on `st` from a host image the plan
// keeps, so building a plan neither allocates (once the pool is warm) nor
// synchronises.
int get_plan(spamm_ctx *ctx, const std::vector<spamm_solve *> &group, hipStream_t st, unsigned long long keep_after,
             Plan **out) {
    std::vector<unsigned long long> ids;
    for (spamm_solve *s : group) ids.push_back(s->id);
    for (Plan *p : ctx->plans)
        if (p->ids == ids) {
            p->last_use = ++ctx->use_clock;
            *out = p;
            return SPAMM_OK;
        }
    const PlanDescs d = plan_descs(group);
    Plan *p = new Plan();
    p->ids = ids;
    p->prec = group[0]->prec;
    p->leaf = group[0]->g.b;
    p->nsolve = (int)group.size();
    p->single = d.single;
    p->damped = std::any_of(group.begin(), group.end(), [](const spamm_solve *s) { return s->damped != 0; });
    Block tb, pb;
    int rc = pool_take(ctx, ctx->free_table, plan_bytes(group), false, &tb);
    if (rc == SPAMM_OK) {
        p->mem = tb.p;
        p->cap = tb.cap;
        rc = pool_take(ctx, ctx->free_pin, sizeof(SolveState) * group.size(), true, &pb);
    }
    if (rc == SPAMM_OK) {
        p->gather_host = (SolveState *)pb.p;
        p->pin_cap = pb.cap;
    }
    if (rc != SPAMM_OK) {
        const std::string keep = g_err;
        free_plan(ctx, p);
        g_err = keep;
        return rc;
    }
    Carve c{p->mem, 0};
    plan_layout(c, d, p, &p->image);
    const hipError_t ce = hipMemcpyAsync(p->mem, p->image.data(), p->image.size(), hipMemcpyHostToDevice, st);
    if (ce != hipSuccess) {
        free_plan(ctx, p);
        return fail(SPAMM_EHIP, "table upload failed: %s", hipGetErrorString(ce));
    }
    p->last_use = ++ctx->use_clock;
    for (size_t i = 0; i < ctx->plans.size();) {
        Plan *q = ctx->plans[i];
        const bool stale = q->last_use <= keep_after && q->prec == p->prec && q->leaf == p->leaf &&
                           q->single == p->single;
        if (stale) {
            free_plan(ctx, q);
            ctx->plans.erase(ctx->plans.begin() + i);
        } else {
            ++i;
        }
    }
    if (ctx->plans.size() >= 8) {
        auto lru = ctx->plans.end();
        for (auto it = ctx->plans.begin(); it != ctx->plans.end(); ++it)
            if ((*it)->last_use <= keep_after && (lru == ctx->plans.end() || (*it)->last_use < (*lru)->last_use))
                lru = it;
        if (lru != ctx->plans.end()) {
            free_plan(ctx, *lru);
            ctx->plans.erase(lru);
        }
    }
    ctx->plans.push_back(p);
    *out = p;
    return SPAMM_OK;
}

// Cull and job list of one table: one launch for small tables.
int enqueue_front(spamm_ctx *ctx, const ProdTable &t, int leaf, int gprec, hipStream_t st) {
    if (front_small(t, leaf, gprec)) {
        TIMED(K_CULL, launch_front_small(t, leaf, gprec, st));
    } else {
        TIMED(K_CULL, launch_cull_tab(t, st));
        HIPCHK(launch_plan_tab(t, leaf, gprec, st));
    }
    return SPAMM_OK;
}

// One Newton-Schulz iteration of every running solve of a plan.
int enqueue_iteration(spamm_ctx *ctx, Plan *p, hipStream_t st) {
    const int kp = kernel_prec(p->prec);
    if (p->single) {
        // zt = z_k^T; y_k = s' (x)_{tau_s} z_k; x_k = zt (x)_tau y_k (+ stop test,
        // map); z_{k+1} = z_k (x)_tau h_k
        HIPCHK(launch_transpose_tab(kp, p->tt, p->leaf, st));
        TIMED(K_PYR, launch_pyramid_tab(p->tt, st));
        TRY(enqueue_front(ctx, p->ty, p->leaf, gemm_prec(p->prec), st));
        TIMED(K_GEMM, launch_gemm_tab(gemm_prec(p->prec), p->leaf, p->ty, st));
        TIMED(K_PYR, launch_pyramid_tab(p->ty, st));
        TRY(enqueue_front(ctx, p->tx, p->leaf, gemm_prec(p->prec), st));
        TIMED(K_GEMM, launch_gemm_tab(gemm_prec(p->prec), p->leaf, p->tx, st));
        const bool fuse = !p->damped && decide_builds_pyramid(p->tx);
        HIPCHK(launch_ns_decide(p->solves, p->nsolve, fuse ? p->tx.prods : nullptr, st));
        if (p->damped) HIPCHK(launch_ns_map(kp, p->tx, p->leaf, st));
        if (!fuse) TIMED(K_PYR, launch_pyramid_tab(p->tx, st));
        TRY(enqueue_front(ctx, p->tz, p->leaf, gemm_prec(p->prec), st));
        TIMED(K_GEMM, launch_gemm_tab(gemm_prec(p->prec), p->leaf, p->tz, st));
        if (decide_builds_pyramid(p->tz)) {
            TIMED(K_PYR, launch_pyramid_advance(p->solves, p->nsolve, p->tz, 1, st));
        } else {
            TIMED(K_PYR, launch_pyramid_tab(p->tz, st));
            HIPCHK(launch_ns_advance(p->solves, p->nsolve, st));
        }
        return SPAMM_OK;
    }
    TRY(enqueue_front(ctx, p->tx, p->leaf, gemm_prec(p->prec), st));
    TIMED(K_GEMM, launch_gemm_tab(gemm_prec(p->prec), p->leaf, p->tx, st));
    const bool fuse = !p->damped && decide_builds_pyramid(p->tx);
    HIPCHK(launch_ns_decide(p->solves, p->nsolve, fuse ? p->tx.prods : nullptr, st));
    if (p->damped) HIPCHK(launch_ns_map(kp, p->tx, p->leaf, st));
    if (!fuse) TIMED(K_PYR, launch_pyramid_tab(p->tx, st));
    TRY(enqueue_front(ctx, p->tyz, p->leaf, gemm_prec(p->prec), st));
    TIMED(K_GEMM, launch_gemm_tab(gemm_prec(p->prec), p->leaf, p->tyz, st));
    if (decide_builds_pyramid(p->tyz)) {
        TIMED(K_PYR, launch_pyramid_advance(p->solves, p->nsolve, p->tyz, 2, st));
    } else {
        TIMED(K_PYR, launch_pyramid_tab(p->tyz, st));
        HIPCHK(launch_ns_advance(p->solves, p->nsolve, st));
    }
    return SPAMM_OK;
}

// Captures one iteration of a plan on the context's graph stream.
int capture_iteration(spamm_ctx *ctx, Plan *p) {
    hipStream_t st = ctx->gstream;
    HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    const int rc = enqueue_iteration(ctx, p, st);
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(st, &graph);
    if (rc < 0) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
    }
    if (e != hipSuccess) return fail(SPAMM_EHIP, "hipStreamEndCapture failed: %s", hipGetErrorString(e));
    hipGraphExec_t exec = nullptr;
    const hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (ie != hipSuccess) {
        (void)hipGraphDestroy(graph);
        return fail(SPAMM_EHIP, "hipGraphInstantiate failed: %s", hipGetErrorString(ie));
    }
    p->graph = graph;
    p->graph_exec = exec;
    return SPAMM_OK;
}

// Arena layout of one solve; returns its size.  With s non-null, also sets
// the solve's pointers into s->mem.
size_t solve_bytes(const Geom &g, int prec, int maxit, int single, spamm_solve *s) {
    Carve c{s ? s->mem : nullptr, 0};
    const size_t tiles = (size_t)g.nb * g.nb * g.b * g.b * elt_size(prec);
    const size_t pyr = (size_t)pyr_len(g.P);
    const size_t nb2 = (size_t)g.nb * g.nb;
    const int nmat = single ? 6 : 5;  // the single instance also holds z^T
    void *tl[6] = {};
    for (int i = 0; i < nmat; ++i) tl[i] = c.take<char>(tiles);
    double *q[6] = {}, *nr[6] = {};
    for (int i = 0; i < nmat; ++i) q[i] = c.take<double>(pyr);
    for (int i = 0; i < nmat; ++i) nr[i] = c.take<double>(2 * nb2);  // leaf norms and their transpose
    int32_t *cnt[3], *kidx[3];
    for (int i = 0; i < 3; ++i) cnt[i] = c.take<int32_t>(nb2);
    for (int i = 0; i < 3; ++i) kidx[i] = c.take<int32_t>(nb2 * g.nb);
    double *part = c.take<double>(2 * nb2);
    double *hr = c.take<double>(maxit + 1);
    double *ht = c.take<double>(maxit + 1);
    int64_t *hn = c.take<int64_t>(3 * (size_t)(maxit + 1));
    SolveState *state = c.take<SolveState>(1);
    if (s) {
        s->y[0] = tl[0];
        s->y[1] = tl[1];
        s->z[0] = tl[2];
        s->z[1] = tl[3];
        s->h = tl[4];
        s->qy[0] = q[0];
        s->qy[1] = q[1];
        s->qz[0] = q[2];
        s->qz[1] = q[3];
        s->qh = q[4];
        s->ny[0] = nr[0];
        s->ny[1] = nr[1];
        s->nz[0] = nr[2];
        s->nz[1] = nr[3];
        s->nh = nr[4];
        s->zt = tl[5];
        s->qzt = q[5];
        s->nzt = nr[5];
        for (int i = 0; i < 3; ++i) {
            s->cnt[i] = cnt[i];
            s->kidx[i] = kidx[i];
        }
        s->part = part;
        s->hist_r = hr;
        s->hist_t = ht;
        s->hist_nR = hn;
        s->state = state;
    }
    return c.off;
}

int validate_ns(spamm_ctx *ctx, const double *s, int64_t n, int64_t ld, double tau, double tol, int maxit,
                const spamm_ns_opts &o) {
    TRY(validate_common(ctx, s, n, ld, o.leaf));
    if (!(tau >= 0.0) || std::isinf(tau)) return fail(SPAMM_EINVAL, "tau must be finite and >= 0");
    if (!(tol > 0.0)) return fail(SPAMM_EINVAL, "tol must be > 0");
    if (maxit < 0 || maxit > 100000) return fail(SPAMM_EINVAL, "maxit must be in [0, 100000]");
    if (!valid_prec(o.prec)) return fail(SPAMM_EINVAL, "unknown precision %d", o.prec);
    if (split_bf16(o.prec) && o.leaf == 16) return fail(SPAMM_EINVAL, "split-bf16 leaves need leaf 32 or 64");
    if (!(o.mu_rel >= 0.0) || std::isinf(o.mu_rel)) return fail(SPAMM_EINVAL, "mu_rel must be finite and >= 0");
    if (std::isnan(o.tau_s) || std::isinf(o.tau_s)) return fail(SPAMM_EINVAL, "tau_s must be finite");
    return SPAMM_OK;
}

spamm_ns_opts default_opts(const spamm_ns_opts *opts) {
    spamm_ns_opts o;
    o.leaf = 32;
    o.prec = SPAMM_F64;
    o.tau_s = -1.0;
    o.mu_rel = 0.0;
    o.stagnation_stop = 0;
    o.damped = 0;
    o.single = 0;
    if (opts) {
        o = *opts;
        if (o.leaf == 0) o.leaf = 32;
    }
    return o;
}

// C = A (x)_tau B on tiles T[0], T[1] -> T[2] (no solve: always runs, parity 0).
ProdDesc plain_product(const Geom &g, double tau, void *const *T, double *const *q, double *const *nr, int32_t *cnt,
                       int32_t *kidx) {
    ProdDesc d{};
    d.n = g.n;
    d.nb = g.nb;
    d.P = g.P;
    d.tau = tau;
    d.A[0] = d.A[1] = T[0];
    d.B[0] = d.B[1] = T[1];
    d.C[0] = d.C[1] = T[2];
    d.nrmA[0] = d.nrmA[1] = nr[0];
    d.nrmB[0] = d.nrmB[1] = nr[1];
    d.rootA[0] = d.rootA[1] = root_of(q[0], g.P);
    d.rootB[0] = d.rootB[1] = root_of(q[1], g.P);
    d.qC[0] = d.qC[1] = q[2];
    d.nrmC[0] = d.nrmC[1] = nr[2];
    d.cnt = cnt;
    d.kidx = kidx;
    d.part = nullptr;
    d.state = nullptr;
    return d;
}

int validate_multiply(spamm_ctx *ctx, const double *A, const double *B, const double *C, int64_t n, int64_t ld,
                      double tau, int leaf, int prec) {
    TRY(validate_common(ctx, A, n, ld, leaf));
    if (!B || !C) return fail(SPAMM_EINVAL, "NULL matrix pointer");
    if (!(tau >= 0.0) || std::isinf(tau)) return fail(SPAMM_EINVAL, "tau must be finite and >= 0");
    if (!valid_prec(prec)) return fail(SPAMM_EINVAL, "unknown precision %d", prec);
    if (split_bf16(prec) && leaf == 16) return fail(SPAMM_EINVAL, "split-bf16 leaves need leaf 32 or 64");
    return SPAMM_OK;
}

void fill_result(const spamm_solve *s, spamm_ns_result *res) {
    if (!res) return;
    const SolveState &h = s->host_state;
    res->iterations = h.k;
    res->resid = h.r;
    res->trace_err = h.t;
    res->scale = s->c;
    res->triples_total = h.triples;
    res->flops_total = 2.0 * (double)s->g.b * s->g.b * s->g.b * (double)h.triples;
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
    void *scr = nullptr;
    TRY(scratch_setup(device, &scr));
    spamm_ctx *ctx = new spamm_ctx();
    ctx->device = device;
    ctx->scratch = scr;
    hipError_t e = hipHostMalloc((void **)&ctx->pinned, 64 * sizeof(double), hipHostMallocDefault);
    if (e != hipSuccess) {
        delete ctx;
        return fail(SPAMM_ENOMEM, "hipHostMalloc failed: %s", hipGetErrorString(e));
    }
    // default-priority stream for graph capture and replay, and two events
    // that order it against the caller's stream
    e = hipStreamCreateWithFlags(&ctx->gstream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ctx->ev_in, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ctx->ev_out, hipEventDisableTiming);
    if (e != hipSuccess) {
        if (ctx->gstream) (void)hipStreamDestroy(ctx->gstream);
        if (ctx->ev_in) (void)hipEventDestroy(ctx->ev_in);
        (void)hipHostFree(ctx->pinned);
        delete ctx;
        return fail(SPAMM_EHIP, "stream/event creation failed: %s", hipGetErrorString(e));
    }
    *out = ctx;
    return SPAMM_OK;
}

int spamm_destroy(spamm_ctx *ctx) {
    if (!ctx) return SPAMM_OK;
    HIPCHK(hipSetDevice(ctx->device));
    HIPCHK(hipDeviceSynchronize());
    for (Plan *p : ctx->plans) free_plan(ctx, p);
    ctx->plans.clear();
    for (spamm_solve *sv : ctx->live) {  // solves begun and never finished
        pool_give(ctx->free_arena, Block{sv->mem, sv->bytes});
        delete sv;
    }
    ctx->live.clear();
    pool_drain(ctx->free_arena, false);
    pool_drain(ctx->free_table, false);
    pool_drain(ctx->free_pin, true);
    for (hipEvent_t e : ctx->pool) HIPCHK(hipEventDestroy(e));
    if (ctx->gstream) HIPCHK(hipStreamDestroy(ctx->gstream));
    for (hipStream_t x : ctx->xstream) HIPCHK(hipStreamDestroy(x));
    for (hipEvent_t e : ctx->xdone) HIPCHK(hipEventDestroy(e));
    if (ctx->ev_in) HIPCHK(hipEventDestroy(ctx->ev_in));
    if (ctx->ev_out) HIPCHK(hipEventDestroy(ctx->ev_out));
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
    TRY(ensure(ctx, S_Q0, (size_t)pyr_len(g.P) * sizeof(double)));
    TRY(ensure(ctx, S_N0, 2 * (size_t)g.nb * g.nb * sizeof(double)));
    double *q = slot_ptr<double>(ctx, S_Q0), *nrm = slot_ptr<double>(ctx, S_N0);
    HIPCHK(hipMemsetAsync(q, 0, (size_t)g.P * g.P * sizeof(double), st));  // virtual blocks read as 0
    HIPCHK(launch_leaf_norms(A, ld, g, q, st));
    TIMED(K_PYR, launch_pyramid(g, q, nrm, q, nrm, 1, st));
    HIPCHK(launch_norms_out(g, q, pyramid, st));
    if (root_norm_host) {
        HIPCHK(hipMemcpyAsync(ctx->pinned, root_of(q, g.P), sizeof(double), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        *root_norm_host = std::sqrt(ctx->pinned[0]);
    }
    return SPAMM_OK;
}

int spamm_multiply(spamm_ctx *ctx, const double *A, const double *B, double *C, int64_t n, int64_t ld,
                   double tau, int leaf, int prec, int32_t *triples, int64_t cap, spamm_stats *stats,
                   void *stream) {
    TRY(validate_multiply(ctx, A, B, C, n, ld, tau, leaf, prec));
    if (triples && cap < 0) return fail(SPAMM_EINVAL, "negative triple capacity");
    TRY(enter(ctx));
    hipStream_t st = (hipStream_t)stream;
    const Geom g = make_geom(n, leaf);
    const int kp = kernel_prec(prec);
    const size_t nb2 = (size_t)g.nb * g.nb;
    for (int m = 0; m < 3; ++m) {
        TRY(ensure(ctx, S_T0 + m, nb2 * g.b * g.b * elt_size(prec)));
        TRY(ensure(ctx, S_Q0 + m, (size_t)pyr_len(g.P) * sizeof(double)));
        TRY(ensure(ctx, S_N0 + m, 2 * nb2 * sizeof(double)));
    }
    TRY(ensure(ctx, S_CNT, nb2 * sizeof(int32_t)));
    TRY(ensure(ctx, S_KIDX, nb2 * g.nb * sizeof(int32_t)));
    TRY(ensure(ctx, S_SCAL, 64 * sizeof(double)));
    double *q[3], *nr[3];
    for (int m = 0; m < 3; ++m) {
        q[m] = slot_ptr<double>(ctx, S_Q0 + m);
        nr[m] = slot_ptr<double>(ctx, S_N0 + m);
        HIPCHK(hipMemsetAsync(q[m], 0, (size_t)g.P * g.P * sizeof(double), st));
    }
    HIPCHK(launch_ingest(kp, A, ld, 0.0, 1.0, g, ctx->buf[S_T0], q[0], st));
    HIPCHK(launch_ingest(kp, B, ld, 0.0, 1.0, g, ctx->buf[S_T1], q[1], st));
    TIMED(K_PYR, launch_pyramid(g, q[0], nr[0], q[1], nr[1], 2, st));

    void *T[3] = {ctx->buf[S_T0], ctx->buf[S_T1], ctx->buf[S_T2]};
    const ProdDesc d = plain_product(g, tau, T, q, nr, slot_ptr<int32_t>(ctx, S_CNT), slot_ptr<int32_t>(ctx, S_KIDX));
    std::vector<ProdDesc> prods{d};
    Carve sizing{nullptr, 0};
    layout_table(sizing, prods.data(), (int)prods.size(), nullptr);
    TRY(ensure(ctx, S_TAB, sizing.off));
    std::vector<char> image;
    Carve c{(char *)ctx->buf[S_TAB], 0};
    ProdTable t = layout_table(c, prods.data(), (int)prods.size(), &image);
    image.resize(c.off);
    HIPCHK(hipMemcpyAsync(ctx->buf[S_TAB], image.data(), image.size(), hipMemcpyHostToDevice, st));
    TRY(enqueue_front(ctx, t, leaf, gemm_prec(prec), st));
    TIMED(K_GEMM, launch_gemm_tab(gemm_prec(prec), leaf, t, st));
    HIPCHK(launch_egress(kp, g, ctx->buf[S_T2], C, ld, 1.0, 0, st));
    int status = SPAMM_OK;
    if (stats || triples) {
        TRY(ensure(ctx, S_OFFS, nb2 * sizeof(int64_t)));
        int64_t *offs = slot_ptr<int64_t>(ctx, S_OFFS);
        int64_t *total = reinterpret_cast<int64_t *>(slot_ptr<double>(ctx, S_SCAL) + 8);
        HIPCHK(launch_count_triples(g, d.cnt, offs, total, st));
        HIPCHK(hipMemcpyAsync(ctx->pinned, total, sizeof(int64_t), hipMemcpyDeviceToHost, st));
        HIPCHK(hipMemcpyAsync(ctx->pinned + 1, d.rootA[0], sizeof(double), hipMemcpyDeviceToHost, st));
        HIPCHK(hipMemcpyAsync(ctx->pinned + 2, d.rootB[0], sizeof(double), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        int64_t retained;
        std::memcpy(&retained, ctx->pinned, sizeof(int64_t));
        if (triples) {
            if (retained > cap)
                status = fail(SPAMM_ECAPACITY, "|R| = %lld exceeds triple capacity %lld", (long long)retained,
                              (long long)cap);
            else
                HIPCHK(launch_write_triples(g, d.cnt, d.kidx, offs, triples, st));
        }
        if (stats) {
            stats->retained = retained;
            stats->possible = (int64_t)g.nb * g.nb * g.nb;
            stats->thr = tau * (std::sqrt(ctx->pinned[1]) * std::sqrt(ctx->pinned[2]));
            stats->flops = 2.0 * (double)leaf * leaf * leaf * (double)retained;
        }
    }
    // the host staging image must outlive its copy
    HIPCHK(hipStreamSynchronize(st));
    return status;
}

int spamm_multiply_noalloc(spamm_ctx *ctx, const double *A, const double *B, double *C, int64_t n, int64_t ld,
                           double tau, int leaf, int prec, void *stream) {
    TRY(validate_multiply(ctx, A, B, C, n, ld, tau, leaf, prec));
    if (!ctx->scratch) return fail(SPAMM_EHIP, "the static scratch of device %d was not located", ctx->device);
    const Geom g = make_geom(n, leaf);
    const size_t nb2 = (size_t)g.nb * g.nb;
    // every buffer of spamm_multiply, carved from this device's static scratch
    Carve c{(char *)ctx->scratch, 0};
    void *T[3];
    double *q[3], *nr[3];
    for (int m = 0; m < 3; ++m) T[m] = c.take<char>(nb2 * g.b * g.b * elt_size(prec));
    for (int m = 0; m < 3; ++m) q[m] = c.take<double>((size_t)pyr_len(g.P));
    for (int m = 0; m < 3; ++m) nr[m] = c.take<double>(2 * nb2);
    int32_t *cnt = c.take<int32_t>(nb2);
    int32_t *kidx = c.take<int32_t>(nb2 * g.nb);
    const ProdDesc d = plain_product(g, tau, T, q, nr, cnt, kidx);
    const ProdTable t = layout_table(c, &d, 1, nullptr);
    if (c.off > (size_t)SPAMM_NOALLOC_BYTES)
        return fail(SPAMM_EINVAL, "n = %lld at leaf %d needs %zu bytes of scratch, more than the static %zu",
                    (long long)n, leaf, c.off, (size_t)SPAMM_NOALLOC_BYTES);
    TRY(enter(ctx));
    hipStream_t st = (hipStream_t)stream;
    const int kp = kernel_prec(prec);
    // the array keeps the previous call's contents: the leaf levels of the
    // pyramids (virtual blocks must read 0) are cleared by a kernel
    for (int m = 0; m < 3; ++m) HIPCHK(launch_fill_zero(q[m], (int64_t)g.P * g.P, st));
    HIPCHK(launch_ingest(kp, A, ld, 0.0, 1.0, g, T[0], q[0], st));
    HIPCHK(launch_ingest(kp, B, ld, 0.0, 1.0, g, T[1], q[1], st));
    TIMED(K_PYR, launch_pyramid(g, q[0], nr[0], q[1], nr[1], 2, st));
    HIPCHK(launch_table_one(d, t, st));
    TRY(enqueue_front(ctx, t, leaf, gemm_prec(prec), st));
    TIMED(K_GEMM, launch_gemm_tab(gemm_prec(prec), leaf, t, st));
    HIPCHK(launch_egress(kp, g, T[2], C, ld, 1.0, 0, st));
    return SPAMM_OK;
}

size_t spamm_solve_footprint(int64_t n, int leaf, int prec, int maxit, int single) {
    if (n <= 0 || !valid_leaf(leaf) || !valid_prec(prec) || maxit < 0) return 0;
    const Geom g = make_geom(n, leaf);
    return solve_bytes(g, prec, maxit, single ? 1 : 0, nullptr);
}

int spamm_solve_begin(spamm_ctx *ctx, const double *s, int64_t n, int64_t ld, double tau, double tol, int maxit,
                      const spamm_ns_opts *opts, spamm_solve **out, void *stream) {
    if (!out) return fail(SPAMM_EINVAL, "NULL output handle");
    *out = nullptr;
    const spamm_ns_opts o = default_opts(opts);
    TRY(validate_ns(ctx, s, n, ld, tau, tol, maxit, o));
    TRY(enter(ctx));
    hipStream_t st = (hipStream_t)stream;
    const Geom g = make_geom(n, o.leaf);

    // input checks and the Gershgorin scale (context scratch, one read-back)
    const int64_t nbk = (n + 31) / 32;
    TRY(ensure(ctx, S_CHECK, (size_t)std::max<int64_t>(3 * nbk * nbk, n) * sizeof(double)));
    TRY(ensure(ctx, S_SCAL, 64 * sizeof(double)));
    double *scal = slot_ptr<double>(ctx, S_SCAL), *check = slot_ptr<double>(ctx, S_CHECK);
    double *pin = ctx->pinned;
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

    spamm_solve *sv = new spamm_solve();
    sv->ctx = ctx;
    sv->id = ctx->next_id++;
    sv->g = g;
    sv->prec = o.prec;
    sv->tau = tau;
    sv->tau_s = o.tau_s < 0.0 ? tau : o.tau_s;
    sv->tol = tol;
    sv->mu = mu;
    sv->c = c;
    sv->maxit = maxit;
    sv->stagnation = o.stagnation_stop ? 1 : 0;
    sv->damped = o.damped ? 1 : 0;
    sv->mem = nullptr;
    sv->single = o.single ? 1 : 0;
    sv->bytes = solve_bytes(g, o.prec, maxit, sv->single, nullptr);
    Block arena;
    int prc = pool_take(ctx, ctx->free_arena, sv->bytes, false, &arena);
    if (prc == SPAMM_ENOMEM && !(ctx->free_arena.empty() && ctx->free_table.empty())) {
        // memory held in the pools goes back to the device, then one retry
        pool_drain(ctx->free_arena, false);
        pool_drain(ctx->free_table, false);
        prc = pool_take(ctx, ctx->free_arena, sv->bytes, false, &arena);
    }
    if (prc != SPAMM_OK) {
        delete sv;
        return fail(SPAMM_ENOMEM, "solve allocation of %zu bytes failed", (size_t)sv->bytes);
    }
    sv->mem = arena.p;
    sv->bytes = arena.cap;
    solve_bytes(g, o.prec, maxit, sv->single, sv);
    const int kp = kernel_prec(o.prec);
    const size_t leafq = (size_t)g.P * g.P * sizeof(double);
    int rc = SPAMM_OK;
    auto chk = [&](hipError_t err, const char *what) {
        if (err != hipSuccess && rc == SPAMM_OK) rc = fail(SPAMM_EHIP, "%s failed: %s", what, hipGetErrorString(err));
    };
    // virtual blocks of every pyramid read as zero; records start empty
    for (double *q : {sv->qy[0], sv->qy[1], sv->qz[0], sv->qz[1], sv->qh, sv->qzt})
        if (q) chk(hipMemsetAsync(q, 0, leafq, st), "memset");
    chk(hipMemsetAsync(sv->hist_nR, 0, 3 * (size_t)(maxit + 1) * sizeof(int64_t), st), "memset");
    chk(launch_ingest(kp, s, ld, mu, c, g, sv->y[0], sv->qy[0], st), "ingest");
    chk(launch_identity(kp, g, sv->z[0], sv->qz[0], st), "identity");
    chk(launch_pyramid(g, sv->qy[0], sv->ny[0], sv->qz[0], sv->nz[0], 2, st), "pyramid");
    SolveState init{};
    init.status = ST_RUNNING;
    init.alpha = 1.0;
    sv->host_state = init;
    chk(hipMemcpyAsync(sv->state, &sv->host_state, sizeof(SolveState), hipMemcpyHostToDevice, st), "state");
    chk(hipStreamSynchronize(st), "synchronise");
    if (rc != SPAMM_OK) {
        pool_give(ctx->free_arena, Block{sv->mem, sv->bytes});
        delete sv;
        return rc;
    }
    // Reserve in the pools the tables and read-back buffer of a plan over
    // every unfinished solve of this group, so that the steps that follow
    // take them from there rather than allocating.
    std::vector<spamm_solve *> group;
    for (spamm_solve *x : ctx->live)
        if (same_group(x, sv)) group.push_back(x);
    group.push_back(sv);
    Block tb, pb;
    rc = pool_take(ctx, ctx->free_table, plan_bytes(group), false, &tb);
    if (rc == SPAMM_OK) {
        pool_give(ctx->free_table, tb);
        rc = pool_take(ctx, ctx->free_pin, sizeof(SolveState) * group.size(), true, &pb);
        if (rc == SPAMM_OK) pool_give(ctx->free_pin, pb);
    }
    if (rc != SPAMM_OK) {
        const std::string keep = g_err;
        pool_give(ctx->free_arena, Block{sv->mem, sv->bytes});
        delete sv;
        g_err = keep;
        return rc;
    }
    ctx->live.push_back(sv);
    *out = sv;
    return SPAMM_OK;
}

}  // extern "C"

namespace {

// Replay streams for `count` plans: the graph stream, then extra ones.
int replay_streams(spamm_ctx *ctx, size_t count) {
    while (ctx->xstream.size() + 1 < count) {
        hipStream_t x = nullptr;
        hipEvent_t e = nullptr;
        HIPCHK(hipStreamCreateWithFlags(&x, hipStreamNonBlocking));
        const hipError_t er = hipEventCreateWithFlags(&e, hipEventDisableTiming);
        if (er != hipSuccess) {
            (void)hipStreamDestroy(x);
            return fail(SPAMM_EHIP, "event creation failed: %s", hipGetErrorString(er));
        }
        ctx->xstream.push_back(x);
        ctx->xdone.push_back(e);
    }
    return SPAMM_OK;
}

}  // namespace

extern "C" {

int spamm_solve_step(spamm_ctx *ctx, spamm_solve *const *solves, int count, int iterations, void *stream) {
    TRY(enter(ctx));
    if (count < 0 || (count > 0 && !solves)) return fail(SPAMM_EINVAL, "bad solve list");
    if (iterations < 1) return fail(SPAMM_EINVAL, "iterations must be >= 1");
    hipStream_t st = (hipStream_t)stream;
    // the listed solves grouped by (precision, leaf, channel) in the caller's
    // order.  A group keeps its stopped solves (the kernels skip them), so
    // its plan and captured graph stay the same while solves stop; groups
    // with no running solve are left out.
    std::vector<std::vector<spamm_solve *>> all;
    for (int i = 0; i < count; ++i) {
        spamm_solve *s = solves[i];
        if (!s || s->ctx != ctx) return fail(SPAMM_EINVAL, "solve %d is NULL or belongs to another context", i);
        for (int j = 0; j < i; ++j)
            if (solves[j] == s) return fail(SPAMM_EINVAL, "solve %d appears twice", i);
        auto it = std::find_if(all.begin(), all.end(),
                               [&](const std::vector<spamm_solve *> &gr) { return same_group(gr[0], s); });
        if (it == all.end())
            all.push_back({s});
        else
            it->push_back(s);
    }
    std::vector<std::vector<spamm_solve *>> groups;
    for (auto &gr : all)
        if (std::any_of(gr.begin(), gr.end(), [](const spamm_solve *s) { return s->host_state.status == ST_RUNNING; }))
            groups.push_back(gr);
    if (groups.empty()) return 0;
    std::vector<Plan *> plans;
    const unsigned long long step_start = ctx->use_clock;
    for (auto &gr : groups) {
        Plan *p = nullptr;
        TRY(get_plan(ctx, gr, st, step_start, &p));
        plans.push_back(p);
    }
    const bool use_graphs = ctx->graphs && !ctx->prof;
    if (use_graphs) {
        // Plan q replays on its own stream (the graph stream for the first):
        // the plans touch disjoint solves, so they run concurrently.  Every
        // replay stream waits for the caller's stream, and the caller's stream
        // waits for all of them (the step also blocks the host).  A plan's
        // iteration is captured on the plan's second step: its first step
        // launches plainly, so a set of solves that lasts one step (a server
        // whose solves join and leave at every step boundary) never pays
        // for a capture.
        for (Plan *p : plans)
            if (!p->graph_exec && p->uses > 0) TRY(capture_iteration(ctx, p));
        TRY(replay_streams(ctx, plans.size()));
        HIPCHK(hipEventRecord(ctx->ev_in, st));
        for (size_t q = 0; q < plans.size(); ++q) {
            hipStream_t rq = q == 0 ? ctx->gstream : ctx->xstream[q - 1];
            HIPCHK(hipStreamWaitEvent(rq, ctx->ev_in, 0));
            if (plans[q]->graph_exec)
                for (int it = 0; it < iterations; ++it) HIPCHK(hipGraphLaunch(plans[q]->graph_exec, rq));
            else
                for (int it = 0; it < iterations; ++it) TRY(enqueue_iteration(ctx, plans[q], rq));
            HIPCHK(launch_gather_states(plans[q]->solves, plans[q]->nsolve, plans[q]->gather, rq));
            HIPCHK(hipMemcpyAsync(plans[q]->gather_host, plans[q]->gather, plans[q]->nsolve * sizeof(SolveState),
                                  hipMemcpyDeviceToHost, rq));
            hipEvent_t done = q == 0 ? ctx->ev_out : ctx->xdone[q - 1];
            HIPCHK(hipEventRecord(done, rq));
            HIPCHK(hipStreamWaitEvent(st, done, 0));
        }
        for (size_t q = 0; q < plans.size(); ++q)
            HIPCHK(hipStreamSynchronize(q == 0 ? ctx->gstream : ctx->xstream[q - 1]));
    } else {
        for (int it = 0; it < iterations; ++it)
            for (Plan *p : plans) TRY(enqueue_iteration(ctx, p, st));
        for (Plan *p : plans) {
            HIPCHK(launch_gather_states(p->solves, p->nsolve, p->gather, st));
            HIPCHK(hipMemcpyAsync(p->gather_host, p->gather, p->nsolve * sizeof(SolveState),
                                  hipMemcpyDeviceToHost, st));
        }
        HIPCHK(hipStreamSynchronize(st));
    }
    for (Plan *p : plans) ++p->uses;
    int running = 0;
    for (size_t gi = 0; gi < groups.size(); ++gi)
        for (size_t i = 0; i < groups[gi].size(); ++i) {
            groups[gi][i]->host_state = plans[gi]->gather_host[i];
            if (groups[gi][i]->host_state.status == ST_RUNNING) ++running;
        }
    return running;
}

}  // extern "C"

namespace {

// Slices of the product representation into W, with six n x ld working
// matrices S, T, Wt, M, Y, Z; returns the first failing status.
int product_rep_body(spamm_ctx *ctx, const double *s, double *W, int64_t n, int64_t ld, const spamm_prodrep_opts &o,
                     int leaf, double *const *buf, spamm_prodrep_result *res, void *stream) {
    hipStream_t st = (hipStream_t)stream;
    double *S = buf[0], *T = buf[1], *Wt = buf[2], *M = buf[3], *Y = buf[4], *Z = buf[5];
    spamm_ns_opts no{};
    no.leaf = leaf;
    no.prec = o.prec;
    no.tau_s = o.tau_s_slice;
    no.stagnation_stop = o.stagnation_stop;
    no.damped = o.damped;
    // c0 = Gershgorin bound of s (the column sums ns_sqrt uses)
    TRY(ensure(ctx, S_CHECK, (size_t)n * sizeof(double)));
    TRY(ensure(ctx, S_SCAL, 64 * sizeof(double)));
    double *out = slot_ptr<double>(ctx, S_SCAL);
    HIPCHK(launch_colsum_max(s, n, ld, 0.0, slot_ptr<double>(ctx, S_CHECK), out, st));
    HIPCHK(hipMemcpyAsync(ctx->pinned, out, sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    const double c0 = ctx->pinned[0];
    spamm_ns_result nr{};
    for (int j = 0; j < o.nslices; ++j) {
        int sj;
        if (j == 0) {
            no.mu_rel = o.mu_rel[0];
            sj = ns_sqrt(ctx, s, Y, W, n, ld, o.tau_slice, o.tol, o.maxit, &no, &nr, stream);
        } else {
            HIPCHK(launch_shift_copy(s, S, n, ld, o.mu_rel[j] * c0, st));
            TRY(spamm_multiply(ctx, S, W, T, n, ld, o.tau_r, leaf, o.prec, nullptr, 0, nullptr, stream));
            HIPCHK(launch_transpose_dense(W, Wt, n, ld, st));
            TRY(spamm_multiply(ctx, Wt, T, M, n, ld, o.tau_r, leaf, o.prec, nullptr, 0, nullptr, stream));
            HIPCHK(launch_sym_part(M, S, n, ld, st));
            no.mu_rel = 0.0;
            sj = ns_sqrt(ctx, S, Y, Z, n, ld, o.tau_slice, o.tol, o.maxit, &no, &nr, stream);
        }
        if (res) {
            res->status[j] = sj;
            res->iterations[j] = nr.iterations;
            res->nslices_done = j + 1;
        }
        if (sj < 0) return sj;
        if (j > 0) {
            TRY(spamm_multiply(ctx, W, Z, T, n, ld, o.tau_r, leaf, o.prec, nullptr, 0, nullptr, stream));
            HIPCHK(hipMemcpyAsync(W, T, (size_t)n * ld * sizeof(double), hipMemcpyDeviceToDevice, st));
        }
    }
    HIPCHK(hipStreamSynchronize(st));
    return SPAMM_OK;
}

}  // namespace

extern "C" {

int spamm_product_rep(spamm_ctx *ctx, const double *s, double *W, int64_t n, int64_t ld,
                      const spamm_prodrep_opts *opts, spamm_prodrep_result *res, void *stream) {
    if (!opts) return fail(SPAMM_EINVAL, "NULL options");
    const spamm_prodrep_opts o = *opts;
    const int leaf = o.leaf == 0 ? 32 : o.leaf;
    TRY(validate_common(ctx, s, n, ld, leaf));
    TRY(enter(ctx));
    if (!W) return fail(SPAMM_EINVAL, "NULL output pointer");
    if (o.nslices < 1 || o.nslices > SPAMM_MAX_SLICES)
        return fail(SPAMM_EINVAL, "nslices must be in [1, %d]", SPAMM_MAX_SLICES);
    if (!o.mu_rel) return fail(SPAMM_EINVAL, "NULL shift list");
    for (int j = 0; j < o.nslices; ++j)
        if (!(o.mu_rel[j] >= 0.0) || std::isinf(o.mu_rel[j])) return fail(SPAMM_EINVAL, "bad shift mu_rel[%d]", j);
    if (!(o.tau_r >= 0.0) || std::isinf(o.tau_r)) return fail(SPAMM_EINVAL, "tau_r must be finite and >= 0");
    if (res) std::memset(res, 0, sizeof(*res));
    const size_t bytes = (size_t)n * ld * sizeof(double);
    double *buf[6] = {};  // S, T, Wt, M, Y, Z
    int rc = SPAMM_OK;
    for (int i = 0; i < 6 && rc == SPAMM_OK; ++i) {
        const hipError_t e = hipMalloc((void **)&buf[i], bytes);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            rc = fail(SPAMM_ENOMEM, "product representation needs 6 x %zu bytes: %s", bytes, hipGetErrorString(e));
        }
    }
    if (rc == SPAMM_OK) rc = product_rep_body(ctx, s, W, n, ld, o, leaf, buf, res, stream);
    (void)hipStreamSynchronize((hipStream_t)stream);
    for (double *b : buf)
        if (b) (void)hipFree(b);
    return rc;
}

int spamm_solve_triples(spamm_ctx *ctx, spamm_solve *s, int which, int32_t *triples, int64_t cap, int64_t *count,
                        void *stream) {
    TRY(enter(ctx));
    if (!s || s->ctx != ctx) return fail(SPAMM_EINVAL, "NULL solve or solve of another context");
    if (which < 0 || which > 2) return fail(SPAMM_EINVAL, "which must be 0 (x), 1 (y) or 2 (z)");
    if (cap < 0 || (cap > 0 && !triples)) return fail(SPAMM_EINVAL, "bad triple buffer");
    hipStream_t st = (hipStream_t)stream;
    const Geom &g = s->g;
    const size_t nb2 = (size_t)g.nb * g.nb;
    TRY(ensure(ctx, S_OFFS, nb2 * sizeof(int64_t)));
    int64_t *offs = slot_ptr<int64_t>(ctx, S_OFFS);
    int64_t *total = reinterpret_cast<int64_t *>(slot_ptr<double>(ctx, S_SCAL) + 8);
    HIPCHK(launch_count_triples(g, s->cnt[which], offs, total, st));
    HIPCHK(hipMemcpyAsync(ctx->pinned, total, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    int64_t m;
    std::memcpy(&m, ctx->pinned, sizeof(int64_t));
    if (count) *count = m;
    if (m > cap) return fail(SPAMM_ECAPACITY, "|R| = %lld exceeds triple capacity %lld", (long long)m, (long long)cap);
    if (m > 0) HIPCHK(launch_write_triples(g, s->cnt[which], s->kidx[which], offs, triples, st));
    HIPCHK(hipStreamSynchronize(st));
    return SPAMM_OK;
}

int spamm_solve_poll(spamm_solve *s, int *done, spamm_ns_result *res) {
    if (!s) return fail(SPAMM_EINVAL, "NULL solve");
    const int st = s->host_state.status;
    if (done) *done = st != ST_RUNNING;
    fill_result(s, res);
    return st == ST_RUNNING ? SPAMM_OK : st;
}

int spamm_solve_finish(spamm_ctx *ctx, spamm_solve *s, double *Y, double *Z, int64_t ld, void *stream) {
    TRY(enter(ctx));
    if (!s || s->ctx != ctx) return fail(SPAMM_EINVAL, "NULL solve or solve of another context");
    if ((Y || Z) && ld < s->g.n)
        return fail(SPAMM_EINVAL, "ld (%lld) < n (%lld)", (long long)ld, (long long)s->g.n);
    hipStream_t st = (hipStream_t)stream;
    const SolveState h = s->host_state;
    const int status = h.status == ST_RUNNING ? SPAMM_NOT_CONVERGED : h.status;
    const int kp = kernel_prec(s->prec);
    const double sc = std::sqrt(s->c);
    const int k = h.k;
    if (Y) HIPCHK(launch_egress(kp, s->g, s->single ? s->y[1] : s->y[h.parity], Y, ld, sc, 0, st));
    if (Z) HIPCHK(launch_egress(kp, s->g, s->z[h.parity], Z, ld, sc, 1, st));
    ctx->hist_r.assign(k + 1, 0.0);
    ctx->hist_t.assign(k + 1, 0.0);
    ctx->hist_nR.assign(3 * (size_t)(k + 1), 0);
    HIPCHK(hipMemcpyAsync(ctx->hist_r.data(), s->hist_r, (k + 1) * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(ctx->hist_t.data(), s->hist_t, (k + 1) * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(ctx->hist_nR.data(), s->hist_nR, 3 * (k + 1) * sizeof(int64_t), hipMemcpyDeviceToHost,
                          st));
    HIPCHK(hipStreamSynchronize(st));
    forget_solve(ctx, s->id);
    ctx->live.erase(std::remove(ctx->live.begin(), ctx->live.end(), s), ctx->live.end());
    pool_return(ctx, ctx->free_arena, Block{s->mem, s->bytes});
    delete s;
    if (status == SPAMM_EDIVERGED) return fail(SPAMM_EDIVERGED, "iteration diverged at k = %d (r = %g)", k, h.r);
    return status;
}

int ns_sqrt(spamm_ctx *ctx, const double *s, double *Y, double *Z, int64_t n, int64_t ld, double tau,
            double tol, int maxit, const spamm_ns_opts *opts, spamm_ns_result *res, void *stream) {
    if (!Y || !Z) return fail(SPAMM_EINVAL, "NULL output pointer");
    spamm_solve *sv = nullptr;
    TRY(spamm_solve_begin(ctx, s, n, ld, tau, tol, maxit, opts, &sv, stream));
    // a few iterations per synchronisation, so a finished solve wastes little
    int rc = SPAMM_OK;
    while (sv->host_state.status == ST_RUNNING) {
        const int left = maxit + 1 - sv->host_state.k;
        rc = spamm_solve_step(ctx, &sv, 1, std::max(1, std::min(4, left)), stream);
        if (rc < 0) break;
    }
    fill_result(sv, res);
    if (rc < 0) {
        const std::string keep = g_err;
        (void)spamm_solve_finish(ctx, sv, nullptr, nullptr, ld, stream);
        g_err = keep;
        return rc;
    }
    return spamm_solve_finish(ctx, sv, Y, Z, ld, stream);
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

int spamm_set_graphs(spamm_ctx *ctx, int enable) {
    if (!ctx) return fail(SPAMM_EINVAL, "NULL context");
    ctx->graphs = enable != 0;
    return SPAMM_OK;
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

int64_t spamm_alloc_count(spamm_ctx *ctx) { return ctx ? ctx->allocs : -1; }

int spamm_set_pool_limit(spamm_ctx *ctx, size_t bytes) {
    TRY(enter(ctx));
    ctx->pool_limit = bytes;
    pool_trim(ctx, bytes);
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
