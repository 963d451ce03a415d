// Internal declarations shared by the kernels and the host engine.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace spk {

// Blocked geometry of one square operand: n logical rows/columns, b x b leaf
// tiles, nb = ceil(n/b) tiles per side, and a quadtree padded to P = 2^L
// leaves per side (virtual blocks beyond nb have zero norm).
struct Geom {
    int64_t n;
    int b;
    int nb;
    int P;
    int L;
};

Geom make_geom(int64_t n, int b);

// Entries in a squared-norm pyramid of leaf side P (levels P, P/2, ..., 1).
int64_t pyr_len(int P);
// Offset of the level of side S inside a pyramid whose leaf level has side P.
int64_t level_off(int P, int S);

enum Prec { P_F64 = 0, P_F32 = 1, P_BF16X3 = 2, P_BF16X6 = 3 };
// leaf products on the bf16 matrix cores (FP32 tiles split into bf16 pieces)
inline bool is_bf16(int gprec) { return gprec == P_BF16X3 || gprec == P_BF16X6; }

// Dispatch order of output tiles: Morton (Z) order of the nb x nb tile grid.
void tile_order(int nb, int32_t *order /* nb*nb */);

// ---------------------------------------------------------------------------
// Newton-Schulz solve state, one per solve, in device memory.  Kernels read
// the current iterate's buffer parity and the running flag from here, so a
// whole iteration is enqueued without the host deciding anything.
// ---------------------------------------------------------------------------
constexpr int ST_RUNNING = 1000;

struct SolveState {
    int status;       // ST_RUNNING, or the final spamm_status
    int k;            // index of the current iterate (updates performed so far)
    int parity;       // y/z buffer holding the current iterate
    int nondecrease;  // consecutive r_k >= 0.99 r_best while r_best < 1/2 or n |t_k| < 1/2
    double r0, r_prev, r, t;  // r_prev: the best (smallest) residual so far
    double alpha, eps;        // damped map of the next update (1, 0 when undamped or switched off)
    int64_t triples;  // retained triples of all products so far
};

struct SolveDesc {
    SolveState *state;
    int64_t n;
    int nb;
    int maxit, stagnation_stop;
    int damped;          // the map's alpha(t), eps(t) are set from t_k (else alpha = 1, eps = 0)
    int single;          // single-channel instance: cnt_y counts y_k of this iteration
    double tol;
    const double *part;  // nb*nb*2: per-tile (sum (I-x)^2, trace x) of the x product
    const int32_t *cnt_x, *cnt_y, *cnt_z;
    double *hist_r, *hist_t;
    int64_t *hist_nR;    // 3 per iteration
};

// ---------------------------------------------------------------------------
// One product C = A (x)_tau B as the kernels see it.  Operands that alternate
// between two buffers are pairs indexed by the solve's parity (a product
// without a solve uses index 0).  A product with a solve runs only while
// that solve is running.
// ---------------------------------------------------------------------------
struct ProdDesc {
    int64_t n;
    int nb, P;
    double tau;
    const void *A[2];
    const void *B[2];
    void *C[2];
    const double *nrmA[2], *nrmB[2];    // leaf norms: nb*nb row-major, then the transpose
    const double *rootA[2], *rootB[2];  // root squared norms
    double *qC[2];                      // C's squared-norm pyramid (leaf level written by the product)
    double *nrmC[2];                    // C's leaf norms (written by the pyramid pass)
    int32_t *cnt;                       // nb*nb retained counts
    int32_t *kidx;                      // nb*nb*nb retained k lists
    double *part;                       // non-null: Newton-Schulz x product (writes per-tile partials)
    int fused_map;                      // x product: the epilogue writes h = 1.5 I - 0.5 x (else x itself,
                                        // mapped afterwards by the damped-map pass)
    const SolveState *state;            // null: always runs, parity 0
};

constexpr int NBUCKET = 64;          // longest-first buckets of the large-table work-list sort
constexpr int PLAN_SMALL_MAX = 16384;  // tables up to this many tiles are sorted by one workgroup
constexpr int PLAN_HIST_ITEMS = 4;     // items per thread and pass of the large-table sort
// Split-bf16 leaf products: consecutive jobs of the longest-first order run in
// groups of this many tiles on one XCD (workgroup w runs on XCD w mod 8), so
// neighbouring tiles share that XCD's L2.
constexpr int BF3_XCD_RUN = 64;

// Split-bf16 products of 64x64 leaves run one workgroup per quad of output tiles
// (2i..2i+1, 2j..2j+1): the quad's workgroup stages each A_ik and B_kj once
// for the tiles of the quad that retain k.  The quad kernel keeps the union of
// the four retained lists in LDS, for at most QUAD_NB_MAX tiles per side.
// BF16x6 quads hold one workgroup per CU (three planes of LDS), so tables on
// the one-launch front (at most FRONT_MAX tiles) keep one tile per workgroup.
constexpr int QUAD_NB_MAX = 1024;
inline bool quad_tiles(int gprec, int leaf, int total_tiles) {
    return leaf == 64 && (gprec == P_BF16X3 || (gprec == P_BF16X6 && total_tiles > 1024));
}

// One output tile of one product, with every pointer already resolved for the
// current parity, so a leaf-product workgroup starts with a single load.
struct Job {
    const void *a_row;    // tile (i, 0) of A; tile (i, k) at a_row + k * b*b elements
    const void *b_col;    // tile (0, j) of B; tile (k, j) at b_col + k * nb*b*b elements
    void *c;              // tile (i, j) of C
    double *qc;           // C's leaf squared norm (i, j)
    double *part;         // Newton-Schulz x product: 2 partial sums of this tile; else null
    const int32_t *list;  // retained k, increasing
    int64_t n;            // logical order
    int nb, cnt, i, j;
    int fused_map;        // with part: write h = 1.5 I - 0.5 x instead of x
    int k0, k1;           // list[0], list[1] when present (the first stages need no list load)
};

// The cull: products of fewer than CULL_BLOCK_NB tiles per side run one wave
// per output tile (k_cull_tab: few registers, many waves in flight); larger
// ones one wave per block of CULL_RI x CULL_J tiles (k_cull_blk), which keeps
// the leaf norms of its rows of A in registers across the block (such a
// product still has at least 1024 blocks).  Each kernel has its own prefix of
// four-wave workgroups over the products of a table, zero for products of the
// other kind.
constexpr int CULL_RI = 4, CULL_J = 16, CULL_BLOCK_NB = 256;
__host__ __device__ inline bool cull_blocked(int nb) { return nb >= CULL_BLOCK_NB; }
__host__ __device__ inline int cull_blk_waves(int nb) {
    return ((nb + CULL_RI - 1) / CULL_RI) * ((nb + CULL_J - 1) / CULL_J);
}
__host__ __device__ inline int cull_blocks(int nb) { return cull_blocked(nb) ? 0 : (nb * nb + 3) / 4; }
__host__ __device__ inline int cull_blk_blocks(int nb) { return cull_blocked(nb) ? (cull_blk_waves(nb) + 3) / 4 : 0; }

// Device-side tables of one set of products, built on the host when the set
// changes and then reused by every launch over that set.
struct ProdTable {
    const ProdDesc *prods;    // device array
    int nprod;
    const int32_t *cull_pre;  // nprod+1 prefix of k_cull_tab blocks (cull_blocks(nb) per product)
    const int32_t *cullb_pre; // nprod+1 prefix of k_cull_blk blocks (cull_blk_blocks(nb) per product)
    const int32_t *tile_pre;  // nprod+1 prefix of nb*nb tiles
    const int32_t *pyr_pre;   // nprod+1 prefix of first-pass pyramid regions
    const int32_t *pyr2_pre;  // nprod+1 prefix of second-pass pyramid blocks (1 per product with P > 32)
    const int32_t *morton;    // concatenated Morton orders, product p's at tile_pre[p]
    int32_t *work;            // tile_pre[nprod] entries: longest-first global tile ids (of the
                              // quads' first tiles, for quad products)
    Job *jobs;                // the same list expanded into job records, four per quad for quad
                              // products (tile (2i+q/2, 2j+q%2) at 4w+q; cnt -1 past the edge)
    int32_t *work_count;      // device scalar: valid entries in `work` (tiles or quads)
    int32_t *hist;            // NBUCKET * hist_blocks scratch for the large-table sort
    int hist_blocks;
    int total_cull, total_cullb, total_tiles, total_pyr, total_pyr2;
    int total_quads;          // sum of ceil(nb/2)^2
    int max_nb;
};

// ---- launchers (all asynchronous on `st`; return the launch error) --------
hipError_t launch_check_input(const double *s, int64_t n, int64_t ld, double *part, double *out3, hipStream_t st);
hipError_t launch_colsum_max(const double *s, int64_t n, int64_t ld, double mu, double *colsum, double *out1,
                             hipStream_t st);
hipError_t launch_ingest(int prec, const double *s, int64_t ld, double mu, double c, const Geom &g, void *tiles,
                         double *qleaf, hipStream_t st);
hipError_t launch_identity(int prec, const Geom &g, void *tiles, double *qleaf, hipStream_t st);
// Leaf squared norms of a row-major FP64 matrix (no tile copy).
hipError_t launch_leaf_norms(const double *s, int64_t ld, const Geom &g, double *qleaf, hipStream_t st);
// Pyramid of one or two operands (squared-norm pyramid q; leaf norms nrm,
// 2*nb*nb doubles: row-major, then transposed).
hipError_t launch_pyramid(const Geom &g, double *q0, double *nrm0, double *q1, double *nrm1, int nops,
                          hipStream_t st);
hipError_t launch_egress(int prec, const Geom &g, const void *tiles, double *out, int64_t ld, double scale,
                         int divide, hipStream_t st);
hipError_t launch_norms_out(const Geom &g, const double *q, double *out, hipStream_t st);
hipError_t launch_count_triples(const Geom &g, const int32_t *cnt, int64_t *offs, int64_t *total,
                                hipStream_t st);
hipError_t launch_write_triples(const Geom &g, const int32_t *cnt, const int32_t *kidx, const int64_t *offs,
                                int32_t *triples, hipStream_t st);

// Dense row-major n x n helpers of the product representation (leading
// dimension ld): dst = src + mu I; dst = src^T; dst = (src + src^T)/2.
hipError_t launch_shift_copy(const double *src, double *dst, int64_t n, int64_t ld, double mu, hipStream_t st);
hipError_t launch_transpose_dense(const double *src, double *dst, int64_t n, int64_t ld, hipStream_t st);
hipError_t launch_sym_part(const double *src, double *dst, int64_t n, int64_t ld, hipStream_t st);

// One-product table set up on the device (descriptor, prefixes, Morton
// order), for callers that cannot stage a table image from the host; and a
// fill kernel clearing doubles (in place of a memset node).
hipError_t launch_table_one(const ProdDesc &d, const ProdTable &t, hipStream_t st);
hipError_t launch_fill_zero(double *p, int64_t count, hipStream_t st);

// Batched stages over a product table.
hipError_t launch_cull_tab(const ProdTable &t, hipStream_t st);
// Longest-first job list for the leaf products of precision gprec on leaf
// tiles of side `leaf` (quads of tiles when quad_tiles(gprec, leaf, total tiles)).
hipError_t launch_plan_tab(const ProdTable &t, int leaf, int gprec, hipStream_t st);
hipError_t launch_gemm_tab(int prec, int leaf, const ProdTable &t, hipStream_t st);
// Tables of at most FRONT_MAX tiles and FRONT_PRODS products (and not quad
// products): cull and job list in one single-workgroup launch, in place of
// launch_cull_tab followed by launch_plan_tab.
constexpr int FRONT_MAX = 1024;
constexpr int FRONT_PRODS = 256;
bool front_small(const ProdTable &t, int leaf, int gprec);
hipError_t launch_front_small(const ProdTable &t, int leaf, int gprec, hipStream_t st);
hipError_t launch_pyramid_tab(const ProdTable &t, hipStream_t st);  // pyramid of each product's C
// Per solve: r_k, t_k, |R| records and the stop decision.
// With xpyr (the x products, one per solve in the solves' order), the block of
// each solve still running after the decision also builds its x product's
// norm pyramid, in place of launch_pyramid_tab; valid when
// decide_builds_pyramid(x table) holds (every P <= 32).
hipError_t launch_ns_decide(const SolveDesc *solves, int nsolve, const ProdDesc *xpyr, hipStream_t st);
bool decide_builds_pyramid(const ProdTable &tx);
// Transpose of each running product's A (current parity) into its C, with
// C's leaf squared norms: tile (i,j) of C is tile (j,i) of A transposed.
hipError_t launch_transpose_tab(int prec, const ProdTable &t, int leaf, hipStream_t st);
// Damped map of every damped running solve's x product, in place:
// h = (sqrt(alpha)/2) (3 I - alpha (eps I + (1 - 2 eps) x)), and h's leaf norms.
hipError_t launch_ns_map(int prec, const ProdTable &t, int leaf, hipStream_t st);
// After a (y, z) update: parity ^= 1, k += 1 for running solves.
hipError_t launch_ns_advance(const SolveDesc *solves, int nsolve, hipStream_t st);
// The pyramids of the update products of table t (per products per solve, in
// the solves' order), then the advance, in one launch; valid when
// decide_builds_pyramid(t) holds (every P <= 32).
hipError_t launch_pyramid_advance(const SolveDesc *solves, int nsolve, const ProdTable &t, int per,
                                  hipStream_t st);
// Copy each solve's state into a contiguous array (for one read-back).
hipError_t launch_gather_states(const SolveDesc *solves, int nsolve, SolveState *out, hipStream_t st);

}  // namespace spk
