// Internal declarations shared by the kernels and the C-ABI host code.
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

enum Prec { P_F64 = 0, P_F32 = 1, P_BF16X3 = 2 };
enum GemmMode { MODE_PLAIN = 0, MODE_NSX = 1 };

// One operand as held on the device between products.
struct Mat {
    void *tiles;   // nb*nb tiles of b*b elements, tile (i,k) at (i*nb+k)*b*b, row-major inside
    double *q;     // squared-norm pyramid, leaves first (P*P), root last
    double *nrm;   // nb*nb leaf norms sqrt(q) for the cull, row-major (i,k)
};

// Cull of one product C = A (x)_tau B into per-tile retained-k lists.
struct CullProb {
    const double *nrmA;   // nb*nb leaf norms of A
    const double *nrmB;   // nb*nb leaf norms of B
    const double *rootA;  // device scalar: root squared norm of A
    const double *rootB;  // device scalar: root squared norm of B
    double tau;
    int32_t *cnt;         // nb*nb: |R_ij|
    int32_t *kidx;        // nb*nb*nb: R_ij at kidx[(i*nb+j)*nb ...], increasing k
};

// Dispatch order of output tiles for the leaf products: the tiles in Morton
// (Z) order, so that a contiguous range of ranks is a compact 2-D block of C.
void tile_order(int nb, int32_t *order /* nb*nb */);

// Leaf products of one C = A (x)_tau B over the culled lists.
struct GemmProb {
    const void *A;
    const void *B;
    void *C;
    const int32_t *cnt;
    const int32_t *kidx;
    double *qC;    // leaf level (P x P) of C's squared-norm pyramid
    double *part;  // MODE_NSX: per tile (sum (I-x)^2, trace x) over the logical block
};

// ---- launchers (all asynchronous on `st`; return the launch error) --------
hipError_t launch_check_input(const double *s, int64_t n, int64_t ld, double *part, double *out3, hipStream_t st);
hipError_t launch_colsum_max(const double *s, int64_t n, int64_t ld, double mu, double *colsum, double *out1,
                             hipStream_t st);
hipError_t launch_ingest(int prec, const double *s, int64_t ld, double mu, double c, const Geom &g, Mat m,
                         hipStream_t st);
hipError_t launch_identity(int prec, const Geom &g, Mat m, hipStream_t st);
hipError_t launch_pyramid(const Geom &g, Mat m, hipStream_t st);
hipError_t launch_pyramid2(const Geom &g, Mat m0, Mat m1, hipStream_t st);
hipError_t launch_cull(const Geom &g, const CullProb *probs, int nprob, hipStream_t st);
// Longest-first work list for one leaf-product launch: every (problem, tile)
// pair, encoded p*nb*nb + t, ordered by decreasing |R_ij| (counting sort in
// one workgroup).  `morton` gives the base order inside each count bucket.
hipError_t launch_lpt_order(const Geom &g, const int32_t *cnt0, const int32_t *cnt1, int nprob,
                            const int32_t *morton, int32_t *work, hipStream_t st);
hipError_t launch_gemm(int prec, int mode, const Geom &g, const int32_t *work, const GemmProb *probs, int nprob,
                       hipStream_t st);
hipError_t launch_ns_reduce(const Geom &g, const double *part, const int32_t *cntX, const int32_t *cntY,
                            const int32_t *cntZ, int k, double *hist_r, double *hist_t, int64_t *hist_nR,
                            double *out2, hipStream_t st);
hipError_t launch_egress(int prec, const Geom &g, const void *tiles, double *out, int64_t ld, double scale,
                         int divide, hipStream_t st);
hipError_t launch_norms_out(const Geom &g, const double *q, double *out, hipStream_t st);
hipError_t launch_count_triples(const Geom &g, const int32_t *cnt, int64_t *offs, int64_t *total,
                                hipStream_t st);
hipError_t launch_write_triples(const Geom &g, const int32_t *cnt, const int32_t *kidx, const int64_t *offs,
                                int32_t *triples, hipStream_t st);

}  // namespace spk
