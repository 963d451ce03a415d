// Leaf products of SpAMM on the gfx950 matrix cores: FP64, FP32 and split
// bf16 (BF16x3, BF16x6) tiles, one workgroup per output tile of a job list
// (per quad of output tiles for BF16x3 at b = 64), with the fused
// Newton-Schulz epilogue.  Kept apart from the other kernels so that counter
// profiles of these kernels can be matched to their source.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "device.h"
#include "internal.h"

namespace spk {

// ---------------------------------------------------------------------------
// Leaf products on MFMA.  One workgroup per output tile, taken from the
// longest-first work list; 64x64 tiles use four waves, each owning a 32x32
// quadrant (2x2 blocks of 16x16), 32x32 and 16x16 tiles one wave.  The
// retained k of the tile are consumed in increasing order, in pipeline
// stages (half a tile of k for 64x64 tiles): each stage of A_ik and B_kj goes
// global -> registers -> one of two LDS buffers, two stages ahead of the
// MFMAs that use it.
// Epilogue: the C tile and its squared norm (of the stored values, FP64);
// for a Newton-Schulz x product the tile written is h = 1.5 I_n - 0.5 x, with
// the FP64 partial sums of (I_n - x)^2 and of the trace over the logical block.
// ---------------------------------------------------------------------------
typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef double d2 __attribute__((ext_vector_type(2)));

// Pointers read from job records are generic; marking them global lets the
// compiler use global (not flat) loads and stores, whose completion is
// tracked apart from LDS traffic.
template <typename T>
using gptr = T __attribute__((address_space(1))) *;
template <typename T>
__device__ inline gptr<T> to_global(T *p) {
    return (gptr<T>)p;
}

template <typename T>
struct Mfma;
template <>
struct Mfma<double> {
    typedef v4d acc_t;
    typedef d2 vec_t;  // 16-byte chunk
    static constexpr int VEC = 2;
    __device__ static inline acc_t mma(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    // accumulator element r of lane l holds row l/16 + 4r, column l%16
    __device__ static inline int row_of(int lane, int r) { return (lane >> 4) + 4 * r; }
};
template <>
struct Mfma<float> {
    typedef v4f acc_t;
    typedef v4f vec_t;
    static constexpr int VEC = 4;
    __device__ static inline acc_t mma(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    // accumulator element r of lane l holds row 4(l/16) + r, column l%16
    __device__ static inline int row_of(int lane, int r) { return 4 * (lane >> 4) + r; }
};

template <typename T, int B>
struct TileCfg {
    static constexpr int WAVES = (B == 64) ? 4 : 1;
    static constexpr int NT = 64 * WAVES;
    static constexpr int Q = (B >= 32) ? 32 : 16;  // rows/cols of C per wave
    static constexpr int NBLK = Q / 16;            // 16x16 MFMA blocks per wave side
    static constexpr int VEC = Mfma<T>::VEC;       // elements per 16-byte chunk
    // k extent of one pipeline stage: FP64 stages are half as deep, which
    // halves the LDS and prefetch registers and raises occupancy (3 waves per
    // SIMD at b = 64, 2 at b = 32); the MFMA sequence is the same
    static constexpr int KS = (sizeof(T) == 8 && B >= 32) ? 16 : ((B == 64) ? 32 : B);
    static constexpr int SPT = B / KS;             // stages per retained triple
    // LDS row strides (elements).  A stage (B x KS) is read by fragments
    // A[row + l%16][k + l/16]: a stride of KS + 16 bytes puts the 16 rows and
    // the k offsets of a 32-lane (FP64) or 64-lane (FP32) access in distinct
    // banks.  B stage (KS x B) is read as B[k + l/16][col + l%16]: a stride of
    // B + 16 elements moves consecutive k rows by half (FP64) or a quarter
    // (FP32) of the 64 banks.
    static constexpr int LDA = KS + VEC;
    static constexpr int LDB = (B == 16) ? 16 : B + 16;
    static constexpr int A_CH = B * KS / VEC / NT;  // 16-byte chunks per thread per stage
    static constexpr int B_CH = KS * B / VEC / NT;
};

template <typename T, int B>
__global__ __launch_bounds__((B == 64 ? 256 : 64)) void k_leaf_gemm(const Job *__restrict__ jobs,
                                                                    const int32_t *__restrict__ work_count) {
    using C = TileCfg<T, B>;
    using M = Mfma<T>;
    typedef typename M::acc_t acc_t;
    typedef typename M::vec_t vec_t;
    // two pipeline buffers for each operand
    __shared__ __attribute__((aligned(16))) T As[2][B * C::LDA];
    __shared__ __attribute__((aligned(16))) T Bs[2][C::KS * C::LDB];
    __shared__ double red[3 * C::WAVES];

    // both loads are issued before the test (the job array always has a
    // record for every block of the grid)
    const int nwork = *work_count;
    const Job J = jobs[blockIdx.x];
    if ((int)blockIdx.x >= nwork) return;
    const bool nsx = J.part != nullptr;
    const int nb = J.nb;
    const int i = J.i, j = J.j;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wr = (C::WAVES == 4) ? (w >> 1) : 0, wc = (C::WAVES == 4) ? (w & 1) : 0;
    const int cnt = J.cnt;
    const gptr<const int32_t> list = to_global(J.list);
    const gptr<const T> Arow = to_global((const T *)J.a_row);
    const gptr<const T> Bcol = to_global((const T *)J.b_col);
    constexpr int64_t TS = (int64_t)B * B;
    const int S = cnt * C::SPT;  // pipeline stages

    acc_t acc[C::NBLK][C::NBLK];
#pragma unroll
    for (int bi = 0; bi < C::NBLK; ++bi)
#pragma unroll
        for (int bj = 0; bj < C::NBLK; ++bj)
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[bi][bj][r] = 0;

    // stage s covers k-columns [ks*KS, ks*KS+KS) of triple (i, j, list[s/SPT])
    auto gload = [&](int s, vec_t *ra, vec_t *rb) {
        const int e = s / C::SPT;
        const int k = e == 0 ? J.k0 : (e == 1 ? J.k1 : list[e]);
        const int ks = s % C::SPT;
        const gptr<const T> a = Arow + (int64_t)k * TS + ks * C::KS;
        const gptr<const vec_t> b = (gptr<const vec_t>)(Bcol + (int64_t)k * nb * TS + (int64_t)ks * C::KS * B);
#pragma unroll
        for (int c = 0; c < C::A_CH; ++c) {
            const int el = (tid + c * C::NT) * C::VEC;
            ra[c] = *(gptr<const vec_t>)(a + (el / C::KS) * B + el % C::KS);
        }
#pragma unroll
        for (int c = 0; c < C::B_CH; ++c) rb[c] = b[tid + c * C::NT];
    };
    auto sstore = [&](int buf, const vec_t *ra, const vec_t *rb) {
#pragma unroll
        for (int c = 0; c < C::A_CH; ++c) {
            const int el = (tid + c * C::NT) * C::VEC;
            *(vec_t *)&As[buf][(el / C::KS) * C::LDA + el % C::KS] = ra[c];
        }
#pragma unroll
        for (int c = 0; c < C::B_CH; ++c) {
            const int el = (tid + c * C::NT) * C::VEC;
            *(vec_t *)&Bs[buf][(el / B) * C::LDB + el % B] = rb[c];
        }
    };
    auto compute = [&](int buf) {
#pragma unroll
        for (int kk = 0; kk < C::KS; kk += 4) {
            T av[C::NBLK], bv[C::NBLK];
#pragma unroll
            for (int bi = 0; bi < C::NBLK; ++bi)
                av[bi] = As[buf][(wr * C::Q + bi * 16 + (lane & 15)) * C::LDA + kk + (lane >> 4)];
#pragma unroll
            for (int bj = 0; bj < C::NBLK; ++bj)
                bv[bj] = Bs[buf][(kk + (lane >> 4)) * C::LDB + wc * C::Q + bj * 16 + (lane & 15)];
#pragma unroll
            for (int bi = 0; bi < C::NBLK; ++bi)
#pragma unroll
                for (int bj = 0; bj < C::NBLK; ++bj) acc[bi][bj] = M::mma(av[bi], bv[bj], acc[bi][bj]);
        }
    };

    // Software pipeline: LDS buffers alternate; register sets R0/R1 hold the
    // stages two and one ahead of the one being multiplied, so every global
    // load has two stages of MFMA work to arrive.  One barrier per stage.
    vec_t ra0[C::A_CH], rb0[C::B_CH], ra1[C::A_CH], rb1[C::B_CH];
    if (S > 0) {
        gload(0, ra0, rb0);
        if (S > 1) gload(1, ra1, rb1);
        sstore(0, ra0, rb0);
        if (S > 2) gload(2, ra0, rb0);
    }
    __syncthreads();
    for (int s = 0; s < S; s += 2) {
        // even stage s: LDS buffer 0; stage s+1 waits in R1, stage s+2 in R0
        if (s + 1 < S) sstore(1, ra1, rb1);
        if (s + 3 < S) gload(s + 3, ra1, rb1);
        compute(0);
        __syncthreads();
        if (s + 1 >= S) break;
        // odd stage s+1: LDS buffer 1; stage s+2 waits in R0, stage s+3 in R1
        if (s + 2 < S) sstore(0, ra0, rb0);
        if (s + 4 < S) gload(s + 4, ra0, rb0);
        compute(1);
        __syncthreads();
    }

    // epilogue
    const gptr<T> Ct = to_global((T *)J.c);
    double qs = 0.0, r2 = 0.0, tr = 0.0;
#pragma unroll
    for (int bi = 0; bi < C::NBLK; ++bi)
#pragma unroll
        for (int bj = 0; bj < C::NBLK; ++bj)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = wr * C::Q + bi * 16 + M::row_of(lane, r);
                const int col = wc * C::Q + bj * 16 + (lane & 15);
                const double x = (double)acc[bi][bj][r];
                T out;
                if (nsx) {
                    const int64_t gi = (int64_t)i * B + row, gj = (int64_t)j * B + col;
                    const bool diag = (gi == gj) && (gi < J.n);
                    const bool logical = (gi < J.n) && (gj < J.n);
                    const double h = (diag ? 1.5 : 0.0) - 0.5 * x;
                    const double ex = (diag ? 1.0 : 0.0) - x;
                    if (logical) r2 += ex * ex;
                    if (diag) tr += x;
                    out = J.fused_map ? (T)h : (T)x;
                } else {
                    out = (T)x;
                }
                Ct[row * B + col] = out;
                const double dv = (double)out;
                qs += dv * dv;
            }
    qs = wave_sum(qs);
    if (nsx) {
        r2 = wave_sum(r2);
        tr = wave_sum(tr);
    }
    if (lane == 0) {
        red[w] = qs;
        red[C::WAVES + w] = r2;
        red[2 * C::WAVES + w] = tr;
    }
    __syncthreads();
    if (tid == 0) {
        double a = 0.0, b = 0.0, c = 0.0;
        for (int x = 0; x < C::WAVES; ++x) {
            a += red[x];
            b += red[C::WAVES + x];
            c += red[2 * C::WAVES + x];
        }
        *to_global(J.qc) = a;
        if (nsx) {
            to_global(J.part)[0] = b;
            to_global(J.part)[1] = c;
        }
    }
}

// ---------------------------------------------------------------------------
// Split-bf16 leaf products.  Operands stay FP32 in HBM (norms and the cull
// use those stored values); while a stage is staged into LDS every element is
// split into NP bf16 planes, each piece the round-to-nearest-even bf16 of
// what the previous pieces leave (every difference is exact in FP32):
//   NP = 2 (BF16x3): x = hi + lo; the block product is hi*hi + hi*lo + lo*hi.
//     The dropped lo*lo term and the split residual are O(2^-16) of |a||b|.
//   NP = 3 (BF16x6): x = hi + mid + lo, exact for every FP32 value (three
//     pieces of 8 significant bits and a sign each cover its 24); the block
//     product is the six terms down to 2^-16: lo*hi, hi*lo, mid*mid, mid*hi,
//     hi*mid, hi*hi, smallest first.  The dropped mid*lo, lo*mid, lo*lo are
//     O(2^-24) of |a||b|, below the FP32 accumulation itself.
// Each 16x16x32 block product runs on the bf16 matrix cores, accumulated in
// FP32.  A is staged row-major (k contiguous per row); B is staged
// transposed (k contiguous per column), the k pairs being packed by the
// conversion itself, so both MFMA operands are single 16-byte LDS reads.
// ---------------------------------------------------------------------------
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f2 __attribute__((ext_vector_type(2)));

template <int B>
struct Bf3Cfg {
    static constexpr int WAVES = (B == 64) ? 4 : 1;
    static constexpr int NT = 64 * WAVES;
    static constexpr int Q = 32;                // rows/cols of C per wave
    static constexpr int NBLK = 2;              // 16x16 blocks per wave side
    static constexpr int KS = 32;               // k of one stage = k of one MFMA
    static constexpr int SPT = B / KS;          // stages per retained triple
    static constexpr int LDK = KS + 8;          // bf16 per LDS row: 16-byte pad keeps 16-lane reads conflict-free
    static constexpr int A_CH = B * KS / 4 / NT;         // float4 chunks of A per thread per stage
    static constexpr int B_UN = (KS / 2) * (B / 4) / NT;  // (k pair, 4 columns) units of B per thread
};

// Split of two FP32 values into NP packed bf16 pairs, p[0] the leading piece.
template <int NP>
__device__ inline void split_pair(float x0, float x1, unsigned (&p)[NP]) {
    f2 v = {x0, x1};
#pragma unroll
    for (int q = 0; q < NP; ++q) {
        p[q] = __builtin_bit_cast(unsigned, __builtin_convertvector(v, bf16x2));
        if (q + 1 < NP) {
            const f2 pv = {__builtin_bit_cast(float, p[q] << 16), __builtin_bit_cast(float, p[q] & 0xffff0000u)};
            v = v - pv;
        }
    }
}

// One 16x16x32 block product of split operands (pieces [0] leading), the
// terms summed smallest first into acc.
template <int NP>
__device__ inline v4f mma_split(const bf16x8 *a, const bf16x8 *b, v4f acc) {
    if constexpr (NP == 2) {
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1], b[0], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], b[1], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], b[0], acc, 0, 0, 0);
    } else {
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[2], b[0], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], b[2], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1], b[1], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1], b[0], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], b[1], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], b[0], acc, 0, 0, 0);
    }
    return acc;
}

template <int B, int NP>
__global__ __launch_bounds__((B == 64 ? 256 : 64)) void k_leaf_gemm_bf3(const Job *__restrict__ jobs,
                                                                        const int32_t *__restrict__ work_count) {
    using C = Bf3Cfg<B>;
    // [buffer][plane][rows x LDK]
    __shared__ __attribute__((aligned(16))) __bf16 As[2][NP][B * C::LDK];
    __shared__ __attribute__((aligned(16))) __bf16 Bt[2][NP][B * C::LDK];
    __shared__ double red[3 * C::WAVES];

    const int nwork = *work_count;
    const Job J = jobs[blockIdx.x];
    if ((int)blockIdx.x >= nwork) return;
    const bool nsx = J.part != nullptr;
    const int nb = J.nb;
    const int i = J.i, j = J.j;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wr = (C::WAVES == 4) ? (w >> 1) : 0, wc = (C::WAVES == 4) ? (w & 1) : 0;
    const int cnt = J.cnt;
    const gptr<const int32_t> list = to_global(J.list);
    const gptr<const float> Arow = to_global((const float *)J.a_row);
    const gptr<const float> Bcol = to_global((const float *)J.b_col);
    constexpr int64_t TS = (int64_t)B * B;
    const int S = cnt * C::SPT;

    // NP = 2: one FP32 accumulator over the whole k list.  NP = 3: each
    // stage's six terms are summed in FP32 from zero and the stage sums in
    // FP64, so the FP32 rounding is that of one 32-k block product.
    constexpr bool ACC64 = NP == 3;
    v4f acc[C::NBLK][C::NBLK];
    double acc64[ACC64 ? C::NBLK : 1][ACC64 ? C::NBLK : 1][4];
#pragma unroll
    for (int bi = 0; bi < C::NBLK; ++bi)
#pragma unroll
        for (int bj = 0; bj < C::NBLK; ++bj)
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[bi][bj][r] = 0.0f;
    if constexpr (ACC64) {
#pragma unroll
        for (int bi = 0; bi < C::NBLK; ++bi)
#pragma unroll
            for (int bj = 0; bj < C::NBLK; ++bj)
#pragma unroll
                for (int r = 0; r < 4; ++r) acc64[bi][bj][r] = 0.0;
    }

    // stage s: k-columns [ks*KS, ks*KS+KS) of triple (i, j, list[s/SPT]).
    // A chunk c: 4 consecutive k of one row.  B unit u: rows 2kp and 2kp+1
    // (a k pair) of 4 consecutive columns 4cg..4cg+3.
    auto gload = [&](int s, v4f *ra, v4f *rb) {
        const int e = s / C::SPT;
        const int k = e == 0 ? J.k0 : (e == 1 ? J.k1 : list[e]);
        const int ks = s % C::SPT;
        const gptr<const float> a = Arow + (int64_t)k * TS + ks * C::KS;
        const gptr<const float> b = Bcol + (int64_t)k * nb * TS + (int64_t)ks * C::KS * B;
#pragma unroll
        for (int c = 0; c < C::A_CH; ++c) {
            const int el = (tid + c * C::NT) * 4;
            ra[c] = *(gptr<const v4f>)(a + (el / C::KS) * B + el % C::KS);
        }
#pragma unroll
        for (int c = 0; c < C::B_UN; ++c) {
            const int u = tid + c * C::NT;
            const int kp = u % (C::KS / 2), cg = u / (C::KS / 2);
            rb[2 * c] = *(gptr<const v4f>)(b + (2 * kp) * B + 4 * cg);
            rb[2 * c + 1] = *(gptr<const v4f>)(b + (2 * kp + 1) * B + 4 * cg);
        }
    };
    auto sstore = [&](int buf, const v4f *ra, const v4f *rb) {
#pragma unroll
        for (int c = 0; c < C::A_CH; ++c) {
            const int el = (tid + c * C::NT) * 4;
            const int row = el / C::KS, k = el % C::KS;
            unsigned p0[NP], p1[NP];
            split_pair<NP>(ra[c][0], ra[c][1], p0);
            split_pair<NP>(ra[c][2], ra[c][3], p1);
            typedef unsigned u2 __attribute__((ext_vector_type(2)));
#pragma unroll
            for (int q = 0; q < NP; ++q) *(u2 *)&As[buf][q][row * C::LDK + k] = u2{p0[q], p1[q]};
        }
#pragma unroll
        for (int c = 0; c < C::B_UN; ++c) {
            const int u = tid + c * C::NT;
            const int kp = u % (C::KS / 2), cg = u / (C::KS / 2);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                unsigned pp[NP];
                split_pair<NP>(rb[2 * c][q], rb[2 * c + 1][q], pp);  // (k, k+1) of column 4cg+q
                const int col = 4 * cg + q;
#pragma unroll
                for (int x = 0; x < NP; ++x) *(unsigned *)&Bt[buf][x][col * C::LDK + 2 * kp] = pp[x];
            }
        }
    };
    auto compute = [&](int buf) {
        // operand layout of the 16x16x32 bf16 MFMA: lane l supplies row (A) or
        // column (B) l%16 at k = 8(l/16) .. 8(l/16)+7
        bf16x8 af[C::NBLK][NP], bf[C::NBLK][NP];
        const int ko = 8 * (lane >> 4);
#pragma unroll
        for (int bi = 0; bi < C::NBLK; ++bi) {
            const int row = wr * C::Q + bi * 16 + (lane & 15);
#pragma unroll
            for (int q = 0; q < NP; ++q) af[bi][q] = *(const bf16x8 *)&As[buf][q][row * C::LDK + ko];
        }
#pragma unroll
        for (int bj = 0; bj < C::NBLK; ++bj) {
            const int col = wc * C::Q + bj * 16 + (lane & 15);
#pragma unroll
            for (int q = 0; q < NP; ++q) bf[bj][q] = *(const bf16x8 *)&Bt[buf][q][col * C::LDK + ko];
        }
#pragma unroll
        for (int bi = 0; bi < C::NBLK; ++bi)
#pragma unroll
            for (int bj = 0; bj < C::NBLK; ++bj) {
                if constexpr (ACC64) {
                    const v4f t = mma_split<NP>(af[bi], bf[bj], v4f{0.0f, 0.0f, 0.0f, 0.0f});
#pragma unroll
                    for (int r = 0; r < 4; ++r) acc64[bi][bj][r] += (double)t[r];
                } else {
                    acc[bi][bj] = mma_split<NP>(af[bi], bf[bj], acc[bi][bj]);
                }
            }
    };

    // same two-stage-ahead software pipeline as the FP32/FP64 kernel
    v4f ra0[C::A_CH], rb0[2 * C::B_UN], ra1[C::A_CH], rb1[2 * C::B_UN];
    if (S > 0) {
        gload(0, ra0, rb0);
        if (S > 1) gload(1, ra1, rb1);
        sstore(0, ra0, rb0);
        if (S > 2) gload(2, ra0, rb0);
    }
    __syncthreads();
    for (int s = 0; s < S; s += 2) {
        if (s + 1 < S) sstore(1, ra1, rb1);
        if (s + 3 < S) gload(s + 3, ra1, rb1);
        compute(0);
        __syncthreads();
        if (s + 1 >= S) break;
        if (s + 2 < S) sstore(0, ra0, rb0);
        if (s + 4 < S) gload(s + 4, ra0, rb0);
        compute(1);
        __syncthreads();
    }

    // epilogue (FP32 tile out; FP64 norms and Newton-Schulz partials)
    const gptr<float> Ct = to_global((float *)J.c);
    double qs = 0.0, r2 = 0.0, tr = 0.0;
#pragma unroll
    for (int bi = 0; bi < C::NBLK; ++bi)
#pragma unroll
        for (int bj = 0; bj < C::NBLK; ++bj)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = wr * C::Q + bi * 16 + 4 * (lane >> 4) + r;
                const int col = wc * C::Q + bj * 16 + (lane & 15);
                double x;
                if constexpr (ACC64)
                    x = acc64[bi][bj][r];
                else
                    x = (double)acc[bi][bj][r];
                float out;
                if (nsx) {
                    const int64_t gi = (int64_t)i * B + row, gj = (int64_t)j * B + col;
                    const bool diag = (gi == gj) && (gi < J.n);
                    const bool logical = (gi < J.n) && (gj < J.n);
                    const double h = (diag ? 1.5 : 0.0) - 0.5 * x;
                    const double ex = (diag ? 1.0 : 0.0) - x;
                    if (logical) r2 += ex * ex;
                    if (diag) tr += x;
                    out = J.fused_map ? (float)h : (float)x;
                } else {
                    out = (float)x;
                }
                Ct[row * B + col] = out;
                const double dv = (double)out;
                qs += dv * dv;
            }
    qs = wave_sum(qs);
    if (nsx) {
        r2 = wave_sum(r2);
        tr = wave_sum(tr);
    }
    if (lane == 0) {
        red[w] = qs;
        red[C::WAVES + w] = r2;
        red[2 * C::WAVES + w] = tr;
    }
    __syncthreads();
    if (tid == 0) {
        double a = 0.0, b = 0.0, c = 0.0;
        for (int x = 0; x < C::WAVES; ++x) {
            a += red[x];
            b += red[C::WAVES + x];
            c += red[2 * C::WAVES + x];
        }
        *to_global(J.qc) = a;
        if (nsx) {
            to_global(J.part)[0] = b;
            to_global(J.part)[1] = c;
        }
    }
}

// ---------------------------------------------------------------------------
// Split-bf16 leaf products of 64x64 tiles (BF16x3, and BF16x6 for tables past
// the one-launch front), one workgroup per quad of output tiles
// (2i+di, 2j+dj), eight waves: waves 2t and 2t+1 own rows 0-31 and 32-63 of
// tile t = 2di+dj (2x4 blocks of 16x16 each), so four waves per SIMD fit and
// the staging of a stage is spread over 512 threads (one A chunk and one B
// unit each).  The workgroup first merges the four retained lists into their
// union in LDS (increasing k, with a 4-bit mask of the tiles that retain k),
// then runs the two-stage-ahead pipeline over the union: a stage stages A_ik
// of each row half and B_kj of each column half that some tile of the mask
// needs, once for the quad, and each wave whose tile retains k multiplies.
// Every tile sees its own retained k in increasing order with the MFMA
// sequence (and, for BF16x6, the FP64 sum of the 32-k stage sums) of the
// one-tile kernel k_leaf_gemm_bf3 (four waves of 32x32 quadrants), and its
// norm and Newton-Schulz partials are summed over the same quadrants in the
// same order, so a quad's tiles come out bitwise as that kernel computes them
// at b = 64.
// A stage holds 32 k.  A planes are rows of 32 bf16 (64 B) whose 16-byte
// chunks are XOR-swizzled by (row/4) mod 4, so the 16 rows of a fragment read
// fall in distinct banks; B planes (columns of k, transposed) keep the padded
// stride of the one-tile kernel, which also keeps the 4-byte k-pair stores
// conflict-free.
// ---------------------------------------------------------------------------
struct Bf3Quad {
    static constexpr int B = 64;
    static constexpr int NT = 512;  // eight waves, two per tile
    static constexpr int KS = 32;
    static constexpr int SPT = B / KS;
    static constexpr int LDA = KS;      // swizzled, unpadded
    static constexpr int LDB = KS + 8;  // padded
    static constexpr int A_CH = B * KS / 4 / NT;               // float4 chunks of one A half per thread per stage
    static constexpr int B_UN = 2 * (KS / 2) * (B / 4) / NT;  // (k pair, 4 columns) units of both B halves per thread
};
static_assert(Bf3Quad::A_CH == 1 && Bf3Quad::B_UN == 1, "stage split assumed below");

__device__ inline int swz_a(int row, int k) {  // bf16 offset of (row, k) in an A plane
    return row * Bf3Quad::LDA + ((((k >> 3) ^ (row >> 2)) & 3) << 3) + (k & 7);
}

// NP = 2 (BF16x3): at most 128 registers per lane, so that two workgroups
// (four waves per SIMD) share a CU.  NP = 3 (BF16x6): the three planes take
// 110 KB of LDS, one workgroup per CU, up to 256 registers.
template <int NP>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(NP == 2 ? 4 : 2, NP == 2 ? 4 : 2))) void
k_leaf_gemm_bf3_quad(const Job *__restrict__ jobs, const int32_t *__restrict__ work_count) {
    using C = Bf3Quad;
    constexpr int B = C::B;
    constexpr int NT = C::NT;
    __shared__ __attribute__((aligned(16))) __bf16 As[2][2][NP][B * C::LDA];
    __shared__ __attribute__((aligned(16))) __bf16 Bt[2][2][NP][B * C::LDB];
    __shared__ unsigned umask[QUAD_NB_MAX / 4];
    __shared__ unsigned ulist[QUAD_NB_MAX];
    __shared__ int wtot[8];
    __shared__ double red[4][3][4];  // [tile][norm, r2, trace][quadrant]

    const int nwork = *work_count;
    if ((int)blockIdx.x >= nwork) return;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int t = w >> 1, rh = w & 1;  // tile of the quad, row half of the tile
    const Job J = jobs[4 * blockIdx.x + t];
    const int nb = jobs[4 * blockIdx.x].nb;
    const gptr<const float> Arow[2] = {to_global((const float *)jobs[4 * blockIdx.x].a_row),
                                       to_global((const float *)jobs[4 * blockIdx.x + 2].a_row)};
    const gptr<const float> Bcol[2] = {to_global((const float *)jobs[4 * blockIdx.x].b_col),
                                       to_global((const float *)jobs[4 * blockIdx.x + 1].b_col)};
    constexpr int64_t TS = (int64_t)B * B;

    // union of the four retained lists (the first wave of each tile adds its bit)
    const int nwords = (nb + 3) / 4;
    for (int x = tid; x < nwords; x += NT) umask[x] = 0u;
    __syncthreads();
    if (rh == 0 && J.cnt > 0) {
        const gptr<const int32_t> list = to_global(J.list);
        for (int e = lane; e < J.cnt; e += 64) {
            const int k = list[e];
            atomicOr(&umask[k >> 2], 1u << (8 * (k & 3) + t));
        }
    }
    __syncthreads();
    const unsigned word = tid < nwords ? umask[tid] : 0u;
    const int mine = (int)((word & 0xffu) != 0) + (int)((word & 0xff00u) != 0) + (int)((word & 0xff0000u) != 0) +
                     (int)((word & 0xff000000u) != 0);
    int incl = mine;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int v = __shfl_up(incl, off, 64);
        if (lane >= off) incl += v;
    }
    if (lane == 63) wtot[w] = incl;
    __syncthreads();
    int pos = incl - mine;
    for (int x = 0; x < w; ++x) pos += wtot[x];
    int U = 0;
#pragma unroll
    for (int x = 0; x < 8; ++x) U += wtot[x];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const unsigned m = (word >> (8 * q)) & 0xfu;
        if (m) ulist[pos++] = (unsigned)(4 * tid + q) | (m << 16);
    }
    __syncthreads();

    const int S = U * C::SPT;
    const int di = t >> 1, dj = t & 1;
    const int hb = tid >> 8;          // the B column half this thread stages
    const int ub = tid & 255;         // its (k pair, 4 columns) unit of that half
    const int kp = ub % (C::KS / 2), cg = ub / (C::KS / 2);

    // NP = 3: each stage's six terms summed in FP32 from zero, the stage sums in
    // FP64, as in k_leaf_gemm_bf3<64, 3>
    constexpr bool ACC64 = NP == 3;
    v4f acc[2][4];
    double acc64[ACC64 ? 2 : 1][ACC64 ? 4 : 1][4];
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 4; ++bj)
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[bi][bj][r] = 0.0f;
    if constexpr (ACC64) {
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
            for (int bj = 0; bj < 4; ++bj)
#pragma unroll
                for (int r = 0; r < 4; ++r) acc64[bi][bj][r] = 0.0;
    }

    auto needA = [](unsigned m, int h) { return (m & (h ? 0xcu : 0x3u)) != 0u; };
    auto needB = [](unsigned m, int h) { return (m & (h ? 0xau : 0x5u)) != 0u; };
    // registers of one stage: [0], [1] one chunk of A halves 0, 1; [2], [3] rows 2kp, 2kp+1 of this thread's B unit
    auto gload = [&](int s, v4f *r) {
        const unsigned e = ulist[s / C::SPT];
        const int k = (int)(e & 0xffffu);
        const unsigned m = e >> 16;
        const int ks = s % C::SPT;
        const int el = tid * 4;
#pragma unroll
        for (int h = 0; h < 2; ++h)
            if (needA(m, h)) {
                const gptr<const float> a = Arow[h] + (int64_t)k * TS + ks * C::KS;
                r[h] = *(gptr<const v4f>)(a + (el / C::KS) * B + el % C::KS);
            }
        if (needB(m, hb)) {
            const gptr<const float> b = Bcol[hb] + (int64_t)k * nb * TS + (int64_t)ks * C::KS * B;
            r[2] = *(gptr<const v4f>)(b + (2 * kp) * B + 4 * cg);
            r[3] = *(gptr<const v4f>)(b + (2 * kp + 1) * B + 4 * cg);
        }
    };
    auto sstore = [&](int buf, int s, const v4f *r) {
        const unsigned m = ulist[s / C::SPT] >> 16;
        typedef unsigned u2 __attribute__((ext_vector_type(2)));
        const int el = tid * 4;
        const int row = el / C::KS, k = el % C::KS;
#pragma unroll
        for (int h = 0; h < 2; ++h)
            if (needA(m, h)) {
                unsigned p0[NP], p1[NP];
                split_pair<NP>(r[h][0], r[h][1], p0);
                split_pair<NP>(r[h][2], r[h][3], p1);
#pragma unroll
                for (int x = 0; x < NP; ++x) *(u2 *)&As[buf][h][x][swz_a(row, k)] = u2{p0[x], p1[x]};
            }
        if (needB(m, hb)) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                unsigned pp[NP];
                split_pair<NP>(r[2][q], r[3][q], pp);  // (k, k+1) of column 4cg+q
                const int col = 4 * cg + q;
#pragma unroll
                for (int x = 0; x < NP; ++x) *(unsigned *)&Bt[buf][hb][x][col * C::LDB + 2 * kp] = pp[x];
            }
        }
    };
    auto compute = [&](int buf, int s) {
        const unsigned m = ulist[s / C::SPT] >> 16;
        if (!((m >> t) & 1u)) return;
        const int ko = 8 * (lane >> 4);
        bf16x8 af[2][NP];
#pragma unroll
        for (int bi = 0; bi < 2; ++bi) {
            const int row = rh * 32 + bi * 16 + (lane & 15);
#pragma unroll
            for (int x = 0; x < NP; ++x) af[bi][x] = *(const bf16x8 *)&As[buf][di][x][swz_a(row, ko)];
        }
#pragma unroll
        for (int bj = 0; bj < 4; ++bj) {
            const int col = bj * 16 + (lane & 15);
            bf16x8 bf[NP];
#pragma unroll
            for (int x = 0; x < NP; ++x) bf[x] = *(const bf16x8 *)&Bt[buf][dj][x][col * C::LDB + ko];
#pragma unroll
            for (int bi = 0; bi < 2; ++bi) {
                if constexpr (ACC64) {
                    const v4f t = mma_split<NP>(af[bi], bf, v4f{0.0f, 0.0f, 0.0f, 0.0f});
#pragma unroll
                    for (int r = 0; r < 4; ++r) acc64[bi][bj][r] += (double)t[r];
                } else {
                    acc[bi][bj] = mma_split<NP>(af[bi], bf, acc[bi][bj]);
                }
            }
        }
    };

    v4f r0[4], r1[4];
    if (S > 0) {
        gload(0, r0);
        if (S > 1) gload(1, r1);
        sstore(0, 0, r0);
        if (S > 2) gload(2, r0);
    }
    __syncthreads();
    for (int s = 0; s < S; s += 2) {
        if (s + 1 < S) sstore(1, s + 1, r1);
        if (s + 3 < S) gload(s + 3, r1);
        compute(0, s);
        __syncthreads();
        if (s + 1 >= S) break;
        if (s + 2 < S) sstore(0, s + 2, r0);
        if (s + 4 < S) gload(s + 4, r0);
        compute(1, s + 1);
        __syncthreads();
    }

    // epilogue: this wave's two quadrants (rh, 0) and (rh, 1) of its tile
    const bool live = J.cnt >= 0;  // tiles past the edge write nothing
    const bool nsx = J.part != nullptr;
    const gptr<float> Ct = to_global((float *)J.c);
#pragma unroll
    for (int wc = 0; wc < 2; ++wc) {
        double qs = 0.0, r2 = 0.0, tr = 0.0;
        if (live) {
#pragma unroll
            for (int bi = 0; bi < 2; ++bi)
#pragma unroll
                for (int bj = 0; bj < 2; ++bj)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int row = rh * 32 + bi * 16 + 4 * (lane >> 4) + r;
                        const int col = wc * 32 + bj * 16 + (lane & 15);
                        double x;
                        if constexpr (ACC64)
                            x = acc64[bi][2 * wc + bj][r];
                        else
                            x = (double)acc[bi][2 * wc + bj][r];
                        float out;
                        if (nsx) {
                            const int64_t gi = (int64_t)J.i * B + row, gj = (int64_t)J.j * B + col;
                            const bool diag = (gi == gj) && (gi < J.n);
                            const bool logical = (gi < J.n) && (gj < J.n);
                            const double h = (diag ? 1.5 : 0.0) - 0.5 * x;
                            const double ex = (diag ? 1.0 : 0.0) - x;
                            if (logical) r2 += ex * ex;
                            if (diag) tr += x;
                            out = J.fused_map ? (float)h : (float)x;
                        } else {
                            out = (float)x;
                        }
                        Ct[row * B + col] = out;
                        const double dv = (double)out;
                        qs += dv * dv;
                    }
        }
        qs = wave_sum(qs);
        r2 = wave_sum(r2);
        tr = wave_sum(tr);
        if (lane == 0) {
            red[t][0][2 * rh + wc] = qs;
            red[t][1][2 * rh + wc] = r2;
            red[t][2][2 * rh + wc] = tr;
        }
    }
    __syncthreads();
    if (live && rh == 0 && lane == 0) {
        double qa = 0.0, r2a = 0.0, tra = 0.0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            qa += red[t][0][q];
            r2a += red[t][1][q];
            tra += red[t][2][q];
        }
        *to_global(J.qc) = qa;
        if (nsx) {
            to_global(J.part)[0] = r2a;
            to_global(J.part)[1] = tra;
        }
    }
}

template <typename T, int B>
static void gemm_launch(const ProdTable &t, hipStream_t st) {
    hipLaunchKernelGGL((k_leaf_gemm<T, B>), dim3(t.total_tiles), dim3(TileCfg<T, B>::NT), 0, st, t.jobs,
                       t.work_count);
}

template <typename T>
static void gemm_dispatch_b(int leaf, const ProdTable &t, hipStream_t st) {
    if (leaf == 64)
        gemm_launch<T, 64>(t, st);
    else if (leaf == 32)
        gemm_launch<T, 32>(t, st);
    else
        gemm_launch<T, 16>(t, st);
}

hipError_t launch_gemm_tab(int prec, int leaf, const ProdTable &t, hipStream_t st) {
    if (prec == P_F64) {
        gemm_dispatch_b<double>(leaf, t, st);
    } else if (prec == P_BF16X3) {
        if (quad_tiles(prec, leaf, t.total_tiles))  // leaf 64
            hipLaunchKernelGGL(k_leaf_gemm_bf3_quad<2>, dim3(t.total_quads), dim3(Bf3Quad::NT), 0, st, t.jobs,
                               t.work_count);
        else if (leaf == 32)
            hipLaunchKernelGGL((k_leaf_gemm_bf3<32, 2>), dim3(t.total_tiles), dim3(64), 0, st, t.jobs,
                               t.work_count);
        else
            return hipErrorInvalidValue;
    } else if (prec == P_BF16X6) {
        if (quad_tiles(prec, leaf, t.total_tiles))
            hipLaunchKernelGGL(k_leaf_gemm_bf3_quad<3>, dim3(t.total_quads), dim3(Bf3Quad::NT), 0, st, t.jobs,
                               t.work_count);
        else if (leaf == 64)
            hipLaunchKernelGGL((k_leaf_gemm_bf3<64, 3>), dim3(t.total_tiles), dim3(256), 0, st, t.jobs,
                               t.work_count);
        else if (leaf == 32)
            hipLaunchKernelGGL((k_leaf_gemm_bf3<32, 3>), dim3(t.total_tiles), dim3(64), 0, st, t.jobs,
                               t.work_count);
        else
            return hipErrorInvalidValue;
    } else {
        gemm_dispatch_b<float>(leaf, t, st);
    }
    return hipGetLastError();
}

}  // namespace spk
