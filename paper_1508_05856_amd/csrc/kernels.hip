// HIP kernels for gfx950 (CDNA4): input checks and ingest, the Frobenius-norm
// pyramid, the two-sided cull and the job lists of the leaf products (whose
// kernels are in leaf_gemm.hip), Newton-Schulz control and map, reductions and
// egress.
//
// Layout in HBM: every operand is tile-major, b x b tiles each contiguous and
// row-major inside, tile (i,k) at offset (i*nb + k)*b*b.  The pyramid holds
// squared norms, leaves first (P x P, P = 2^L >= nb), then each parent level.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "device.h"
#include "internal.h"

namespace spk {

Geom make_geom(int64_t n, int b) {
    Geom g;
    g.n = n;
    g.b = b;
    g.nb = (int)((n + b - 1) / b);
    g.L = 0;
    while ((1 << g.L) < g.nb) g.L++;
    g.P = 1 << g.L;
    return g;
}

int64_t pyr_len(int P) {
    int64_t s = 0;
    for (int64_t S = P; S >= 1; S >>= 1) s += S * S;
    return s;
}

int64_t level_off(int P, int S) {
    int64_t o = 0;
    for (int64_t T = P; T > S; T >>= 1) o += T * T;
    return o;
}

void tile_order(int nb, int32_t *order) {
    int P = 1;
    while (P < nb) P <<= 1;
    int m = 0;
    for (int64_t z = 0; z < (int64_t)P * P; ++z) {
        int i = 0, j = 0;
        for (int bit = 0; (1 << bit) < P; ++bit) {
            j |= (int)((z >> (2 * bit)) & 1) << bit;
            i |= (int)((z >> (2 * bit + 1)) & 1) << bit;
        }
        if (i < nb && j < nb) order[m++] = i * nb + j;
    }
}

// ---------------------------------------------------------------------------
// Device-side set-up of a one-product table (the allocation-free product):
// the product descriptor, the prefix arrays and the Morton order of its
// nb x nb tiles, the same order tile_order lists on the host, built in
// chunks of 4096 Morton codes with a block scan for the compaction.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void k_table_one(ProdDesc d, ProdTable t) {
    __shared__ int wsum[16];
    __shared__ int carry;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int nb = d.nb, P = d.P;
    if (tid == 0) {
        *const_cast<ProdDesc *>(t.prods) = d;
        const int32_t nb2 = nb * nb;
        int32_t *cull = const_cast<int32_t *>(t.cull_pre), *cullb = const_cast<int32_t *>(t.cullb_pre);
        int32_t *tile = const_cast<int32_t *>(t.tile_pre);
        int32_t *pyr = const_cast<int32_t *>(t.pyr_pre), *pyr2 = const_cast<int32_t *>(t.pyr2_pre);
        cull[0] = cullb[0] = tile[0] = pyr[0] = pyr2[0] = 0;
        cull[1] = cull_blocks(nb);
        cullb[1] = cull_blk_blocks(nb);
        tile[1] = nb2;
        pyr[1] = P <= 32 ? 1 : (P / 32) * (P / 32);
        pyr2[1] = P > 32 ? 1 : 0;
        carry = 0;
    }
    __syncthreads();
    int32_t *morton = const_cast<int32_t *>(t.morton);
    const int64_t PP = (int64_t)P * P;
    for (int64_t base = 0; base < PP; base += 4 * 1024) {
        int idx[4], valid[4], mine = 0;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t z = base + 4 * tid + u;
            int i = 0, j = 0;
            for (int bit = 0; (1 << bit) < P; ++bit) {
                j |= (int)((z >> (2 * bit)) & 1) << bit;
                i |= (int)((z >> (2 * bit + 1)) & 1) << bit;
            }
            valid[u] = (z < PP && i < nb && j < nb) ? 1 : 0;
            idx[u] = i * nb + j;
            mine += valid[u];
        }
        int incl = mine;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const int v = __shfl_up(incl, off, 64);
            if (lane >= off) incl += v;
        }
        if (lane == 63) wsum[w] = incl;
        __syncthreads();
        int pos = carry + incl - mine;
        for (int x = 0; x < w; ++x) pos += wsum[x];
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (valid[u]) morton[pos++] = idx[u];
        __syncthreads();
        if (tid == 0) {
            int tot = 0;
            for (int x = 0; x < 16; ++x) tot += wsum[x];
            carry += tot;
        }
        __syncthreads();
    }
}

hipError_t launch_table_one(const ProdDesc &d, const ProdTable &t, hipStream_t st) {
    hipLaunchKernelGGL(k_table_one, dim3(1), dim3(1024), 0, st, d, t);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_fill_zero(double *__restrict__ p, int64_t count) {
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < count; e += (int64_t)gridDim.x * 256) p[e] = 0.0;
}

hipError_t launch_fill_zero(double *p, int64_t count, hipStream_t st) {
    const int64_t blocks = (count + 255) / 256;
    hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)(blocks < 1024 ? (blocks > 0 ? blocks : 1) : 1024)), dim3(256), 0,
                       st, p, count);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Input checks: max |s - s^T|, max |s|, and a non-finite flag, per 32x32 block
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_check_input(const double *__restrict__ s, int64_t n, int64_t ld,
                                                      double *__restrict__ part) {
    __shared__ double tileT[32][33];
    __shared__ double sh[4];
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
    const int64_t r0 = (int64_t)blockIdx.y * 32, c0 = (int64_t)blockIdx.x * 32;
    // the mirrored block s[c0.., r0..], stored transposed
    for (int m = 0; m < 32; m += 8) {
        const int64_t r = c0 + ty + m, c = r0 + tx;
        tileT[tx][ty + m] = (r < n && c < n) ? s[r * ld + c] : 0.0;
    }
    __syncthreads();
    double dmax = 0.0, amax = 0.0, bad = 0.0;
    for (int m = 0; m < 32; m += 8) {
        const int64_t r = r0 + ty + m, c = c0 + tx;
        if (r < n && c < n) {
            const double v = s[r * ld + c];
            if (!isfinite(v)) bad = 1.0;
            amax = fmax(amax, fabs(v));
            const double d = fabs(v - tileT[ty + m][tx]);
            dmax = fmax(dmax, d);
        }
    }
    dmax = block_max<256>(dmax, sh);
    amax = block_max<256>(amax, sh);
    bad = block_max<256>(bad, sh);
    if (threadIdx.x == 0) {
        const int64_t b = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
        part[3 * b + 0] = dmax;
        part[3 * b + 1] = amax;
        part[3 * b + 2] = bad;
    }
}

// Max over `count` strided entries (stride, offset), single block.
__global__ __launch_bounds__(1024) void k_reduce_max(const double *__restrict__ x, int64_t count, int stride,
                                                      int offset, double *__restrict__ out) {
    __shared__ double sh[16];
    double m = 0.0;
    for (int64_t i = threadIdx.x; i < count; i += 1024) m = fmax(m, x[i * stride + offset]);
    m = block_max<1024>(m, sh);
    if (threadIdx.x == 0) *out = m;
}

hipError_t launch_check_input(const double *s, int64_t n, int64_t ld, double *part, double *out3,
                              hipStream_t st) {
    const int nbk = (int)((n + 31) / 32);
    hipLaunchKernelGGL(k_check_input, dim3(nbk, nbk), dim3(256), 0, st, s, n, ld, part);
    for (int c = 0; c < 3; ++c)
        hipLaunchKernelGGL(k_reduce_max, dim3(1), dim3(1024), 0, st, part, (int64_t)nbk * nbk, 3, c, out3 + c);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Gershgorin bound: column j sums |s_ij + [i==j] mu| over i = 0..n-1 in order.
// For an exactly symmetric s this is the row sum taken left to right.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_colsum(const double *__restrict__ s, int64_t n, int64_t ld, double mu,
                                                double *__restrict__ colsum) {
    const int64_t j = (int64_t)blockIdx.x * 64 + threadIdx.x;
    if (j >= n) return;
    // The sum stays strictly sequential in i; the loads of a group of U rows
    // are issued together so that enough memory requests are in flight.
    constexpr int U = 16;
    double acc = 0.0;
    int64_t i = 0;
    for (; i + U <= n; i += U) {
        double v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = s[(i + u) * ld + j];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            double x = v[u];
            if (i + u == j) x = x + mu;
            acc += fabs(x);
        }
    }
    for (; i < n; ++i) {
        double x = s[i * ld + j];
        if (i == j) x = x + mu;
        acc += fabs(x);
    }
    colsum[j] = acc;
}

hipError_t launch_colsum_max(const double *s, int64_t n, int64_t ld, double mu, double *colsum, double *out1,
                             hipStream_t st) {
    hipLaunchKernelGGL(k_colsum, dim3((unsigned)((n + 63) / 64)), dim3(64), 0, st, s, n, ld, mu, colsum);
    hipLaunchKernelGGL(k_reduce_max, dim3(1), dim3(1024), 0, st, colsum, n, 1, 0, out1);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Ingest: s' = (s + mu I)/c into tile-major storage of type T, zero padded,
// with each tile's squared norm taken of the stored values.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_ingest(const double *__restrict__ s, int64_t ld, double mu, double c,
                                                 Geom g, T *__restrict__ tiles, double *__restrict__ qleaf) {
    __shared__ double sh[4];
    const int t = blockIdx.x;
    const int i = t / g.nb, k = t % g.nb;
    const int b = g.b;
    T *dst = tiles + (int64_t)t * b * b;
    double q = 0.0;
    for (int e = threadIdx.x; e < b * b; e += 256) {
        const int r = e / b, cc = e % b;
        const int64_t gi = (int64_t)i * b + r, gj = (int64_t)k * b + cc;
        double v = 0.0;
        if (gi < g.n && gj < g.n) {
            v = s[gi * ld + gj];
            if (gi == gj) v = v + mu;
            v = v / c;
        }
        const T tv = (T)v;
        dst[e] = tv;
        const double dv = (double)tv;
        q += dv * dv;
    }
    q = block_sum<256>(q, sh);
    if (threadIdx.x == 0) qleaf[(int64_t)i * g.P + k] = q;
}

// Leaf squared norms of a row-major FP64 matrix read once, with no tile copy
// (the norm pass of spamm_norms): one workgroup per leaf, its loads issued
// together before the sums.
__global__ __launch_bounds__(256) void k_leaf_norms(const double *__restrict__ s, int64_t ld, Geom g,
                                                    double *__restrict__ qleaf) {
    __shared__ double sh[4];
    const int t = blockIdx.x;
    const int i = t / g.nb, k = t % g.nb;
    const int b = g.b, per = b * b / 256;  // 16, 4 or 1 elements per thread
    double v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
        v[u] = 0.0;
        if (u < per) {
            const int e = threadIdx.x + u * 256, r = e / b, cc = e % b;
            const int64_t gi = (int64_t)i * b + r, gj = (int64_t)k * b + cc;
            if (gi < g.n && gj < g.n) v[u] = s[gi * ld + gj];
        }
    }
    double q = 0.0;
#pragma unroll
    for (int u = 0; u < 16; ++u) q += v[u] * v[u];
    q = block_sum<256>(q, sh);
    if (threadIdx.x == 0) qleaf[(int64_t)i * g.P + k] = q;
}

hipError_t launch_leaf_norms(const double *s, int64_t ld, const Geom &g, double *qleaf, hipStream_t st) {
    hipLaunchKernelGGL(k_leaf_norms, dim3((unsigned)g.nb * g.nb), dim3(256), 0, st, s, ld, g, qleaf);
    return hipGetLastError();
}

template <typename T>
__global__ __launch_bounds__(256) void k_identity(Geom g, T *__restrict__ tiles, double *__restrict__ qleaf) {
    const int t = blockIdx.x;
    const int i = t / g.nb, k = t % g.nb;
    const int b = g.b;
    T *dst = tiles + (int64_t)t * b * b;
    for (int e = threadIdx.x; e < b * b; e += 256) {
        const int r = e / b, cc = e % b;
        const int64_t gi = (int64_t)i * b + r, gj = (int64_t)k * b + cc;
        dst[e] = (T)((gi == gj && gi < g.n) ? 1.0 : 0.0);
    }
    if (threadIdx.x == 0) {
        int64_t ones = 0;
        if (i == k) {
            const int64_t lo = (int64_t)i * b, hi = lo + b < g.n ? lo + b : g.n;
            ones = hi > lo ? hi - lo : 0;
        }
        qleaf[(int64_t)i * g.P + k] = (double)ones;
    }
}

hipError_t launch_ingest(int prec, const double *s, int64_t ld, double mu, double c, const Geom &g, void *tiles,
                         double *qleaf, hipStream_t st) {
    const unsigned nt = (unsigned)g.nb * g.nb;
    if (prec == P_F64)
        hipLaunchKernelGGL(k_ingest<double>, dim3(nt), dim3(256), 0, st, s, ld, mu, c, g, (double *)tiles, qleaf);
    else
        hipLaunchKernelGGL(k_ingest<float>, dim3(nt), dim3(256), 0, st, s, ld, mu, c, g, (float *)tiles, qleaf);
    return hipGetLastError();
}

hipError_t launch_identity(int prec, const Geom &g, void *tiles, double *qleaf, hipStream_t st) {
    const unsigned nt = (unsigned)g.nb * g.nb;
    if (prec == P_F64)
        hipLaunchKernelGGL(k_identity<double>, dim3(nt), dim3(256), 0, st, g, (double *)tiles, qleaf);
    else
        hipLaunchKernelGGL(k_identity<float>, dim3(nt), dim3(256), 0, st, g, (float *)tiles, qleaf);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Norm pyramid: a block reduces an R x R region (R = min(S, 32)) of the level
// of side S through up to five parent levels, each parent's squared norm
// being (q00 + q01) + (q10 + q11).  On the leaf level (leaf != 0) it also
// writes the leaf norms sqrt(q) of the real blocks, which the cull reads.
// ---------------------------------------------------------------------------
__device__ void pyramid_region(double *q, double *nrm, int P, int S, int nb, int leaf, int region, double *buf) {
    const int R = S < 32 ? S : 32;
    const int G = S / R;  // regions per side
    const int gy = region / G, gx = region % G;
    const double *lvl = q + dev_level_off(P, S);
    for (int e = threadIdx.x; e < R * R; e += blockDim.x) {
        const int r = e / R, c = e % R;
        const int64_t gr = (int64_t)gy * R + r, gc = (int64_t)gx * R + c;
        const double v = lvl[gr * S + gc];
        buf[e] = v;
        if (leaf && gr < nb && gc < nb) {
            const double nv = sqrt(v);
            nrm[gr * nb + gc] = nv;                          // (i, k) row-major
            nrm[(int64_t)nb * nb + gc * nb + gr] = nv;       // transposed copy for B-side reads
        }
    }
    __syncthreads();
    int s = R;
    int Scur = S;
    while (s > 1) {
        const int h = s / 2;
        double v = 0.0;
        const int e = threadIdx.x;
        if (e < h * h) {
            const int pr = e / h, pc = e % h;
            const double q00 = buf[(2 * pr) * s + 2 * pc], q01 = buf[(2 * pr) * s + 2 * pc + 1];
            const double q10 = buf[(2 * pr + 1) * s + 2 * pc], q11 = buf[(2 * pr + 1) * s + 2 * pc + 1];
            v = (q00 + q01) + (q10 + q11);
        }
        __syncthreads();
        const int Spar = Scur / 2;
        if (e < h * h) {
            buf[e] = v;
            const int pr = e / h, pc = e % h;
            const int64_t gr = (int64_t)gy * h + pr, gc = (int64_t)gx * h + pc;
            q[dev_level_off(P, Spar) + gr * Spar + gc] = v;
        }
        __syncthreads();
        s = h;
        Scur = Spar;
    }
}

__global__ __launch_bounds__(256) void k_pyramid(double *q0, double *nrm0, double *q1, double *nrm1, int P, int S,
                                                 int nb, int leaf) {
    __shared__ double buf[32 * 32];
    if (blockIdx.y == 0)
        pyramid_region(q0, nrm0, P, S, nb, leaf, blockIdx.x, buf);
    else
        pyramid_region(q1, nrm1, P, S, nb, leaf, blockIdx.x, buf);
}

hipError_t launch_pyramid(const Geom &g, double *q0, double *nrm0, double *q1, double *nrm1, int nops,
                          hipStream_t st) {
    int S = g.P;
    int leaf = 1;
    while (true) {
        const int R = S < 32 ? S : 32;
        const int G = S / R;
        hipLaunchKernelGGL(k_pyramid, dim3(G * G, nops), dim3(256), 0, st, q0, nrm0, q1, nrm1, g.P, S, g.nb, leaf);
        leaf = 0;
        if (G == 1) break;
        S = G;
    }
    return hipGetLastError();
}

// Pyramid of each running product's C: pass 1 on the leaf level, pass 2 (one
// block per product with P > 32) from level P/32 to the root.
__global__ __launch_bounds__(256) void k_pyramid_tab1(const ProdDesc *__restrict__ prods,
                                                      const int32_t *__restrict__ pre, int nprod) {
    __shared__ double buf[32 * 32];
    const int p = find_slot(pre, nprod, blockIdx.x);
    const ProdDesc &d = prods[p];
    if (!prod_running(d)) return;
    const int par = prod_parity(d);
    pyramid_region(d.qC[par], d.nrmC[par], d.P, d.P, d.nb, 1, blockIdx.x - pre[p], buf);
}

__global__ __launch_bounds__(256) void k_pyramid_tab2(const ProdDesc *__restrict__ prods,
                                                      const int32_t *__restrict__ pre, int nprod) {
    __shared__ double buf[32 * 32];
    const int p = find_slot(pre, nprod, blockIdx.x);
    const ProdDesc &d = prods[p];
    if (!prod_running(d)) return;
    const int par = prod_parity(d);
    pyramid_region(d.qC[par], d.nrmC[par], d.P, d.P / 32, d.nb, 0, 0, buf);
}

hipError_t launch_pyramid_tab(const ProdTable &t, hipStream_t st) {
    hipLaunchKernelGGL(k_pyramid_tab1, dim3(t.total_pyr), dim3(256), 0, st, t.prods, t.pyr_pre, t.nprod);
    if (t.total_pyr2 > 0)
        hipLaunchKernelGGL(k_pyramid_tab2, dim3(t.total_pyr2), dim3(256), 0, st, t.prods, t.pyr2_pre, t.nprod);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Cull: for output tile (i,j) keep every k with ||A_ik|| ||B_kj|| >= thr,
// thr = tau * (||A|| * ||B||), in increasing k.  Flat enumeration: since a
// parent's squared norm is a sum of non-negative children, every ancestor
// triple of a kept leaf triple is kept, so this equals the recursive set.
// One wave per output tile, or per block of CULL_RI x CULL_J tiles for large
// products; for each tile lane l tests k = kb + l, a ballot gives the kept k
// of the group of 64 and each kept lane writes its k at its rank.  Rows of A's leaf norms and columns of B's
// (from the transposed copy) are read coalesced.
// ---------------------------------------------------------------------------
// Cull of tile t of a running product by one wave (lane = lane index);
// returns the count, and the first two kept k in k0, k1 (-1 when absent).
// The norms of CULL_TU groups of 64 k are loaded before any of their
// compares and list stores, so a wave waits one round trip per 64*CULL_TU k
// rather than one per group (the stores would order later loads behind them).
constexpr int CULL_TU = 4;
__device__ inline int cull_tile(const ProdDesc &d, int t, int lane, int &k0, int &k1) {
    const int par = prod_parity(d);
    const int nb = d.nb;
    const int i = t / nb, j = t % nb;
    const double thr = d.tau * (sqrt(*d.rootA[par]) * sqrt(*d.rootB[par]));
    const double *na = d.nrmA[par] + (int64_t)i * nb;
    const double *nbt = d.nrmB[par] + (int64_t)nb * nb + (int64_t)j * nb;  // ||B_kj|| at nbt[k]
    int32_t *out = d.kidx + (int64_t)t * nb;
    int base = 0;
    k0 = k1 = -1;
    for (int kc = 0; kc < nb; kc += 64 * CULL_TU) {
        double pa[CULL_TU], pb[CULL_TU];
#pragma unroll
        for (int u = 0; u < CULL_TU; ++u) {
            const int k = kc + 64 * u + lane;
            pa[u] = k < nb ? na[k] : 0.0;
            pb[u] = k < nb ? nbt[k] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < CULL_TU; ++u) {
            const int kb = kc + 64 * u;
            if (kb >= nb) break;  // wave-uniform
            const int k = kb + lane;
            const bool keep = k < nb && !(pa[u] * pb[u] < thr);
            const unsigned long long mask = __ballot(keep);
            if (keep) out[base + __popcll(mask & ((1ull << lane) - 1ull))] = k;
            if (base < 2 && mask) {  // wave-uniform
                unsigned long long m = mask;
                int f = base;
                while (f < 2 && m) {
                    const int kk = kb + __ffsll((long long)m) - 1;
                    if (f == 0) k0 = kk; else k1 = kk;
                    m &= m - 1ull;
                    ++f;
                }
            }
            base += __popcll(mask);
        }
    }
    return base;
}

__global__ __launch_bounds__(256) void k_cull_tab(const ProdDesc *__restrict__ prods,
                                                  const int32_t *__restrict__ pre, int nprod) {
    const int p = find_slot(pre, nprod, blockIdx.x);
    const ProdDesc &d = prods[p];
    if (!prod_running(d)) return;
    const int t = (blockIdx.x - pre[p]) * 4 + (threadIdx.x >> 6);
    if (t >= d.nb * d.nb) return;
    const int lane = threadIdx.x & 63;
    int k0, k1;
    const int cnt = cull_tile(d, t, lane, k0, k1);
    if (lane == 0) d.cnt[t] = cnt;
}

template <typename T>
using gptr = T __attribute__((address_space(1))) *;

// Cull of a block of tiles (rows i0..i1-1, at most CULL_RI; columns
// j0..j1-1) by one wave, for nb <= 64 * CULL_U: the leaf norms of the block's
// rows of A stay in registers and B's columns come CULL_JG at a time, all
// their loads issued together (the first group's with A's), so a wave waits
// one memory round trip per CULL_JG columns and reads each of A's rows once
// for CULL_J tiles.  Lists, counts and order are those of cull_tile.
constexpr int CULL_U = 8, CULL_JG = 4;
__device__ inline void cull_block_regs(const ProdDesc &d, int i0, int i1, int j0, int j1, int lane) {
    const int par = prod_parity(d);
    const int nb = d.nb;
    const double thr = d.tau * (sqrt(*d.rootA[par]) * sqrt(*d.rootB[par]));
    const gptr<const double> nA = (gptr<const double>)d.nrmA[par];
    const gptr<const double> nBt = (gptr<const double>)(d.nrmB[par] + (int64_t)nb * nb);  // ||B_kj|| at [j*nb + k]
    const gptr<int32_t> kidx = (gptr<int32_t>)d.kidx;
    const gptr<int32_t> cnt = (gptr<int32_t>)d.cnt;
    double pa[CULL_RI][CULL_U], b[CULL_JG][CULL_U];
    auto load_cols = [&](int jg) {
#pragma unroll
        for (int c = 0; c < CULL_JG; ++c) {
            if (jg + c >= j1) break;  // wave-uniform
#pragma unroll
            for (int u = 0; u < CULL_U; ++u) {
                const int k = 64 * u + lane;
                b[c][u] = k < nb ? nBt[(int64_t)(jg + c) * nb + k] : 0.0;
            }
        }
    };
#pragma unroll
    for (int r = 0; r < CULL_RI; ++r) {
        if (i0 + r >= i1) break;  // wave-uniform
#pragma unroll
        for (int u = 0; u < CULL_U; ++u) {
            const int k = 64 * u + lane;
            pa[r][u] = k < nb ? nA[(int64_t)(i0 + r) * nb + k] : 0.0;
        }
    }
    load_cols(j0);
    unsigned long long inb[CULL_U];  // lanes whose k = 64u + lane < nb
#pragma unroll
    for (int u = 0; u < CULL_U; ++u) inb[u] = __builtin_amdgcn_ballot_w64(64 * u + lane < nb);
    for (int jg = j0; jg < j1; jg += CULL_JG) {
#pragma unroll
        for (int c = 0; c < CULL_JG; ++c) {
            const int j = jg + c;
            if (j >= j1) break;  // wave-uniform
#pragma unroll
            for (int r = 0; r < CULL_RI; ++r) {
                if (i0 + r >= i1) break;  // wave-uniform
                const int t = __builtin_amdgcn_readfirstlane((i0 + r) * nb + j);
                const gptr<int32_t> out = kidx + (int64_t)t * nb;
                int base = 0;
#pragma unroll
                for (int u = 0; u < CULL_U; ++u) {
                    if (64 * u >= nb) break;  // wave-uniform
                    const int k = 64 * u + lane;
                    const bool pass = !(pa[r][u] * b[c][u] < thr);
                    const bool keep = k < nb && pass;
                    // the ballot of the compare alone, masked by the lanes of k < nb
                    const unsigned long long mask = __builtin_amdgcn_ballot_w64(pass) & inb[u];
                    // rank of this lane among the kept lanes below it
                    const unsigned rank = __builtin_amdgcn_mbcnt_hi((unsigned)(mask >> 32),
                                                                    __builtin_amdgcn_mbcnt_lo((unsigned)mask, 0u));
                    if (keep) out[base + (int)rank] = k;
                    base += __popcll(mask);
                }
                if (lane == 0) cnt[t] = base;
            }
        }
        if (jg + CULL_JG < j1) load_cols(jg + CULL_JG);
    }
}

__global__ __launch_bounds__(256) void k_cull_blk(const ProdDesc *__restrict__ prods,
                                                  const int32_t *__restrict__ pre, int nprod) {
    const int p = find_slot(pre, nprod, blockIdx.x);
    const ProdDesc &d = prods[p];
    if (!prod_running(d)) return;
    const int nb = d.nb;
    const int wv = (blockIdx.x - pre[p]) * 4 + (threadIdx.x >> 6);
    if (wv >= cull_blk_waves(nb)) return;  // whole waves
    const int lane = threadIdx.x & 63;
    const int nbj = (nb + CULL_J - 1) / CULL_J;
    const int i0 = (wv / nbj) * CULL_RI, j0 = (wv % nbj) * CULL_J;
    const int i1 = min(i0 + CULL_RI, nb), j1 = min(j0 + CULL_J, nb);
    if (nb <= 64 * CULL_U) {
        cull_block_regs(d, i0, i1, j0, j1, lane);
        return;
    }
    for (int i = i0; i < i1; ++i)
        for (int j = j0; j < j1; ++j) {
            int k0, k1;
            const int t = i * nb + j;
            const int c = cull_tile(d, t, lane, k0, k1);
            if (lane == 0) d.cnt[t] = c;
        }
}

hipError_t launch_cull_tab(const ProdTable &t, hipStream_t st) {
    if (t.total_cull > 0)
        hipLaunchKernelGGL(k_cull_tab, dim3(t.total_cull), dim3(256), 0, st, t.prods, t.cull_pre, t.nprod);
    if (t.total_cullb > 0)
        hipLaunchKernelGGL(k_cull_blk, dim3(t.total_cullb), dim3(256), 0, st, t.prods, t.cullb_pre, t.nprod);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Longest-first work list: the tiles of all running products, ordered by
// decreasing retained count, so the heaviest tiles are dispatched first and
// a launch ends on short tiles.  Order inside a count bucket is whatever the
// atomics give; no product depends on it.  Entries are global tile ids
// tile_pre[p] + (i*nb + j); the base order is Morton within each product.
// Small tables: one workgroup, one bucket per count.  Large tables: NBUCKET
// coarse buckets (count capped), per-workgroup histograms, a scan, a scatter.
// ---------------------------------------------------------------------------
// With quad set, an item is a quad of tiles, named by its first tile (both
// indices even; the other tiles return -1), and its count is the largest of
// its tiles' counts.  Going through the tiles in Morton order visits the quads
// in Morton order of the quad grid.
__device__ inline int item_count(const ProdDesc *prods, const int32_t *tile_pre, const int32_t *morton, int nprod,
                                 int g, int quad, int &p, int &t) {
    p = find_slot(tile_pre, nprod, g);
    const ProdDesc &d = prods[p];
    if (!prod_running(d)) return -1;
    t = morton[g];
    if (!quad) return d.cnt[t];
    const int nb = d.nb, i = t / nb, j = t % nb;
    if ((i | j) & 1) return -1;
    int c = d.cnt[t];
    if (j + 1 < nb) c = max(c, d.cnt[t + 1]);
    if (i + 1 < nb) {
        c = max(c, d.cnt[t + nb]);
        if (j + 1 < nb) c = max(c, d.cnt[t + nb + 1]);
    }
    return c;
}

// Job record of tile t of product p for element size esz (pointers resolved
// for the product's current parity).
// Job record of tile t of product d at parity par, with the tile's first two
// retained k given.
__device__ inline Job make_job_kp(const ProdDesc &d, int par, int t, int cnt, int b, int esz, int k0, int k1) {
    const int nb = d.nb, i = t / nb, j = t % nb;
    const int64_t ts = (int64_t)b * b * esz;
    Job J;
    J.a_row = (const char *)d.A[par] + (int64_t)i * nb * ts;
    J.b_col = (const char *)d.B[par] + (int64_t)j * ts;
    J.c = (char *)d.C[par] + (int64_t)t * ts;
    J.qc = d.qC[par] + (int64_t)i * d.P + j;
    J.part = d.part ? d.part + 2 * (int64_t)t : nullptr;
    J.list = d.kidx + (int64_t)t * nb;
    J.n = d.n;
    J.nb = nb;
    J.cnt = cnt;
    J.i = i;
    J.j = j;
    J.fused_map = d.fused_map;
    J.k0 = cnt > 0 ? k0 : 0;
    J.k1 = cnt > 1 ? k1 : 0;
    return J;
}

// The same at the product's current parity, with the first two retained k
// read from the tile's list.
__device__ inline Job make_job(const ProdDesc &d, int t, int cnt, int b, int esz) {
    const int32_t *list = d.kidx + (int64_t)t * d.nb;
    return make_job_kp(d, prod_parity(d), t, cnt, b, esz, cnt > 0 ? list[0] : 0, cnt > 1 ? list[1] : 0);
}

// Slot of entry idx of a longest-first list of `count` entries after the XCD
// runs: each window of 8*run entries is transposed so that entries
// q*run .. q*run+run-1 of the window land on workgroups that run on XCD q
// (workgroup w runs on XCD w mod 8); the partial last window keeps its order.
__device__ inline int xcd_slot(int idx, int count, int run) {
    if (run <= 1) return idx;
    const int W = 8 * run;
    if (idx >= count / W * W) return idx;
    const int q = idx % W;
    return idx - q + (q % run) * 8 + q / run;
}

// Small tables (<= PLAN_ITEMS * 1024 tiles, the tables without hist_blocks):
// every thread loads its items once, with independent loads, and keeps each
// item's count and tile id packed in one register for the histogram and the
// scatter.  That keeps the kernel under 48 registers, so its four waves per
// SIMD fit where a single leaf-product workgroup (160 registers a wave) has
// retired: on a GPU busy with other solves' leaf products the planner of a
// solve is placed as soon as one of their workgroups ends.
constexpr int PLAN_ITEMS = PLAN_SMALL_MAX / 1024;
static_assert(PLAN_SMALL_MAX < (1 << 16), "tile ids and counts are packed in 16 bits each");

__global__ __launch_bounds__(1024) void k_plan_small(const ProdDesc *__restrict__ prods,
                                                     const int32_t *__restrict__ tile_pre,
                                                     const int32_t *__restrict__ morton, int nprod, int max_nb,
                                                     int quad, int32_t *__restrict__ work,
                                                     int32_t *__restrict__ work_count) {
    extern __shared__ int hist[];  // max_nb + 1 bins
    const int total = tile_pre[nprod];
    for (int c = threadIdx.x; c <= max_nb; c += 1024) hist[c] = 0;
    unsigned it[PLAN_ITEMS];  // (count + 1) << 16 | tile id; 0 when the thread has no item there
#pragma unroll
    for (int q = 0; q < PLAN_ITEMS; ++q) {
        const int g = threadIdx.x + q * 1024;
        it[q] = 0u;
        if (g < total) {
            int p, t;
            const int c = item_count(prods, tile_pre, morton, nprod, g, quad, p, t);
            if (c >= 0) it[q] = ((unsigned)(c + 1) << 16) | (unsigned)(tile_pre[p] + t);
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < PLAN_ITEMS; ++q)
        if (it[q]) atomicAdd(&hist[(int)(it[q] >> 16) - 1], 1);
    __syncthreads();
    if (threadIdx.x == 0) {
        int run = 0;
        for (int c = max_nb; c >= 0; --c) {
            const int h = hist[c];
            hist[c] = run;
            run += h;
        }
        *work_count = run;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < PLAN_ITEMS; ++q)
        if (it[q]) work[atomicAdd(&hist[(int)(it[q] >> 16) - 1], 1)] = (int)(it[q] & 0xffffu);
}

__device__ inline int bucket_of(int c) { return c < NBUCKET - 1 ? c : NBUCKET - 1; }

// The large-table passes give each thread PLAN_HIST_ITEMS items whose count
// chains (Morton order, product state, count) are issued together, and read
// the table's prefix from LDS when it fits.
constexpr int PRE_LDS = 1024;

__global__ __launch_bounds__(256) void k_plan_hist(const ProdDesc *__restrict__ prods,
                                                   const int32_t *__restrict__ tile_pre,
                                                   const int32_t *__restrict__ morton, int nprod, int nblk,
                                                   int quad, int32_t *__restrict__ hist) {
    __shared__ int h[NBUCKET];
    __shared__ int s_pre[PRE_LDS + 1];
    const bool lds = nprod <= PRE_LDS;
    if (lds)
        for (int x = threadIdx.x; x <= nprod; x += 256) s_pre[x] = tile_pre[x];
    for (int b = threadIdx.x; b < NBUCKET; b += 256) h[b] = 0;
    __syncthreads();
    const int32_t *pre = lds ? s_pre : tile_pre;
    const int total = pre[nprod];
    const int chunk = (total + nblk - 1) / nblk;
    const int lo = blockIdx.x * chunk, hi = lo + chunk < total ? lo + chunk : total;
    for (int base = lo; base < hi; base += 256 * PLAN_HIST_ITEMS) {
        int c[PLAN_HIST_ITEMS];
#pragma unroll
        for (int q = 0; q < PLAN_HIST_ITEMS; ++q) {
            const int g = base + threadIdx.x + q * 256;
            int p, t;
            c[q] = g < hi ? item_count(prods, pre, morton, nprod, g, quad, p, t) : -1;
        }
#pragma unroll
        for (int q = 0; q < PLAN_HIST_ITEMS; ++q)
            if (c[q] >= 0) atomicAdd(&h[bucket_of(c[q])], 1);
    }
    __syncthreads();
    for (int b = threadIdx.x; b < NBUCKET; b += 256) hist[b * nblk + blockIdx.x] = h[b];
}

// Exclusive scan of hist in the order (bucket descending, block ascending).
__global__ __launch_bounds__(1024) void k_plan_scan(int32_t *__restrict__ hist, int nblk,
                                                    int32_t *__restrict__ work_count) {
    __shared__ int wsum[16];
    const int m = NBUCKET * nblk;
    const int per = (m + 1023) / 1024;
    const int lo = threadIdx.x * per, hi = lo + per < m ? lo + per : m;
    auto at = [&](int L) -> int32_t & {  // L-th entry in scan order
        const int b = NBUCKET - 1 - L / nblk, w = L % nblk;
        return hist[b * nblk + w];
    };
    int s = 0;
    for (int L = lo; L < hi; ++L) s += at(L);
    // exclusive prefix of the threads' sums: within each wave by shuffles,
    // then over the 16 wave totals
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int incl = s;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int v = __shfl_up(incl, off, 64);
        if (lane >= off) incl += v;
    }
    if (lane == 63) wsum[wv] = incl;
    __syncthreads();
    int run = incl - s;
    for (int x = 0; x < wv; ++x) run += wsum[x];
    if (threadIdx.x == 1023) *work_count = run + s;
    for (int L = lo; L < hi; ++L) {
        const int v = at(L);
        at(L) = run;
        run += v;
    }
}

__global__ __launch_bounds__(256) void k_plan_scatter(const ProdDesc *__restrict__ prods,
                                                      const int32_t *__restrict__ tile_pre,
                                                      const int32_t *__restrict__ morton, int nprod, int nblk,
                                                      int quad, const int32_t *__restrict__ hist,
                                                      int32_t *__restrict__ work) {
    __shared__ int cur[NBUCKET];
    __shared__ int s_pre[PRE_LDS + 1];
    const bool lds = nprod <= PRE_LDS;
    if (lds)
        for (int x = threadIdx.x; x <= nprod; x += 256) s_pre[x] = tile_pre[x];
    for (int q = threadIdx.x; q < NBUCKET; q += 256) cur[q] = hist[q * nblk + blockIdx.x];
    __syncthreads();
    const int32_t *pre = lds ? s_pre : tile_pre;
    const int total = pre[nprod];
    const int chunk = (total + nblk - 1) / nblk;
    const int lo = blockIdx.x * chunk, hi = lo + chunk < total ? lo + chunk : total;
    for (int base = lo; base < hi; base += 256 * PLAN_HIST_ITEMS) {
        int c[PLAN_HIST_ITEMS], id[PLAN_HIST_ITEMS];
#pragma unroll
        for (int q = 0; q < PLAN_HIST_ITEMS; ++q) {
            const int g = base + threadIdx.x + q * 256;
            int p = 0, t = 0;
            c[q] = g < hi ? item_count(prods, pre, morton, nprod, g, quad, p, t) : -1;
            id[q] = c[q] >= 0 ? pre[p] + t : 0;
        }
#pragma unroll
        for (int q = 0; q < PLAN_HIST_ITEMS; ++q)
            if (c[q] >= 0) work[atomicAdd(&cur[bucket_of(c[q])], 1)] = id[q];
    }
}

// Expands the sorted tile ids into job records, one thread per entry, at the
// slots of the XCD runs (xcd_slot): the window's order in time barely
// changes, and neighbouring tiles meet in one L2.  With quad set, entry w is
// a quad and gets the four records 4w .. 4w+3.
__global__ __launch_bounds__(256) void k_make_jobs(const ProdDesc *__restrict__ prods,
                                                   const int32_t *__restrict__ tile_pre, int nprod,
                                                   const int32_t *__restrict__ work,
                                                   const int32_t *__restrict__ work_count, int b, int esz, int run,
                                                   int quad, Job *__restrict__ jobs) {
    const int idx = blockIdx.x * 256 + threadIdx.x;
    const int count = *work_count;
    if (idx >= count) return;
    const int gid = work[idx];
    const int p = find_slot(tile_pre, nprod, gid);
    const int t = gid - tile_pre[p];
    const ProdDesc &d = prods[p];
    const int w = xcd_slot(idx, count, run);
    if (!quad) {
        jobs[w] = make_job(d, t, d.cnt[t], b, esz);
        return;
    }
    const int nb = d.nb, i = t / nb, j = t % nb;
    for (int q = 0; q < 4; ++q) {
        const int ti = i + (q >> 1), tj = j + (q & 1);
        Job J;
        if (ti < nb && tj < nb) {
            J = make_job(d, ti * nb + tj, d.cnt[ti * nb + tj], b, esz);
        } else {  // past the edge of an odd nb: no tile, never loaded or written
            J = make_job(d, t, 0, b, esz);
            J.cnt = -1;
        }
        jobs[4 * w + q] = J;
    }
}

// Tables of at most FRONT_MAX tiles and FRONT_PRODS products (launch-bound
// solves): cull, longest-first order and job records in one workgroup, one
// launch instead of three.  Such tables have nb <= 32, so their leaf norms
// fit in LDS: one round of parallel loads brings the table's prefix, every
// product's threshold, state and pointers, and both operands' leaf norms into
// LDS; the cull then reads LDS only, with 64/L tiles per wave (L lanes per
// tile, L the power of two >= the largest nb, lane = k).  The counts and
// first two retained k stay in LDS for the order and the job records.  The
// lists and counts written, and the order, are those of k_cull_tab and
// k_plan_small.
__global__ __launch_bounds__(1024) void k_front_small(const ProdDesc *__restrict__ prods,
                                                      const int32_t *__restrict__ tile_pre,
                                                      const int32_t *__restrict__ morton, int nprod, int max_nb,
                                                      int b, int esz, int run, Job *__restrict__ jobs,
                                                      int32_t *__restrict__ work_count) {
    __shared__ int s_pre[FRONT_PRODS + 1];
    __shared__ int s_par[FRONT_PRODS];  // parity, or -1 when the product is not running
    __shared__ int s_nbk[FRONT_PRODS];
    __shared__ double s_thr[FRONT_PRODS];
    __shared__ int32_t *s_kidx[FRONT_PRODS];
    __shared__ int32_t *s_cntp[FRONT_PRODS];
    __shared__ const double *s_nra[FRONT_PRODS], *s_nrb[FRONT_PRODS];  // leaf norms at the current parity
    __shared__ double s_na[FRONT_MAX], s_nb[FRONT_MAX];  // A's leaf norms, B's transposed, product q's at s_pre[q]
    __shared__ int s_cnt[FRONT_MAX], s_k0[FRONT_MAX], s_k1[FRONT_MAX];
    __shared__ int s_total;
    extern __shared__ int hist[];  // max_nb + 1 bins
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int ntile = tile_pre[nprod];
    const int mort = tid < ntile ? morton[tid] : 0;  // read now, used by the ordering
    for (int x = tid; x <= nprod; x += 1024) s_pre[x] = tile_pre[x];
    for (int c = tid; c <= max_nb; c += 1024) hist[c] = 0;
    for (int q = tid; q < nprod; q += 1024) {
        const ProdDesc &d = prods[q];
        const int par = prod_running(d) ? prod_parity(d) : -1;
        s_par[q] = par;
        s_nbk[q] = d.nb;
        s_kidx[q] = d.kidx;
        s_cntp[q] = d.cnt;
        if (par >= 0) {
            s_thr[q] = d.tau * (sqrt(*d.rootA[par]) * sqrt(*d.rootB[par]));
            s_nra[q] = d.nrmA[par];
            s_nrb[q] = d.nrmB[par] + (int64_t)d.nb * d.nb;
        }
    }
    __syncthreads();
    const int total = s_pre[nprod];
    for (int g = tid; g < total; g += 1024) {
        const int q = find_slot(s_pre, nprod, g);
        if (s_par[q] < 0) continue;
        const int x = g - s_pre[q];
        s_na[g] = s_nra[q][x];
        s_nb[g] = s_nrb[q][x];
    }
    __syncthreads();
    // cull: lane l tests k = l % L of tile l / L of the wave's group
    int L = 1;
    while (L < max_nb) L <<= 1;
    const int per = 64 / L, sub = lane / L, k = lane % L;
    const unsigned long long lmask = L == 64 ? ~0ull : ((1ull << L) - 1ull);
    for (int g0 = per * wv; g0 < total; g0 += 16 * per) {
        const int g = g0 + sub;
        int q = 0, nb = 1, t = 0;
        bool keep = false, live = false;
        if (g < total) {
            q = find_slot(s_pre, nprod, g);
            live = s_par[q] >= 0;
            if (live) {
                nb = s_nbk[q];
                t = g - s_pre[q];
                const int i = t / nb, j = t % nb;
                if (k < nb) {
                    const double prod = s_na[s_pre[q] + i * nb + k] * s_nb[s_pre[q] + j * nb + k];
                    keep = !(prod < s_thr[q]);
                }
            }
        }
        const unsigned long long mine = (__ballot(keep) >> (L * sub)) & lmask;
        if (keep) s_kidx[q][(int64_t)t * nb + __popcll(mine & ((1ull << k) - 1ull))] = k;
        if (g < total && k == 0) {
            int cnt = -1, k0 = -1, k1 = -1;
            if (live) {
                cnt = __popcll(mine);
                if (mine) {
                    k0 = __ffsll((long long)mine) - 1;
                    const unsigned long long rest = mine & (mine - 1ull);
                    if (rest) k1 = __ffsll((long long)rest) - 1;
                }
                s_cntp[q][t] = cnt;
            }
            s_cnt[g] = cnt;
            s_k0[g] = k0;
            s_k1[g] = k1;
        }
    }
    __syncthreads();
    // longest-first order over the items in Morton order, one item per thread
    int c = -1, gt = 0, q = 0, t = 0;
    if (tid < total) {
        q = find_slot(s_pre, nprod, tid);
        t = mort;
        gt = s_pre[q] + t;
        c = s_cnt[gt];
        if (c >= 0) atomicAdd(&hist[c], 1);
    }
    __syncthreads();
    if (tid == 0) {
        int r = 0;
        for (int x = max_nb; x >= 0; --x) {
            const int h = hist[x];
            hist[x] = r;
            r += h;
        }
        *work_count = r;
        s_total = r;
    }
    __syncthreads();
    if (c >= 0) {
        const int idx = atomicAdd(&hist[c], 1);
        jobs[xcd_slot(idx, s_total, run)] = make_job_kp(prods[q], s_par[q], t, c, b, esz, s_k0[gt], s_k1[gt]);
    }
}

bool front_small(const ProdTable &t, int leaf, int gprec) {
    return t.total_tiles <= FRONT_MAX && t.nprod <= FRONT_PRODS && !quad_tiles(gprec, leaf, t.total_tiles);
}

hipError_t launch_front_small(const ProdTable &t, int leaf, int gprec, hipStream_t st) {
    const int esz = gprec == P_F64 ? 8 : 4;
    const int run = is_bf16(gprec) ? BF3_XCD_RUN : 1;
    hipLaunchKernelGGL(k_front_small, dim3(1), dim3(1024), (t.max_nb + 1) * sizeof(int), st, t.prods, t.tile_pre,
                       t.morton, t.nprod, t.max_nb, leaf, esz, run, t.jobs, t.work_count);
    return hipGetLastError();
}

hipError_t launch_plan_tab(const ProdTable &t, int leaf, int gprec, hipStream_t st) {
    const int esz = gprec == P_F64 ? 8 : 4;
    const int quad = quad_tiles(gprec, leaf, t.total_tiles) ? 1 : 0;
    // FP64 products of large tables (beyond one-workgroup sorting) also run
    // in XCD runs: their operands stream from HBM, and neighbouring tiles of
    // a run share A rows and B columns in one L2
    const int run = is_bf16(gprec) ? (quad ? BF3_XCD_RUN / 4 : BF3_XCD_RUN)
                                   : (gprec == P_F64 && t.total_tiles > PLAN_SMALL_MAX ? BF3_XCD_RUN : 1);
    if (t.hist_blocks == 0) {
        hipLaunchKernelGGL(k_plan_small, dim3(1), dim3(1024), (t.max_nb + 1) * sizeof(int), st, t.prods, t.tile_pre,
                           t.morton, t.nprod, t.max_nb, quad, t.work, t.work_count);
    } else {
        hipLaunchKernelGGL(k_plan_hist, dim3(t.hist_blocks), dim3(256), 0, st, t.prods, t.tile_pre, t.morton,
                           t.nprod, t.hist_blocks, quad, t.hist);
        hipLaunchKernelGGL(k_plan_scan, dim3(1), dim3(1024), 0, st, t.hist, t.hist_blocks, t.work_count);
        hipLaunchKernelGGL(k_plan_scatter, dim3(t.hist_blocks), dim3(256), 0, st, t.prods, t.tile_pre, t.morton,
                           t.nprod, t.hist_blocks, quad, t.hist, t.work);
    }
    const int items = quad ? t.total_quads : t.total_tiles;
    hipLaunchKernelGGL(k_make_jobs, dim3((items + 255) / 256), dim3(256), 0, st, t.prods, t.tile_pre, t.nprod,
                       t.work, t.work_count, leaf, esz, run, quad, t.jobs);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Newton-Schulz control, one workgroup per solve: r_k = sqrt(sum of per-tile
// (I-x)^2), t_k = (n - trace)/n and the retained-triple counts, summed in a
// fixed order, then the stop tests in the order: r_k < tol (OK); r_k not
// finite or > 10 max(r_0, sqrt(n)) (diverged); two consecutive
// r_k >= 0.99 r_best, r_best = min(r_0..r_{k-1}), while r_best < 1/2 or
// n |t_k| < 1/2 (stagnated, opt-in); k == maxit (not converged).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void k_ns_decide(const SolveDesc *__restrict__ solves,
                                                    const ProdDesc *__restrict__ xpyr) {
    __shared__ double sh[16];
    __shared__ double buf[32 * 32];
    __shared__ int s_run;
    const SolveDesc &sd = solves[blockIdx.x];
    SolveState *st = sd.state;
    if (st->status != ST_RUNNING) return;
    const int k = st->k;
    const int64_t ntiles = (int64_t)sd.nb * sd.nb;
    // the y product of the single instance precedes x_k; the dual instance's
    // y and z products, and the single instance's z product, belong to k-1
    const bool have_y = sd.single || k > 0, have_z = k > 0;
    double r2 = 0.0, tr = 0.0, cx = 0.0, cy = 0.0, cz = 0.0;
    for (int64_t e = threadIdx.x; e < ntiles; e += 1024) {
        r2 += sd.part[2 * e];
        tr += sd.part[2 * e + 1];
        cx += (double)sd.cnt_x[e];
        if (have_y) cy += (double)sd.cnt_y[e];
        if (have_z) cz += (double)sd.cnt_z[e];
    }
    r2 = block_sum<1024>(r2, sh);
    tr = block_sum<1024>(tr, sh);
    cx = block_sum<1024>(cx, sh);
    cy = block_sum<1024>(cy, sh);
    cz = block_sum<1024>(cz, sh);
    if (threadIdx.x == 0) {
        const double r = sqrt(r2);
        const double tk = ((double)sd.n - tr) / (double)sd.n;
        sd.hist_r[k] = r;
        sd.hist_t[k] = tk;
        sd.hist_nR[3 * k] = (int64_t)cx;
        if (sd.single) {
            sd.hist_nR[3 * k + 1] = (int64_t)cy;
            if (k > 0) sd.hist_nR[3 * (k - 1) + 2] = (int64_t)cz;
        } else if (k > 0) {
            sd.hist_nR[3 * (k - 1) + 1] = (int64_t)cy;
            sd.hist_nR[3 * (k - 1) + 2] = (int64_t)cz;
        }
        st->triples += (int64_t)cx + (int64_t)cy + (int64_t)cz;
        st->r = r;
        st->t = tk;
        if (k == 0) st->r0 = r;
        int status = ST_RUNNING;
        if (r < sd.tol) {
            status = 0;  // SPAMM_OK
        } else if (!isfinite(r) || r > 10.0 * fmax(st->r0, sqrt((double)sd.n))) {
            status = -3;  // SPAMM_EDIVERGED
        } else {
            if (sd.stagnation_stop && k > 0) {
                // progress against the best residual so far, counted only once
                // every eigenvalue of an exact iterate is within 1/2 of 1 (best r
                // below 1/2, or n |t_k| below 1/2 since exact iterates keep x in
                // (0, 1]): there an exact update shrinks r by more than 2x, so a
                // step gaining under 1% is the floor
                const bool settled = st->r_prev < 0.5 || fabs(tk) * (double)sd.n < 0.5;
                st->nondecrease = (settled && r >= 0.99 * st->r_prev) ? st->nondecrease + 1 : 0;
                if (st->nondecrease >= 2) status = 2;  // SPAMM_STAGNATED
            }
            if (status == ST_RUNNING) {
                if (k == 0 || r < st->r_prev) st->r_prev = r;  // best residual so far
                if (k == sd.maxit) status = 1;  // SPAMM_NOT_CONVERGED
            }
        }
        // damped map (Sec. 4.2): scaling alpha(t) and stabilisation eps(t) of the
        // trace error, both switched off once t_k < 0.1 (the sigmoids never reach
        // 1 and 0 exactly; eps(0) alone would hold r above sqrt(n) 1.7e-11)
        double alpha = 1.0, eps = 0.0;
        if (sd.damped && tk >= 0.1) {
            alpha = 1.0 + 1.85 / (1.0 + exp(-50.0 * (tk - 0.35)));
            eps = 0.1 / (1.0 + exp(-75.0 * (tk - 0.30)));
        }
        st->alpha = alpha;
        st->eps = eps;
        st->status = status;
        s_run = status == ST_RUNNING;
    }
    // the x product's pyramid (P <= 32: one region) for a solve still running
    if (xpyr == nullptr) return;
    __syncthreads();
    if (!s_run) return;
    const ProdDesc &d = xpyr[blockIdx.x];
    const int par = prod_parity(d);
    pyramid_region(d.qC[par], d.nrmC[par], d.P, d.P, d.nb, 1, 0, buf);
}

// Tile transpose, one workgroup per output tile, through LDS (b <= 64).
template <typename T>
__global__ __launch_bounds__(256) void k_transpose_tab(const ProdDesc *__restrict__ prods,
                                                       const int32_t *__restrict__ pre, int nprod, int b) {
    __shared__ T buf[64][65];
    __shared__ double sh[4];
    const int p = find_slot(pre, nprod, blockIdx.x);
    const ProdDesc &d = prods[p];
    if (!prod_running(d)) return;
    const int par = prod_parity(d);
    const int nb = d.nb, t = blockIdx.x - pre[p], i = t / nb, j = t % nb;
    const T *src = (const T *)d.A[par] + ((int64_t)j * nb + i) * b * b;
    T *dst = (T *)d.C[par] + (int64_t)t * b * b;
    for (int e = threadIdx.x; e < b * b; e += 256) buf[e / b][e % b] = src[e];
    __syncthreads();
    double q = 0.0;
    for (int e = threadIdx.x; e < b * b; e += 256) {
        const T v = buf[e % b][e / b];
        dst[e] = v;
        q += (double)v * (double)v;
    }
    q = block_sum<256>(q, sh);
    if (threadIdx.x == 0) d.qC[par][(int64_t)i * d.P + j] = q;
}

hipError_t launch_transpose_tab(int prec, const ProdTable &t, int leaf, hipStream_t st) {
    if (prec == P_F64)
        hipLaunchKernelGGL(k_transpose_tab<double>, dim3(t.total_tiles), dim3(256), 0, st, t.prods, t.tile_pre,
                           t.nprod, leaf);
    else
        hipLaunchKernelGGL(k_transpose_tab<float>, dim3(t.total_tiles), dim3(256), 0, st, t.prods, t.tile_pre,
                           t.nprod, leaf);
    return hipGetLastError();
}

// Damped map, one workgroup per tile of the x products of a table, in place.
// An off-diagonal tile with no retained triple holds exact zeros and maps to
// zeros (its squared norm, 0, is already written), so it is skipped.
template <typename T>
__global__ __launch_bounds__(256) void k_ns_map(const ProdDesc *__restrict__ prods, const int32_t *__restrict__ pre,
                                                int nprod, int b) {
    __shared__ double sh[4];
    const int g = blockIdx.x;
    const int p = find_slot(pre, nprod, g);
    const ProdDesc &d = prods[p];
    if (d.part == nullptr || d.fused_map || !prod_running(d)) return;
    const int par = prod_parity(d);
    const int nb = d.nb, t = g - pre[p], i = t / nb, j = t % nb;
    if (i != j && d.cnt[t] == 0) return;
    const double alpha = d.state->alpha, eps = d.state->eps;
    const bool plain = (alpha == 1.0 && eps == 0.0);
    const double hs = 0.5 * sqrt(alpha), om = 1.0 - 2.0 * eps;
    T *tile = (T *)d.C[par] + (int64_t)t * b * b;
    double q = 0.0;
    for (int e = threadIdx.x; e < b * b; e += 256) {
        const int r = e / b, c = e % b;
        const int64_t gi = (int64_t)i * b + r, gj = (int64_t)j * b + c;
        const bool diag = (gi == gj) && (gi < d.n);
        const double x = (double)tile[e];
        const double h = plain ? (diag ? 1.5 : 0.0) - 0.5 * x
                               : hs * ((diag ? 3.0 : 0.0) - alpha * ((diag ? eps : 0.0) + om * x));
        const T out = (T)h;
        tile[e] = out;
        q += (double)out * (double)out;
    }
    q = block_sum<256>(q, sh);
    if (threadIdx.x == 0) d.qC[par][(int64_t)i * d.P + j] = q;
}

hipError_t launch_ns_map(int prec, const ProdTable &t, int leaf, hipStream_t st) {
    if (prec == P_F64)
        hipLaunchKernelGGL(k_ns_map<double>, dim3(t.total_tiles), dim3(256), 0, st, t.prods, t.tile_pre, t.nprod,
                           leaf);
    else
        hipLaunchKernelGGL(k_ns_map<float>, dim3(t.total_tiles), dim3(256), 0, st, t.prods, t.tile_pre, t.nprod,
                           leaf);
    return hipGetLastError();
}

__global__ __launch_bounds__(64) void k_ns_advance(const SolveDesc *__restrict__ solves, int nsolve) {
    const int i = blockIdx.x * 64 + threadIdx.x;
    if (i >= nsolve) return;
    SolveState *st = solves[i].state;
    if (st->status != ST_RUNNING) return;
    st->parity ^= 1;
    st->k += 1;
}

// The update products' pyramids built by the block of their solve, which
// then advances it: one launch in place of k_pyramid_tab1 and k_ns_advance,
// for tables whose every pyramid is one region (P <= 32).  Products
// per*s .. per*s+per-1 of the table belong to solve s.
__global__ __launch_bounds__(256) void k_pyramid_advance(const SolveDesc *__restrict__ solves,
                                                         const ProdDesc *__restrict__ prods, int per) {
    __shared__ double buf[32 * 32];
    const int s = blockIdx.x;
    SolveState *st = solves[s].state;
    if (st->status != ST_RUNNING) return;  // the same for every thread of the block
    for (int q = 0; q < per; ++q) {
        const ProdDesc &d = prods[s * per + q];
        const int par = prod_parity(d);
        pyramid_region(d.qC[par], d.nrmC[par], d.P, d.P, d.nb, 1, 0, buf);
        __syncthreads();
    }
    if (threadIdx.x == 0) {  // every thread has read the parity
        st->parity ^= 1;
        st->k += 1;
    }
}

__global__ __launch_bounds__(64) void k_gather_states(const SolveDesc *__restrict__ solves, int nsolve,
                                                      SolveState *__restrict__ out) {
    const int i = blockIdx.x * 64 + threadIdx.x;
    if (i < nsolve) out[i] = *solves[i].state;
}

hipError_t launch_ns_decide(const SolveDesc *solves, int nsolve, const ProdDesc *xpyr, hipStream_t st) {
    hipLaunchKernelGGL(k_ns_decide, dim3(nsolve), dim3(1024), 0, st, solves, xpyr);
    return hipGetLastError();
}

bool decide_builds_pyramid(const ProdTable &tx) { return tx.total_pyr == tx.nprod && tx.total_pyr2 == 0; }

hipError_t launch_ns_advance(const SolveDesc *solves, int nsolve, hipStream_t st) {
    hipLaunchKernelGGL(k_ns_advance, dim3((nsolve + 63) / 64), dim3(64), 0, st, solves, nsolve);
    return hipGetLastError();
}

hipError_t launch_pyramid_advance(const SolveDesc *solves, int nsolve, const ProdTable &t, int per,
                                  hipStream_t st) {
    hipLaunchKernelGGL(k_pyramid_advance, dim3(nsolve), dim3(256), 0, st, solves, t.prods, per);
    return hipGetLastError();
}

hipError_t launch_gather_states(const SolveDesc *solves, int nsolve, SolveState *out, hipStream_t st) {
    hipLaunchKernelGGL(k_gather_states, dim3((nsolve + 63) / 64), dim3(64), 0, st, solves, nsolve, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Egress: tile-major T -> row-major FP64, times or divided by `scale`.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_egress(const T *__restrict__ tiles, Geom g, double *__restrict__ out,
                                                 int64_t ld, double scale, int divide) {
    const int t = blockIdx.x;
    const int i = t / g.nb, k = t % g.nb;
    const int b = g.b;
    const T *src = tiles + (int64_t)t * b * b;
    for (int e = threadIdx.x; e < b * b; e += 256) {
        const int r = e / b, c = e % b;
        const int64_t gi = (int64_t)i * b + r, gj = (int64_t)k * b + c;
        if (gi < g.n && gj < g.n) {
            const double v = (double)src[e];
            out[gi * ld + gj] = divide ? v / scale : v * scale;
        }
    }
}

hipError_t launch_egress(int prec, const Geom &g, const void *tiles, double *out, int64_t ld, double scale,
                         int divide, hipStream_t st) {
    const unsigned nt = (unsigned)g.nb * g.nb;
    if (prec == P_F64)
        hipLaunchKernelGGL(k_egress<double>, dim3(nt), dim3(256), 0, st, (const double *)tiles, g, out, ld, scale,
                           divide);
    else
        hipLaunchKernelGGL(k_egress<float>, dim3(nt), dim3(256), 0, st, (const float *)tiles, g, out, ld, scale,
                           divide);
    return hipGetLastError();
}

// sqrt of every pyramid entry (squared norms -> norms).
__global__ __launch_bounds__(256) void k_sqrt(const double *__restrict__ q, double *__restrict__ out, int64_t m) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e < m) out[e] = sqrt(q[e]);
}

hipError_t launch_norms_out(const Geom &g, const double *q, double *out, hipStream_t st) {
    const int64_t m = pyr_len(g.P);
    hipLaunchKernelGGL(k_sqrt, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, st, q, out, m);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Dense row-major helpers of the product representation (32 x 32 blocks
// through LDS for the transposed reads).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_shift_copy(const double *__restrict__ src, double *__restrict__ dst,
                                                    int64_t n, int64_t ld, double mu) {
    const int64_t r = blockIdx.y;
    for (int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x; c < n; c += (int64_t)gridDim.x * 256) {
        double v = src[r * ld + c];
        if (r == c) v += mu;
        dst[r * ld + c] = v;
    }
}

// mode 0: dst = src^T; mode 1: dst = (src + src^T)/2 (each pair summed in the
// order src_ij + src_ji, which is commutative, so dst is exactly symmetric)
__global__ __launch_bounds__(256) void k_transpose_sym(const double *__restrict__ src, double *__restrict__ dst,
                                                       int64_t n, int64_t ld, int mode) {
    __shared__ double tileT[32][33];
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
    const int64_t r0 = (int64_t)blockIdx.y * 32, c0 = (int64_t)blockIdx.x * 32;
    for (int m = 0; m < 32; m += 8) {  // block (c0, r0) of src, stored transposed
        const int64_t r = c0 + ty + m, c = r0 + tx;
        tileT[tx][ty + m] = (r < n && c < n) ? src[r * ld + c] : 0.0;
    }
    __syncthreads();
    for (int m = 0; m < 32; m += 8) {
        const int64_t r = r0 + ty + m, c = c0 + tx;
        if (r < n && c < n) {
            const double t = tileT[ty + m][tx];  // src[c][r]
            dst[r * ld + c] = mode == 0 ? t : 0.5 * (src[r * ld + c] + t);
        }
    }
}

hipError_t launch_shift_copy(const double *src, double *dst, int64_t n, int64_t ld, double mu, hipStream_t st) {
    const unsigned gx = (unsigned)std::min<int64_t>((n + 255) / 256, 64);
    hipLaunchKernelGGL(k_shift_copy, dim3(gx, (unsigned)n), dim3(256), 0, st, src, dst, n, ld, mu);
    return hipGetLastError();
}

hipError_t launch_transpose_dense(const double *src, double *dst, int64_t n, int64_t ld, hipStream_t st) {
    const unsigned nbk = (unsigned)((n + 31) / 32);
    hipLaunchKernelGGL(k_transpose_sym, dim3(nbk, nbk), dim3(256), 0, st, src, dst, n, ld, 0);
    return hipGetLastError();
}

hipError_t launch_sym_part(const double *src, double *dst, int64_t n, int64_t ld, hipStream_t st) {
    const unsigned nbk = (unsigned)((n + 31) / 32);
    hipLaunchKernelGGL(k_transpose_sym, dim3(nbk, nbk), dim3(256), 0, st, src, dst, n, ld, 1);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Retained-triple export: exclusive scan of per-tile counts in (i,j) order
// (single block), then every tile scatters its (i,j,k) records.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void k_scan_counts(const int32_t *__restrict__ cnt, int64_t m,
                                                       int64_t *__restrict__ offs, int64_t *__restrict__ total) {
    __shared__ int64_t part[1024];
    const int64_t per = (m + 1023) / 1024;
    const int64_t lo = threadIdx.x * per, hi = lo + per < m ? lo + per : m;
    int64_t s = 0;
    for (int64_t e = lo; e < hi; ++e) s += cnt[e];
    part[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t run = 0;
        for (int x = 0; x < 1024; ++x) {
            const int64_t v = part[x];
            part[x] = run;
            run += v;
        }
        *total = run;
    }
    __syncthreads();
    int64_t run = part[threadIdx.x];
    for (int64_t e = lo; e < hi; ++e) {
        offs[e] = run;
        run += cnt[e];
    }
}

__global__ __launch_bounds__(64) void k_write_triples(const int32_t *__restrict__ cnt,
                                                       const int32_t *__restrict__ kidx,
                                                       const int64_t *__restrict__ offs, int nb,
                                                       int32_t *__restrict__ trip) {
    const int64_t t = blockIdx.x;
    const int i = (int)(t / nb), j = (int)(t % nb);
    const int c = cnt[t];
    const int64_t o = offs[t];
    for (int e = threadIdx.x; e < c; e += 64) {
        trip[3 * (o + e) + 0] = i;
        trip[3 * (o + e) + 1] = j;
        trip[3 * (o + e) + 2] = kidx[t * nb + e];
    }
}

hipError_t launch_count_triples(const Geom &g, const int32_t *cnt, int64_t *offs, int64_t *total,
                                hipStream_t st) {
    hipLaunchKernelGGL(k_scan_counts, dim3(1), dim3(1024), 0, st, cnt, (int64_t)g.nb * g.nb, offs, total);
    return hipGetLastError();
}

hipError_t launch_write_triples(const Geom &g, const int32_t *cnt, const int32_t *kidx, const int64_t *offs,
                                int32_t *triples, hipStream_t st) {
    hipLaunchKernelGGL(k_write_triples, dim3((unsigned)g.nb * g.nb), dim3(64), 0, st, cnt, kidx, offs, g.nb,
                       triples);
    return hipGetLastError();
}

}  // namespace spk
