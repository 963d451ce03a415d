// Device-side helpers shared by the kernel sources: fixed-order wave and
// block reductions, and the product-table lookups of batched launches.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.h"

namespace spk {

__device__ inline int64_t dev_level_off(int P, int S) {
    int64_t o = 0;
    for (int64_t T = P; T > S; T >>= 1) o += T * T;
    return o;
}

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ inline double wave_max(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

// Block-wide sum in a fixed order: lanes by xor-butterfly, then waves 0..W-1.
template <int NT>
__device__ inline double block_sum(double v, double *sh) {
    v = wave_sum(v);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[w] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < NT / 64; ++i) t += sh[i];
    return t;  // valid in thread 0
}

template <int NT>
__device__ inline double block_max(double v, double *sh) {
    v = wave_max(v);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[w] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < NT / 64; ++i) t = fmax(t, sh[i]);
    return t;
}

// Product tables.  Every batched launch covers all products of a table; a
// block finds its product by binary search in a prefix array and returns at
// once when the product's solve is not running.
__device__ inline int find_slot(const int32_t *pre, int n, int x) {
    // largest p in [0, n) with pre[p] <= x  (pre[0] = 0 <= x < pre[n])
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (pre[mid] <= x)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

__device__ inline bool prod_running(const ProdDesc &d) { return d.state == nullptr || d.state->status == ST_RUNNING; }
__device__ inline int prod_parity(const ProdDesc &d) { return d.state ? d.state->parity : 0; }

}  // namespace spk
