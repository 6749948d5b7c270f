// Block-wide sums of many per-thread accumulators, and the sum over blocks of
// a grid's partials; both in a fixed order (results are bitwise repeatable).
#pragma once
#include "st_internal.hpp"

namespace st {

// out[d] = sum over the THREADS threads of the block of v[d], for d < nd
// (nd <= N); out is in LDS and visible to the whole block on return.
// The values pass through LDS in chunks of RC_CHUNK: thread t writes its
// chunk, then each group of THREADS / RC_CHUNK lanes adds the column of one
// value (RC_CHUNK independent LDS reads) and finishes with xor shuffles inside
// the group.  A shuffle tree per value instead (six dependent cross-lane
// rounds each) serialises: with 66 values it costs ~20 us per workgroup.
constexpr int RC_CHUNK = 8;
template <int N, int THREADS>
__device__ __forceinline__ void block_sum_many(const double (&v)[N], int nd, double* out) {
    constexpr int LPV = THREADS / RC_CHUNK;   // lanes per value
    static_assert(LPV <= 64 && 64 % LPV == 0, "value groups must tile a wave");
    __shared__ double stage[RC_CHUNK][THREADS];
    const int t = threadIdx.x;
    const int k = t / LPV, s = t - (t / LPV) * LPV;
#pragma unroll
    for (int c0 = 0; c0 < N; c0 += RC_CHUNK) {
        if (c0 >= nd) break;   // uniform over the block
#pragma unroll
        for (int q = 0; q < RC_CHUNK; ++q)
            if (c0 + q < N) stage[q][t] = v[c0 + q];
        __syncthreads();
        double a = 0.0;
#pragma unroll
        for (int u = 0; u < RC_CHUNK; ++u) a += stage[k][s + LPV * u];
#pragma unroll
        for (int o = LPV / 2; o > 0; o >>= 1) a += __shfl_xor(a, o, 64);
        if (s == 0 && c0 + k < nd) out[c0 + k] = a;
        __syncthreads();
    }
}

// sums[d] = sum over blocks b < nb of part[b * stride + d], d < nd, by one
// block of THREADS threads.  Up to 64 values per round: w (the value count
// rounded up to a power of two) lanes cover the values of one contiguous row,
// the THREADS / w groups of them take the blocks g, g + THREADS / w, ... (loads
// unrolled so that several are in flight), and a fixed tree adds the groups.
// sums is in LDS and visible to the whole block on return.
template <int THREADS>
__device__ __forceinline__ void sum_block_partials(const double* __restrict__ part, int nb,
                                                   long long stride, int nd, double* sums) {
    __shared__ double gsum[THREADS];
    const int t = threadIdx.x;
    for (int d0 = 0; d0 < nd; d0 += 64) {
        const int m = nd - d0 < 64 ? nd - d0 : 64;
        int w = 1;
        while (w < m) w <<= 1;
        const int G = THREADS / w;
        const int d = t & (w - 1), g = t / w;
        double v = 0.0;
        if (d < m) {
#pragma unroll 8
            for (int b = g; b < nb; b += G) v += part[(long long)b * stride + d0 + d];
        }
        gsum[t] = v;
        __syncthreads();
        for (int h = G / 2; h > 0; h >>= 1) {
            if (g < h) gsum[t] += gsum[t + h * w];
            __syncthreads();
        }
        if (g == 0 && d < m) sums[d0 + d] = gsum[t];
        __syncthreads();
    }
}

}  // namespace st
