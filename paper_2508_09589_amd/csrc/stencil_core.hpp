// 27-point stencil rows of a coarse level, shared by the stand-alone stencil
// apply and the fused smoother kernels.
//
// Stencil layout: st[d][plane][j][i], d = (dn+1)*9 + (dj+1)*3 + (di+1) holds
// A(node, node + (di, dj, dn)); plane = plane_map[n] so that time levels with
// identical rows share storage.  Storage is FP64, FP32 or BF16 (upper half of
// an FP32, round to nearest even).
//
// BF16 stencils keep their three in-plane centres (di = dj = 0, d = 4, 13, 22)
// in FP32 instead, compensated so that rounding leaves the sums over each
// time offset intact: cen[g][plane][r] (g = dn + 1) makes every row's sum over
// the 9 entries of offset dn exact (forward apply), cen[3 + g][plane][r] makes
// the matching column sums exact (transposed apply).  Those sums fix how the
// operator acts on fields that are constant in space; an insulated domain has
// near-null modes of that kind, which plain BF16 rounding would perturb.
#pragma once
#include <type_traits>

#include "st_internal.hpp"

namespace st {

__device__ __forceinline__ float bf16_to_f32(uint16_t h) {
    return __uint_as_float(((unsigned)h) << 16);
}
__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
    unsigned u = __float_as_uint(f);
    const unsigned lsb = (u >> 16) & 1u;
    u += 0x7fffu + lsb;   // round to nearest even
    return (uint16_t)(u >> 16);
}

template <typename S> __device__ __forceinline__ float ldc(const S* p);
template <> __device__ __forceinline__ float ldc<float>(const float* p) { return *p; }
template <> __device__ __forceinline__ float ldc<uint16_t>(const uint16_t* p) {
    return bf16_to_f32(*p);
}
template <typename TC, typename S> __device__ __forceinline__ TC ldcoef(const S* p) {
    return (TC)ldc<S>(p);
}
template <> __device__ __forceinline__ double ldcoef<double, double>(const double* p) {
    return *p;
}

// Rows of y = A x (TRANS: A^T x) at in-plane position r = j (nx+1) + i for the
// time levels n0 <= n < n1; emit(n, idx, value) receives each one.  The
// thread keeps the x values of levels n-1, n, n+1 around r in registers (9 new
// loads per level).  The 27 coefficients of a row depend on the plane index
// only, so they are loaded again only when plane_map changes (time-invariant
// operators load them a handful of times per column).
template <typename T, typename S, typename TC, bool TRANS, typename Emit>
__device__ __forceinline__ void stencil_march_rows(int nx, int ny, int nt, int nplanes,
                                                   const S* __restrict__ st,
                                                   const float* __restrict__ cen,
                                                   const int* __restrict__ pmap,
                                                   const T* __restrict__ x, int r, int n0, int n1,
                                                   Emit&& emit) {
    constexpr bool CEN = std::is_same<S, uint16_t>::value;   // compensated FP32 centres
    const int rowp = nx + 1;
    const int P = rowp * (ny + 1);
    const int j = r / rowp, i = r - j * rowp;
    const long long DS = (long long)P * nplanes;
    unsigned valid = 0;
    int off[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        const int di = q % 3 - 1, dj = q / 3 - 1;
        off[q] = dj * rowp + di;
        if (i + di >= 0 && i + di <= nx && j + dj >= 0 && j + dj <= ny) valid |= 1u << q;
    }
    auto load_plane = [&](int n, TC u[9]) {
        if (n < 0 || n > nt) {
#pragma unroll
            for (int q = 0; q < 9; ++q) u[q] = (TC)0;
            return;
        }
        const T* xp = x + (long long)n * P + r;
#pragma unroll
        for (int q = 0; q < 9; ++q) u[q] = ((valid >> q) & 1u) ? (TC)xp[off[q]] : (TC)0;
    };
    TC xm[9], xc[9], xp[9], c[27];
    load_plane(n0 - 1, xm);
    load_plane(n0, xc);
    int key0 = -2, key1 = -2, key2 = -2;
    for (int n = n0; n < n1; ++n) {
        load_plane(n + 1, xp);
        const int pm = n > 0 ? pmap[n - 1] : -1;
        const int pc = pmap[n];
        const int pp = n < nt ? pmap[n + 1] : -1;
        const bool same = TRANS ? (pm == key0 && pc == key1 && pp == key2) : (pc == key1);
        if (!same) {
            key0 = pm;
            key1 = pc;
            key2 = pp;
            if (!TRANS) {
                const S* sp = st + (long long)pc * P + r;
#pragma unroll
                for (int d = 0; d < 27; ++d) {
                    if (CEN && d % 9 == 4)
                        c[d] = (TC)cen[(long long)(d / 9) * DS + (long long)pc * P + r];
                    else
                        c[d] = ldcoef<TC, S>(sp + (long long)d * DS);
                }
            } else {
#pragma unroll
                for (int dn = -1; dn <= 1; ++dn) {
                    const int pl = dn < 0 ? pm : (dn == 0 ? pc : pp);
#pragma unroll
                    for (int q = 0; q < 9; ++q) {
                        const int d = (dn + 1) * 9 + q;
                        if (CEN && q == 4)
                            c[d] = pl >= 0 ? (TC)cen[(long long)(4 - dn) * DS + (long long)pl * P + r]
                                           : (TC)0;
                        else
                            c[d] = (pl >= 0 && ((valid >> q) & 1u))
                                       ? ldcoef<TC, S>(st + (long long)(26 - d) * DS + (long long)pl * P + r + off[q])
                                       : (TC)0;
                    }
                }
            }
        }
        TC acc = 0;
#pragma unroll
        for (int q = 0; q < 9; ++q) acc += c[q] * xm[q];
#pragma unroll
        for (int q = 0; q < 9; ++q) acc += c[9 + q] * xc[q];
#pragma unroll
        for (int q = 0; q < 9; ++q) acc += c[18 + q] * xp[q];
        emit(n, (long long)n * P + r, acc);
#pragma unroll
        for (int q = 0; q < 9; ++q) {
            xm[q] = xc[q];
            xc[q] = xp[q];
        }
    }
}

}  // namespace st
