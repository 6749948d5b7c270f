// 27-point stencil rows of a coarse level: the row march of the FP64 stencil
// apply and of the fused small-level smoother kernels (the stand-alone FP32
// applies take the wave form, k_stencil_wave).
//
// Stencil layout: st[d][plane][j][i], d = (dn+1)*9 + (dj+1)*3 + (di+1) holds
// A(node, node + (di, dj, dn)); plane = plane_map[n] so that time levels with
// identical rows share storage.  Storage is FP64, FP32 or BF16 (upper half of
// an FP32, round to nearest even).
//
// The FP32 and BF16 copies are stored in symmetric form.  Every time-offset
// block of a Galerkin level is symmetric in space,
//     A(p, p + (dn, dj, di)) = A(q, q + (dn, -dj, -di)),  q = p + (0, dj, di),
// so of the nine in-plane entries q = (dj+1)*3 + (di+1) of a time offset only
// q >= 4 (the centre and the four "upper" neighbours) are stored; entry q < 4
// of row r is entry 8 - q of the neighbour row r + off_q.  FP32: sym[g*5 +
// q - 4][plane][r] (15 per row, g = dn + 1).  BF16: sym[g*4 + q - 5][plane][r]
// (12 per row), the three centres in FP32 instead, compensated so that
// rounding leaves the sums over each time offset intact: cen[g][plane][r] =
// the exact FP64 sum of the nine values the apply uses for row r and offset
// dn minus the eight rounded off-centre ones.  By the symmetry the transposed
// apply uses the same values for its column sums, so the same centres serve
// it.  Those sums fix how the operator acts on fields that are constant in
// space; an insulated domain has near-null modes of that kind, which plain
// BF16 rounding would perturb.  The FP64 stencil keeps all 27 entries.
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

// Address of element e of an array whose base is the same for the whole
// wave: a scalar base plus a 32-bit per-lane byte offset (no 64-bit vector
// address per load).
template <typename S> __device__ __forceinline__ const S* at_elem(const S* base, unsigned e) {
    return (const S*)((const char*)base + e * (unsigned)sizeof(S));
}
// The same with the base moved to scalar registers explicitly (it is
// wave-uniform), so that the compiler cannot fold it into a 64-bit per-lane
// address.
template <typename S> __device__ __forceinline__ const S* at_elem_u(const S* base, unsigned e) {
    typedef const S __attribute__((address_space(1))) GS;
    const unsigned long long v = (unsigned long long)base;
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)v);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(v >> 32));
    GS* g = (GS*)(((unsigned long long)hi << 32) | lo);
    // the 32-bit offset is formed here, next to its load (a hoisted 64-bit
    // copy would defeat the scalar-base addressing form)
    unsigned b = e * (unsigned)sizeof(S);
    asm volatile("" : "+v"(b));
    return (const S*)((const __attribute__((address_space(1))) char*)g + b);
}

// Index of stored entry (g, q), q >= 4 (q >= 5 for BF16, whose centres live
// in the FP32 array), in a symmetric stencil array.
template <bool BF16> __device__ __forceinline__ int sym_index(int g, int q) {
    return BF16 ? g * 4 + (q - 5) : g * 5 + (q - 4);
}

// Rows of y = A x (TRANS: A^T x) at in-plane position r = j (nx+1) + i for the
// time levels n0 <= n < n1; emit(n, idx, value) receives each one.  The
// thread keeps the x values of levels n-1, n, n+1 around r in registers (9 new
// loads per level).  The 27 coefficients of a row depend on the plane index
// only, so they are loaded again only when plane_map changes (time-invariant
// operators load them a handful of times per column).
//
// Loads of x are guarded lane by lane (a neighbour outside the plane would
// read another row, or outside the array): the three of one grid row share an
// address and differ by immediate offsets, and on interior waves the guards
// cost no branch.  Loads of coefficients are not guarded, so that a reload of
// a row's coefficients has no branch (each would close with a wait for its
// load): a neighbour outside the plane reads row r itself, and the number it
// gets meets an x value of zero.  Their addresses are a wave-uniform base
// (plane and entry) plus a 32-bit lane offset.
template <typename T, typename S, typename TC, bool TRANS, typename Emit>
__device__ __forceinline__ void stencil_march_rows(int nx, int ny, int nt, int nplanes,
                                                   const S* __restrict__ st,
                                                   const float* __restrict__ cen,
                                                   const int* __restrict__ pmap,
                                                   const T* __restrict__ x, int r, int n0, int n1,
                                                   Emit&& emit) {
    constexpr bool CEN = std::is_same<S, uint16_t>::value;   // compensated FP32 centres
    constexpr bool SYM = !std::is_same<S, double>::value;     // symmetric (15- or 12-entry) storage
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
    // in-plane index of neighbour q for a coefficient load (r outside the plane)
    auto ce = [&](int q) -> unsigned { return (unsigned)(((valid >> q) & 1u) ? r + off[q] : r); };
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
        const int pm = n > 0 ? __builtin_amdgcn_readfirstlane(pmap[n - 1]) : -1;
        const int pc = __builtin_amdgcn_readfirstlane(pmap[n]);
        const int pp = n < nt ? __builtin_amdgcn_readfirstlane(pmap[n + 1]) : -1;
        const bool same = TRANS ? (pm == key0 && pc == key1 && pp == key2) : (pc == key1);
        if (!same) {
            key0 = pm;
            key1 = pc;
            key2 = pp;
            if (!TRANS) {
                const long long pb = (long long)pc * P;
#pragma unroll
                for (int g = 0; g < 3; ++g)
#pragma unroll
                    for (int q = 0; q < 9; ++q) {
                        if (SYM) {
                            // row r's entry (g, q): stored at r for q >= 4,
                            // the neighbour's (g, 8 - q) for q < 4
                            if (CEN && q == 4) {
                                c[g * 9 + q] = (TC)*at_elem_u(cen + (long long)g * DS + pb, (unsigned)r);
                            } else {
                                const int qs = q >= 4 ? q : 8 - q;
                                c[g * 9 + q] = ldcoef<TC, S>(at_elem_u(
                                    st + (long long)sym_index<CEN>(g, qs) * DS + pb,
                                    q >= 4 ? (unsigned)r : ce(q)));
                            }
                        } else {
                            c[g * 9 + q] = ldcoef<TC, S>(
                                at_elem_u(st + (long long)(g * 9 + q) * DS + pb, (unsigned)r));
                        }
                    }
            } else {
#pragma unroll
                for (int dn = -1; dn <= 1; ++dn) {
                    // plane of level n + dn (plane 0 past either end, where
                    // the x level is zero)
                    const int pl = dn < 0 ? (pm < 0 ? 0 : pm) : (dn == 0 ? pc : (pp < 0 ? 0 : pp));
                    const long long pb = (long long)pl * P;
                    const int gt = 1 - dn;   // time-offset group of the row that points back
#pragma unroll
                    for (int q = 0; q < 9; ++q) {
                        const int d = (dn + 1) * 9 + q;
                        // A^T(r, r + off_q) at offset dn = entry (gt, 8 - q) of
                        // row r + off_q on level n + dn; in symmetric storage
                        // that is entry (gt, q) of row r itself
                        if (SYM) {
                            if (CEN && q == 4) {
                                c[d] = (TC)*at_elem_u(cen + (long long)gt * DS + pb, (unsigned)r);
                            } else {
                                const bool own = q > 4;
                                c[d] = ldcoef<TC, S>(at_elem_u(
                                    st + (long long)sym_index<CEN>(gt, own ? q : 8 - q) * DS + pb,
                                    own ? (unsigned)r : ce(q)));
                            }
                        } else {
                            c[d] = ldcoef<TC, S>(
                                at_elem_u(st + (long long)(26 - d) * DS + pb, ce(q)));
                        }
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
