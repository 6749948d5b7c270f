// Coarse-level kernels of the space-time multigrid hierarchy (paper §3.2):
// 27-point stencil application and its transpose, masked trilinear restriction
// (P_m^T) and prolongation (P_m) for space and time semi-coarsening (§3.2.1)
// and for full space-time coarsening (how = 3, the paper's comparison),
// coarse Dirichlet masks, and the pieces of the Galerkin construction
// A_{l+1} = P_m^T A_l P_m by probing with 27 colours.
//
// Stencil layout and storage precisions: see stencil_core.hpp.
#include "st_internal.hpp"
#include "stencil_core.hpp"

namespace st {

static inline unsigned grid_for(long long n, int threads = 256, long long cap = 65535) {
    long long nb = (n + threads - 1) / threads;
    if (nb < 1) nb = 1;
    if (nb > cap) nb = cap;
    return (unsigned)nb;
}

// ---------------------------------------------------------------------------
// y = A x (or A^T x) with the same epilogue as the fine apply:
//   v = A x;  if b: v = b - v;  if invd: v *= invd;  v *= scale.
template <typename T, typename S, typename TC, bool TRANS>
__global__ __launch_bounds__(256) void k_stencil_march(
    int nx, int ny, int nt, int nplanes, const S* __restrict__ st, const float* __restrict__ cen,
    const int* __restrict__ pmap, const T* __restrict__ x, T* __restrict__ y, const T* __restrict__ b,
    const T* __restrict__ invd, const double* __restrict__ scale, const int* __restrict__ skip,
    int nchunk, int gx, int nblk, int per_xcd) {
    if (skip && *skip) return;
    // Workgroup (node block bx, time chunk by): the 2-D grid's, or with
    // per_xcd > 0 an XCD-aware order over a 1-D grid -- hardware workgroup b
    // runs on XCD b % 8, so each XCD takes a contiguous range of (bx, by) and
    // the rows above and below a block, whose coefficients the symmetric
    // form reads, come from the same L2.
    int bx = blockIdx.x, by = blockIdx.y;
    if (per_xcd > 0) {
        const int bid = blockIdx.x;
        const int lin = (bid & 7) * per_xcd + (bid >> 3);
        if (lin >= nblk) return;
        by = lin / gx;
        bx = lin - by * gx;
    }
    const int P = (nx + 1) * (ny + 1);
    const int r = bx * blockDim.x + threadIdx.x;
    if (r >= P) return;
    const int n0 = by * nchunk;
    if (n0 > nt) return;
    const int n1 = min(n0 + nchunk, nt + 1);
    const TC sc = scale ? (TC)(*scale) : (TC)1;
    stencil_march_rows<T, S, TC, TRANS>(nx, ny, nt, nplanes, st, cen, pmap, x, r, n0, n1,
                                        [&](int, long long idx, TC acc) {
                                            TC v = acc;
                                            if (b) v = (TC)b[idx] - v;
                                            if (invd) v *= (TC)invd[idx];
                                            y[idx] = (T)(v * sc);
                                        });
}

// Lane l of the wave receives v of lane l - 1 (lane_prev) or l + 1
// (lane_next); the lanes at the ends of the wave receive zero.  A DPP
// whole-wave shift, no LDS.
__device__ __forceinline__ float lane_prev(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v),
                                                                 0x138, 0xf, 0xf, true));
}
__device__ __forceinline__ float lane_next(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v),
                                                                 0x130, 0xf, 0xf, true));
}
// The same for FP64 values: both 32-bit halves shifted.
__device__ __forceinline__ double lane_prev(double v) {
    typedef int i32x2 __attribute__((ext_vector_type(2)));
    i32x2 h = __builtin_bit_cast(i32x2, v);
    h.x = __builtin_amdgcn_update_dpp(0, h.x, 0x138, 0xf, 0xf, true);
    h.y = __builtin_amdgcn_update_dpp(0, h.y, 0x138, 0xf, 0xf, true);
    return __builtin_bit_cast(double, h);
}
__device__ __forceinline__ double lane_next(double v) {
    typedef int i32x2 __attribute__((ext_vector_type(2)));
    i32x2 h = __builtin_bit_cast(i32x2, v);
    h.x = __builtin_amdgcn_update_dpp(0, h.x, 0x130, 0xf, 0xf, true);
    h.y = __builtin_amdgcn_update_dpp(0, h.y, 0x130, 0xf, 0xf, true);
    return __builtin_bit_cast(double, h);
}

// FP32 apply (TRANS: transposed apply) with the in-plane neighbours taken
// from adjacent lanes.  A wave covers 64 consecutive in-plane nodes and
// produces the 62 inside them (lanes 0 and 63 only load): per time level it
// loads three node segments, one per grid row j-1, j, j+1.  Consecutive lanes
// hold consecutive in-plane indices, also across the end of a grid row, so
// lane l +- 1 holds node r +- 1; where that is not a neighbour (i = 0 or
// i = nx, or a row outside the plane) the coefficient is set to zero at load
// time, and a segment load outside the plane is clamped into it (a finite
// value times zero).  The coefficient of row r for its left neighbour r - 1
// is kept by lane l - 1 (moved there once, when the coefficients are
// loaded), which forms the nine products with its own x values; one shift
// per level brings their sum to lane l (the right neighbours likewise): two
// lane shifts per level instead of one per product.
//
// Three loads per level instead of nine leave the registers for loading x
// two levels ahead (b and invd one level ahead): level k lives in register
// set (k - n0 + 1) mod 4 from its load (two steps before its first use) to
// its last use, and the loop is unrolled by four so that each set has a
// fixed name.  x, b, invd and y go through buffer resources: a level outside
// [0, nt] (or past the chunk) and the stores of the two loading-only lanes
// take an offset past the resource's end, which reads zero and writes
// nothing, so that no load or store sits behind a branch (a branch's join
// makes the compiler wait for every load in flight, the ones ahead too).
// Arrays up to 2 GiB (the offsets are 32-bit).  Same epilogue as
// k_stencil_march; HB, HD: b and invd given.
constexpr int SW_OUT = 62;
constexpr unsigned SW_OOB = 0x80000000u;   // offset past the end of every resource here

__device__ __forceinline__ __amdgpu_buffer_rsrc_t lv_rsrc(const void* p, long long bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}
template <typename T> __device__ __forceinline__ T lv_ld(__amdgpu_buffer_rsrc_t r, unsigned off);
template <> __device__ __forceinline__ float lv_ld<float>(__amdgpu_buffer_rsrc_t r, unsigned off) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
template <> __device__ __forceinline__ double lv_ld<double>(__amdgpu_buffer_rsrc_t r, unsigned off) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
__device__ __forceinline__ void lv_st(float v, __amdgpu_buffer_rsrc_t r, unsigned off) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, off, 0, 0);
}
__device__ __forceinline__ void lv_st(double v, __amdgpu_buffer_rsrc_t r, unsigned off) {
    typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, off, 0, 0);
}

template <typename T, typename S, bool HB, bool HD, bool TRANS>
__global__ __launch_bounds__(256) void k_stencil_wave(
    int nx, int ny, int nt, int nplanes, const S* __restrict__ st, const float* __restrict__ cen,
    const int* __restrict__ pmap, const T* __restrict__ x, T* __restrict__ y,
    const T* __restrict__ b, const T* __restrict__ invd, const double* __restrict__ scale,
    const int* __restrict__ skip, int nchunk, int gx, int nblk, int per_xcd) {
    if (skip && *skip) return;
    int bx = blockIdx.x, by = blockIdx.y;
    if (per_xcd > 0) {
        const int bid = blockIdx.x;
        const int lin = (bid & 7) * per_xcd + (bid >> 3);
        if (lin >= nblk) return;
        by = lin / gx;
        bx = lin - by * gx;
    }
    constexpr bool CEN = std::is_same<S, uint16_t>::value;
    constexpr bool SYM = !std::is_same<S, double>::value;   // symmetric (15- or 12-entry) storage
    constexpr unsigned ES = sizeof(T);
    const int rowp = nx + 1;
    const int P = rowp * (ny + 1);
    const int lane = threadIdx.x & 63;
    const int first = (bx * 4 + (int)(threadIdx.x >> 6)) * SW_OUT;   // first output node of the wave
    if (first >= P) return;
    const int n0 = by * nchunk;
    if (n0 > nt) return;
    const int n1 = min(n0 + nchunk, nt + 1);
    const int rl = first + lane - 1;                 // this lane's node (-1 or >= P on halo lanes)
    const bool out = lane >= 1 && lane <= SW_OUT && rl < P;
    const int r = min(max(rl, 0), P - 1);            // in-plane node for coefficient, b, invd loads
    const int j = r / rowp, i = r - j * rowp;
    unsigned valid = 0;
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        const int di = q % 3 - 1, dj = q / 3 - 1;
        if (i + di >= 0 && i + di <= nx && j + dj >= 0 && j + dj <= ny) valid |= 1u << q;
    }
    const unsigned PB = (unsigned)P * ES;            // bytes per level
    unsigned seg[3];                                 // byte offset of the segment load per grid row
#pragma unroll
    for (int d = 0; d < 3; ++d) seg[d] = (unsigned)min(max(rl + (d - 1) * rowp, 0), P - 1) * ES;
    const unsigned rb = (unsigned)r * ES;
    const unsigned ob = out ? rb : SW_OOB;           // store offset within a level
    const long long DS = (long long)P * nplanes;
    const T sc = scale ? (T)(*scale) : (T)1;
    const long long vbytes = (long long)(nt + 1) * P * ES;
    const __amdgpu_buffer_rsrc_t xr = lv_rsrc(x, vbytes), yr = lv_rsrc(y, vbytes);
    const __amdgpu_buffer_rsrc_t br = lv_rsrc(b, HB ? vbytes : 0), dr = lv_rsrc(invd, HD ? vbytes : 0);
    // the plane indices of the chunk's levels, one per lane, read back with
    // readlane: a load of pmap[n] inside the loop would be a vector load whose
    // wait also drains the levels loaded ahead.  The transpose also takes the
    // levels before and after the chunk (nchunk + 2 <= 64); a level outside
    // [0, nt] reads plane 0, whose numbers meet a zero x.
    const int pl0 = TRANS ? n0 - 1 : n0;
    const int pk = pl0 + lane;
    const int pml = (pk < (TRANS ? n1 + 1 : n1) && pk >= 0 && pk <= nt) ? pmap[pk] : 0;

    // level k (zero outside [0, nt]; not needed past n1)
    auto load_level = [&](int k, T (&u)[3]) __attribute__((always_inline)) {
        const unsigned kb = (k >= 0 && k <= min(nt, n1)) ? (unsigned)k * PB : SW_OOB;
#pragma unroll
        for (int d = 0; d < 3; ++d) u[d] = lv_ld<T>(xr, kb + seg[d]);
    };
    T c[27];
    // c[(dn + 1) * 9 + q] multiplies x at level n + dn, in-plane node r + off_q.
    // Forward: entry (dn + 1, q) of row r on level n's plane pc.  Transpose:
    // entry (1 - dn, 8 - q) of row r + off_q on level n + dn's plane (pm, pc,
    // pp); in symmetric storage that is entry (1 - dn, q) of row r itself
    // for q > 4.  FP64 storage holds all 27 entries of every row: the
    // transpose reads entry 26 - ((dn + 1) * 9 + q) of row r + off_q.
    auto load_coefs = [&](int pm, int pc, int pp) __attribute__((always_inline)) {
#pragma unroll
        for (int g = 0; g < 3; ++g)
#pragma unroll
            for (int q = 0; q < 9; ++q) {
                const int di = q % 3 - 1, dj = q / 3 - 1;
                const bool ok = (valid >> q) & 1u;
                const unsigned nb = ok ? (unsigned)(r + dj * rowp + di) : (unsigned)r;
                const int gs = TRANS ? 2 - g : g;
                const long long pb = (long long)(TRANS ? (g == 0 ? pm : (g == 1 ? pc : pp)) : pc) * P;
                T v;
                if (!SYM) {
                    const int dd = TRANS ? 26 - (g * 9 + q) : g * 9 + q;
                    v = ldcoef<T, S>(at_elem_u(st + (long long)dd * DS + pb, TRANS ? nb : (unsigned)r));
                } else if (CEN && q == 4) {
                    v = *at_elem_u(cen + (long long)gs * DS + pb, (unsigned)r);
                } else if (!TRANS) {
                    // row r's entry (g, q): stored at r for q >= 4, the
                    // neighbour's (g, 8 - q) for q < 4
                    const int qs = q >= 4 ? q : 8 - q;
                    v = ldcoef<T, S>(at_elem_u(st + (long long)sym_index<CEN>(gs, qs) * DS + pb,
                                               q >= 4 ? (unsigned)r : nb));
                } else {
                    const bool own = q > 4;
                    v = ldcoef<T, S>(at_elem_u(
                        st + (long long)sym_index<CEN>(gs, own ? q : 8 - q) * DS + pb,
                        own ? (unsigned)r : nb));
                }
                v = ok ? v : (T)0;
                // a left-neighbour coefficient moves to the lane of that
                // neighbour, a right-neighbour one likewise
                c[g * 9 + q] = di < 0 ? lane_next(v) : (di > 0 ? lane_prev(v) : v);
            }
    };
    // sums over one level's three rows: the node's own column into acc, the
    // products its left and right neighbours need into sl and sr
    auto row_sum = [&](const T* cg, const T (&u)[3], T& acc, T& sl, T& sr)
        __attribute__((always_inline)) {
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            sl += cg[d * 3 + 0] * u[d];
            acc += cg[d * 3 + 1] * u[d];
            sr += cg[d * 3 + 2] * u[d];
        }
    };
    // The chunk's first three levels of x (and b, invd of its first level)
    // are loaded while the plane indices, then the first coefficients, come
    // in: the first step needs all of them, so the coefficients' waits drain
    // nothing that is loaded ahead.
    T R0[3], R1[3], R2[3], R3[3];
    T b0 = 0, b1 = 0, d0 = 1, d1 = 1;
    if (HB) b0 = lv_ld<T>(br, (unsigned)n0 * PB + rb);
    if (HD) d0 = lv_ld<T>(dr, (unsigned)n0 * PB + rb);
    load_level(n0 - 1, R0);
    load_level(n0, R1);
    load_level(n0 + 1, R2);
    int key = __builtin_amdgcn_readlane(pml, 0), keyc = 0, keyp = 0;
    if (TRANS) {
        keyc = __builtin_amdgcn_readlane(pml, 1);
        keyp = __builtin_amdgcn_readlane(pml, 2);
    }
    load_coefs(key, TRANS ? keyc : key, keyp);
    // step n: levels n - 1, n, n + 1 of x in A, B, C and b, invd of level n
    // in bc, dc; level n + 2 of x goes into D, b and invd of level n + 1 into
    // bn, dn.  The scheduling barrier keeps those loads ahead of the
    // arithmetic, so that its waits leave them in flight.
    auto step = [&](int n, const T (&A)[3], const T (&B)[3], const T (&C)[3], T (&D)[3], T bc,
                    T dc, T& bn, T& dn)
        __attribute__((always_inline)) {
        // steps past the chunk (n >= n1) keep the last planes, load nothing
        // and store nothing
        const int i0 = min(n, n1 - 1) - n0;
        const int p0 = __builtin_amdgcn_readlane(pml, i0);
        if (TRANS) {
            const int p1 = __builtin_amdgcn_readlane(pml, i0 + 1);
            const int p2 = __builtin_amdgcn_readlane(pml, i0 + 2);
            if (p0 != key || p1 != keyc || p2 != keyp) {
                key = p0;
                keyc = p1;
                keyp = p2;
                load_coefs(p0, p1, p2);
            }
        } else if (p0 != key) {
            key = p0;
            load_coefs(p0, p0, p0);
        }
        load_level(n + 2, D);
        const unsigned nb = n + 1 < n1 ? (unsigned)(n + 1) * PB + rb : SW_OOB;
        if (HB) bn = lv_ld<T>(br, nb);
        if (HD) dn = lv_ld<T>(dr, nb);
        __builtin_amdgcn_sched_barrier(0);
        T acc = 0, sl = 0, sr = 0;
        row_sum(c, A, acc, sl, sr);
        row_sum(c + 9, B, acc, sl, sr);
        row_sum(c + 18, C, acc, sl, sr);
        // lane l - 1 holds the products with node r - 1 that row r needs
        T v = acc + lane_prev(sl) + lane_next(sr);
        if (HB) v = bc - v;
        if (HD) v *= dc;
        lv_st(v * sc, yr, out && n < n1 ? (unsigned)n * PB + rb : SW_OOB);
    };
    // no exit between the four steps: a load whose value only a later step
    // uses would be moved behind such an exit, after the arithmetic
    for (int n = n0; n < n1; n += 4) {
        step(n, R0, R1, R2, R3, b0, d0, b1, d1);
        step(n + 1, R1, R2, R3, R0, b1, d1, b0, d0);
        step(n + 2, R2, R3, R0, R1, b0, d0, b1, d1);
        step(n + 3, R3, R0, R1, R2, b1, d1, b0, d0);
    }
}

template <typename T, typename S, typename TC>
static void stencil_dispatch(hipStream_t s, const Level& L, const S* st, int trans, const void* x,
                             void* y, const void* b, const void* invd, const double* scale,
                             const int* skip, bool row_march) {
    const int P = (L.nx + 1) * (L.ny + 1);
    // applies run as k_stencil_wave (4 x 62 nodes per block) where its
    // 32-bit buffer offsets reach every level
    const bool wave =
        !row_march && (long long)(L.nt + 1) * P * (long long)sizeof(T) < (long long)SW_OOB;
    const int gx = wave ? (P + 4 * SW_OUT - 1) / (4 * SW_OUT) : (P + 255) / 256;
    // (k_stencil_wave runs its levels four at a time; 64 levels per chunk
    // rather than 32 drop half its extra loads at the chunk boundaries; its
    // transpose keeps the planes of nchunk + 2 levels in one register)
    int nchunk = wave && !trans ? 64 : 32;
    while (nchunk > (wave ? 4 : 2) && (long long)gx * ((L.nt + 1 + nchunk - 1) / nchunk) < 2048)
        nchunk /= 2;
    const int gy = (L.nt + 1 + nchunk - 1) / nchunk;
    const int nblk = gx * gy;
    // XCD-aware order (each XCD takes a contiguous range of blocks, so the
    // grid rows above and below a block, which its neighbours read too, come
    // from the same L2): for k_stencil_wave always (512^2 x 1024 hierarchy:
    // 293 -> 271 ms of stencil applies per solve), for k_stencil_march where
    // the coefficients change in time (every level reloads them, and
    // neighbouring blocks share rows of them: on a 256^2 x 256 hierarchy 32 ->
    // 29.5 ms per solve); a time-constant operator measured faster in the
    // plain order with k_stencil_march (369 ms against 440)
    const bool tv = 2 * L.nplanes > L.nt + 1;
    const int per_xcd = (tv || wave) ? (nblk + 7) / 8 : 0;
    const dim3 grid = per_xcd > 0 ? dim3(8 * per_xcd) : dim3(gx, gy);
    if (wave) {
        auto pick = [&](auto tr) {
            constexpr bool TR = decltype(tr)::value;
            return b ? (invd ? k_stencil_wave<T, S, true, true, TR> : k_stencil_wave<T, S, true, false, TR>)
                     : (invd ? k_stencil_wave<T, S, false, true, TR> : k_stencil_wave<T, S, false, false, TR>);
        };
        auto kern = trans ? pick(std::true_type{}) : pick(std::false_type{});
        hipLaunchKernelGGL(kern, grid, dim3(256), 0, s, L.nx, L.ny, L.nt, L.nplanes, st, L.cen32,
                           L.plane_map, (const T*)x, (T*)y, (const T*)b, (const T*)invd, scale,
                           skip, nchunk, gx, nblk, per_xcd);
        return;
    }
    if (trans)
        hipLaunchKernelGGL((k_stencil_march<T, S, TC, true>), grid, dim3(256), 0, s, L.nx, L.ny,
                           L.nt, L.nplanes, st, L.cen32, L.plane_map, (const T*)x, (T*)y,
                           (const T*)b, (const T*)invd, scale, skip, nchunk, gx, nblk, per_xcd);
    else
        hipLaunchKernelGGL((k_stencil_march<T, S, TC, false>), grid, dim3(256), 0, s, L.nx, L.ny,
                           L.nt, L.nplanes, st, L.cen32, L.plane_map, (const T*)x, (T*)y,
                           (const T*)b, (const T*)invd, scale, skip, nchunk, gx, nblk, per_xcd);
}

void launch_stencil_apply(hipStream_t s, const Level& L, int prec, int trans, const void* x,
                          void* y, const void* b, const void* invd, const double* scale,
                          const int* skip, bool row_march) {
    if (prec == 0)
        stencil_dispatch<double, double, double>(s, L, L.st64, trans, x, y, b, invd, scale, skip,
                                                 row_march);
    else if (L.sprec == 2)
        stencil_dispatch<float, uint16_t, float>(s, L, L.st16, trans, x, y, b, invd, scale, skip,
                                                 row_march);
    else
        stencil_dispatch<float, float, float>(s, L, L.st32, trans, x, y, b, invd, scale, skip,
                                              row_march);
}

// Row j of in-plane index r on rows of length rowp, without an integer
// division: a reciprocal multiply (double, exact to one step for r < 2^31)
// corrected by one step either way.
__device__ __forceinline__ int row_of(int r, int rowp, double inv) {
    int j = (int)((double)r * inv);
    if (j * rowp > r)
        --j;
    else if ((j + 1) * rowp <= r)
        ++j;
    return j;
}

// Transfers run one thread per in-plane node and a grid row per time level
// (looping when there are more levels than grid rows).
static inline dim3 plane_grid(const Level& L) {
    const long long P = (long long)(L.nx + 1) * (L.ny + 1);
    const long long gy = L.nt + 1 < 65535 ? L.nt + 1 : 65535;
    return dim3((unsigned)((P + 255) / 256), (unsigned)gy);
}

// ---------------------------------------------------------------------------
// Restriction b_c = P_m^T r_f = P^T N_f r_f.  Space: coarse (I, J, n) gathers
// fine (2I+a, 2J+c, n), a, c in {-1, 0, 1}, weight w(a) w(c) with w(0) = 1,
// w(+-1) = 1/2.  Time: coarse (i, j, N) gathers fine (i, j, 2N+a).
//
// Space semi-coarsening, the common case and the one on the largest grids:
// a thread takes one coarse node through TR_LV time levels at a time, all of
// their loads issued before any sum (each level on its own would wait a
// whole memory latency for a few bytes).  Loads are unconditional: a
// neighbour outside the plane reads the centre and is not summed.  The sum
// takes the terms in the same order as the definition, skipping the same
// ones.
constexpr int TR_LV = 2;
template <typename T>
__global__ void k_restrict_space(int nxf, int nyf, int nt, int nxc, int nyc, double inv_rowc,
                                 const uint8_t* __restrict__ maskf, const T* __restrict__ rf,
                                 T* __restrict__ bc) {
    const int rowc = nxc + 1, Pc = rowc * (nyc + 1);
    const long long rowf = nxf + 1, Pf = rowf * (nyf + 1);
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= Pc) return;
    const int J = row_of(r, rowc, inv_rowc), I = r - J * rowc;
    long long fo[9];   // in-plane index of fine neighbour q (the centre when outside)
    unsigned in = 0;
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        const int fj = 2 * J + q / 3 - 1, fi = 2 * I + q % 3 - 1;
        const bool ok = fj >= 0 && fj <= nyf && fi >= 0 && fi <= nxf;
        fo[q] = ok ? (long long)fj * rowf + fi : (long long)(2 * J) * rowf + 2 * I;
        if (ok) in |= 1u << q;
    }
    for (int n0 = blockIdx.y * TR_LV; n0 <= nt; n0 += gridDim.y * TR_LV) {
        T v[TR_LV][9];
        uint8_t mk[TR_LV][9];
#pragma unroll
        for (int u = 0; u < TR_LV; ++u) {
            const long long pf = (long long)min(n0 + u, nt) * Pf;   // past nt: not stored
#pragma unroll
            for (int q = 0; q < 9; ++q) {
                v[u][q] = rf[pf + fo[q]];
                mk[u][q] = maskf[pf + fo[q]];
            }
        }
#pragma unroll
        for (int u = 0; u < TR_LV; ++u) {
            if (n0 + u > nt) break;
            double acc = 0.0;
#pragma unroll
            for (int q = 0; q < 9; ++q) {
                const double w = (q / 3 == 1 ? 1.0 : 0.5) * (q % 3 == 1 ? 1.0 : 0.5);
                if (((in >> q) & 1u) && !mk[u][q]) acc += w * (double)v[u][q];
            }
            bc[(long long)(n0 + u) * Pc + r] = (T)acc;
        }
    }
}

// Time semi-coarsening (how = 2) and full space-time coarsening (how = 3).
template <typename T, int how>
__global__ void k_restrict(int nxf, int nyf, int ntf, int nxc, int nyc, int ntc,
                           double inv_rowc, const uint8_t* __restrict__ maskf,
                           const T* __restrict__ rf, T* __restrict__ bc) {
    const int rowc = nxc + 1, Pc = rowc * (nyc + 1);
    const long long rowf = nxf + 1, Pf = rowf * (nyf + 1);
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= Pc) return;
    const int J = row_of(r, rowc, inv_rowc), I = r - J * rowc;
    for (int n = blockIdx.y; n <= ntc; n += gridDim.y) {
        const long long idx = (long long)n * Pc + r;
        double acc = 0.0;
        if (how == 2) {
            for (int a = -1; a <= 1; ++a) {
                const int fn = 2 * n + a;
                if (fn < 0 || fn > ntf) continue;   // uniform
                const long long f = (long long)fn * Pf + r;
                const T v = rf[f];
                if (!maskf[f]) acc += (a == 0 ? 1.0 : 0.5) * (double)v;
            }
        } else {   // full space-time coarsening: the product of both
            for (int d = -1; d <= 1; ++d) {
                const int fn = 2 * n + d;
                if (fn < 0 || fn > ntf) continue;
                const double wd = d == 0 ? 1.0 : 0.5;
                for (int c = -1; c <= 1; ++c) {
                    const int fj = 2 * J + c;
                    if (fj < 0 || fj > nyf) continue;
                    const double wc = wd * (c == 0 ? 1.0 : 0.5);
                    for (int a = -1; a <= 1; ++a) {
                        const int fi = 2 * I + a;
                        if (fi < 0 || fi > nxf) continue;
                        const long long f = (long long)fn * Pf + (long long)fj * rowf + fi;
                        if (maskf[f]) continue;
                        acc += wc * (a == 0 ? 1.0 : 0.5) * (double)rf[f];
                    }
                }
            }
        }
        bc[idx] = (T)acc;
    }
}

// Grid of a transfer that takes lv time levels per thread and step.
// Space restriction (P_m^T, nxf = 2 nxc, nyf = 2 nyc) with the horizontal
// weights taken across lanes.  A wave covers fine columns 2 I0 - 1 ..
// 2 I0 + 62 of the fine rows 2J - 1, 2J, 2J + 1: each lane sums its column
// over the three rows (weights 1/2, 1, 1/2; masked fine nodes left out), and
// the odd lanes, which sit on even fine columns, add half of each
// neighbour's column sum to their own: coarse nodes I0 .. I0 + 30.  Fine
// values and masks come through buffer resources, so that a row or column
// outside the grid reads zero without a branch; all loads of a batch of
// RW_LV time levels are issued before its arithmetic.  Sums in FP64, as in
// k_restrict_space.
constexpr int RW_OUT = 31, RW_LV = 4;

template <typename T>
__global__ __launch_bounds__(256) void k_restrict_wave(int nxf, int nyf, int nt, int nxc, int nyc,
                                                       int nseg, int nchunk,
                                                       const uint8_t* __restrict__ maskf,
                                                       const T* __restrict__ rf, T* __restrict__ bc) {
    const int lane = threadIdx.x & 63;
    const int w = blockIdx.x * 4 + (int)(threadIdx.x >> 6);   // wave over (coarse row, segment)
    const int J = w / nseg;
    if (J > nyc) return;
    const int I0 = (w - J * nseg) * RW_OUT;
    const int n0 = blockIdx.y * nchunk;
    if (n0 > nt) return;
    const int n1 = min(n0 + nchunk, nt + 1);
    const int fi = 2 * I0 - 1 + lane;                          // this lane's fine column
    const int I = fi >> 1;                                     // coarse column of an odd lane
    const bool out = (lane & 1) && lane <= 2 * RW_OUT - 1 && I <= nxc;
    const int rowf = nxf + 1, rowc = nxc + 1;
    const unsigned Pf = (unsigned)rowf * (unsigned)(nyf + 1), Pc = (unsigned)rowc * (unsigned)(nyc + 1);
    unsigned fo[3];                                            // in-plane fine node of row d
    unsigned fin = 0;                                          // bit d: that node is in the grid
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const int fj = 2 * J + d - 1;
        const bool ok = fi >= 0 && fi <= nxf && fj >= 0 && fj <= nyf;
        fo[d] = ok ? (unsigned)(fj * rowf + fi) : 0u;
        if (ok) fin |= 1u << d;
    }
    const long long nl = nt + 1;
    const __amdgpu_buffer_rsrc_t rr = lv_rsrc(rf, nl * Pf * (long long)sizeof(T));
    const __amdgpu_buffer_rsrc_t mr = lv_rsrc(maskf, nl * Pf);
    const __amdgpu_buffer_rsrc_t cr = lv_rsrc(bc, nl * Pc * (long long)sizeof(T));
    const unsigned co = (unsigned)(J * rowc + I);
    for (int nb = n0; nb < n1; nb += RW_LV) {
        T v[RW_LV][3];
        unsigned char m[RW_LV][3];
#pragma unroll
        for (int u = 0; u < RW_LV; ++u) {
            // levels past the chunk read nothing and store nothing
            const bool lv = nb + u < n1;
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                // a node outside the grid (or a level past the chunk) reads
                // at an offset past both resources' ends: zero, no access
                const bool ok = lv && ((fin >> d) & 1u);
                const unsigned e = (unsigned)(nb + u) * Pf + fo[d];
                v[u][d] = lv_ld<T>(rr, ok ? e * (unsigned)sizeof(T) : SW_OOB);
                m[u][d] = __builtin_amdgcn_raw_buffer_load_b8(mr, ok ? e : SW_OOB, 0, 0);
            }
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < RW_LV; ++u) {
            double col = 0.0;
#pragma unroll
            for (int d = 0; d < 3; ++d)
                col += (m[u][d] ? 0.0 : (d == 1 ? 1.0 : 0.5)) * (double)v[u][d];
            const double r = col + 0.5 * (lane_prev(col) + lane_next(col));
            const bool st = out && nb + u < n1;
            lv_st((T)r, cr, st ? ((unsigned)(nb + u) * Pc + co) * (unsigned)sizeof(T) : SW_OOB);
        }
    }
}

static inline dim3 level_grid(const Level& L, int lv) {
    const long long P = (long long)(L.nx + 1) * (L.ny + 1);
    const long long steps = (L.nt + 1 + lv - 1) / lv;
    return dim3((unsigned)((P + 255) / 256), (unsigned)(steps < 65535 ? steps : 65535));
}

void launch_restrict(hipStream_t s, const Level& F, const Level& C, int prec, const void* rf,
                     void* bc) {
    const double inv = 1.0 / (C.nx + 1);
    const long long Pf = (long long)(F.nx + 1) * (F.ny + 1);
    const size_t es = prec == 0 ? 8 : 4;
    if (C.how == 1 && F.nx == 2 * C.nx && F.ny == 2 * C.ny &&
        (long long)(C.nt + 1) * Pf * (long long)es < (long long)SW_OOB) {
        // wave form: 31 coarse nodes per wave, chunks of 32 levels (fewer
        // while the grid does not fill the chip)
        const int nseg = (C.nx + 1 + RW_OUT - 1) / RW_OUT;
        const long long waves = (long long)(C.ny + 1) * nseg;
        const unsigned gx = (unsigned)((waves + 3) / 4);
        int nchunk = 32;
        while (nchunk > RW_LV && (long long)gx * ((C.nt + 1 + nchunk - 1) / nchunk) < 2048)
            nchunk /= 2;
        const dim3 grid(gx, (unsigned)((C.nt + 1 + nchunk - 1) / nchunk));
        if (prec == 0)
            hipLaunchKernelGGL(k_restrict_wave<double>, grid, dim3(256), 0, s, F.nx, F.ny, C.nt,
                               C.nx, C.ny, nseg, nchunk, F.mask, (const double*)rf, (double*)bc);
        else
            hipLaunchKernelGGL(k_restrict_wave<float>, grid, dim3(256), 0, s, F.nx, F.ny, C.nt,
                               C.nx, C.ny, nseg, nchunk, F.mask, (const float*)rf, (float*)bc);
        return;
    }
    if (C.how == 1) {
        const dim3 grid = level_grid(C, TR_LV);
        if (prec == 0)
            hipLaunchKernelGGL(k_restrict_space<double>, grid, dim3(256), 0, s, F.nx, F.ny, C.nt,
                               C.nx, C.ny, inv, F.mask, (const double*)rf, (double*)bc);
        else
            hipLaunchKernelGGL(k_restrict_space<float>, grid, dim3(256), 0, s, F.nx, F.ny, C.nt,
                               C.nx, C.ny, inv, F.mask, (const float*)rf, (float*)bc);
        return;
    }
    const dim3 grid = plane_grid(C);
#define RS_LAUNCH(T, H)                                                                         \
    hipLaunchKernelGGL((k_restrict<T, H>), grid, dim3(256), 0, s, F.nx, F.ny, F.nt, C.nx, C.ny,  \
                       C.nt, inv, F.mask, (const T*)rf, (T*)bc)
    if (prec == 0) {
        if (C.how == 2)
            RS_LAUNCH(double, 2);
        else
            RS_LAUNCH(double, 3);
    } else {
        if (C.how == 2)
            RS_LAUNCH(float, 2);
        else
            RS_LAUNCH(float, 3);
    }
#undef RS_LAUNCH
}

// Prolongation x_f (+)= P_m e_c: zero at fine Dirichlet nodes.
//
// Space semi-coarsening: as the restriction, TP_LV time levels per thread
// and step with every load issued first; the four coarse neighbours are
// loaded without a branch (a missing second one repeats the first) and the
// parity cases selected afterwards.
constexpr int TP_LV = 4;
template <typename T, bool ACC>
__global__ void k_prolong_space(int nxf, int nyf, int nt, int nxc, int nyc, double inv_rowf,
                                const uint8_t* __restrict__ maskf, const T* __restrict__ ec,
                                T* __restrict__ xf) {
    const int rowf = nxf + 1, Pf = rowf * (nyf + 1);
    const long long rowc = nxc + 1, Pc = rowc * (nyc + 1);
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= Pf) return;
    const int j = row_of(r, rowf, inv_rowf), i = r - j * rowf;
    const bool io = i & 1, jo = j & 1;
    const long long c00 = (long long)(j >> 1) * rowc + (i >> 1);
    const long long c01 = c00 + (io ? 1 : 0), c10 = c00 + (jo ? rowc : 0);
    const long long c11 = c10 + (io ? 1 : 0);
    for (int n0 = blockIdx.y * TP_LV; n0 <= nt; n0 += gridDim.y * TP_LV) {
        T a[TP_LV][4], xo[TP_LV];
        uint8_t mk[TP_LV];
#pragma unroll
        for (int u = 0; u < TP_LV; ++u) {
            const int n = min(n0 + u, nt);   // past nt: not stored
            const long long pc = (long long)n * Pc, idx = (long long)n * Pf + r;
            a[u][0] = ec[pc + c00];
            a[u][1] = ec[pc + c01];
            a[u][2] = ec[pc + c10];
            a[u][3] = ec[pc + c11];
            mk[u] = maskf[idx];
            xo[u] = ACC ? xf[idx] : (T)0;
        }
#pragma unroll
        for (int u = 0; u < TP_LV; ++u) {
            if (n0 + u > nt) break;
            const double a00 = (double)a[u][0], a01 = (double)a[u][1];
            const double a10 = (double)a[u][2], a11 = (double)a[u][3];
            const double vx = 0.5 * (a00 + a01), vy = 0.5 * (a00 + a10);
            const double vxy = 0.25 * (a00 + a01 + a10 + a11);
            const double v = mk[u] ? 0.0 : (io ? (jo ? vxy : vx) : (jo ? vy : a00));
            const long long idx = (long long)(n0 + u) * Pf + r;
            xf[idx] = ACC ? (T)((double)xo[u] + v) : (T)v;
        }
    }
}

// Time semi-coarsening (how = 2) and full space-time coarsening (how = 3).
template <typename T, int how>
__global__ void k_prolong(int nxf, int nyf, int ntf, int nxc, int nyc, int ntc,
                          double inv_rowf, const uint8_t* __restrict__ maskf,
                          const T* __restrict__ ec, T* __restrict__ xf, int accumulate) {
    const int rowf = nxf + 1, Pf = rowf * (nyf + 1);
    const long long rowc = nxc + 1, Pc = rowc * (nyc + 1);
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= Pf) return;
    const int j = row_of(r, rowf, inv_rowf), i = r - j * rowf;
    for (int n = blockIdx.y; n <= ntf; n += gridDim.y) {
        const long long idx = (long long)n * Pf + r;
        double v = 0.0;
        const bool dir = maskf[idx] != 0;
        if (!dir) {
            if (how == 2) {
                const int n0 = n >> 1;
                if (!(n & 1))
                    v = (double)ec[(long long)n0 * Pc + r];
                else
                    v = 0.5 * ((double)ec[(long long)n0 * Pc + r] +
                               (double)ec[(long long)(n0 + 1) * Pc + r]);
            } else {   // full: trilinear, one or two coarse nodes per axis
                const int kn = (n & 1) ? 2 : 1, kj = (j & 1) ? 2 : 1, ki = (i & 1) ? 2 : 1;
                const double w = ((n & 1) ? 0.5 : 1.0) * ((j & 1) ? 0.5 : 1.0) * ((i & 1) ? 0.5 : 1.0);
                for (int dn = 0; dn < kn; ++dn)
                    for (int dj = 0; dj < kj; ++dj)
                        for (int di = 0; di < ki; ++di)
                            v += (double)ec[(long long)((n >> 1) + dn) * Pc +
                                            (long long)((j >> 1) + dj) * rowc + (i >> 1) + di];
                v *= w;
            }
        }
        if (accumulate)
            xf[idx] = (T)((double)xf[idx] + v);
        else
            xf[idx] = (T)v;
    }
}

void launch_prolong(hipStream_t s, const Level& F, const Level& C, int prec, const void* ec,
                    void* xf, int accumulate) {
    const double inv = 1.0 / (F.nx + 1);
    if (C.how == 1) {
        const dim3 grid = level_grid(F, TP_LV);
#define PS_LAUNCH(T, A)                                                                        \
    hipLaunchKernelGGL((k_prolong_space<T, A>), grid, dim3(256), 0, s, F.nx, F.ny, F.nt, C.nx,  \
                       C.ny, inv, F.mask, (const T*)ec, (T*)xf)
        if (prec == 0) {
            if (accumulate)
                PS_LAUNCH(double, true);
            else
                PS_LAUNCH(double, false);
        } else {
            if (accumulate)
                PS_LAUNCH(float, true);
            else
                PS_LAUNCH(float, false);
        }
#undef PS_LAUNCH
        return;
    }
    const dim3 grid = plane_grid(F);
#define PL_LAUNCH(T, H)                                                                        \
    hipLaunchKernelGGL((k_prolong<T, H>), grid, dim3(256), 0, s, F.nx, F.ny, F.nt, C.nx, C.ny,   \
                       C.nt, inv, F.mask, (const T*)ec, (T*)xf, accumulate)
    if (prec == 0) {
        if (C.how == 2)
            PL_LAUNCH(double, 2);
        else
            PL_LAUNCH(double, 3);
    } else {
        if (C.how == 2)
            PL_LAUNCH(float, 2);
        else
            PL_LAUNCH(float, 3);
    }
#undef PL_LAUNCH
}

// Coarse Dirichlet mask: a coarse node is Dirichlet when every fine node in the
// support of its prolongation column is Dirichlet (its P_m column is zero).
__global__ void k_coarse_mask(int how, int nxf, int nyf, int ntf, int nxc, int nyc, int ntc,
                              const uint8_t* __restrict__ maskf, uint8_t* __restrict__ maskc) {
    const long long rowc = nxc + 1, Pc = rowc * (nyc + 1);
    const long long Nc = Pc * (ntc + 1);
    const long long rowf = nxf + 1, Pf = rowf * (nyf + 1);
    for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < Nc;
         idx += (long long)gridDim.x * blockDim.x) {
        const int n = (int)(idx / Pc);
        const long long r = idx - n * Pc;
        const int J = (int)(r / rowc), I = (int)(r - (long long)J * rowc);
        bool any_free = false;
        if (how == 1) {
            for (int c = -1; c <= 1; ++c)
                for (int a = -1; a <= 1; ++a) {
                    const int fj = 2 * J + c, fi = 2 * I + a;
                    if (fj < 0 || fj > nyf || fi < 0 || fi > nxf) continue;
                    any_free |= !maskf[(long long)n * Pf + (long long)fj * rowf + fi];
                }
        } else if (how == 2) {
            for (int a = -1; a <= 1; ++a) {
                const int fn = 2 * n + a;
                if (fn < 0 || fn > ntf) continue;
                any_free |= !maskf[(long long)fn * Pf + r];
            }
        } else {
            for (int d = -1; d <= 1; ++d)
                for (int c = -1; c <= 1; ++c)
                    for (int a = -1; a <= 1; ++a) {
                        const int fn = 2 * n + d, fj = 2 * J + c, fi = 2 * I + a;
                        if (fn < 0 || fn > ntf || fj < 0 || fj > nyf || fi < 0 || fi > nxf) continue;
                        any_free |= !maskf[(long long)fn * Pf + (long long)fj * rowf + fi];
                    }
        }
        maskc[idx] = any_free ? 0 : 1;
    }
}

void launch_coarse_mask(hipStream_t s, const Level& F, const Level& C) {
    hipLaunchKernelGGL(k_coarse_mask, dim3(grid_for(C.nn)), dim3(256), 0, s, C.how, F.nx, F.ny,
                       F.nt, C.nx, C.ny, C.nt, F.mask, C.mask);
}

// ---------------------------------------------------------------------------
// Galerkin by probing.  Colour c = (cn, cj, ci) in {0,1,2}^3 marks the coarse
// nodes with (n mod 3, j mod 3, i mod 3) = c.  Two nodes of one colour are at
// least 3 apart in some direction, so within the 3x3x3 stencil of any row at
// most one of them appears: y = P_m^T A P_m e_c read at row C is the entry of
// the unique offset d that lands on colour c.
__global__ void k_probe_fill(int nx, int ny, int nt, int color, const uint8_t* __restrict__ mask,
                             double* __restrict__ e) {
    const long long row = nx + 1, P = row * (ny + 1), N = P * (nt + 1);
    const int ci = color % 3, cj = (color / 3) % 3, cn = color / 9;
    for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < N;
         idx += (long long)gridDim.x * blockDim.x) {
        const int n = (int)(idx / P);
        const long long r = idx - n * P;
        const int j = (int)(r / row), i = (int)(r - (long long)j * row);
        e[idx] = (i % 3 == ci && j % 3 == cj && n % 3 == cn && !(mask && mask[idx])) ? 1.0 : 0.0;
    }
}

void launch_probe_fill(hipStream_t s, const Level& C, int color, double* e) {
    hipLaunchKernelGGL(k_probe_fill, dim3(grid_for(C.nn)), dim3(256), 0, s, C.nx, C.ny, C.nt,
                       color, C.mask, e);
}

__device__ __forceinline__ int off_to_colour(int v, int c) {
    // offset d in {-1, 0, 1} with (v + d) mod 3 == c
    const int d = ((c - v % 3) % 3 + 3) % 3;   // 0, 1, 2
    return d == 2 ? -1 : d;
}

// Writes the full (uncompressed, nplanes = nt+1) stencil entry of colour c.
__global__ void k_probe_extract(int nx, int ny, int nt, int color, const double* __restrict__ yc,
                                double* __restrict__ st) {
    const long long row = nx + 1, P = row * (ny + 1), N = P * (nt + 1);
    const int ci = color % 3, cj = (color / 3) % 3, cn = color / 9;
    for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < N;
         idx += (long long)gridDim.x * blockDim.x) {
        const int n = (int)(idx / P);
        const long long r = idx - n * P;
        const int j = (int)(r / row), i = (int)(r - (long long)j * row);
        const int di = off_to_colour(i, ci), dj = off_to_colour(j, cj), dn = off_to_colour(n, cn);
        const bool inside = i + di >= 0 && i + di <= nx && j + dj >= 0 && j + dj <= ny &&
                            n + dn >= 0 && n + dn <= nt;
        const int d = (dn + 1) * 9 + (dj + 1) * 3 + (di + 1);
        st[(long long)d * N + idx] = inside ? yc[idx] : 0.0;
    }
}

void launch_probe_extract(hipStream_t s, const Level& C, int color, const double* yc, double* st) {
    hipLaunchKernelGGL(k_probe_extract, dim3(grid_for(C.nn)), dim3(256), 0, s, C.nx, C.ny, C.nt,
                       color, yc, st);
}

// Identity rows on coarse Dirichlet nodes (their probed rows are zero).
__global__ void k_identity_rows(long long N, const uint8_t* __restrict__ mask,
                                double* __restrict__ st) {
    for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < N;
         idx += (long long)gridDim.x * blockDim.x) {
        if (!mask[idx]) continue;
        for (int d = 0; d < 27; ++d) st[(long long)d * N + idx] = d == 13 ? 1.0 : 0.0;
    }
}

void launch_identity_rows(hipStream_t s, const Level& C, double* st) {
    hipLaunchKernelGGL(k_identity_rows, dim3(grid_for(C.nn)), dim3(256), 0, s, C.nn, C.mask, st);
}

// neq[n] = 1 when time level n of the uncompressed stencil differs (bitwise)
// from time level n-1.
__global__ void k_plane_equal(int nx, int ny, int nt, const double* __restrict__ st,
                              int* __restrict__ neq) {
    const long long P = (long long)(nx + 1) * (ny + 1), N = P * (nt + 1);
    const int n = blockIdx.y + 1;
    bool diff = false;
    for (long long r = blockIdx.x * (long long)blockDim.x + threadIdx.x; r < P;
         r += (long long)gridDim.x * blockDim.x) {
        for (int d = 0; d < 27; ++d) {
            const double a = st[(long long)d * N + (long long)n * P + r];
            const double b = st[(long long)d * N + (long long)(n - 1) * P + r];
            diff |= __double_as_longlong(a) != __double_as_longlong(b);
        }
    }
    if (__any(diff) && (threadIdx.x % 64) == 0) atomicOr(&neq[n], 1);
}

void launch_plane_equal(hipStream_t s, const Level& C, const double* st, int* neq) {
    if (C.nt < 1) return;
    const long long P = (long long)(C.nx + 1) * (C.ny + 1);
    unsigned gx = grid_for(P, 256, 64);
    hipLaunchKernelGGL(k_plane_equal, dim3(gx, C.nt), dim3(256), 0, s, C.nx, C.ny, C.nt, st, neq);
}

// Copy one contiguous block of P values (one stencil entry of one time level).
__global__ void k_plane_move(long long P, const double* __restrict__ in, double* __restrict__ out) {
    for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < P;
         t += (long long)gridDim.x * blockDim.x)
        out[t] = in[t];
}

// In-place compaction: the distinct planes are moved one entry d at a time in
// increasing d, so no source is overwritten before it is read (the compressed
// position of (d, p) never exceeds its uncompressed position).
void launch_plane_compact(hipStream_t s, const Level& C, double* st, const int* src_plane,
                          int ndistinct) {
    const long long P = (long long)(C.nx + 1) * (C.ny + 1);
    const int nold = C.nt + 1;
    for (int d = 0; d < 27; ++d)
        for (int p = 0; p < ndistinct; ++p) {
            const long long from = (long long)d * nold * P + (long long)src_plane[p] * P;
            const long long to = (long long)d * ndistinct * P + (long long)p * P;
            if (from == to) continue;
            hipLaunchKernelGGL(k_plane_move, dim3(grid_for(P)), dim3(256), 0, s, P, st + from,
                               st + to);
        }
}

// Expand a compressed stencil to [27][nt+1][ny+1][nx+1].
__global__ void k_stencil_expand(int nx, int ny, int nt, int nplanes, const double* __restrict__ st,
                                 const int* __restrict__ pmap, double* __restrict__ out) {
    const long long P = (long long)(nx + 1) * (ny + 1), N = P * (nt + 1);
    for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < 27 * N;
         t += (long long)gridDim.x * blockDim.x) {
        const int d = (int)(t / N);
        const long long idx = t - (long long)d * N;
        const int n = (int)(idx / P);
        const long long r = idx - (long long)n * P;
        out[t] = st[(long long)d * nplanes * P + (long long)pmap[n] * P + r];
    }
}

void launch_stencil_expand(hipStream_t s, const Level& L, double* out) {
    hipLaunchKernelGGL(k_stencil_expand, dim3(grid_for(27 * L.nn)), dim3(256), 0, s, L.nx, L.ny,
                       L.nt, L.nplanes, L.st64, L.plane_map, out);
}

// Inverse diagonal from the centre entry (d = 13).
__global__ void k_stencil_invdiag(int nx, int ny, int nt, int nplanes,
                                  const double* __restrict__ st, const int* __restrict__ pmap,
                                  double* __restrict__ invd64, float* __restrict__ invd32) {
    const long long row = nx + 1, P = row * (ny + 1), N = P * (nt + 1);
    for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < N;
         idx += (long long)gridDim.x * blockDim.x) {
        const int n = (int)(idx / P);
        const long long r = idx - n * P;
        const double d = st[(long long)13 * nplanes * P + (long long)pmap[n] * P + r];
        const double v = 1.0 / d;
        invd64[idx] = v;
        if (invd32) invd32[idx] = (float)v;
    }
}

void launch_stencil_invdiag(hipStream_t s, const Level& L, double* invd64, float* invd32) {
    hipLaunchKernelGGL(k_stencil_invdiag, dim3(grid_for(L.nn)), dim3(256), 0, s, L.nx, L.ny, L.nt,
                       L.nplanes, L.st64, L.plane_map, invd64, invd32);
}

// Symmetric FP32 / BF16 copies of the FP64 stencil (layout in
// stencil_core.hpp), with the compensated FP32 centres of the BF16 form: per
// plane, node r and time offset g = dn + 1, over the nine values v_q the apply
// uses (v_q = A_{g,q}(r) for q >= 4, A_{g,8-q}(r + off_q) for q < 4 and an
// in-domain neighbour):
//     cen[g] = sum_q v_q - sum_{q != 4} bf16(v_q).
__global__ void k_stencil_sym(int nx, int ny, int nplanes, const double* __restrict__ st,
                              float* __restrict__ o32, uint16_t* __restrict__ o16,
                              float* __restrict__ cen) {
    const int rowp = nx + 1;
    const long long P = (long long)rowp * (ny + 1);
    const long long DS = P * nplanes;
    for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < DS;
         t += (long long)gridDim.x * blockDim.x) {
        const int pl = (int)(t / P);
        const long long r = t - (long long)pl * P;
        const int j = (int)(r / rowp), i = (int)(r - (long long)j * rowp);
        const double* sp = st + (long long)pl * P;
        for (int g = 0; g < 3; ++g) {
            double sum = 0.0, rounded = 0.0;
            for (int q = 0; q < 9; ++q) {
                double v;
                if (q >= 4) {
                    v = sp[(long long)(g * 9 + q) * DS + r];
                    if (o32) o32[(long long)(g * 5 + q - 4) * DS + t] = (float)v;
                    if (o16 && q > 4) o16[(long long)(g * 4 + q - 5) * DS + t] = f32_to_bf16((float)v);
                } else {
                    const int di = q % 3 - 1, dj = q / 3 - 1;
                    if (i + di < 0 || i + di > nx || j + dj < 0 || j + dj > ny) continue;
                    v = sp[(long long)(g * 9 + 8 - q) * DS + r + dj * rowp + di];
                }
                sum += v;
                if (q != 4) rounded += (double)bf16_to_f32(f32_to_bf16((float)v));
            }
            if (cen) cen[(long long)g * DS + t] = (float)(sum - rounded);
        }
    }
}

void launch_stencil_cast(hipStream_t s, const Level& L, float* st32, uint16_t* st16) {
    const long long m = (long long)L.nplanes * (L.nx + 1) * (L.ny + 1);
    hipLaunchKernelGGL(k_stencil_sym, dim3(grid_for(m)), dim3(256), 0, s, L.nx, L.ny, L.nplanes,
                       L.st64, st32, st16, st16 ? L.cen32 : nullptr);
}

// ---------------------------------------------------------------------------
template <typename A, typename B>
__global__ void k_cast(long long n, const A* __restrict__ in, B* __restrict__ out,
                       const double* __restrict__ scale) {
    const double sc = scale ? *scale : 1.0;
    for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < n;
         t += (long long)gridDim.x * blockDim.x)
        out[t] = (B)((double)in[t] * sc);
}

void launch_cast(hipStream_t s, long long n, int from, int to, const void* in, void* out,
                 const double* scale) {
    const unsigned nb = grid_for(n);
    if (from == 0 && to == 0)
        hipLaunchKernelGGL((k_cast<double, double>), dim3(nb), dim3(256), 0, s, n,
                           (const double*)in, (double*)out, scale);
    else if (from == 0 && to == 1)
        hipLaunchKernelGGL((k_cast<double, float>), dim3(nb), dim3(256), 0, s, n,
                           (const double*)in, (float*)out, scale);
    else if (from == 1 && to == 0)
        hipLaunchKernelGGL((k_cast<float, double>), dim3(nb), dim3(256), 0, s, n,
                           (const float*)in, (double*)out, scale);
    else
        hipLaunchKernelGGL((k_cast<float, float>), dim3(nb), dim3(256), 0, s, n,
                           (const float*)in, (float*)out, scale);
}

template <typename T>
__global__ void k_fill(long long n, T* __restrict__ p, T v) {
    for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < n;
         t += (long long)gridDim.x * blockDim.x)
        p[t] = v;
}

void launch_fill(hipStream_t s, long long n, int prec, void* p, double v) {
    const unsigned nb = grid_for(n);
    if (prec == 0)
        hipLaunchKernelGGL(k_fill<double>, dim3(nb), dim3(256), 0, s, n, (double*)p, v);
    else if (prec == 1)
        hipLaunchKernelGGL(k_fill<float>, dim3(nb), dim3(256), 0, s, n, (float*)p, (float)v);
    else
        hipLaunchKernelGGL(k_fill<int>, dim3(nb), dim3(256), 0, s, n, (int*)p, (int)v);
}

}  // namespace st
