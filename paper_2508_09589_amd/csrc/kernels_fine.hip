// Fine-level kernels: SIMP coefficients, the matrix-free stabilised space-time
// Q1 operator and its transpose, its diagonal, the consistent load, the density
// sensitivities and the constant-coefficient tensor operator of the filter.
//
// Operator (paper §3.1.1, §3.1.2).  For a dx x dx x dt brick the element matrix
// is k_e A + C_e B with A = Mt (x) Kq and B = U (x) Mq, where Kq is the 2-D
// bilinear stiffness (independent of dx for square elements), Mq the 2-D mass,
// Mt = dt/6 [[2,1],[1,2]] and U = [[0,0],[-1,1]] (the capacity term plus the
// artificial time diffusion C dt/2 collapses to this upwind block).  Summing
// slab s (elements between time levels s and s+1) gives, with K_s, M_s the
// 2-D operators weighted by the slab's k and C,
//   y_s     += dt/6 K_s (2 x_s + x_{s+1})
//   y_{s+1} += dt/6 K_s (x_s + 2 x_{s+1}) + M_s (x_{s+1} - x_s)
// and for the transpose the capacity part moves to  y_s -= M_s x_{s+1},
// y_{s+1} += M_s x_{s+1}.  A workgroup owns a tile of (i, j) node columns
// and marches through a chunk of time levels, so every x value is loaded once
// per chunk from its plane and the stiffness of the lower plane is reused when
// the coefficients do not change in time.  Dirichlet nodes: inputs are masked
// to zero and rows become identity rows (N J N + I - N).
#include <type_traits>

#include "st_internal.hpp"

namespace st {

__device__ __forceinline__ bool on_patch(const PatchSet& P, int nx, int ny, int i, int j) {
    bool r = false;
#pragma unroll
    for (int q = 0; q < ST_MAX_PATCHES; ++q) {
        if (q < P.n) {
            const int e = P.edge[q];
            const int lo = P.lo[q], hi = P.hi[q];
            if (e == ST_EDGE_X1_LO) r |= (i == 0 && j >= lo && j <= hi);
            else if (e == ST_EDGE_X1_HI) r |= (i == nx && j >= lo && j <= hi);
            else if (e == ST_EDGE_X2_LO) r |= (j == 0 && i >= lo && i <= hi);
            else r |= (j == ny && i >= lo && i <= hi);
        }
    }
    return r;
}

// ---------------------------------------------------------------------------
// SIMP (§2.2): k, C and their derivatives per element.
__global__ void k_simp(long long ne, const double* __restrict__ rho, double kins, double kcon,
                       double pk, double cins, double ccon, double pc, double* __restrict__ k,
                       double* __restrict__ c, double* __restrict__ dk, double* __restrict__ dc,
                       float* __restrict__ k32, float* __restrict__ c32, int cuniform) {
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < ne;
         e += (long long)gridDim.x * blockDim.x) {
        const double r = rho[e];
        const double kv = kins + (kcon - kins) * pow(r, pk);
        k[e] = kv;
        dk[e] = pk * (kcon - kins) * pow(r, pk - 1.0);
        if (k32) k32[e] = (float)kv;
        if (!cuniform) {
            const double cv = cins + (ccon - cins) * pow(r, pc);
            c[e] = cv;
            dc[e] = pc * (ccon - cins) * pow(r, pc - 1.0);
            if (c32) c32[e] = (float)cv;
        }
    }
}

void launch_simp(hipStream_t s, long long ne, const double* rho, const st_material* m, double* k,
                 double* c, double* dk, double* dc, float* k32, float* c32, int cuniform) {
    long long nb = (ne + 255) / 256;
    if (nb > 65535) nb = 65535;
    hipLaunchKernelGGL(k_simp, dim3((unsigned)nb), dim3(256), 0, s, ne, rho, m->k_ins, m->k_con,
                       m->p_k, m->c_ins, m->c_con, m->p_c, k, c, dk, dc, k32, c32, cuniform);
}

// ---------------------------------------------------------------------------
// Matrix-free apply, LDS-tiled.
// A workgroup of 64 x 4 threads owns a tile of 64 node columns x 8 node rows
// and marches through a chunk of time levels.  Per level the tile's x window
// (10 x 66 values, halo included) and per slab its coefficient window (9 x 65
// elements) are loaded once, coalesced, into LDS; the loads of level s + 2 and
// slab s + 2 are issued before the arithmetic of slab s, and those of b of
// level s + 1 after its outputs, so every load has one iteration to
// arrive (three x buffers, two coefficient buffers, one barrier per level).  A thread reads its 3 x 4 stencil window of the two levels of a slab
// from LDS and produces 2 outputs of one column.  Workgroups are numbered so
// that the eight XCDs (separate L2 caches) each get a contiguous range of
// tiles: the halo rows a tile shares with its neighbours are then read from
// the same L2.
// Raw buffer access: base and size in a resource held in scalar registers,
// 32-bit byte offsets per lane (no 64-bit address arithmetic per load).  One
// resource per array serves the whole launch: it spans the whole array, and
// the time level (or slab) is selected by the scalar offset operand, which the
// range check includes.  The offsets need arrays below 4 GiB (checked on the
// host).  An access at or past the resource's size reads zero without a
// memory access.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void* p, long long bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}
template <typename T>
__device__ __forceinline__ T buf_ld(__amdgpu_buffer_rsrc_t r, unsigned off, unsigned soff);
template <>
__device__ __forceinline__ float buf_ld<float>(__amdgpu_buffer_rsrc_t r, unsigned off, unsigned soff) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, soff, 0));
}
template <>
__device__ __forceinline__ double buf_ld<double>(__amdgpu_buffer_rsrc_t r, unsigned off, unsigned soff) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, soff, 0));
}
template <typename T>
__device__ __forceinline__ void buf_st(T v, __amdgpu_buffer_rsrc_t r, unsigned off, unsigned soff);
template <>
__device__ __forceinline__ void buf_st<float>(float v, __amdgpu_buffer_rsrc_t r, unsigned off,
                                              unsigned soff) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, off, soff, 0);
}
template <>
__device__ __forceinline__ void buf_st<double>(double v, __amdgpu_buffer_rsrc_t r, unsigned off,
                                               unsigned soff) {
    typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, off, soff, 0);
}
// Reciprocal of a Jacobi diagonal: the hardware estimate (1 ulp) in FP32, a
// correctly rounded division in FP64.
__device__ __forceinline__ float recip(float d) { return __builtin_amdgcn_rcpf(d); }
__device__ __forceinline__ double recip(double d) { return 1.0 / d; }
// Scalar offsets must be wave-uniform values in scalar registers.
__device__ __forceinline__ unsigned uniform(unsigned v) { return __builtin_amdgcn_readfirstlane(v); }
// Keeps a value computed before a loop from being recomputed inside it.
template <typename T> __device__ __forceinline__ void pin_value(T& v) { asm volatile("" : "+v"(v)); }

constexpr int FA_TX = 64, FA_RY = 2, FA_TY = 4 * FA_RY;
constexpr int FA_DEPTH_TCONST = 3;   // load distance (loop iterations), see k_fine_apply

template <typename TIN, typename TOUT, typename TC, bool TRANS, bool TCONST, bool CUNI, bool SMOOTH>
__global__ __launch_bounds__(256) void k_fine_apply(
    FineGeom g, const TC* __restrict__ kc, const TC* __restrict__ cc, const TIN* __restrict__ x,
    TOUT* __restrict__ y, const TOUT* __restrict__ b, int jacobi,
    const double* __restrict__ scale, const int* __restrict__ skip, int gx, int gy, int nchunk,
    int per_xcd, int mask_in, int dir_rows) {
    constexpr int RY = FA_RY, TX = FA_TX, TY = FA_TY;
    constexpr int WX = TX + 2, NW = WX * (TY + 2);            // x window
    constexpr int EX = TX + 1, NE = EX * (TY + 1);            // element window
    constexpr int LW = (NW + 255) / 256, LE = (NE + 255) / 256;
    __shared__ TC xs[3][NW];
    __shared__ TC ks[2][NE];
    __shared__ TC cs[CUNI ? 1 : 2][CUNI ? 1 : NE];

    if (skip && *skip) return;
    // SMOOTH: y = scale D^{-1} A x off the Dirichlet rows, scale x on them
    // (the smoother's basis vectors); the scale goes into the reciprocal
    // diagonal once instead of into every output.
    if (SMOOTH) {
        jacobi = 1;
        b = nullptr;
        dir_rows = 1;
    }
    // XCD-aware tile order: hardware workgroup b runs on XCD b % 8.
    const int bid = blockIdx.x;
    const int lin = (bid & 7) * per_xcd + (bid >> 3);
    const int tiles = gx * gy;
    const int bz = lin / tiles;
    const int rem = lin - bz * tiles;
    const int by = rem / gx, bx = rem - by * gx;
    const int nx = g.nx, ny = g.ny, nt = g.nt;
    const int n0 = (int)uniform((unsigned)(bz * nchunk));
    if (n0 > nt) return;                      // uniform over the workgroup
    const int n1 = (int)uniform((unsigned)min(n0 + nchunk, nt + 1));
    const int tx = threadIdx.x, ry0 = threadIdx.y * RY;
    const int tid = threadIdx.y * 64 + tx;
    const int i0 = bx * TX, jb = by * TY;
    const int rowp = nx + 1;
    const long long P = (long long)rowp * (ny + 1);
    const long long slab = (long long)nx * ny;

    // Byte offsets of the window entries tid + 256 r this thread loads; dead
    // entries (outside the grid or, with mask_in, on a patch) load offset 0
    // and are replaced by zero.
    unsigned xlive = 0, elive = 0;
    unsigned xo[LW], eo[LE];
#pragma unroll
    for (int r = 0; r < LW; ++r) {
        const int e = tid + 256 * r;
        const int row = e / WX, col = e - (e / WX) * WX;
        const int gi = i0 - 1 + col, gj = jb - 1 + row;
        const bool live = e < NW && gi >= 0 && gi <= nx && gj >= 0 && gj <= ny &&
                          !(mask_in && on_patch(g.patches, nx, ny, gi, gj));
        if (live) xlive |= 1u << r;
        xo[r] = live ? (unsigned)(gj * rowp + gi) * (unsigned)sizeof(TIN) : 0u;
    }
#pragma unroll
    for (int r = 0; r < LE; ++r) {
        const int e = tid + 256 * r;
        const int row = e / EX, col = e - (e / EX) * EX;
        const int ei = i0 - 1 + col, ej = jb - 1 + row;
        const bool live = e < NE && ei >= 0 && ei < nx && ej >= 0 && ej < ny;
        if (live) elive |= 1u << r;
        eo[r] = live ? (unsigned)(ej * nx + ei) * (unsigned)sizeof(TC) : 0u;
    }
    // Loads run DEPTH loop iterations ahead, in DEPTH register sets used by
    // iterations in turn (the loop is unrolled so that every set is named
    // statically).  Three iterations of cover for the FP32 time-constant
    // kernels (measured on the large grid: 731 us with one, 617 with two,
    // 605 with three, 601 with four); the time-varying and FP64 kernels
    // hold more registers per set and keep one (more sets cost them more
    // occupancy than they hide latency).
    constexpr int DEPTH = (TCONST && sizeof(TC) == 4) ? FA_DEPTH_TCONST : 1;
    TC pk[DEPTH][LE], pc[DEPTH][CUNI ? 1 : LE];
    // One resource per array for the launch (see buf_rsrc).
    const unsigned pin = (unsigned)(P * (long long)sizeof(TIN));
    const unsigned pout = (unsigned)(P * (long long)sizeof(TOUT));
    const unsigned pcoef = TCONST ? 0u : (unsigned)(slab * (long long)sizeof(TC));
    const long long levels = nt + 1, cslabs = TCONST ? 1 : nt;
    const auto rsx = buf_rsrc(x, levels * P * (long long)sizeof(TIN));
    const auto rsy = buf_rsrc(y, levels * P * (long long)sizeof(TOUT));
    const auto rsb = buf_rsrc(b, b ? levels * P * (long long)sizeof(TOUT) : 0);
    const auto rsk = buf_rsrc(kc, cslabs * slab * (long long)sizeof(TC));
    const auto rsc = buf_rsrc(cc, CUNI ? 0 : cslabs * slab * (long long)sizeof(TC));
    // The loaded values are only touched when they are written to LDS one
    // iteration later (dead entries are zeroed there), so no wait for the
    // loads is placed before the arithmetic in between.
    TIN lx[DEPTH][LW];
    auto fetch_x = [&](int n, int q) {
        const unsigned so = uniform((unsigned)n * pin);
#pragma unroll
        for (int r = 0; r < LW; ++r) lx[q][r] = buf_ld<TIN>(rsx, xo[r], so);
    };
    auto put_x = [&](int n, int q) {
        TC* d = xs[n % 3];
        const unsigned live = (mask_in && g.ic_dir && n == 0) ? 0u : xlive;
#pragma unroll
        for (int r = 0; r < LW; ++r)
            if (tid + 256 * r < NW) d[tid + 256 * r] = ((live >> r) & 1u) ? (TC)lx[q][r] : (TC)0;
    };
    auto fetch_c = [&](int s, int q) {
        const unsigned so = TCONST ? 0u : uniform((unsigned)s * pcoef);
#pragma unroll
        for (int r = 0; r < LE; ++r) {
            pk[q][r] = buf_ld<TC>(rsk, eo[r], so);
            if (!CUNI) pc[q][r] = buf_ld<TC>(rsc, eo[r], so);
        }
    };
    auto put_c = [&](int s, int q) {
#pragma unroll
        for (int r = 0; r < LE; ++r)
            if (tid + 256 * r < NE) {
                const bool v = (elive >> r) & 1u;
                ks[s & 1][tid + 256 * r] = v ? pk[q][r] : (TC)0;
                if (!CUNI) cs[s & 1][tid + 256 * r] = v ? pc[q][r] : (TC)0;
            }
    };
    // Capacity of the elements around this thread's nodes when it is uniform.
    unsigned cval = 0;
    if (CUNI) {
#pragma unroll
        for (int m = 0; m < RY + 1; ++m)
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const int ei = i0 + tx + c - 1, ej = jb + ry0 + m - 1;
                if (ei >= 0 && ei < nx && ej >= 0 && ej < ny) cval |= 1u << (m * 2 + c);
            }
    }
    TC ke[RY + 1][2], ce[RY + 1][2];
    // time-constant coefficients are read once: the time-step and mass
    // factors go into them there instead of into every level's products
    const TC fk = TCONST ? (TC)g.dt6 : (TC)1, fc = TCONST ? (TC)g.mw : (TC)1;
    auto read_c = [&](int s) {
#pragma unroll
        for (int m = 0; m < RY + 1; ++m)
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                ke[m][c] = fk * ks[s & 1][(ry0 + m) * EX + tx + c];
                ce[m][c] = fc * (CUNI ? (((cval >> (m * 2 + c)) & 1u) ? (TC)g.c0 : (TC)0)
                                      : cs[CUNI ? 0 : (s & 1)][CUNI ? 0 : (ry0 + m) * EX + tx + c]);
            }
    };
    auto read_x = [&](int n, TC u[RY + 2][3]) {
        const TC* sx = xs[n % 3];
#pragma unroll
        for (int m = 0; m < RY + 2; ++m)
#pragma unroll
            for (int c = 0; c < 3; ++c) u[m][c] = sx[(ry0 + m) * WX + tx + c];
    };

    // time-step and mass factors still to apply (1 where read_c did)
    const TC kt = TCONST ? (TC)1 : (TC)g.dt6;
    const TC mw = TCONST ? (TC)1 : (TC)g.mw;
    const TC sc = scale ? (TC)(*scale) : (TC)1;
    // 6 * stiffness and 36/dx^2 * mass at row m of the window.
    auto stiff = [&](const TC u[RY + 2][3], int m) -> TC {
        const TC kSW = ke[m][0], kSE = ke[m][1], kNW = ke[m + 1][0], kNE = ke[m + 1][1];
        TC v = (TC)4 * u[m + 1][1] * (kSW + kSE + kNW + kNE);
        v -= u[m + 1][0] * (kSW + kNW);
        v -= u[m + 1][2] * (kSE + kNE);
        v -= u[m][1] * (kSW + kSE);
        v -= u[m + 2][1] * (kNW + kNE);
        v -= (TC)2 * (kSW * u[m][0] + kSE * u[m][2] + kNW * u[m + 2][0] + kNE * u[m + 2][2]);
        return v;
    };
    auto mass = [&](const TC u[RY + 2][3], int m) -> TC {
        const TC cSW = ce[m][0], cSE = ce[m][1], cNW = ce[m + 1][0], cNE = ce[m + 1][1];
        // the factor 2 goes onto the coefficient sums (the same exact
        // scaling; with time-constant coefficients they are loop-invariant)
        TC v = (TC)4 * u[m + 1][1] * (cSW + cSE + cNW + cNE);
        v += u[m + 1][0] * ((TC)2 * (cSW + cNW));
        v += u[m + 1][2] * ((TC)2 * (cSE + cNE));
        v += u[m][1] * ((TC)2 * (cSW + cSE));
        v += u[m + 2][1] * ((TC)2 * (cNW + cNE));
        v += cSW * u[m][0] + cSE * u[m][2] + cNW * u[m + 2][0] + cNE * u[m + 2][2];
        return v;
    };

    // Own outputs: column i, rows jb + ry0 + m.
    const int i = i0 + tx;
    unsigned own = 0, opatch = 0;
#pragma unroll
    for (int m = 0; m < RY; ++m) {
        const int j = jb + ry0 + m;
        if (i <= nx && j <= ny) {
            own |= 1u << m;
            if (on_patch(g.patches, nx, ny, i, j)) opatch |= 1u << m;
        }
    }
    // Byte offsets (within a level) of the own outputs; only owned rows are
    // loaded or stored.
    unsigned oo[RY];
#pragma unroll
    for (int m = 0; m < RY; ++m) oo[m] = ((own >> m) & 1u) ? (unsigned)((jb + ry0 + m) * rowp + i) : 0u;
    // b and (Dirichlet rows) x of the own outputs of one level, loaded an
    // iteration before they are used.
    // Every load is issued unconditionally (straight-line code lets the
    // compiler wait for exactly the loads a use needs): an absent b is a
    // zero-size buffer, and a row that is not a Dirichlet row reads x at an
    // offset past the end of the buffer -- both read as zero without a memory
    // access.
    TOUT bv[DEPTH][RY];
    TIN xd[DEPTH][RY];
    constexpr unsigned OOB = 0x7FFFFFF0u;
    auto fetch_bd = [&](int n, int q) {
        const unsigned sob = uniform((unsigned)n * pout);
        // x of the Dirichlet rows: a resource over level n alone, so that
        // the rows that are not Dirichlet rows read past its end (zero, no
        // memory access) whatever the level
        const auto rxn = buf_rsrc(x + (long long)n * P, P * (long long)sizeof(TIN));
        const bool ic = dir_rows && g.ic_dir && n == 0;
#pragma unroll
        for (int m = 0; m < RY; ++m) {
            bv[q][m] = buf_ld<TOUT>(rsb, oo[m] * (unsigned)sizeof(TOUT), sob);
            const bool dr = ic || (dir_rows && ((opatch >> m) & 1u));
            xd[q][m] = buf_ld<TIN>(rxn, dr ? oo[m] * (unsigned)sizeof(TIN) : OOB, 0u);
        }
    };
    // jacobi: the output is scaled by the inverse diagonal of the operator,
    // formed here from the coefficients already staged for the apply (per
    // element A_aa = 2 dt / 9 k and, on the element's upper time face,
    // B_aa = dx^2 / 9 C; App. A) instead of being streamed from memory:
    //   diag(s) = 8 kt (Sk(s - 1) + Sk(s)) + 4 mw Sc(s - 1),
    // Sk, Sc = sums over the four elements around the node in a slab; a
    // Dirichlet row has the unit diagonal.
    // rdiag: the reciprocal of that diagonal.
    auto emit = [&](int n, int m, TC v, TC rdiag, int q) {
        if (!((own >> m) & 1u)) return;
        const bool dir = dir_rows && ((g.ic_dir && n == 0) || ((opatch >> m) & 1u));
        if (SMOOTH) {
            // rdiag carries the scale already
            const TC val = dir ? (TC)xd[q][m] * sc : v * rdiag;
            buf_st<TOUT>((TOUT)val, rsy, oo[m] * (unsigned)sizeof(TOUT), uniform((unsigned)n * pout));
            return;
        }
        TC val = dir ? (TC)xd[q][m] : v;
        if (b) val = (TC)bv[q][m] - val;
        if (jacobi && !dir) val *= rdiag;
        buf_st<TOUT>((TOUT)(val * sc), rsy, oo[m] * (unsigned)sizeof(TOUT), uniform((unsigned)n * pout));
    };

    const int sa = max(n0 - 1, 0);
    const int sb = min(n1 - 1, nt - 1);
    TC ulo[RY + 2][3], uhi[RY + 2][3];
    TC Plo[RY], Rlo[RY], acc[RY], dacc[RY];
    // Iteration s of the loop puts level s + 1 (and slab s + 1) into LDS from
    // register set (s - sa) % DEPTH, then reloads that set with level (slab)
    // s + 1 + DEPTH; it emits level s with b and Dirichlet x from the same
    // set, loaded DEPTH iterations before, and then loads level s + DEPTH
    // into it.  Indices past the chunk's end load the last level / slab again
    // (cache hits that keep the loop free of branches around loads).
    const int xl = sb + 1, cl = sb;
    fetch_x(sa, 0);
    fetch_c(sa, 0);
    put_x(sa, 0);
    put_c(sa, 0);
#pragma unroll
    for (int d = 0; d < DEPTH; ++d) {
        fetch_x(min(sa + 1 + d, xl), d);
        if (!TCONST) fetch_c(min(sa + 1 + d, cl), d);
        fetch_bd(min(sa + d, xl), d);
    }
    __syncthreads();
    read_c(sa);
#pragma unroll
    for (int m = 0; m < RY; ++m) {
        acc[m] = 0;
        dacc[m] = 0;
        Plo[m] = 0;
        Rlo[m] = 0;
    }
    // Time-constant coefficients: the diagonal of a row is the same on every
    // level but the first (no slab below) and the last (none above).
    TC rmid[RY], rfirst[RY], rlast[RY];
    if (TCONST) {
        read_x(sa, ulo);
#pragma unroll
        for (int m = 0; m < RY; ++m) {
            Plo[m] = kt * stiff(ulo, m);
            Rlo[m] = mw * mass(ulo, m);
            const TC dl = (TC)8 * kt * (ke[m][0] + ke[m][1] + ke[m + 1][0] + ke[m + 1][1]);
            const TC du = (TC)4 * mw * (ce[m][0] + ce[m][1] + ce[m + 1][0] + ce[m + 1][1]);
            rmid[m] = (SMOOTH ? sc : (TC)1) / (dl + dl + du);
            rfirst[m] = (SMOOTH ? sc : (TC)1) / dl;
            rlast[m] = (SMOOTH ? sc : (TC)1) / (dl + du);
            pin_value(rmid[m]);
            pin_value(rfirst[m]);
        }
    }
    auto step = [&](int s, int q) {
        put_x(s + 1, q);
        if (!TCONST && s + 1 <= sb) put_c(s + 1, q);
        __syncthreads();
        fetch_x(min(s + 1 + DEPTH, xl), q);
        if (!TCONST) fetch_c(min(s + 1 + DEPTH, cl), q);
        if (!TCONST) read_x(s, ulo);
        read_x(s + 1, uhi);
#pragma unroll
        for (int m = 0; m < RY; ++m) {
            const TC Pv = TCONST ? Plo[m] : kt * stiff(ulo, m);
            const TC Qv = kt * stiff(uhi, m);
            const TC Sv = mw * mass(uhi, m);
            TC bottom = (TC)2 * Pv + Qv;
            TC top = Pv + (TC)2 * Qv;
            if (TRANS) {
                bottom -= Sv;
                top += Sv;
            } else {
                const TC Rv = TCONST ? Rlo[m] : mw * mass(ulo, m);
                top += Sv - Rv;
            }
            if (TCONST) {
                if (s >= n0) emit(s, m, acc[m] + bottom, s == 0 ? rfirst[m] : rmid[m], q);
                Plo[m] = Qv;
                Rlo[m] = Sv;
            } else {
                const TC sk = ke[m][0] + ke[m][1] + ke[m + 1][0] + ke[m + 1][1];
                const TC sc4 = ce[m][0] + ce[m][1] + ce[m + 1][0] + ce[m + 1][1];
                const TC dlo = (TC)8 * kt * sk;
                const TC rd = SMOOTH ? recip(dacc[m] + dlo) * sc
                                     : (jacobi ? recip(dacc[m] + dlo) : (TC)1);
                if (s >= n0) emit(s, m, acc[m] + bottom, rd, q);
                dacc[m] = dlo + (TC)4 * mw * sc4;
            }
            acc[m] = top;
        }
        if (!TCONST && s + 1 <= sb) read_c(s + 1);
        // b of level s + DEPTH: issued after this level's outputs, so
        // waiting for them never waits for the x / coefficient loads above
        fetch_bd(min(s + DEPTH, xl), q);
    };
    int s = sa;
    for (; s + DEPTH - 1 <= sb; s += DEPTH) {
#pragma unroll
        for (int d = 0; d < DEPTH; ++d) step(s + d, d);
    }
#pragma unroll
    for (int d = 0; d < DEPTH - 1; ++d)
        if (s + d <= sb) step(s + d, d);
    if (sb + 1 == nt && nt >= n0 && nt < n1) {
        // level nt was emitted by no step; its b and x come from the set of
        // the step after the last one
        const int q = (sb + 1 - sa) % DEPTH;
#pragma unroll
        for (int m = 0; m < RY; ++m)
            emit(nt, m, acc[m],
                 TCONST ? rlast[m]
                        : (SMOOTH ? recip(dacc[m]) * sc : (jacobi ? recip(dacc[m]) : (TC)1)),
                 q);
    }
}

template <typename TIN, typename TOUT, typename TC>
static void fine_dispatch(hipStream_t s, const FineGeom& g, const TC* kc, const TC* cc, int trans,
                          const void* x, void* y, const void* b, int jacobi,
                          const double* scale, const int* skip, int mask_in, int dir_rows) {
    const int gx = (g.nx + 1 + FA_TX - 1) / FA_TX, gy = (g.ny + 1 + FA_TY - 1) / FA_TY;
    const long long tiles = (long long)gx * gy;
    // Time levels per workgroup: 32 when the grid is many times the 2048
    // workgroups the chip holds at once (256 CUs x 8); otherwise the fewest
    // chunks that still fill those 2048 slots, split evenly (a grid of 1.4
    // rounds leaves most of the chip idle in its second round), at least 8.
    const int nl = g.nt + 1;
    int nchunk = 32;
    if (tiles * ((nl + 31) / 32) < 4 * 2048) {
        const long long gzw = (2048 + tiles - 1) / tiles;
        nchunk = (int)((nl + gzw - 1) / gzw);
        if (nchunk > 32) nchunk = 32;
        if (nchunk < 8) nchunk = 8;
    }
    const long long gz = (g.nt + 1 + nchunk - 1) / nchunk;
    const long long per_xcd = (tiles * gz + 7) / 8;
    dim3 grid((unsigned)(8 * per_xcd)), block(64, 4);
    const TIN* xi = (const TIN*)x;
    TOUT* yo = (TOUT*)y;
    const TOUT* bi = (const TOUT*)b;
    const int px = (int)per_xcd;
    // The smoother's basis applies (Jacobi-scaled, no b, Dirichlet rows
    // copied) get their own instantiation when input, output and arithmetic
    // share one precision.
    constexpr bool ONE = std::is_same<TIN, TOUT>::value && std::is_same<TIN, TC>::value;
    const bool smooth = ONE && jacobi && !b && dir_rows;
#define FA_LAUNCH(TR, TCN, CU)                                                                 \
    do {                                                                                       \
        if (smooth)                                                                            \
            hipLaunchKernelGGL((k_fine_apply<TIN, TOUT, TC, TR, TCN, CU, ONE>), grid, block, 0, s, \
                               g, kc, cc, xi, yo, bi, jacobi, scale, skip, gx, gy, nchunk, px,     \
                               mask_in, dir_rows);                                             \
        else                                                                                   \
            hipLaunchKernelGGL((k_fine_apply<TIN, TOUT, TC, TR, TCN, CU, false>), grid, block, 0, \
                               s, g, kc, cc, xi, yo, bi, jacobi, scale, skip, gx, gy, nchunk, px,  \
                               mask_in, dir_rows);                                             \
    } while (0)
    const bool cu = g.cuniform != 0;
    if (g.tconst) {
        if (trans) {
            if (cu) FA_LAUNCH(true, true, true); else FA_LAUNCH(true, true, false);
        } else {
            if (cu) FA_LAUNCH(false, true, true); else FA_LAUNCH(false, true, false);
        }
    } else {
        if (trans) {
            if (cu) FA_LAUNCH(true, false, true); else FA_LAUNCH(true, false, false);
        } else {
            if (cu) FA_LAUNCH(false, false, true); else FA_LAUNCH(false, false, false);
        }
    }
#undef FA_LAUNCH
}

// prec_in / prec_out: 0 = double, 1 = float.  compute64: arithmetic and
// coefficients in FP64 (else FP32).
void launch_fine_apply(hipStream_t s, const FineGeom& g, const Coef& cf, int prec_in, int prec_out,
                       int compute64, int trans, const void* x, void* y, const void* b,
                       int jacobi, const double* scale, const int* skip, int mask_in,
                       int dir_rows) {
    if (compute64) {
        if (prec_in == 0 && prec_out == 0)
            fine_dispatch<double, double, double>(s, g, cf.k64, cf.c64, trans, x, y, b, jacobi,
                                                  scale, skip, mask_in, dir_rows);
        else if (prec_in == 1 && prec_out == 0)
            fine_dispatch<float, double, double>(s, g, cf.k64, cf.c64, trans, x, y, b, jacobi, scale,
                                                 skip, mask_in, dir_rows);
        else
            fine_dispatch<double, float, double>(s, g, cf.k64, cf.c64, trans, x, y, b, jacobi, scale,
                                                 skip, mask_in, dir_rows);
    } else {
        fine_dispatch<float, float, float>(s, g, cf.k32, cf.c32, trans, x, y, b, jacobi, scale, skip,
                                           mask_in, dir_rows);
    }
}

// ---------------------------------------------------------------------------
// Diagonal of the fine operator: per element, A_aa = 2 dt / 9 for every node and
// B_aa = dx^2 / 9 for the nodes on the element's upper time face.
__global__ void k_fine_invdiag(FineGeom g, const double* __restrict__ kc,
                               const double* __restrict__ cc, double dx, double dt,
                               double* __restrict__ invd64, float* __restrict__ invd32,
                               uint8_t* __restrict__ mask) {
    const int nx = g.nx, ny = g.ny, nt = g.nt;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (i > nx || j > ny) return;
    const long long P = (long long)(nx + 1) * (ny + 1);
    const long long slab = (long long)nx * ny;
    const bool qv[4] = {i >= 1 && j >= 1, i < nx && j >= 1, i >= 1 && j < ny, i < nx && j < ny};
    const long long qoff[4] = {(long long)(j - 1) * nx + (i - 1), (long long)(j - 1) * nx + i,
                               (long long)j * nx + (i - 1), (long long)j * nx + i};
    const bool patch = on_patch(g.patches, nx, ny, i, j);
    auto sums = [&](int s, double& ks, double& cs) {
        const long long base = g.tconst ? 0 : (long long)s * slab;
        ks = 0;
        cs = 0;
        for (int q = 0; q < 4; ++q)
            if (qv[q]) {
                ks += kc[base + qoff[q]];
                cs += g.cuniform ? g.c0 : cc[base + qoff[q]];
            }
    };
    for (int n = 0; n <= nt; ++n) {
        double kb = 0, cb = 0, ka = 0, ca = 0;
        if (n >= 1) sums(n - 1, kb, cb);
        if (n < nt) sums(n, ka, ca);
        const bool dir = (g.ic_dir && n == 0) || patch;
        const double d = (2.0 * dt / 9.0) * (kb + ka) + (dx * dx / 9.0) * cb;
        const double inv = dir ? 1.0 : 1.0 / d;
        const long long idx = (long long)n * P + (long long)j * (nx + 1) + i;
        invd64[idx] = inv;
        if (invd32) invd32[idx] = (float)inv;
        if (mask) mask[idx] = dir ? 1 : 0;
    }
}

void launch_fine_invdiag(hipStream_t s, const FineGeom& g, const Coef& cf, double dx, double dt,
                         double* invd64, float* invd32, uint8_t* mask) {
    dim3 grid((g.nx + 1 + 63) / 64, g.ny + 1);
    hipLaunchKernelGGL(k_fine_invdiag, grid, dim3(64), 0, s, g, cf.k64, cf.c64, dx, dt, invd64,
                       invd32, mask);
}

// ---------------------------------------------------------------------------
// Consistent load of a uniform source: each element adds q0 V_e / 8 to its nodes.
__global__ void k_load_uniform(FineGeom g, double w, double* __restrict__ f) {
    const int nx = g.nx, ny = g.ny, nt = g.nt;
    const long long P = (long long)(nx + 1) * (ny + 1);
    const long long N = P * (nt + 1);
    for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < N;
         idx += (long long)gridDim.x * blockDim.x) {
        const int n = (int)(idx / P);
        const long long r = idx - n * P;
        const int j = (int)(r / (nx + 1)), i = (int)(r - (long long)j * (nx + 1));
        const int cx = (i == 0 || i == nx) ? 1 : 2;
        const int cy = (j == 0 || j == ny) ? 1 : 2;
        const int ct = (n == 0 || n == nt) ? 1 : 2;
        f[idx] = w * (double)(cx * cy * ct);
    }
}

void launch_load_uniform(hipStream_t s, const FineGeom& g, double q0, double dx, double dt,
                         double* f) {
    const long long N = (long long)(g.nx + 1) * (g.ny + 1) * (g.nt + 1);
    long long nb = (N + 255) / 256;
    if (nb > 65535) nb = 65535;
    hipLaunchKernelGGL(k_load_uniform, dim3((unsigned)nb), dim3(256), 0, s, g,
                       q0 * dx * dx * dt / 8.0, f);
}

// Dirichlet lifting vector: the initial condition on the t = 0 plane, zero
// elsewhere (patch nodes of later levels are T = 0).
__global__ void k_ic_lift(FineGeom g, const double* __restrict__ ic, double* __restrict__ gv) {
    const long long P = (long long)(g.nx + 1) * (g.ny + 1);
    const long long N = P * (g.nt + 1);
    for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < N;
         idx += (long long)gridDim.x * blockDim.x)
        gv[idx] = (idx < P && g.ic_dir) ? ic[idx] : 0.0;
}

void launch_ic_lift_vector(hipStream_t s, const FineGeom& g, const double* ic, double* gvec) {
    const long long N = (long long)(g.nx + 1) * (g.ny + 1) * (g.nt + 1);
    long long nb = (N + 255) / 256;
    if (nb > 65535) nb = 65535;
    hipLaunchKernelGGL(k_ic_lift, dim3((unsigned)nb), dim3(256), 0, s, g, ic, gvec);
}

// f_m = N (f - J g) + g.
__global__ void k_lift(long long n, const uint8_t* __restrict__ mask, const double* __restrict__ f,
                       const double* __restrict__ Jg, const double* __restrict__ gv,
                       double* __restrict__ fm) {
    for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < n;
         idx += (long long)gridDim.x * blockDim.x)
        fm[idx] = mask[idx] ? gv[idx] : f[idx] - Jg[idx];
}

void launch_lift(hipStream_t s, long long n, const uint8_t* mask, const double* f,
                 const double* Jg, const double* g, double* fm) {
    long long nb = (n + 255) / 256;
    if (nb > 65535) nb = 65535;
    hipLaunchKernelGGL(k_lift, dim3((unsigned)nb), dim3(256), 0, s, n, mask, f, Jg, g, fm);
}

__global__ void k_mask_vec(long long n, const uint8_t* __restrict__ mask,
                           const double* __restrict__ in, double* __restrict__ out) {
    for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < n;
         idx += (long long)gridDim.x * blockDim.x)
        out[idx] = mask[idx] ? 0.0 : in[idx];
}

void launch_mask_vec(hipStream_t s, long long n, const uint8_t* mask, const double* in,
                     double* out) {
    long long nb = (n + 255) / 256;
    if (nb > 65535) nb = 65535;
    hipLaunchKernelGGL(k_mask_vec, dim3((unsigned)nb), dim3(256), 0, s, n, mask, in, out);
}

// ---------------------------------------------------------------------------
// Sensitivities (§3.3.3): g_e = -lambda_e^T (k'_e A + C'_e B) s_e.  With
// A = Mt (x) Kq:  lambda^T A s = dt/6 [2 lb.Kq sb + lb.Kq st + lt.Kq sb + 2 lt.Kq st];
// with B = U (x) Mq:  lambda^T B s = lt.Mq (st - sb).  A thread owns one
// element column; a time-constant design sums over slabs in order.
__device__ __forceinline__ void kq4(const double s[4], double o[4]) {
    // 6 * Kq s with local order (0,0), (1,0), (0,1), (1,1)
    o[0] = 4 * s[0] - s[1] - s[2] - 2 * s[3];
    o[1] = -s[0] + 4 * s[1] - 2 * s[2] - s[3];
    o[2] = -s[0] - 2 * s[1] + 4 * s[2] - s[3];
    o[3] = -2 * s[0] - s[1] - s[2] + 4 * s[3];
}
__device__ __forceinline__ void mq4(const double s[4], double o[4]) {
    // 36 / dx^2 * Mq s
    o[0] = 4 * s[0] + 2 * s[1] + 2 * s[2] + s[3];
    o[1] = 2 * s[0] + 4 * s[1] + s[2] + 2 * s[3];
    o[2] = 2 * s[0] + s[1] + 4 * s[2] + 2 * s[3];
    o[3] = s[0] + 2 * s[1] + 2 * s[2] + 4 * s[3];
}

__global__ void k_sensitivity(FineGeom g, double dx, double dt, const double* __restrict__ T,
                              const double* __restrict__ lam, const double* __restrict__ dk,
                              const double* __restrict__ dc, double* __restrict__ out,
                              int sum_slabs) {
    const int nx = g.nx, ny = g.ny, nt = g.nt;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (i >= nx || j >= ny) return;
    const long long rowp = nx + 1;
    const long long P = rowp * (ny + 1);
    const long long slab = (long long)nx * ny;
    const long long e2 = (long long)j * nx + i;
    const long long c0 = (long long)j * rowp + i;
    const long long loc[4] = {c0, c0 + 1, c0 + rowp, c0 + rowp + 1};
    double acc = 0.0;
    for (int s = 0; s < nt; ++s) {
        double sb[4], st_[4], lb[4], lt[4];
        for (int a = 0; a < 4; ++a) {
            sb[a] = T[(long long)s * P + loc[a]];
            st_[a] = T[(long long)(s + 1) * P + loc[a]];
            lb[a] = lam[(long long)s * P + loc[a]];
            lt[a] = lam[(long long)(s + 1) * P + loc[a]];
        }
        double kb[4], kt[4], md[4], ds[4];
        kq4(sb, kb);
        kq4(st_, kt);
        for (int a = 0; a < 4; ++a) ds[a] = st_[a] - sb[a];
        mq4(ds, md);
        double lbkb = 0, lbkt = 0, ltkb = 0, ltkt = 0, ltm = 0;
        for (int a = 0; a < 4; ++a) {
            lbkb += lb[a] * kb[a];
            lbkt += lb[a] * kt[a];
            ltkb += lt[a] * kb[a];
            ltkt += lt[a] * kt[a];
            ltm += lt[a] * md[a];
        }
        const double la = (dt / 36.0) * (2 * lbkb + lbkt + ltkb + 2 * ltkt);
        const double lb_ = (dx * dx / 36.0) * ltm;
        const long long e = g.tconst ? e2 : (long long)s * slab + e2;
        const double dcv = g.cuniform ? 0.0 : dc[e];
        const double ge = -(dk[e] * la + dcv * lb_);
        if (sum_slabs)
            acc += ge;
        else
            out[(long long)s * slab + e2] = ge;
    }
    if (sum_slabs) out[e2] = acc;
}

void launch_sensitivity(hipStream_t s, const FineGeom& g, double dx, double dt, const double* T,
                        const double* lam, const double* dk, const double* dc, double* out,
                        int sum_slabs) {
    dim3 grid((g.nx + 63) / 64, g.ny);
    hipLaunchKernelGGL(k_sensitivity, grid, dim3(64), 0, s, g, dx, dt, T, lam, dk, dc, out,
                       sum_slabs);
}

// ---------------------------------------------------------------------------
// Constant-coefficient tensor operator on a full box with natural boundaries:
//   H = dxx (Mt (x) My (x) Sx + Mt (x) Sy (x) Mx) + dtt St (x) My (x) Mx + Mt (x) My (x) Mx
// with 1-D assembled linear-element mass M and stiffness S.  It is the nodal
// Helmholtz operator of the PDE filter (§3.3.2) and, with dxx = dtt = 0, the
// consistent space-time mass used for a nodal heat source.
__device__ __forceinline__ void w1d(int i, int n, double h, double m[3], double st[3]) {
    const bool lo = i > 0, hi = i < n;
    const int cnt = (int)lo + (int)hi;
    m[0] = lo ? h / 6.0 : 0.0;
    m[2] = hi ? h / 6.0 : 0.0;
    m[1] = cnt * h / 3.0;
    st[0] = lo ? -1.0 / h : 0.0;
    st[2] = hi ? -1.0 / h : 0.0;
    st[1] = cnt / h;
}

__global__ void k_tensor_op(int nx, int ny, int nt, double dx, double dt, double dxx, double dtt,
                            const double* __restrict__ x, double* __restrict__ y,
                            const double* __restrict__ b, const double* __restrict__ invd,
                            const int* __restrict__ skip) {
    if (skip && *skip) return;
    const long long rowp = nx + 1;
    const long long P = rowp * (ny + 1);
    const long long N = P * (nt + 1);
    for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < N;
         idx += (long long)gridDim.x * blockDim.x) {
        const int n = (int)(idx / P);
        const long long r = idx - n * P;
        const int j = (int)(r / rowp), i = (int)(r - (long long)j * rowp);
        double mx[3], sx[3], my[3], sy[3], mt[3], stt[3];
        w1d(i, nx, dx, mx, sx);
        w1d(j, ny, dx, my, sy);
        w1d(n, nt, dt, mt, stt);
        double acc = 0.0;
        for (int a = 0; a < 3; ++a) {
            if (mt[a] == 0.0) continue;
            for (int c = 0; c < 3; ++c) {
                if (my[c] == 0.0) continue;
                const double* xp = x + idx + (long long)(a - 1) * P + (long long)(c - 1) * rowp;
                for (int d = 0; d < 3; ++d) {
                    if (mx[d] == 0.0) continue;
                    const double w = dxx * (mt[a] * my[c] * sx[d] + mt[a] * sy[c] * mx[d]) +
                                     dtt * stt[a] * my[c] * mx[d] + mt[a] * my[c] * mx[d];
                    acc += w * xp[d - 1];
                }
            }
        }
        double v = b ? b[idx] - acc : acc;
        if (invd) v *= invd[idx];
        y[idx] = v;
    }
}

void launch_tensor_op(hipStream_t s, int nx, int ny, int nt, double dx, double dt, double dxx,
                      double dtt, const double* x, double* y, const double* b, const double* invd,
                      const int* skip) {
    const long long N = (long long)(nx + 1) * (ny + 1) * (nt + 1);
    long long nb = (N + 255) / 256;
    if (nb > 65535) nb = 65535;
    hipLaunchKernelGGL(k_tensor_op, dim3((unsigned)nb), dim3(256), 0, s, nx, ny, nt, dx, dt, dxx,
                       dtt, x, y, b, invd, skip);
}

__global__ void k_tensor_invdiag(int nx, int ny, int nt, double dx, double dt, double dxx,
                                 double dtt, double* __restrict__ invd) {
    const long long rowp = nx + 1;
    const long long P = rowp * (ny + 1);
    const long long N = P * (nt + 1);
    for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < N;
         idx += (long long)gridDim.x * blockDim.x) {
        const int n = (int)(idx / P);
        const long long r = idx - n * P;
        const int j = (int)(r / rowp), i = (int)(r - (long long)j * rowp);
        double mx[3], sx[3], my[3], sy[3], mt[3], stt[3];
        w1d(i, nx, dx, mx, sx);
        w1d(j, ny, dx, my, sy);
        w1d(n, nt, dt, mt, stt);
        const double d = dxx * (mt[1] * my[1] * sx[1] + mt[1] * sy[1] * mx[1]) +
                         dtt * stt[1] * my[1] * mx[1] + mt[1] * my[1] * mx[1];
        invd[idx] = 1.0 / d;
    }
}

void launch_tensor_invdiag(hipStream_t s, int nx, int ny, int nt, double dx, double dt,
                           double dxx, double dtt, double* invd) {
    const long long N = (long long)(nx + 1) * (ny + 1) * (nt + 1);
    long long nb = (N + 255) / 256;
    if (nb > 65535) nb = 65535;
    hipLaunchKernelGGL(k_tensor_invdiag, dim3((unsigned)nb), dim3(256), 0, s, nx, ny, nt, dx, dt,
                       dxx, dtt, invd);
}

// Element -> node: nodal[a] = w * sum of the element values around a.
__global__ void k_elem_to_node(int nx, int ny, int nt, double w, const double* __restrict__ e,
                               double* __restrict__ nodal) {
    const long long rowp = nx + 1;
    const long long P = rowp * (ny + 1);
    const long long N = P * (nt + 1);
    for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < N;
         idx += (long long)gridDim.x * blockDim.x) {
        const int n = (int)(idx / P);
        const long long r = idx - n * P;
        const int j = (int)(r / rowp), i = (int)(r - (long long)j * rowp);
        double acc = 0.0;
        for (int en = n - 1; en <= n; ++en) {
            if (en < 0 || en >= nt) continue;
            for (int ej = j - 1; ej <= j; ++ej) {
                if (ej < 0 || ej >= ny) continue;
                for (int ei = i - 1; ei <= i; ++ei) {
                    if (ei < 0 || ei >= nx) continue;
                    acc += e[((long long)en * ny + ej) * nx + ei];
                }
            }
        }
        nodal[idx] = w * acc;
    }
}

void launch_elem_to_node(hipStream_t s, int nx, int ny, int nt, double w, const double* e,
                         double* nodal) {
    const long long N = (long long)(nx + 1) * (ny + 1) * (nt + 1);
    long long nb = (N + 255) / 256;
    if (nb > 65535) nb = 65535;
    hipLaunchKernelGGL(k_elem_to_node, dim3((unsigned)nb), dim3(256), 0, s, nx, ny, nt, w, e,
                       nodal);
}

// Node -> element: mean of the element's 8 nodal values.
__global__ void k_node_to_elem(int nx, int ny, int nt, const double* __restrict__ nodal,
                               double* __restrict__ e) {
    const long long rowp = nx + 1;
    const long long P = rowp * (ny + 1);
    const long long NE = (long long)nx * ny * nt;
    for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < NE;
         idx += (long long)gridDim.x * blockDim.x) {
        const long long sl = (long long)nx * ny;
        const int n = (int)(idx / sl);
        const long long r = idx - n * sl;
        const int j = (int)(r / nx), i = (int)(r - (long long)j * nx);
        const long long c = (long long)n * P + (long long)j * rowp + i;
        const double s = nodal[c] + nodal[c + 1] + nodal[c + rowp] + nodal[c + rowp + 1] +
                         nodal[c + P] + nodal[c + P + 1] + nodal[c + P + rowp] +
                         nodal[c + P + rowp + 1];
        e[idx] = 0.125 * s;
    }
}

void launch_node_to_elem(hipStream_t s, int nx, int ny, int nt, const double* nodal, double* e) {
    const long long NE = (long long)nx * ny * nt;
    long long nb = (NE + 255) / 256;
    if (nb > 65535) nb = 65535;
    hipLaunchKernelGGL(k_node_to_elem, dim3((unsigned)nb), dim3(256), 0, s, nx, ny, nt, nodal, e);
}

}  // namespace st
