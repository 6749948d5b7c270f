// Fused Jacobi-GMRES smoother for the small coarse levels (paper §3.2: at most
// 10 GMRES iterations with Jacobi preconditioning on every non-coarsest level).
//
// On a level of a few thousand to a few hundred thousand nodes every kernel of
// the generic smoother (stencil apply, multi-dot, its reduction, maxpy + norm,
// its reduction with the Givens update) is a few microseconds of work behind a
// launch, so the smoothing is launch-bound.  Here one iteration is two kernels:
//   apply:  v_{j+1} = D^{-1} A v_j with the projections <v_d, v_{j+1}>, d <= j,
//           reduced per workgroup in the same pass;
//   maxpy:  every workgroup sums the apply's workgroup partials itself (fixed
//           order, so all agree bitwise), subtracts the projections and
//           reduces ||v_{j+1}||^2 per workgroup.
// The next apply's workgroups each sum those norm partials and apply the
// Givens rotation of the finished column themselves (identical arithmetic in
// every workgroup); workgroup 0 records it in the level's KState.  No kernel
// waits on another workgroup, and no device-scope fence is needed: each
// kernel reads only what earlier kernels on the stream wrote.
//
// Basis vectors are stored unnormalised, as in the generic smoother:
// KState::scale[d] = 1 / ||w_d||.
#include "st_internal.hpp"
#include "stencil_core.hpp"

namespace st {

constexpr int SM_THREADS = 256;
constexpr int SM_MAXB = 512;       // most workgroups of a fused smoother kernel
constexpr int SM_MAXCHUNK = 4;     // most time levels one apply thread marches through

__device__ __forceinline__ double sm_wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    return v;
}

// Per-workgroup sums of nd accumulators into out[0..nd).
template <int ND>
__device__ void sm_block_partials(const double (&acc)[ND], int nd, double* __restrict__ out) {
    __shared__ double red[SM_THREADS / 64][ND];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int d = 0; d < ND; ++d)
        if (d < nd) {
            const double v = sm_wave_sum(acc[d]);
            if (lane == 0) red[wave][d] = v;
        }
    __syncthreads();
    if ((int)threadIdx.x < nd) {
        double v = 0.0;
#pragma unroll
        for (int w = 0; w < SM_THREADS / 64; ++w) v += red[w][threadIdx.x];
        out[threadIdx.x] = v;
    }
}

// sums[d] = sum_b part[b * stride + d], d < nd, in a fixed order (every
// workgroup computes the same values).  Result in LDS.
__device__ void sm_sum_partials(const double* __restrict__ part, int nb, int stride, int nd,
                                double* sums) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int d = wave; d < nd; d += SM_THREADS / 64) {
        double v = 0.0;
        for (int b = lane; b < nb; b += 64) v += part[(long long)b * stride + d];
        v = sm_wave_sum(v);
        if (lane == 0) sums[d] = v;
    }
    __syncthreads();
}

// Givens update of Hessenberg column jm from ||w|| = sqrt(hn2), the
// projections ks->hcol, the earlier rotations and the unrotated g_jm (one
// thread, inputs staged in LDS).  col[] returns the rotated column; write:
// also store it in ks.
// Nothing it reads is written by a kernel that runs it (the carry of g sits
// in gcarry[jm & 1], the next one goes to the other slot), so every
// workgroup of a kernel sees the same inputs.
struct SmGivens {
    double col[SMAX];
    double g0, g1;      // g[jm], g[jm + 1] after the rotation
    double scale_next;  // 1 / ||w||
    int done;
};

// What the Givens update of column jm reads from the KState, staged in LDS
// by the whole workgroup (parallel loads) before one thread uses it.
struct SmStage {
    double col[SMAX], cs[SMAX], sn[SMAX];
    double gj, rtol, ref;
    int maxit;
};

__device__ void sm_stage_load(const KState* ks, int jm, SmStage& st) {
    const int t = threadIdx.x;
    if (t <= jm) st.col[t] = ks->hcol[t];
    if (t < jm) {
        st.cs[t] = ks->cs[t];
        st.sn[t] = ks->sn[t];
    }
    if (t == 64) st.gj = ks->gcarry[jm & 1];
    if (t == 65) st.rtol = ks->rtol;
    if (t == 66) st.ref = ks->ref;
    if (t == 67) st.maxit = ks->maxit;
}

__device__ SmGivens sm_givens(const SmStage& st, KState* ks, int jm, double hn2, bool write) {
    SmGivens o;
#pragma unroll
    for (int i = 0; i < SMAX; ++i) o.col[i] = i <= jm ? st.col[i] : 0.0;
    const double gj = st.gj;
    const double hn = sqrt(hn2);
    double hnorm2 = hn * hn;
#pragma unroll
    for (int i = 0; i < SMAX; ++i)
        if (i <= jm) hnorm2 += o.col[i] * o.col[i];
#pragma unroll
    for (int i = 0; i < SMAX - 1; ++i)
        if (i < jm) {
            const double a = o.col[i], b = o.col[i + 1];
            o.col[i] = st.cs[i] * a + st.sn[i] * b;
            o.col[i + 1] = -st.sn[i] * a + st.cs[i] * b;
        }
    double hj = 0.0;
#pragma unroll
    for (int i = 0; i < SMAX; ++i)
        if (i == jm) hj = o.col[i];
    const double r = hypot(hj, hn);
    double cc = 1.0, ss = 0.0;
    if (r != 0.0) {
        cc = hj / r;
        ss = hn / r;
    }
#pragma unroll
    for (int i = 0; i < SMAX; ++i)
        if (i == jm) o.col[i] = r;
    o.g0 = cc * gj;
    o.g1 = -ss * gj;
    o.scale_next = hn > 0.0 ? 1.0 / hn : 0.0;
    const double est = fabs(o.g1);
    const bool bad = !isfinite(est) || !isfinite(hn);
    const bool conv = est <= st.rtol * st.ref;
    const bool brk = hn <= 1e-14 * sqrt(hnorm2);
    const int k = jm + 1;
    o.done = (conv || brk || bad || k >= st.maxit) ? 1 : 0;
    if (write) {
#pragma unroll
        for (int i = 0; i < SMAX; ++i)
            if (i <= jm) ks->H[i][jm] = o.col[i];
        ks->cs[jm] = cc;
        ks->sn[jm] = ss;
        ks->g[jm] = o.g0;
        ks->g[jm + 1] = o.g1;
        ks->gcarry[(jm + 1) & 1] = o.g1;
        ks->scale[jm + 1] = o.scale_next;
        ks->k = k;
        ks->est = est;
        ks->bad |= bad ? 1 : 0;
        ks->done = o.done;
    }
    return o;
}

// ---------------------------------------------------------------------------
// Start from x0 = 0: w = D^{-1} b, per-workgroup ||w||^2; workgroup 0 resets
// the KState.
template <typename T>
__global__ __launch_bounds__(SM_THREADS) void k_sm_scale(long long n, const T* __restrict__ b,
                                                         const T* __restrict__ invd,
                                                         T* __restrict__ w,
                                                         double* __restrict__ npart, KState* ks,
                                                         int maxit, double rtol) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        ks->maxit = maxit;
        ks->rtol = rtol;
        ks->scale_update = 1;
        ks->done = 0;
        ks->bad = 0;
        ks->k = 0;
    }
    double acc[1] = {0.0};
    for (long long i = blockIdx.x * (long long)SM_THREADS + threadIdx.x; i < n;
         i += (long long)gridDim.x * SM_THREADS) {
        const T v = (T)(b[i] * invd[i]);
        w[i] = v;
        acc[0] += (double)v * (double)v;
    }
    sm_block_partials<1>(acc, 1, npart + blockIdx.x);
}

// phase 0: w = V_0 = D^{-1} (b - A x0) with per-workgroup ||w||^2 (the first
//          kernel of a smoothing from a given x0; workgroup 0 resets the KState).
// phase 1: iteration j: finish the previous step from the norm partials
//          (initial beta for j = 0, Givens update of column j - 1 otherwise),
//          then V_{j+1} = D^{-1} A V_j scale_j with per-workgroup <V_d, V_{j+1}>,
//          d <= j.
template <typename T, typename S, typename TC, bool TRANS>
__global__ __launch_bounds__(SM_THREADS) void k_sm_apply(
    int nx, int ny, int nt, int nplanes, const S* __restrict__ st, const float* __restrict__ cen,
    const int* __restrict__ pmap, const T* __restrict__ x, T* __restrict__ y,
    const T* __restrict__ b, const T* __restrict__ invd, const T* __restrict__ V, long long ld,
    int j, int phase,
    KState* ks, const double* __restrict__ npart, int nbn, double* __restrict__ dpart,
    double* __restrict__ npart_out, int maxit, double rtol, int nchunk) {
    __shared__ double sums[1];
    __shared__ double sc_s;
    __shared__ int done_s;
    __shared__ SmStage stg;
    TC sc = (TC)1;
    if (phase == 1) {
        // Workgroup 0 may set ks->done during this kernel; a workgroup that
        // reads the new value stops, as its own Givens update would tell it.
        if (threadIdx.x == 0) done_s = ks->done;
        __syncthreads();
        if (done_s) return;
        if (j > 0) sm_stage_load(ks, j - 1, stg);
        sm_sum_partials(npart, nbn, 1, 1, sums);
        if (threadIdx.x == 0) {
            const bool write = blockIdx.x == 0 && blockIdx.y == 0;
            if (j == 0) {
                const double beta = sqrt(sums[0]);
                const int bad = !isfinite(beta);
                const int done = (beta == 0.0) || bad;
                const double s0 = beta > 0.0 ? 1.0 / beta : 0.0;
                if (write) {
                    ks->beta = beta;
                    ks->ref = beta;
                    ks->g[0] = beta;
                    ks->gcarry[0] = beta;
                    ks->scale[0] = s0;
                    ks->k = 0;
                    ks->est = beta;
                    ks->bad = bad;
                    ks->done = done;
                }
                sc_s = s0;
                done_s = done;
            } else {
                const SmGivens o = sm_givens(stg, ks, j - 1, sums[0], write);
                sc_s = o.scale_next;
                done_s = o.done;
            }
        }
        __syncthreads();
        if (done_s) return;
        sc = (TC)sc_s;
    } else if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) {
        ks->maxit = maxit;
        ks->rtol = rtol;
        ks->scale_update = 1;
        ks->done = 0;
        ks->bad = 0;
        ks->k = 0;
    }
    const int P = (nx + 1) * (ny + 1);
    const int r = blockIdx.x * SM_THREADS + threadIdx.x;
    const int n0 = blockIdx.y * nchunk;
    const int n1 = min(n0 + nchunk, nt + 1);
    double acc[SMAX];
#pragma unroll
    for (int d = 0; d < SMAX; ++d) acc[d] = 0.0;
    if (r < P && n0 <= nt) {
        stencil_march_rows<T, S, TC, TRANS>(
            nx, ny, nt, nplanes, st, cen, pmap, x, r, n0, n1, [&](int, long long idx, TC a) {
                TC v = a;
                if (phase == 0) v = (TC)b[idx] - v;
                v *= (TC)invd[idx];
                const T o = (T)(v * sc);
                y[idx] = o;
                const double od = (double)o;
                if (phase == 0) {
                    acc[0] += od * od;
                } else {
#pragma unroll
                    for (int d = 0; d < SMAX; ++d)
                        if (d <= j) acc[d] += (double)V[(long long)d * ld + idx] * od;
                }
            });
    }
    const int blk = blockIdx.y * gridDim.x + blockIdx.x;
    if (phase == 0)
        sm_block_partials<SMAX>(acc, 1, npart_out + blk);
    else
        sm_block_partials<SMAX>(acc, j + 1, dpart + (long long)blk * SMAX);
}

// w = V_{j+1} -= sum_{d <= j} coef_d V_d with the projections summed from the
// apply's workgroup partials; per-workgroup ||w||^2.  Workgroup 0 records the
// projections in the KState (the Givens update reads them).
template <typename T>
__global__ __launch_bounds__(SM_THREADS) void k_sm_maxpy(long long n, T* __restrict__ w,
                                                         const T* __restrict__ V, long long ld,
                                                         int j, KState* ks,
                                                         const double* __restrict__ dpart,
                                                         int nbd, double* __restrict__ npart) {
    if (ks->done) return;
    __shared__ double sums[SMAX];
    __shared__ double coef[SMAX];
    sm_sum_partials(dpart, nbd, SMAX, j + 1, sums);
    if ((int)threadIdx.x <= j) {
        const double sd = ks->scale[threadIdx.x];
        const double h = sums[threadIdx.x] * sd;
        coef[threadIdx.x] = h * sd;
        if (blockIdx.x == 0) {
            ks->hcol[threadIdx.x] = h;
            ks->coef[threadIdx.x] = h * sd;
        }
    }
    __syncthreads();
    double acc[1] = {0.0};
    const long long stride = (long long)gridDim.x * SM_THREADS;
    if (sizeof(T) == 4 && ld % 4 == 0) {
        const long long n4 = n >> 2;
        for (long long q = blockIdx.x * (long long)SM_THREADS + threadIdx.x; q < n4; q += stride) {
            float4 xv = *reinterpret_cast<const float4*>(w + 4 * q);
#pragma unroll
            for (int d = 0; d < SMAX; ++d)
                if (d <= j) {
                    const float4 v = *reinterpret_cast<const float4*>(V + (long long)d * ld + 4 * q);
                    const float cd = (float)coef[d];
                    xv.x -= cd * v.x; xv.y -= cd * v.y; xv.z -= cd * v.z; xv.w -= cd * v.w;
                }
            *reinterpret_cast<float4*>(w + 4 * q) = xv;
            acc[0] += (double)(xv.x * xv.x + xv.y * xv.y + xv.z * xv.z + xv.w * xv.w);
        }
        for (long long i = 4 * n4 + blockIdx.x * (long long)SM_THREADS + threadIdx.x; i < n;
             i += stride) {
            float v = (float)w[i];
#pragma unroll
            for (int d = 0; d < SMAX; ++d)
                if (d <= j) v -= (float)coef[d] * (float)V[(long long)d * ld + i];
            w[i] = (T)v;
            acc[0] += (double)v * (double)v;
        }
    } else {
        for (long long i = blockIdx.x * (long long)SM_THREADS + threadIdx.x; i < n; i += stride) {
            double v = (double)w[i];
#pragma unroll
            for (int d = 0; d < SMAX; ++d)
                if (d <= j) v -= coef[d] * (double)V[(long long)d * ld + i];
            const T o = (T)v;
            w[i] = o;
            acc[0] += (double)o * (double)o;
        }
    }
    sm_block_partials<1>(acc, 1, npart + blockIdx.x);
}

// x = (zero_x0 ? 0 : x) + sum_d y_d V_d, after finishing the last column (its
// Givens update, when the cycle has not stopped earlier) and the triangular
// solve for y -- both done by every workgroup, in LDS.
template <typename T>
__global__ __launch_bounds__(SM_THREADS) void k_sm_update(long long n, T* __restrict__ x,
                                                          const T* __restrict__ V, long long ld,
                                                          KState* ks,
                                                          const double* __restrict__ npart,
                                                          int nbn, int its, int zero_x0) {
    __shared__ double Hs[SMAX][SMAX];
    __shared__ double gs[SMAX + 1];
    __shared__ double scl[SMAX + 1];
    __shared__ double ys[SMAX];
    __shared__ double sums[1];
    __shared__ int k_s, done_s, kin_s;
    __shared__ SmStage stg;
    if (threadIdx.x == 0) {
        done_s = ks->done;
        kin_s = ks->k;
    }
    __syncthreads();
    const int done0 = done_s;
    const int k0 = done0 ? kin_s : its - 1;   // columns already in ks->H
    for (int e = threadIdx.x; e < SMAX * SMAX; e += SM_THREADS) {
        const int i = e / SMAX, c = e - i * SMAX;
        Hs[i][c] = (c < k0 && i <= c) ? ks->H[i][c] : 0.0;
    }
    if ((int)threadIdx.x <= SMAX) {
        gs[threadIdx.x] = (int)threadIdx.x <= k0 ? ks->g[threadIdx.x] : 0.0;
        scl[threadIdx.x] = (int)threadIdx.x <= k0 ? ks->scale[threadIdx.x] : 0.0;
    }
    if (!done0) {
        sm_stage_load(ks, its - 1, stg);
        sm_sum_partials(npart, nbn, 1, 1, sums);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int k = k0;
        if (!done0) {
            // the KState is not written here: other workgroups still read it
            const SmGivens o = sm_givens(stg, ks, its - 1, sums[0], false);
#pragma unroll
            for (int i = 0; i < SMAX; ++i)
                if (i < its) Hs[i][its - 1] = o.col[i];
            gs[its - 1] = o.g0;
            gs[its] = o.g1;
            k = its;
        }
        for (int i = k - 1; i >= 0; --i) {
            double v = gs[i];
            for (int c = i + 1; c < k; ++c) v -= Hs[i][c] * ys[c];
            ys[i] = Hs[i][i] != 0.0 ? v / Hs[i][i] : 0.0;
        }
        for (int i = 0; i < k; ++i) ys[i] *= scl[i];
        k_s = k;
    }
    __syncthreads();
    const int k = k_s;
    if (k == 0 && !zero_x0) return;
    const long long stride = (long long)gridDim.x * SM_THREADS;
    for (long long i = blockIdx.x * (long long)SM_THREADS + threadIdx.x; i < n; i += stride) {
        double v = zero_x0 ? 0.0 : (double)x[i];
        for (int d = 0; d < k; ++d) v += ys[d] * (double)V[(long long)d * ld + i];
        x[i] = (T)v;
    }
}

// ---------------------------------------------------------------------------
// Host side.
static inline int sm_vec_blocks(long long n) {
    long long nb = (n + 4LL * SM_THREADS - 1) / (4LL * SM_THREADS);
    if (nb < 1) nb = 1;
    if (nb > SM_MAXB) nb = SM_MAXB;
    return (int)nb;
}

bool sm_fused_plan(const Level& L, int* nchunk, int* gx, int* gy) {
    const int P = (L.nx + 1) * (L.ny + 1);
    const int x = (P + SM_THREADS - 1) / SM_THREADS;
    for (int c = 1; c <= SM_MAXCHUNK; c *= 2) {
        const int y = (L.nt + 1 + c - 1) / c;
        if ((long long)x * y <= SM_MAXB) {
            *nchunk = c;
            *gx = x;
            *gy = y;
            return true;
        }
    }
    return false;
}

size_t sm_partials_doubles() { return (size_t)SM_MAXB * SMAX + 2 * SM_MAXB; }

template <typename T, typename S, typename TC>
static void sm_apply_launch(hipStream_t s, const Level& L, const S* st, int trans, const void* x,
                            void* y, const void* b, const void* invd, const void* V, int j,
                            int phase, KState* ks, const double* npart, int nbn, double* dpart,
                            double* npart_out, int maxit, double rtol, int nchunk, int gx,
                            int gy) {
    if (trans)
        hipLaunchKernelGGL((k_sm_apply<T, S, TC, true>), dim3(gx, gy), dim3(SM_THREADS), 0, s,
                           L.nx, L.ny, L.nt, L.nplanes, st, L.cen32, L.plane_map, (const T*)x, (T*)y,
                           (const T*)b, (const T*)invd, (const T*)V, L.ld, j, phase, ks, npart,
                           nbn, dpart, npart_out, maxit, rtol, nchunk);
    else
        hipLaunchKernelGGL((k_sm_apply<T, S, TC, false>), dim3(gx, gy), dim3(SM_THREADS), 0, s,
                           L.nx, L.ny, L.nt, L.nplanes, st, L.cen32, L.plane_map, (const T*)x, (T*)y,
                           (const T*)b, (const T*)invd, (const T*)V, L.ld, j, phase, ks, npart,
                           nbn, dpart, npart_out, maxit, rtol, nchunk);
}

static void sm_apply_dispatch(hipStream_t s, const Level& L, int prec, int trans, const void* x,
                              void* y, const void* b, const void* invd, const void* V, int j,
                              int phase, KState* ks, const double* npart, int nbn, double* dpart,
                              double* npart_out, int maxit, double rtol, int nchunk, int gx,
                              int gy) {
    if (prec == 0)
        sm_apply_launch<double, double, double>(s, L, L.st64, trans, x, y, b, invd, V, j, phase,
                                                ks, npart, nbn, dpart, npart_out, maxit, rtol,
                                                nchunk, gx, gy);
    else if (L.sprec == 2)
        sm_apply_launch<float, uint16_t, float>(s, L, L.st16, trans, x, y, b, invd, V, j, phase,
                                                ks, npart, nbn, dpart, npart_out, maxit, rtol,
                                                nchunk, gx, gy);
    else
        sm_apply_launch<float, float, float>(s, L, L.st32, trans, x, y, b, invd, V, j, phase, ks,
                                             npart, nbn, dpart, npart_out, maxit, rtol, nchunk,
                                             gx, gy);
}

// Partials buffer: [SM_MAXB][SMAX] projections, then two norm regions of
// SM_MAXB (the norms written by one kernel are read by the next, which may
// write norms of its own only in phase 0 -- it then reads none).
void launch_sm_init(hipStream_t s, const Level& L, int prec, int trans, const void* b,
                    const void* x, int zero_x0, const void* invd, void* V0, KState* ks,
                    double* part, int maxit, double rtol, int* nbn) {
    double* npart = part + (size_t)SM_MAXB * SMAX;
    if (zero_x0) {
        const int nb = sm_vec_blocks(L.nn);
        if (prec == 0)
            hipLaunchKernelGGL(k_sm_scale<double>, dim3(nb), dim3(SM_THREADS), 0, s, L.nn,
                               (const double*)b, (const double*)invd, (double*)V0, npart, ks,
                               maxit, rtol);
        else
            hipLaunchKernelGGL(k_sm_scale<float>, dim3(nb), dim3(SM_THREADS), 0, s, L.nn,
                               (const float*)b, (const float*)invd, (float*)V0, npart, ks, maxit,
                               rtol);
        *nbn = nb;
        return;
    }
    int nchunk, gx, gy;
    sm_fused_plan(L, &nchunk, &gx, &gy);
    sm_apply_dispatch(s, L, prec, trans, x, V0, b, invd, nullptr, 0, 0, ks, nullptr, 0, nullptr,
                      npart, maxit, rtol, nchunk, gx, gy);
    *nbn = gx * gy;
}

void launch_sm_iteration(hipStream_t s, const Level& L, int prec, int trans, const void* invd,
                         void* V, int j, KState* ks, double* part, int* nbn) {
    double* dpart = part;
    double* npart = part + (size_t)SM_MAXB * SMAX;
    int nchunk, gx, gy;
    sm_fused_plan(L, &nchunk, &gx, &gy);
    const size_t vb = prec == 0 ? 8 : 4;
    char* Vc = (char*)V;
    const void* vj = Vc + (size_t)j * L.ld * vb;
    void* vj1 = Vc + (size_t)(j + 1) * L.ld * vb;
    sm_apply_dispatch(s, L, prec, trans, vj, vj1, nullptr, invd, V, j, 1, ks, npart, *nbn, dpart,
                      nullptr, 0, 0.0, nchunk, gx, gy);
    const int nb = sm_vec_blocks(L.nn);
    if (prec == 0)
        hipLaunchKernelGGL(k_sm_maxpy<double>, dim3(nb), dim3(SM_THREADS), 0, s, L.nn,
                           (double*)vj1, (const double*)V, L.ld, j, ks, dpart, gx * gy, npart);
    else
        hipLaunchKernelGGL(k_sm_maxpy<float>, dim3(nb), dim3(SM_THREADS), 0, s, L.nn,
                           (float*)vj1, (const float*)V, L.ld, j, ks, dpart, gx * gy, npart);
    *nbn = nb;
}

void launch_sm_update(hipStream_t s, const Level& L, int prec, void* x, const void* V, KState* ks,
                      const double* part, int nbn, int its, int zero_x0) {
    const double* npart = part + (size_t)SM_MAXB * SMAX;
    const int nb = sm_vec_blocks(L.nn);
    if (prec == 0)
        hipLaunchKernelGGL(k_sm_update<double>, dim3(nb), dim3(SM_THREADS), 0, s, L.nn,
                           (double*)x, (const double*)V, L.ld, ks, npart, nbn, its, zero_x0);
    else
        hipLaunchKernelGGL(k_sm_update<float>, dim3(nb), dim3(SM_THREADS), 0, s, L.nn, (float*)x,
                           (const float*)V, L.ld, ks, npart, nbn, its, zero_x0);
}

}  // namespace st
