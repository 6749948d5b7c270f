// Krylov kernels: classical Gram-Schmidt projections, vector updates, Givens
// rotations and the least-squares solve of GMRES (Saad & Schultz) and FGMRES
// (Saad), all with the small scalar work on the device (paper §3.2).
//
// Reductions are deterministic: every block reduces its threads in a fixed
// tree, writes one partial per quantity, and the last block to arrive (an
// arrival counter) sums the partials in block order and finalises.  The grid
// size depends only on the vector length, so two runs give bitwise equal sums.
//
// Basis vectors are stored unnormalised; KState::scale[d] = 1/||w_d|| turns
// them into the orthonormal v_d inside the scalar coefficients, so no pass is
// spent on normalising a vector.
#include "st_internal.hpp"
#include "reduce_core.hpp"

namespace st {

// Blocks of the vectorised reductions: four elements per thread per step.
// Streaming reductions use at most four blocks of 256 threads per CU: measured
// on MI355X this is where the multi-dot and maxpy kernels stream fastest
// (one block per CU leaves a single wave per SIMD to hide latency, more
// blocks only lengthen the tail).
constexpr long long MAX_RED_GRID = 1024;

static inline unsigned red_grid4(long long n) {
    long long nb = (n + 8LL * VEC_THREADS - 1) / (8LL * VEC_THREADS);
    if (nb < 1) nb = 1;
    if (nb > MAX_RED_GRID) nb = MAX_RED_GRID;
    return (unsigned)nb;
}

static inline unsigned red_grid(long long n) {
    long long nb = (n + 4LL * VEC_THREADS - 1) / (4LL * VEC_THREADS);
    if (nb < 1) nb = 1;
    if (nb > MAX_RED_GRID) nb = MAX_RED_GRID;
    return (unsigned)nb;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    return v;
}

template <typename T> __device__ __forceinline__ double ldd(const T* p) { return (double)*p; }

// ---------------------------------------------------------------------------
// Vectorised variants: four consecutive elements per thread per step (one
// 16-byte load for FP32, two for FP64), all pointers aligned to 4 elements and
// the basis stride a multiple of 4; the host picks them only when that holds.
template <typename T> struct V4;
template <> struct V4<float> { using type = float4; };
template <> struct V4<double> { using type = double4; };

template <typename T>
__device__ __forceinline__ void ld4(const T* p, double o[4]) {
    const typename V4<T>::type v = *reinterpret_cast<const typename V4<T>::type*>(p);
    o[0] = (double)v.x; o[1] = (double)v.y; o[2] = (double)v.z; o[3] = (double)v.w;
}
template <typename T>
__device__ __forceinline__ void st4(T* p, const double o[4]) {
    typename V4<T>::type v;
    v.x = (T)o[0]; v.y = (T)o[1]; v.z = (T)o[2]; v.w = (T)o[3];
    *reinterpret_cast<typename V4<T>::type*>(p) = v;
}

static inline bool al4(const void* p, size_t esz) {
    return ((uintptr_t)p % (4 * esz)) == 0;
}

// ---------------------------------------------------------------------------
// Scalar finalisation (thread 0 of the last block).
__device__ void kstate_solve_y(KState* ks) {
    const int k = ks->k;
    for (int i = k - 1; i >= 0; --i) {
        double v = ks->g[i];
        for (int c = i + 1; c < k; ++c) v -= ks->H[i][c] * ks->y[c];
        const double d = ks->H[i][i];
        ks->y[i] = d != 0.0 ? v / d : 0.0;
    }
    if (ks->scale_update)
        for (int i = 0; i < k; ++i) ks->y[i] *= ks->scale[i];
}

__device__ void kstate_finalize(KState* ks, int mode, int j, const double* sums, int nd) {
    switch (mode) {
    case FIN_INIT_SELF:
    case FIN_INIT_REF: {
        const double beta = sqrt(sums[0]);
        ks->beta = beta;
        if (mode == FIN_INIT_SELF) ks->ref = beta;
        ks->g[0] = beta;
        ks->scale[0] = beta > 0.0 ? 1.0 / beta : 0.0;
        ks->k = 0;
        ks->est = beta;
        ks->bad = !isfinite(beta);
        ks->done = (beta == 0.0) || ks->bad || (mode == FIN_INIT_REF && beta <= ks->rtol * ks->ref);
        break;
    }
    case FIN_PROJ1:
        for (int d = 0; d < nd; ++d) {
            const double h = sums[d] * ks->scale[d];
            ks->hcol[d] = h;
            ks->coef[d] = h * ks->scale[d];
        }
        break;
    case FIN_PROJ2:
        for (int d = 0; d < nd; ++d) {
            const double h = sums[d] * ks->scale[d];
            ks->hcol[d] += h;
            ks->coef[d] = h * ks->scale[d];
        }
        break;
    case FIN_GIVENS: {
        // Column j of the Hessenberg matrix is rotated in place in ks->H.
        const double hn = sqrt(sums[0]);
        double hnorm2 = hn * hn;
        for (int i = 0; i <= j; ++i) {
            const double v = ks->hcol[i];
            ks->H[i][j] = v;
            hnorm2 += v * v;
        }
        for (int i = 0; i < j; ++i) {
            const double a = ks->H[i][j], b = ks->H[i + 1][j];
            ks->H[i][j] = ks->cs[i] * a + ks->sn[i] * b;
            ks->H[i + 1][j] = -ks->sn[i] * a + ks->cs[i] * b;
        }
        const double hj = ks->H[j][j];
        const double r = hypot(hj, hn);
        double c = 1.0, sn = 0.0;
        if (r != 0.0) {
            c = hj / r;
            sn = hn / r;
        }
        ks->cs[j] = c;
        ks->sn[j] = sn;
        ks->H[j][j] = r;
        ks->g[j + 1] = -sn * ks->g[j];
        ks->g[j] = c * ks->g[j];
        ks->scale[j + 1] = hn > 0.0 ? 1.0 / hn : 0.0;
        ks->k = j + 1;
        ks->est = fabs(ks->g[j + 1]);
        const bool bad = !isfinite(ks->est) || !isfinite(hn);
        const bool conv = ks->est <= ks->rtol * ks->ref;
        const bool brk = hn <= 1e-14 * sqrt(hnorm2);
        ks->bad |= bad;
        if (conv || brk || bad || ks->k >= ks->maxit) {
            ks->done = 1;
            kstate_solve_y(ks);
        }
        break;
    }
    case FIN_DCGS2: {
        // sums = [s_0..s_{KMAX-1}, t_0..t_{KMAX-1}, alpha, beta, gamma] for
        // the current vector u (stored times scale[j]) and w = A z_j:
        // s = Q^T u, t = Q^T w (entries below j), alpha = u.u, beta = u.w,
        // gamma = w.w.
        const double* sv = sums;
        const double* tv = sums + KMAX;
        const double alpha = sums[2 * KMAX], beta = sums[2 * KMAX + 1], gamma = sums[2 * KMAX + 2];
        double ss = 0.0, st = 0.0, tt = 0.0;
        for (int i = 0; i < j; ++i) {
            ss += sv[i] * sv[i];
            st += sv[i] * tv[i];
            tt += tv[i] * tv[i];
        }
        const double nu = sqrt(fmax(alpha - ss, 0.0));
        bool bad = !isfinite(nu) || !(nu > 0.0) || !isfinite(gamma);
        const double nuinv = bad ? 0.0 : 1.0 / nu;
        // column j-1 becomes final: u = (w_{j-1} orthogonalised once) / eta,
        // and u = nu q_j + Q s, so H[0..j-1][j-1] += eta s, H[j][j-1] = eta nu
        if (j >= 1) {
            double col[KMAX + 1];
            for (int i = 0; i < j; ++i) col[i] = ks->hcol[i] + ks->d_eta * sv[i];
            col[j] = ks->d_eta * nu;
            for (int i = 0; i < j - 1; ++i) {
                const double a = col[i], b = col[i + 1];
                col[i] = ks->cs[i] * a + ks->sn[i] * b;
                col[i + 1] = -ks->sn[i] * a + ks->cs[i] * b;
            }
            const double r = hypot(col[j - 1], col[j]);
            double c = 1.0, sn = 0.0;
            if (r != 0.0) {
                c = col[j - 1] / r;
                sn = col[j] / r;
            }
            col[j - 1] = r;
            for (int i = 0; i < j; ++i) ks->H[i][j - 1] = col[i];
            ks->cs[j - 1] = c;
            ks->sn[j - 1] = sn;
            const double gj = ks->g[j - 1];
            ks->g[j] = -sn * gj;
            ks->g[j - 1] = c * gj;
        }
        // column j, provisional: t, c = q_j . w, eta from Pythagoras
        const double cj = (beta - st) * nuinv;
        for (int i = 0; i < j; ++i) {
            ks->hcol[i] = tv[i];
            ks->ds[i] = sv[i];
        }
        ks->hcol[j] = cj;
        const double eta = sqrt(fmax(gamma - tt - cj * cj, 0.0));
        const bool brk = !(eta > 1e-14 * sqrt(gamma));
        // provisional residual estimate with column j as it stands
        double p0 = cj, p1 = eta;
        {
            double col[KMAX + 1];
            for (int i = 0; i < j; ++i) col[i] = tv[i];
            col[j] = cj;
            for (int i = 0; i < j; ++i) {
                const double a = col[i], b = col[i + 1];
                col[i] = ks->cs[i] * a + ks->sn[i] * b;
                col[i + 1] = -ks->sn[i] * a + ks->cs[i] * b;
            }
            p0 = col[j];
        }
        const double r = hypot(p0, p1);
        const double est = r != 0.0 ? fabs(p1 / r * ks->g[j]) : fabs(ks->g[j]);
        ks->est = est;
        ks->k = j + 1;
        ks->d_nuinv = nuinv;
        ks->d_c = cj;
        ks->d_eta = eta;
        ks->d_etainv = brk ? 0.0 : 1.0 / eta;
        ks->d_brk = brk ? 1 : 0;
        ks->scale[j + 1] = 1.0;   // the update pass stores u_{j+1} normalised
        bad = bad || !isfinite(est);
        ks->bad |= bad;
        ks->pending = (est <= ks->rtol * ks->ref || brk || bad || j + 1 >= ks->maxit) ? 1 : 0;
        break;
    }
    case FIN_DCGS2_LAST: {
        // sums = [s'_0..s'_j, alpha'] of u_{j+1} against q_0..q_j: column j final
        double col[KMAX + 2];
        for (int i = 0; i <= j; ++i) col[i] = ks->hcol[i];
        if (ks->d_brk) {
            col[j + 1] = 0.0;
        } else {
            double ss = 0.0;
            for (int i = 0; i <= j; ++i) {
                col[i] += ks->d_eta * sums[i];
                ss += sums[i] * sums[i];
            }
            col[j + 1] = ks->d_eta * sqrt(fmax(sums[j + 1] - ss, 0.0));
        }
        for (int i = 0; i < j; ++i) {
            const double a = col[i], b = col[i + 1];
            col[i] = ks->cs[i] * a + ks->sn[i] * b;
            col[i + 1] = -ks->sn[i] * a + ks->cs[i] * b;
        }
        const double r = hypot(col[j], col[j + 1]);
        double c = 1.0, sn = 0.0;
        if (r != 0.0) {
            c = col[j] / r;
            sn = col[j + 1] / r;
        }
        col[j] = r;
        for (int i = 0; i <= j; ++i) ks->H[i][j] = col[i];
        ks->cs[j] = c;
        ks->sn[j] = sn;
        const double gj = ks->g[j];
        ks->g[j + 1] = -sn * gj;
        ks->g[j] = c * gj;
        ks->est = fabs(ks->g[j + 1]);
        ks->bad |= !isfinite(ks->est);
        ks->k = j + 1;
        ks->done = 1;
        ks->pending = 0;
        kstate_solve_y(ks);
        break;
    }
    default:
        break;
    }
}

// The same finalisation done by a whole workgroup (every thread calls it):
// the projections are scaled in parallel, and for the Givens update the
// column and the earlier rotations are loaded into LDS in parallel before one
// thread applies the rotations -- the serial part then touches LDS only, not a
// chain of dependent global loads.  Arithmetic and its order are those of
// kstate_finalize.
__device__ void kstate_finalize_block(KState* ks, int mode, int j, const double* sums, int nd) {
    __shared__ double fcol[KMAX + 1], fcs[KMAX], fsn[KMAX], fg[KMAX + 1], fsc[KMAX + 1];
    __shared__ double fH[KMAX][KMAX + 1];
    __shared__ double fy[KMAX];
    __shared__ int fdone, fk;
    const int t = threadIdx.x;
    if (mode == FIN_PROJ1 || mode == FIN_PROJ2) {
        if (t < nd) {
            const double sd = ks->scale[t];
            const double h = sums[t] * sd;
            if (mode == FIN_PROJ1)
                ks->hcol[t] = h;
            else
                ks->hcol[t] += h;
            ks->coef[t] = h * sd;
        }
        return;
    }
    if (mode != FIN_GIVENS) {
        if (t == 0) kstate_finalize(ks, mode, j, sums, nd);
        return;
    }
    if (t <= j) fcol[t] = ks->hcol[t];
    if (t < j) {
        fcs[t] = ks->cs[t];
        fsn[t] = ks->sn[t];
    }
    __syncthreads();
    if (t == 0) {
        const double hn = sqrt(sums[0]);
        double hnorm2 = hn * hn;
        for (int i = 0; i <= j; ++i) hnorm2 += fcol[i] * fcol[i];
        for (int i = 0; i < j; ++i) {
            const double a = fcol[i], b = fcol[i + 1];
            fcol[i] = fcs[i] * a + fsn[i] * b;
            fcol[i + 1] = -fsn[i] * a + fcs[i] * b;
        }
        const double hj = fcol[j];
        const double r = hypot(hj, hn);
        double c = 1.0, sn = 0.0;
        if (r != 0.0) {
            c = hj / r;
            sn = hn / r;
        }
        fcol[j] = r;
        const double gj = ks->g[j];
        ks->cs[j] = c;
        ks->sn[j] = sn;
        ks->g[j + 1] = -sn * gj;
        ks->g[j] = c * gj;
        ks->scale[j + 1] = hn > 0.0 ? 1.0 / hn : 0.0;
        ks->k = j + 1;
        const double est = fabs(-sn * gj);
        ks->est = est;
        const bool bad = !isfinite(est) || !isfinite(hn);
        const bool conv = est <= ks->rtol * ks->ref;
        const bool brk = hn <= 1e-14 * sqrt(hnorm2);
        ks->bad |= bad;
        const int done = (conv || brk || bad || j + 1 >= ks->maxit) ? 1 : 0;
        if (done) ks->done = 1;
        fdone = done;
        fk = j + 1;
        fg[j] = c * gj;
    }
    __syncthreads();
    if (t <= j) ks->H[t][j] = fcol[t];
    if (!fdone) return;
    // Least-squares solve R y = g (R upper triangular, k x k) in LDS.
    const int k = fk;
    for (int e = t; e < k * k; e += blockDim.x) {
        const int i = e / k, c = e - i * k;
        if (i <= c) fH[i][c] = c == j ? fcol[i] : ks->H[i][c];
    }
    if (t < j) fg[t] = ks->g[t];
    if (t < k) fsc[t] = ks->scale[t];
    __syncthreads();
    if (t == 0) {
        for (int i = k - 1; i >= 0; --i) {
            double v = fg[i];
            for (int c = i + 1; c < k; ++c) v -= fH[i][c] * fy[c];
            const double d = fH[i][i];
            fy[i] = d != 0.0 ? v / d : 0.0;
        }
    }
    __syncthreads();
    if (t < k) ks->y[t] = ks->scale_update ? fy[t] * fsc[t] : fy[t];
}

// Block reduction of MAXD accumulators into partials[blockIdx][.].  Grids of
// at most FUSE_MAX blocks then finalise in the last block to arrive (arrival
// counter); larger grids leave the partials to k_reduce_finalize, launched
// right after them on the stream: a device-scope fence per block costs more
// than one extra launch once there are more than a handful of blocks.
constexpr int FUSE_MAX = 16;

template <int MAXD>
__device__ void block_finish(double (&acc)[MAXD], int nd, double* __restrict__ partials,
                             KState* ks, int mode, int j, double* out) {
    __shared__ double bsum[MAXD];
    __shared__ double sums[MAXD];
    __shared__ int amlast;
    block_sum_many<MAXD, VEC_THREADS>(acc, nd, bsum);
    for (int d = threadIdx.x; d < nd; d += VEC_THREADS)
        partials[(long long)blockIdx.x * MAXD + d] = bsum[d];
    if (gridDim.x > FUSE_MAX) return;   // uniform over the grid
    __threadfence();
    __syncthreads();
    unsigned* counter = ks ? &ks->counter : (unsigned*)(partials + PARTIALS_COUNTER);
    if (threadIdx.x == 0) {
        const unsigned prev = atomicAdd(counter, 1u);
        amlast = (prev == gridDim.x - 1);
    }
    __syncthreads();
    if (!amlast) return;
    __threadfence();
    sum_block_partials<VEC_THREADS>(partials, (int)gridDim.x, MAXD, nd, sums);
    if (threadIdx.x == 0) *counter = 0u;
    if (ks)
        kstate_finalize_block(ks, mode, j, sums, nd);
    else if (threadIdx.x == 0)
        for (int d = 0; d < nd; ++d) out[d] = sums[d];
}

// One block: sum the partials of a reduction grid (block order) and finalise.
// A full-size workgroup, so that the partial sums keep many loads in flight.
constexpr int RF_THREADS = 1024;
template <int MAXD>
__global__ __launch_bounds__(RF_THREADS) void k_reduce_finalize(const double* __restrict__ partials,
                                                                int nb, int nd, KState* ks,
                                                                int mode, int j, double* out) {
    __shared__ double sums[MAXD];
    if (ks && ks->done && mode != FIN_INIT_SELF && mode != FIN_INIT_REF) return;
    sum_block_partials<RF_THREADS>(partials, nb, MAXD, nd, sums);
    if (ks)
        kstate_finalize_block(ks, mode, j, sums, nd);
    else if (threadIdx.x == 0)
        for (int d = 0; d < nd; ++d) out[d] = sums[d];
}

template <int MAXD>
static void finish(hipStream_t s, unsigned nb, int nd, double* partials, KState* ks, int mode,
                   int j, double* out) {
    if ((int)nb <= FUSE_MAX) return;
    hipLaunchKernelGGL(k_reduce_finalize<MAXD>, dim3(1), dim3(RF_THREADS), 0, s, partials,
                       (int)nb, nd, ks, mode, j, out);
}

// ---------------------------------------------------------------------------
// w = invd .* b (invd optional), ||w||^2 -> FIN_INIT_*.
template <typename T>
__global__ __launch_bounds__(VEC_THREADS) void k_scale_norm(long long n, const T* __restrict__ b,
                                                            const T* __restrict__ invd,
                                                            T* __restrict__ w,
                                                            double* __restrict__ partials,
                                                            KState* ks, int mode) {
    double acc[1] = {0.0};
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        T v = b[i];
        if (invd) v *= invd[i];
        w[i] = v;
        acc[0] += (double)v * (double)v;
    }
    block_finish<1>(acc, 1, partials, ks, mode, 0, nullptr);
}

template <typename T>
__global__ __launch_bounds__(VEC_THREADS) void k_scale_norm4(long long n, const T* __restrict__ b,
                                                             const T* __restrict__ invd,
                                                             T* __restrict__ w,
                                                             double* __restrict__ partials,
                                                             KState* ks, int mode) {
    double acc[1] = {0.0};
    const long long n4 = n >> 2;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < n4; q += stride) {
        typename V4<T>::type bv = *reinterpret_cast<const typename V4<T>::type*>(b + 4 * q);
        if (invd) {
            const typename V4<T>::type dv = *reinterpret_cast<const typename V4<T>::type*>(invd + 4 * q);
            bv.x *= dv.x; bv.y *= dv.y; bv.z *= dv.z; bv.w *= dv.w;
        }
        *reinterpret_cast<typename V4<T>::type*>(w + 4 * q) = bv;
        acc[0] += (double)bv.x * (double)bv.x + (double)bv.y * (double)bv.y +
                  (double)bv.z * (double)bv.z + (double)bv.w * (double)bv.w;
    }
    for (long long i = 4 * n4 + blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += stride) {
        T v = b[i];
        if (invd) v *= invd[i];
        w[i] = v;
        acc[0] += (double)v * (double)v;
    }
    block_finish<1>(acc, 1, partials, ks, mode, 0, nullptr);
}

__global__ void k_init_state(KState* ks, int maxit, double rtol, int scale_update,
                             const double* ref) {
    if (threadIdx.x == 0) {
        ks->maxit = maxit;
        ks->rtol = rtol;
        ks->scale_update = scale_update;
        ks->done = 0;
        ks->bad = 0;
        ks->k = 0;
        ks->counter = 0u;
        if (ref) ks->ref = *ref;
    }
}

void launch_init_state(hipStream_t s, KState* ks, int maxit, double rtol, int scale_update,
                       const double* ref) {
    hipLaunchKernelGGL(k_init_state, dim3(1), dim3(64), 0, s, ks, maxit, rtol, scale_update, ref);
}

void launch_scale_norm(hipStream_t s, long long n, int prec, const void* b, const void* invd,
                       void* w, double* partials, KState* ks, int mode, int maxit, double rtol,
                       int scale_update) {
    (void)maxit;
    (void)rtol;
    (void)scale_update;
    const unsigned nb = red_grid(n);
    const size_t es = prec ? 4 : 8;
    if (al4(b, es) && al4(w, es) && (!invd || al4(invd, es))) {
        const unsigned nb4 = red_grid4(n);
        if (prec == 0)
            hipLaunchKernelGGL(k_scale_norm4<double>, dim3(nb4), dim3(VEC_THREADS), 0, s, n,
                               (const double*)b, (const double*)invd, (double*)w, partials, ks, mode);
        else
            hipLaunchKernelGGL(k_scale_norm4<float>, dim3(nb4), dim3(VEC_THREADS), 0, s, n,
                               (const float*)b, (const float*)invd, (float*)w, partials, ks, mode);
        finish<1>(s, nb4, 1, partials, ks, mode, 0, nullptr);
        return;
    }
    if (prec == 0)
        hipLaunchKernelGGL(k_scale_norm<double>, dim3(nb), dim3(VEC_THREADS), 0, s, n,
                           (const double*)b, (const double*)invd, (double*)w, partials, ks, mode);
    else
        hipLaunchKernelGGL(k_scale_norm<float>, dim3(nb), dim3(VEC_THREADS), 0, s, n,
                           (const float*)b, (const float*)invd, (float*)w, partials, ks, mode);
    finish<1>(s, nb, 1, partials, ks, mode, 0, nullptr);
}

// w = invd .* b without the norm (the s-step smoother's first vector: its
// norm comes out of the Gram pass).
template <typename T>
__global__ __launch_bounds__(VEC_THREADS) void k_scale(long long n, const T* __restrict__ b,
                                                       const T* __restrict__ invd,
                                                       T* __restrict__ w, int vec) {
    const long long stride = (long long)gridDim.x * blockDim.x;
    const long long t0 = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    long long tail = 0;
    if (vec) {
        const long long n4 = n >> 2;
        for (long long q = t0; q < n4; q += stride) {
            typename V4<T>::type bv = *reinterpret_cast<const typename V4<T>::type*>(b + 4 * q);
            const typename V4<T>::type dv = *reinterpret_cast<const typename V4<T>::type*>(invd + 4 * q);
            bv.x *= dv.x; bv.y *= dv.y; bv.z *= dv.z; bv.w *= dv.w;
            *reinterpret_cast<typename V4<T>::type*>(w + 4 * q) = bv;
        }
        tail = 4 * n4;
    }
    for (long long i = tail + t0; i < n; i += stride) w[i] = b[i] * invd[i];
}

void launch_scale(hipStream_t s, long long n, int prec, const void* b, const void* invd, void* w) {
    const size_t es = prec ? 4 : 8;
    const int vec = al4(b, es) && al4(w, es) && al4(invd, es);
    const unsigned nb = vec ? red_grid4(n) : red_grid(n);
    if (prec == 0)
        hipLaunchKernelGGL(k_scale<double>, dim3(nb), dim3(VEC_THREADS), 0, s, n, (const double*)b,
                           (const double*)invd, (double*)w, vec);
    else
        hipLaunchKernelGGL(k_scale<float>, dim3(nb), dim3(VEC_THREADS), 0, s, n, (const float*)b,
                           (const float*)invd, (float*)w, vec);
}

// ---------------------------------------------------------------------------
// Multi-dot: h_d = <V_d, w>, d < nd (mode FIN_PROJ1 / FIN_INIT_*).
template <typename TW, typename TV, int MAXD>
__global__ __launch_bounds__(VEC_THREADS) void k_mdot(long long n, const TW* __restrict__ w,
                                                      const TV* __restrict__ V, long long ldv,
                                                      int nd, double* __restrict__ partials,
                                                      KState* ks, int mode, int j) {
    if (ks && ks->done) return;
    double acc[MAXD];
#pragma unroll
    for (int d = 0; d < MAXD; ++d) acc[d] = 0.0;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        const double wv = (double)w[i];
#pragma unroll
        for (int d = 0; d < MAXD; ++d)
            if (d < nd) acc[d] += (double)V[(long long)d * ldv + i] * wv;
    }
    block_finish<MAXD>(acc, nd, partials, ks, mode, j, nullptr);
}

// w -= sum_d coef_d V_d, then either ||w||^2 (FIN_GIVENS) or the
// re-orthogonalisation projections <V_d, w> (FIN_PROJ2).
template <typename TW, typename TV, int MAXD>
__global__ __launch_bounds__(VEC_THREADS) void k_maxpy(long long n, TW* __restrict__ w,
                                                       const TV* __restrict__ V, long long ldv,
                                                       int nd, double* __restrict__ partials,
                                                       KState* ks, int mode, int j) {
    if (ks->done) return;
    __shared__ double c[MAXD];
    if (threadIdx.x < MAXD) c[threadIdx.x] = (int)threadIdx.x < nd ? ks->coef[threadIdx.x] : 0.0;
    __syncthreads();
    double acc[MAXD];
#pragma unroll
    for (int d = 0; d < MAXD; ++d) acc[d] = 0.0;
    const bool redot = mode == FIN_PROJ2;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        double wv = (double)w[i];
#pragma unroll
        for (int d = 0; d < MAXD; ++d)
            if (d < nd) wv -= c[d] * (double)V[(long long)d * ldv + i];
        const TW wo = (TW)wv;
        w[i] = wo;
        const double wr = (double)wo;
        if (redot) {
#pragma unroll
            for (int d = 0; d < MAXD; ++d)
                if (d < nd) acc[d] += (double)V[(long long)d * ldv + i] * wr;
        } else {
            acc[0] += wr * wr;
        }
    }
    block_finish<MAXD>(acc, redot ? nd : 1, partials, ks, mode, j, nullptr);
}

template <typename TW, typename TV, int MAXD>
__global__ __launch_bounds__(VEC_THREADS) void k_mdot4(long long n, const TW* __restrict__ w,
                                                       const TV* __restrict__ V, long long ldv,
                                                       int nd, double* __restrict__ partials,
                                                       KState* ks, int mode, int j) {
    if (ks && ks->done) return;
    double acc[MAXD];
#pragma unroll
    for (int d = 0; d < MAXD; ++d) acc[d] = 0.0;
    const long long n4 = n >> 2;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < n4; q += stride) {
        if (sizeof(TW) == 4 && sizeof(TV) == 4) {
            // FP32 storage: the four products are summed in FP32, the running
            // sum is FP64.
            const float4 x = *reinterpret_cast<const float4*>(w + 4 * q);
#pragma unroll
            for (int d = 0; d < MAXD; ++d)
                if (d < nd) {
                    const float4 v = *reinterpret_cast<const float4*>(V + (long long)d * ldv + 4 * q);
                    acc[d] += (double)(v.x * x.x + v.y * x.y + v.z * x.z + v.w * x.w);
                }
        } else {
            double wv[4];
            ld4(w + 4 * q, wv);
#pragma unroll
            for (int d = 0; d < MAXD; ++d)
                if (d < nd) {
                    double vv[4];
                    ld4(V + (long long)d * ldv + 4 * q, vv);
                    acc[d] += vv[0] * wv[0] + vv[1] * wv[1] + vv[2] * wv[2] + vv[3] * wv[3];
                }
        }
    }
    for (long long i = 4 * n4 + blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += stride) {
        const double wv = (double)w[i];
#pragma unroll
        for (int d = 0; d < MAXD; ++d)
            if (d < nd) acc[d] += (double)V[(long long)d * ldv + i] * wv;
    }
    block_finish<MAXD>(acc, nd, partials, ks, mode, j, nullptr);
}

// w -= sum_d coef_d V_d and ||w||^2 (FIN_GIVENS) -- the vectorised path has no
// re-orthogonalisation mode.
template <typename TW, typename TV, int MAXD>
__global__ __launch_bounds__(VEC_THREADS) void k_maxpy4(long long n, TW* __restrict__ w,
                                                        const TV* __restrict__ V, long long ldv,
                                                        int nd, double* __restrict__ partials,
                                                        KState* ks, int mode, int j) {
    if (ks->done) return;
    __shared__ double c[MAXD];
    if (threadIdx.x < MAXD) c[threadIdx.x] = (int)threadIdx.x < nd ? ks->coef[threadIdx.x] : 0.0;
    __syncthreads();
    double acc[1] = {0.0};
    const long long n4 = n >> 2;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < n4; q += stride) {
        double wv[4];
        if (sizeof(TW) == 4) {
            // FP32 storage: FP32 arithmetic, the basis read as float4
            float4 x = *reinterpret_cast<const float4*>(w + 4 * q);
#pragma unroll
            for (int d = 0; d < MAXD; ++d)
                if (d < nd) {
                    const float4 v = *reinterpret_cast<const float4*>(V + (long long)d * ldv + 4 * q);
                    const float cd = (float)c[d];
                    x.x -= cd * v.x; x.y -= cd * v.y; x.z -= cd * v.z; x.w -= cd * v.w;
                }
            wv[0] = x.x; wv[1] = x.y; wv[2] = x.z; wv[3] = x.w;
        } else {
            ld4(w + 4 * q, wv);
#pragma unroll
            for (int d = 0; d < MAXD; ++d)
                if (d < nd) {
                    double vv[4];
                    ld4(V + (long long)d * ldv + 4 * q, vv);
                    const double cd = c[d];
                    wv[0] -= cd * vv[0]; wv[1] -= cd * vv[1]; wv[2] -= cd * vv[2]; wv[3] -= cd * vv[3];
                }
        }
        // round to the storage type before the norm, as the scalar path does
        typename V4<TW>::type o;
        o.x = (TW)wv[0]; o.y = (TW)wv[1]; o.z = (TW)wv[2]; o.w = (TW)wv[3];
        *reinterpret_cast<typename V4<TW>::type*>(w + 4 * q) = o;
        if (sizeof(TW) == 4)
            acc[0] += (double)((float)o.x * (float)o.x + (float)o.y * (float)o.y +
                               (float)o.z * (float)o.z + (float)o.w * (float)o.w);
        else
            acc[0] += (double)o.x * (double)o.x + (double)o.y * (double)o.y +
                      (double)o.z * (double)o.z + (double)o.w * (double)o.w;
    }
    for (long long i = 4 * n4 + blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += stride) {
        double wv = (double)w[i];
#pragma unroll
        for (int d = 0; d < MAXD; ++d)
            if (d < nd) wv -= c[d] * (double)V[(long long)d * ldv + i];
        const TW wo = (TW)wv;
        w[i] = wo;
        acc[0] += (double)wo * (double)wo;
    }
    if (mode == FIN_NONE) return;   // uniform: no reduction wanted
    block_finish<1>(acc, 1, partials, ks, mode, j, nullptr);
}

// CGS2 middle passes in one stream (FP64 outer basis): w' = w - sum_d coef_d
// V_d with the first projections, stored, and the second projections V_d . w'
// accumulated from the stored values -- the same sums, in the same order, as
// a maxpy followed by a separate multi-dot over w'.
template <int MAXD>
__global__ __launch_bounds__(VEC_THREADS) void k_maxpy_mdot4(long long n, double* __restrict__ w,
                                                             const double* __restrict__ V,
                                                             long long ldv, int nd,
                                                             double* __restrict__ partials,
                                                             KState* ks, int j) {
    if (ks->done) return;
    __shared__ double c[MAXD];
    if (threadIdx.x < MAXD) c[threadIdx.x] = (int)threadIdx.x < nd ? ks->coef[threadIdx.x] : 0.0;
    __syncthreads();
    double acc[MAXD];
#pragma unroll
    for (int d = 0; d < MAXD; ++d) acc[d] = 0.0;
    const long long n4 = n >> 2;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < n4; q += stride) {
        double wv[4];
        ld4(w + 4 * q, wv);
#pragma unroll
        for (int d = 0; d < MAXD; ++d)
            if (d < nd) {
                double vv[4];
                ld4(V + (long long)d * ldv + 4 * q, vv);
                const double cd = c[d];
                wv[0] -= cd * vv[0]; wv[1] -= cd * vv[1]; wv[2] -= cd * vv[2]; wv[3] -= cd * vv[3];
            }
        st4(w + 4 * q, wv);
#pragma unroll
        for (int d = 0; d < MAXD; ++d)
            if (d < nd) {
                double vv[4];
                ld4(V + (long long)d * ldv + 4 * q, vv);
                acc[d] += vv[0] * wv[0] + vv[1] * wv[1] + vv[2] * wv[2] + vv[3] * wv[3];
            }
    }
    for (long long i = 4 * n4 + blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += stride) {
        double wv = w[i];
#pragma unroll
        for (int d = 0; d < MAXD; ++d)
            if (d < nd) wv -= c[d] * V[(long long)d * ldv + i];
        w[i] = wv;
#pragma unroll
        for (int d = 0; d < MAXD; ++d)
            if (d < nd) acc[d] += V[(long long)d * ldv + i] * wv;
    }
    block_finish<MAXD>(acc, nd, partials, ks, FIN_PROJ2, j, nullptr);
}

// Delayed CGS2 (outer FGMRES, FP64 basis).  Step j holds clean q_0..q_{j-1}
// in V[0..j-1], the current vector u (once orthogonalised, not yet cleaned;
// its value is V[j] * scale[j]) and w = A z_j in V[j+1].  One pass forms all
// inner products that step needs; after the finalisation the second pass
// writes q_j = (u - Q s) / nu over V[j] and u_{j+1} = (w - Q t - c q_j) / eta
// over V[j+1].  Step j thereby re-orthogonalises q_j (lagging by one step)
// and orthogonalises w once: two streams over the basis instead of the three
// of classical CGS2.
constexpr int DC_MAXD = 2 * KMAX + 3;
static_assert(DC_MAXD <= RED_WIDTH, "reduction width");

__global__ __launch_bounds__(VEC_THREADS) void k_dcgs2_dots(long long n, const double* __restrict__ V,
                                                           long long ldv, int j,
                                                           double* __restrict__ partials,
                                                           KState* ks) {
    if (ks->done) return;
    const double us = ks->scale[j];
    double acc[DC_MAXD];
#pragma unroll
    for (int d = 0; d < DC_MAXD; ++d) acc[d] = 0.0;
    const double* U = V + (long long)j * ldv;
    const double* W = V + (long long)(j + 1) * ldv;
    const long long n4 = n >> 2;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < n4; q += stride) {
        double uv[4], wv[4];
        ld4(U + 4 * q, uv);
        ld4(W + 4 * q, wv);
        uv[0] *= us; uv[1] *= us; uv[2] *= us; uv[3] *= us;
#pragma unroll
        for (int d = 0; d < KMAX; ++d)
            if (d < j) {
                double qv[4];
                ld4(V + (long long)d * ldv + 4 * q, qv);
                acc[d] += qv[0] * uv[0] + qv[1] * uv[1] + qv[2] * uv[2] + qv[3] * uv[3];
                acc[KMAX + d] += qv[0] * wv[0] + qv[1] * wv[1] + qv[2] * wv[2] + qv[3] * wv[3];
            }
        acc[2 * KMAX] += uv[0] * uv[0] + uv[1] * uv[1] + uv[2] * uv[2] + uv[3] * uv[3];
        acc[2 * KMAX + 1] += uv[0] * wv[0] + uv[1] * wv[1] + uv[2] * wv[2] + uv[3] * wv[3];
        acc[2 * KMAX + 2] += wv[0] * wv[0] + wv[1] * wv[1] + wv[2] * wv[2] + wv[3] * wv[3];
    }
    for (long long i = 4 * n4 + blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += stride) {
        const double u = U[i] * us, w = W[i];
#pragma unroll
        for (int d = 0; d < KMAX; ++d)
            if (d < j) {
                const double qv = V[(long long)d * ldv + i];
                acc[d] += qv * u;
                acc[KMAX + d] += qv * w;
            }
        acc[2 * KMAX] += u * u;
        acc[2 * KMAX + 1] += u * w;
        acc[2 * KMAX + 2] += w * w;
    }
    // layout [s_0..s_{KMAX-1}, t_0..t_{KMAX-1}, alpha, beta, gamma] (zeros past j)
    block_finish<DC_MAXD>(acc, DC_MAXD, partials, ks, FIN_DCGS2, j, nullptr);
}

void launch_dcgs2_dots(hipStream_t s, long long n, const double* V, long long ldv, int j,
                       double* partials, KState* ks) {
    const unsigned nb4 = red_grid4(n);
    hipLaunchKernelGGL(k_dcgs2_dots, dim3(nb4), dim3(VEC_THREADS), 0, s, n, V, ldv, j, partials, ks);
    finish<DC_MAXD>(s, nb4, DC_MAXD, partials, ks, FIN_DCGS2, j, nullptr);
}

__global__ __launch_bounds__(VEC_THREADS) void k_dcgs2_update(long long n, double* __restrict__ V,
                                                             long long ldv, int j, KState* ks) {
    if (ks->done) return;
    __shared__ double cs_[KMAX], ct_[KMAX];
    if (threadIdx.x < KMAX) {
        cs_[threadIdx.x] = (int)threadIdx.x < j ? ks->ds[threadIdx.x] : 0.0;
        ct_[threadIdx.x] = (int)threadIdx.x < j ? ks->hcol[threadIdx.x] : 0.0;
    }
    __syncthreads();
    const double us = ks->scale[j] * ks->d_nuinv;   // q_j = (us u_stored - Q s nuinv) ...
    const double nuinv = ks->d_nuinv, c = ks->d_c, etainv = ks->d_etainv;
    double* U = V + (long long)j * ldv;
    double* W = V + (long long)(j + 1) * ldv;
    const long long n4 = n >> 2;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < n4; q += stride) {
        double uv[4], wv[4];
        ld4(U + 4 * q, uv);
        ld4(W + 4 * q, wv);
        double qs[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int d = 0; d < KMAX; ++d)
            if (d < j) {
                double qv[4];
                ld4(V + (long long)d * ldv + 4 * q, qv);
                const double a = cs_[d], b = ct_[d];
                qs[0] += a * qv[0]; qs[1] += a * qv[1]; qs[2] += a * qv[2]; qs[3] += a * qv[3];
                wv[0] -= b * qv[0]; wv[1] -= b * qv[1]; wv[2] -= b * qv[2]; wv[3] -= b * qv[3];
            }
        double qj[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            qj[e] = uv[e] * us - qs[e] * nuinv;
            wv[e] = (wv[e] - c * qj[e]) * etainv;
        }
        st4(U + 4 * q, qj);
        st4(W + 4 * q, wv);
    }
    for (long long i = 4 * n4 + blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += stride) {
        double qs = 0.0, w = W[i];
#pragma unroll
        for (int d = 0; d < KMAX; ++d)
            if (d < j) {
                const double qv = V[(long long)d * ldv + i];
                qs += cs_[d] * qv;
                w -= ct_[d] * qv;
            }
        const double qj = U[i] * us - qs * nuinv;
        U[i] = qj;
        W[i] = (w - c * qj) * etainv;
    }
}

void launch_dcgs2_update(hipStream_t s, long long n, double* V, long long ldv, int j, KState* ks) {
    const unsigned nb4 = red_grid4(n);
    hipLaunchKernelGGL(k_dcgs2_update, dim3(nb4), dim3(VEC_THREADS), 0, s, n, V, ldv, j, ks);
}

bool launch_maxpy_mdot(hipStream_t s, long long n, double* w, const double* V, long long ldv,
                       int nd, double* partials, KState* ks, int j) {
    if (!(ldv % 4 == 0 && al4(w, 8) && al4(V, 8)) || nd > KMAX) return false;
    const unsigned nb4 = red_grid4(n);
    hipLaunchKernelGGL((k_maxpy_mdot4<KMAX>), dim3(nb4), dim3(VEC_THREADS), 0, s, n, w, V, ldv,
                       nd, partials, ks, j);
    finish<KMAX>(s, nb4, nd, partials, ks, FIN_PROJ2, j, nullptr);
    return true;
}

template <int MAXD>
static void mdot_dispatch(hipStream_t s, long long n, int pw, int pv, const void* w,
                          const void* V, long long ldv, int nd, double* partials, KState* ks,
                          int mode, int j) {
    const unsigned nb = red_grid(n);
    const bool vec = pw == pv && ldv % 4 == 0 && al4(w, pw ? 4 : 8) && al4(V, pv ? 4 : 8);
    if (vec) {
        const unsigned nb4 = red_grid4(n);
        if (pw == 0)
            hipLaunchKernelGGL((k_mdot4<double, double, MAXD>), dim3(nb4), dim3(VEC_THREADS), 0, s,
                               n, (const double*)w, (const double*)V, ldv, nd, partials, ks, mode, j);
        else
            hipLaunchKernelGGL((k_mdot4<float, float, MAXD>), dim3(nb4), dim3(VEC_THREADS), 0, s,
                               n, (const float*)w, (const float*)V, ldv, nd, partials, ks, mode, j);
        finish<MAXD>(s, nb4, nd, partials, ks, mode, j, nullptr);
        return;
    }
    if (pw == 0 && pv == 0)
        hipLaunchKernelGGL((k_mdot<double, double, MAXD>), dim3(nb), dim3(VEC_THREADS), 0, s, n,
                           (const double*)w, (const double*)V, ldv, nd, partials, ks, mode, j);
    else if (pw == 1 && pv == 1)
        hipLaunchKernelGGL((k_mdot<float, float, MAXD>), dim3(nb), dim3(VEC_THREADS), 0, s, n,
                           (const float*)w, (const float*)V, ldv, nd, partials, ks, mode, j);
    else if (pw == 0 && pv == 1)
        hipLaunchKernelGGL((k_mdot<double, float, MAXD>), dim3(nb), dim3(VEC_THREADS), 0, s, n,
                           (const double*)w, (const float*)V, ldv, nd, partials, ks, mode, j);
    else
        hipLaunchKernelGGL((k_mdot<float, double, MAXD>), dim3(nb), dim3(VEC_THREADS), 0, s, n,
                           (const float*)w, (const double*)V, ldv, nd, partials, ks, mode, j);
    finish<MAXD>(s, nb, nd, partials, ks, mode, j, nullptr);
}

void launch_mdot(hipStream_t s, long long n, int prec_w, int prec_v, const void* w,
                 const void* V, long long ldv, int nd, double* partials, KState* ks, int mode,
                 int j, int maxd) {
    if (maxd <= 1)
        mdot_dispatch<1>(s, n, prec_w, prec_v, w, V, ldv, nd, partials, ks, mode, j);
    else if (maxd <= SMAX)
        mdot_dispatch<SMAX>(s, n, prec_w, prec_v, w, V, ldv, nd, partials, ks, mode, j);
    else
        mdot_dispatch<KMAX>(s, n, prec_w, prec_v, w, V, ldv, nd, partials, ks, mode, j);
}

template <int MAXD>
static void maxpy_dispatch(hipStream_t s, long long n, int pw, int pv, void* w, const void* V,
                           long long ldv, int nd, double* partials, KState* ks, int mode, int j) {
    const unsigned nb = red_grid(n);
    const bool vec = (mode == FIN_GIVENS || mode == FIN_NONE) && pw == pv && ldv % 4 == 0 &&
                     al4(w, pw ? 4 : 8) && al4(V, pv ? 4 : 8);
    if (vec) {
        const unsigned nb4 = red_grid4(n);
        if (pw == 0)
            hipLaunchKernelGGL((k_maxpy4<double, double, MAXD>), dim3(nb4), dim3(VEC_THREADS), 0,
                               s, n, (double*)w, (const double*)V, ldv, nd, partials, ks, mode, j);
        else
            hipLaunchKernelGGL((k_maxpy4<float, float, MAXD>), dim3(nb4), dim3(VEC_THREADS), 0, s,
                               n, (float*)w, (const float*)V, ldv, nd, partials, ks, mode, j);
        if (mode != FIN_NONE) finish<1>(s, nb4, 1, partials, ks, mode, j, nullptr);
        return;
    }
    if (pw == 0 && pv == 0)
        hipLaunchKernelGGL((k_maxpy<double, double, MAXD>), dim3(nb), dim3(VEC_THREADS), 0, s, n,
                           (double*)w, (const double*)V, ldv, nd, partials, ks, mode, j);
    else
        hipLaunchKernelGGL((k_maxpy<float, float, MAXD>), dim3(nb), dim3(VEC_THREADS), 0, s, n,
                           (float*)w, (const float*)V, ldv, nd, partials, ks, mode, j);
    if (mode != FIN_NONE) finish<MAXD>(s, nb, mode == FIN_PROJ2 ? nd : 1, partials, ks, mode, j, nullptr);
}

void launch_maxpy(hipStream_t s, long long n, int prec_w, int prec_v, void* w, const void* V,
                  long long ldv, int nd, double* partials, KState* ks, int mode, int j, int maxd) {
    if (maxd <= SMAX)
        maxpy_dispatch<SMAX>(s, n, prec_w, prec_v, w, V, ldv, nd, partials, ks, mode, j);
    else
        maxpy_dispatch<KMAX>(s, n, prec_w, prec_v, w, V, ldv, nd, partials, ks, mode, j);
}

// x = (zero ? 0 : x) + sum_{d < k} y_d V_d.
template <typename TX, typename TV>
__global__ __launch_bounds__(VEC_THREADS) void k_update(long long n, TX* __restrict__ x,
                                                        const TV* __restrict__ V, long long ldv,
                                                        const KState* __restrict__ ks,
                                                        int zero_x0) {
    const int k = ks->k;
    if (k == 0 && !zero_x0) return;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        double v = zero_x0 ? 0.0 : (double)x[i];
        for (int d = 0; d < k; ++d) v += ks->y[d] * (double)V[(long long)d * ldv + i];
        x[i] = (TX)v;
    }
}

template <typename TX, typename TV>
__global__ __launch_bounds__(VEC_THREADS) void k_update4(long long n, TX* __restrict__ x,
                                                         const TV* __restrict__ V, long long ldv,
                                                         const KState* __restrict__ ks,
                                                         int zero_x0) {
    const int k = ks->k;
    if (k == 0 && !zero_x0) return;
    const long long n4 = n >> 2;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < n4; q += stride) {
        double xv[4] = {0.0, 0.0, 0.0, 0.0};
        if (!zero_x0) ld4(x + 4 * q, xv);
        for (int d = 0; d < k; ++d) {
            double vv[4];
            ld4(V + (long long)d * ldv + 4 * q, vv);
            const double yd = ks->y[d];
            xv[0] += yd * vv[0]; xv[1] += yd * vv[1]; xv[2] += yd * vv[2]; xv[3] += yd * vv[3];
        }
        st4(x + 4 * q, xv);
    }
    for (long long i = 4 * n4 + blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += stride) {
        double v = zero_x0 ? 0.0 : (double)x[i];
        for (int d = 0; d < k; ++d) v += ks->y[d] * (double)V[(long long)d * ldv + i];
        x[i] = (TX)v;
    }
}

void launch_update(hipStream_t s, long long n, int prec_x, int prec_v, void* x, const void* V,
                   long long ldv, KState* ks, int zero_x0, int maxd) {
    (void)maxd;
    long long nb = (n + VEC_THREADS - 1) / VEC_THREADS;
    if (nb > 65535) nb = 65535;
    const bool vec = ldv % 4 == 0 && al4(x, prec_x ? 4 : 8) && al4(V, prec_v ? 4 : 8);
    if (vec) {
        const unsigned nb4 = red_grid4(n);
        if (prec_x == 0 && prec_v == 0)
            hipLaunchKernelGGL((k_update4<double, double>), dim3(nb4), dim3(VEC_THREADS), 0, s, n,
                               (double*)x, (const double*)V, ldv, ks, zero_x0);
        else if (prec_x == 0 && prec_v == 1)
            hipLaunchKernelGGL((k_update4<double, float>), dim3(nb4), dim3(VEC_THREADS), 0, s, n,
                               (double*)x, (const float*)V, ldv, ks, zero_x0);
        else
            hipLaunchKernelGGL((k_update4<float, float>), dim3(nb4), dim3(VEC_THREADS), 0, s, n,
                               (float*)x, (const float*)V, ldv, ks, zero_x0);
        return;
    }
    if (prec_x == 0 && prec_v == 0)
        hipLaunchKernelGGL((k_update<double, double>), dim3((unsigned)nb), dim3(VEC_THREADS), 0, s,
                           n, (double*)x, (const double*)V, ldv, ks, zero_x0);
    else if (prec_x == 0 && prec_v == 1)
        hipLaunchKernelGGL((k_update<double, float>), dim3((unsigned)nb), dim3(VEC_THREADS), 0, s,
                           n, (double*)x, (const float*)V, ldv, ks, zero_x0);
    else
        hipLaunchKernelGGL((k_update<float, float>), dim3((unsigned)nb), dim3(VEC_THREADS), 0, s,
                           n, (float*)x, (const float*)V, ldv, ks, zero_x0);
}

// Plain dot product into out[0] (deterministic).
__global__ __launch_bounds__(VEC_THREADS) void k_dot(long long n, const double* __restrict__ a,
                                                     const double* __restrict__ b,
                                                     double* __restrict__ partials,
                                                     double* __restrict__ out) {
    double acc[1] = {0.0};
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        acc[0] += a[i] * b[i];
    block_finish<1>(acc, 1, partials, nullptr, FIN_SUM, 0, out);
}

void launch_dot(hipStream_t s, long long n, const double* a, const double* b, double* partials,
                double* out) {
    const unsigned nb = red_grid(n);
    hipLaunchKernelGGL(k_dot, dim3(nb), dim3(VEC_THREADS), 0, s, n, a, b, partials, out);
    finish<1>(s, nb, 1, partials, nullptr, FIN_SUM, 0, out);
}

// ---------------------------------------------------------------------------
// Coarsest level: Jacobi-preconditioned GMRES(restart), at most maxit
// iterations, stopping at rtol times the initial preconditioned residual, in
// FP64, in one workgroup (§3.2: the coarse grid solver).
constexpr int CT = 1024;

__device__ __forceinline__ double block_sum_1(double v, double* sh) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    v = wave_sum(v);
    __syncthreads();
    if (lane == 0) sh[wave] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0) {
        for (int w = 0; w < CT / 64; ++w) t += sh[w];
        sh[CT / 64] = t;
    }
    __syncthreads();
    return sh[CT / 64];
}

// LDS layout: the current basis vector v_j and the work vector w (2n doubles)
// when they fit (USE_LDS), otherwise both live in global memory.
template <typename TIO, bool USE_LDS>
__global__ __launch_bounds__(CT) void k_coarse_gmres(
    int nx, int ny, int nt, int nplanes, const double* __restrict__ st,
    const int* __restrict__ pmap, const double* __restrict__ invd, const TIO* __restrict__ bio,
    TIO* __restrict__ xio, double* __restrict__ V, double* __restrict__ work, int maxit,
    int restart, double rtol, int zero_x0, int trans) {
    const int row = nx + 1, P = row * (ny + 1), n = P * (nt + 1);
    const long long DS = (long long)P * nplanes;
    extern __shared__ double dyn[];
    double* x = work;
    double* w = USE_LDS ? dyn : work + n;
    double* vj = USE_LDS ? dyn + n : work + 2 * n;
    __shared__ double H[KMAX + 1][KMAX];
    __shared__ double cs[KMAX], sn[KMAX], g[KMAX + 1], y[KMAX], h[KMAX + 1];
    __shared__ double sh[CT / 64 + 1];
    __shared__ int flag;
    const int tid = threadIdx.x;

    // Plane map in LDS; each thread's node coordinates computed once (a thread
    // owns nodes tid, tid + CT, ...; at most CMAXN of them are cached).
    __shared__ int pm[1025];
    for (int q = tid; q <= nt && q < 1025; q += CT) pm[q] = pmap[q];
    constexpr int CMAXN = 4;
    int cn[CMAXN], cj[CMAXN], ci[CMAXN];
#pragma unroll
    for (int u = 0; u < CMAXN; ++u) {
        const int idx = tid + u * CT;
        const int nn0 = idx / P, r = idx - nn0 * P;
        cn[u] = nn0;
        cj[u] = r / row;
        ci[u] = r - cj[u] * row;
    }
    __syncthreads();
    const bool pm_lds = nt < 1025;
    // (A v)[idx] for a vector in LDS/global, forward or transposed stencil;
    // u is the index of idx among this thread's nodes.
    auto apply = [&](const double* in, int idx, int u) -> double {
        int nn0, j, i;
        if (u < CMAXN) {
            nn0 = cn[u];
            j = cj[u];
            i = ci[u];
        } else {
            nn0 = idx / P;
            const int r = idx - nn0 * P;
            j = r / row;
            i = r - j * row;
        }
        const int r = j * row + i;
        double acc = 0.0;
#pragma unroll
        for (int dn = -1; dn <= 1; ++dn) {
            const int nn = nn0 + dn;
            if (nn < 0 || nn > nt) continue;
            const int pl = pm_lds ? (trans ? pm[nn] : pm[nn0]) : (trans ? pmap[nn] : pmap[nn0]);
#pragma unroll
            for (int dj = -1; dj <= 1; ++dj) {
                const int jj = j + dj;
                if (jj < 0 || jj > ny) continue;
#pragma unroll
                for (int di = -1; di <= 1; ++di) {
                    const int ii = i + di;
                    if (ii < 0 || ii > nx) continue;
                    const int d = (dn + 1) * 9 + (dj + 1) * 3 + (di + 1);
                    const int nb = nn * P + jj * row + ii;
                    const double a = trans ? st[(long long)(26 - d) * DS + (long long)pl * P + jj * row + ii]
                                           : st[(long long)d * DS + (long long)pl * P + r];
                    acc += a * in[nb];
                }
            }
        }
        return acc;
    };

    for (int i = tid; i < n; i += CT) x[i] = zero_x0 ? 0.0 : (double)xio[i];
    __syncthreads();
    double loc = 0.0;
    for (int i = tid, u = 0; i < n; i += CT, ++u) {
        const double v = invd[i] * ((double)bio[i] - (zero_x0 ? 0.0 : apply(x, i, u)));
        w[i] = v;
        loc += v * v;
    }
    double beta = sqrt(block_sum_1(loc, sh));
    const double ref = beta;
    int its = 0;
    bool finished = !(beta > 0.0) || !isfinite(beta);
    while (!finished) {
        const double ib = 1.0 / beta;
        for (int i = tid; i < n; i += CT) {
            const double v = w[i] * ib;
            vj[i] = v;
            V[i] = v;
        }
        if (tid < KMAX + 1) g[tid] = 0.0;
        __syncthreads();
        if (tid == 0) g[0] = beta;
        int k = 0;
        bool stop = false;
        for (int jcol = 0; jcol < restart && !stop; ++jcol) {
            __syncthreads();
            for (int i = tid, u = 0; i < n; i += CT, ++u) w[i] = invd[i] * apply(vj, i, u);
            __syncthreads();
            // h_d = <v_d, w>, d <= jcol: 32 lanes per d, 4 independent sums
            {
                const int d = tid >> 5, q = tid & 31;
                double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
                if (d <= jcol) {
                    const double* vd = V + (long long)d * n;
                    int i = q;
                    for (; i + 224 < n; i += 256) {
                        double t[8];
#pragma unroll
                        for (int u = 0; u < 8; ++u) t[u] = vd[i + 32 * u];
                        a0 += t[0] * w[i] + t[4] * w[i + 128];
                        a1 += t[1] * w[i + 32] + t[5] * w[i + 160];
                        a2 += t[2] * w[i + 64] + t[6] * w[i + 192];
                        a3 += t[3] * w[i + 96] + t[7] * w[i + 224];
                    }
                    for (; i < n; i += 32) a0 += vd[i] * w[i];
                }
                double a = (a0 + a1) + (a2 + a3);
#pragma unroll
                for (int o = 16; o > 0; o >>= 1) a += __shfl_down(a, o, 32);
                if (q == 0 && d <= jcol) h[d] = a;
            }
            __syncthreads();
            loc = 0.0;
            for (int i = tid; i < n; i += CT) {
                // eight independent loads per step keep the L2 latency hidden
                double v0 = w[i], v1 = 0.0;
                int d = 0;
                for (; d + 7 <= jcol; d += 8) {
                    double t[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) t[u] = V[(long long)(d + u) * n + i];
#pragma unroll
                    for (int u = 0; u < 8; u += 2) {
                        v0 -= h[d + u] * t[u];
                        v1 -= h[d + u + 1] * t[u + 1];
                    }
                }
                for (; d <= jcol; ++d) v0 -= h[d] * V[(long long)d * n + i];
                const double v = v0 + v1;
                w[i] = v;
                loc += v * v;
            }
            const double hn = sqrt(block_sum_1(loc, sh));
            if (tid == 0) {
                double hn2 = hn * hn;
                for (int i = 0; i <= jcol; ++i) {
                    H[i][jcol] = h[i];
                    hn2 += h[i] * h[i];
                }
                for (int i = 0; i < jcol; ++i) {
                    const double a = H[i][jcol], bb = H[i + 1][jcol];
                    H[i][jcol] = cs[i] * a + sn[i] * bb;
                    H[i + 1][jcol] = -sn[i] * a + cs[i] * bb;
                }
                const double hj = H[jcol][jcol];
                const double r = hypot(hj, hn);
                double c = 1.0, s_ = 0.0;
                if (r != 0.0) {
                    c = hj / r;
                    s_ = hn / r;
                }
                cs[jcol] = c;
                sn[jcol] = s_;
                H[jcol][jcol] = r;
                g[jcol + 1] = -s_ * g[jcol];
                g[jcol] = c * g[jcol];
                const double est = fabs(g[jcol + 1]);
                int f = 0;
                if (est <= rtol * ref) f = 1;
                if (hn <= 1e-14 * sqrt(hn2) || !isfinite(est)) f = 2;
                if (its + 1 >= maxit) f |= 4;
                flag = f;
            }
            __syncthreads();
            ++its;
            k = jcol + 1;
            const int f = flag;
            if (f) {
                stop = true;
                finished = true;
            } else if (jcol + 1 < restart) {
                const double ih = 1.0 / hn;
                for (int i = tid; i < n; i += CT) {
                    const double v = w[i] * ih;
                    vj[i] = v;
                    V[(long long)(jcol + 1) * n + i] = v;
                }
            }
        }
        __syncthreads();
        if (tid == 0) {
            for (int i = k - 1; i >= 0; --i) {
                double v = g[i];
                for (int c = i + 1; c < k; ++c) v -= H[i][c] * y[c];
                y[i] = H[i][i] != 0.0 ? v / H[i][i] : 0.0;
            }
        }
        __syncthreads();
        for (int i = tid; i < n; i += CT) {
            double v0 = x[i], v1 = 0.0;
            int d = 0;
            for (; d + 7 < k; d += 8) {
                double t[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) t[u] = V[(long long)(d + u) * n + i];
#pragma unroll
                for (int u = 0; u < 8; u += 2) {
                    v0 += y[d + u] * t[u];
                    v1 += y[d + u + 1] * t[u + 1];
                }
            }
            for (; d < k; ++d) v0 += y[d] * V[(long long)d * n + i];
            x[i] = v0 + v1;
        }
        __syncthreads();
        if (finished || its >= maxit) break;
        loc = 0.0;
        for (int i = tid, u = 0; i < n; i += CT, ++u) {
            const double v = invd[i] * ((double)bio[i] - apply(x, i, u));
            w[i] = v;
            loc += v * v;
        }
        beta = sqrt(block_sum_1(loc, sh));
        if (!(beta > 0.0) || !isfinite(beta)) break;
    }
    __syncthreads();
    for (int i = tid; i < n; i += CT) xio[i] = (TIO)x[i];
}

// work must hold 3 n doubles (x, and w / v_j when they do not fit in LDS).
void launch_coarse_solve(hipStream_t s, const Level& L, int prec_io, int trans, const void* b,
                         void* x, double* V, double* work, int maxit, int restart, double rtol,
                         int zero_x0) {
    const long long n = L.nn;
    const size_t lds = (size_t)2 * n * sizeof(double);
    const bool use_lds = lds <= 48 * 1024;   // with ~14 KB static LDS: within 64 KB per block
    const size_t dyn = use_lds ? lds : 0;
    if (prec_io == 0) {
        if (use_lds)
            hipLaunchKernelGGL((k_coarse_gmres<double, true>), dim3(1), dim3(CT), dyn, s, L.nx, L.ny,
                               L.nt, L.nplanes, L.st64, L.plane_map, L.invd64, (const double*)b,
                               (double*)x, V, work, maxit, restart, rtol, zero_x0, trans);
        else
            hipLaunchKernelGGL((k_coarse_gmres<double, false>), dim3(1), dim3(CT), 0, s, L.nx, L.ny,
                               L.nt, L.nplanes, L.st64, L.plane_map, L.invd64, (const double*)b,
                               (double*)x, V, work, maxit, restart, rtol, zero_x0, trans);
    } else {
        if (use_lds)
            hipLaunchKernelGGL((k_coarse_gmres<float, true>), dim3(1), dim3(CT), dyn, s, L.nx, L.ny,
                               L.nt, L.nplanes, L.st64, L.plane_map, L.invd64, (const float*)b,
                               (float*)x, V, work, maxit, restart, rtol, zero_x0, trans);
        else
            hipLaunchKernelGGL((k_coarse_gmres<float, false>), dim3(1), dim3(CT), 0, s, L.nx, L.ny,
                               L.nt, L.nplanes, L.st64, L.plane_map, L.invd64, (const float*)b,
                               (float*)x, V, work, maxit, restart, rtol, zero_x0, trans);
    }
}

// ---------------------------------------------------------------------------
// Jacobi-preconditioned conjugate gradients for the filter system, scalars on
// the device.  scal: [0] rz, [1] alpha, [2] beta, [3] rr, [4] rz_new.
__global__ __launch_bounds__(VEC_THREADS) void k_cg_pq(long long n, const double* __restrict__ p,
                                                       const double* __restrict__ q,
                                                       double* __restrict__ partials,
                                                       double* __restrict__ scal) {
    double acc[1] = {0.0};
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        acc[0] += p[i] * q[i];
    block_finish<1>(acc, 1, partials, nullptr, FIN_SUM, 0, scal + 5);
}

__global__ __launch_bounds__(VEC_THREADS) void k_cg_update(
    long long n, double* __restrict__ x, double* __restrict__ r, double* __restrict__ z,
    const double* __restrict__ p, const double* __restrict__ q, const double* __restrict__ invd,
    double* __restrict__ partials, double* __restrict__ scal) {
    const double alpha = scal[0] / scal[5];
    double acc[2] = {0.0, 0.0};
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        x[i] += alpha * p[i];
        const double rv = r[i] - alpha * q[i];
        r[i] = rv;
        const double zv = invd[i] * rv;
        z[i] = zv;
        acc[0] += rv * zv;
        acc[1] += rv * rv;
    }
    block_finish<2>(acc, 2, partials, nullptr, FIN_SUM, 0, scal + 6);
}

__global__ void k_cg_p(long long n, const double* __restrict__ z, double* __restrict__ p,
                       double* __restrict__ scal, int first) {
    const double beta = first ? 0.0 : scal[6] / scal[0];
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        p[i] = z[i] + beta * p[i];
    // rz <- rz_new after every thread has read the old value: done by the host
    // through step 3 (below) on the next launch.
}

// r = b, z = invd .* b, p = z; sums r.z, r.r -> scal[6], scal[7].
__global__ __launch_bounds__(VEC_THREADS) void k_cg_init(long long n, const double* __restrict__ b,
                                                         double* __restrict__ r,
                                                         double* __restrict__ z,
                                                         double* __restrict__ p,
                                                         const double* __restrict__ invd,
                                                         double* __restrict__ partials,
                                                         double* __restrict__ scal) {
    double acc[2] = {0.0, 0.0};
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        const double rv = b[i];
        const double zv = invd[i] * rv;
        r[i] = rv;
        z[i] = zv;
        p[i] = zv;
        acc[0] += rv * zv;
        acc[1] += rv * rv;
    }
    block_finish<2>(acc, 2, partials, nullptr, FIN_SUM, 0, scal + 6);
}

__global__ void k_cg_roll(double* scal) {
    if (threadIdx.x == 0) {
        scal[0] = scal[6];
        scal[3] = scal[7];
    }
}

void launch_cg_step(hipStream_t s, int step, long long n, double* x, double* r, double* z,
                    double* p, const double* q, const double* invd, double* partials,
                    double* scal, const int* skip) {
    (void)skip;
    const unsigned nb = red_grid(n);
    long long nb2 = (n + VEC_THREADS - 1) / VEC_THREADS;
    if (nb2 > 65535) nb2 = 65535;
    switch (step) {
    case 0:   // p . q
        hipLaunchKernelGGL(k_cg_pq, dim3(nb), dim3(VEC_THREADS), 0, s, n, p, q, partials, scal);
        finish<1>(s, nb, 1, partials, nullptr, FIN_SUM, 0, scal + 5);
        break;
    case 1:   // x, r, z updates and r.z, r.r
        hipLaunchKernelGGL(k_cg_update, dim3(nb), dim3(VEC_THREADS), 0, s, n, x, r, z, p, q, invd,
                           partials, scal);
        finish<2>(s, nb, 2, partials, nullptr, FIN_SUM, 0, scal + 6);
        break;
    case 2:   // p = z + beta p
        hipLaunchKernelGGL(k_cg_p, dim3((unsigned)nb2), dim3(VEC_THREADS), 0, s, n, z, p, scal, 0);
        break;
    case 3:   // p = z (first iteration)
        hipLaunchKernelGGL(k_cg_p, dim3((unsigned)nb2), dim3(VEC_THREADS), 0, s, n, z, p, scal, 1);
        break;
    case 4:   // roll scalars
        hipLaunchKernelGGL(k_cg_roll, dim3(1), dim3(64), 0, s, scal);
        break;
    case 5:   // init from b (= q argument): r = b, z = p = invd .* b
        hipLaunchKernelGGL(k_cg_init, dim3(nb), dim3(VEC_THREADS), 0, s, n, q, r, z, p, invd,
                           partials, scal);
        finish<2>(s, nb, 2, partials, nullptr, FIN_SUM, 0, scal + 6);
        break;
    }
}

}  // namespace st
