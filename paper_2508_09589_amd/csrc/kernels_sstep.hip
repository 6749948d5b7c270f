// s-step form of the Jacobi-GMRES smoother (§3.2): the Krylov vectors
// w_0 = D^{-1}(b - A x0), w_{j+1} = D^{-1} A w_j are made by plain operator
// applies (no orthogonalisation between them), one pass forms their Gram
// matrix G = W^T W, and one workgroup solves the scaled normal equations of
// min || w_0 - sum_j y_j w_{j+1} ||.  In exact arithmetic this is the GMRES
// iterate with the same stopping rule; it reads every basis vector once for
// the inner products instead of once per later Arnoldi step.
//
// Reductions are deterministic: fixed trees inside a workgroup, partials summed
// in workgroup order by the solve kernel.
#include "st_internal.hpp"
#include "reduce_core.hpp"

namespace st {

constexpr int GR_THREADS = 256;
constexpr int GR_MAXNV = SMAX + 1;
constexpr int GR_MAXP = GR_MAXNV * (GR_MAXNV + 1) / 2;
constexpr long long GR_MAX_BLOCKS = 1024;
// Smallest accepted pivot of the scaled normal equations (the squared sine
// of the angle between a new basis vector and the earlier ones).  The
// monomial basis loses about a decade per vector; below ~1e-11 the pivot is
// rounding and the equations no longer carry information, so the basis is cut
// before that vector.
constexpr double SSTEP_MIN_PIVOT = 1e-11;

// [GR_MAXP][GR_MAX_BLOCKS] workgroup partials, then GR_MAXP summed entries.
size_t gram_partials_doubles() { return (size_t)GR_MAX_BLOCKS * GR_MAXP + GR_MAXP; }

static unsigned gram_grid(long long n) {
    long long nb = (n + 8LL * GR_THREADS - 1) / (8LL * GR_THREADS);
    if (nb < 1) nb = 1;
    if (nb > GR_MAX_BLOCKS) nb = GR_MAX_BLOCKS;
    return (unsigned)nb;
}

__device__ __forceinline__ double gr_wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    return v;
}

template <typename T> struct GrVec;
template <> struct GrVec<float> { using type = float4; };
template <> struct GrVec<double> { using type = double4; };

// part[p][block] (row stride GR_MAX_BLOCKS), p = index of the pair (a <= b)
// in row-major upper order.
// Four consecutive elements per thread per step when the basis is aligned
// (ld a multiple of 4, base 16-byte aligned), a scalar tail after them.
template <typename T, int NV>
__global__ __launch_bounds__(GR_THREADS) void k_gram(long long n, const T* __restrict__ V,
                                                     long long ld, int vec,
                                                     double* __restrict__ part) {
    constexpr int NP = NV * (NV + 1) / 2;
    double acc[NP];
#pragma unroll
    for (int p = 0; p < NP; ++p) acc[p] = 0.0;
    const long long stride = (long long)gridDim.x * blockDim.x;
    const long long t0 = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    long long tail = 0;
    if (vec) {
        const long long n4 = n >> 2;
        for (long long q = t0; q < n4; q += stride) {
            typename GrVec<T>::type v[NV];
#pragma unroll
            for (int d = 0; d < NV; ++d)
                v[d] = *reinterpret_cast<const typename GrVec<T>::type*>(V + (long long)d * ld + 4 * q);
            int p = 0;
#pragma unroll
            for (int a = 0; a < NV; ++a)
#pragma unroll
                for (int b = a; b < NV; ++b) {
                    acc[p] += (double)v[a].x * (double)v[b].x + (double)v[a].y * (double)v[b].y +
                              (double)v[a].z * (double)v[b].z + (double)v[a].w * (double)v[b].w;
                    ++p;
                }
        }
        tail = 4 * n4;
    }
    for (long long i = tail + t0; i < n; i += stride) {
        double v[NV];
#pragma unroll
        for (int d = 0; d < NV; ++d) v[d] = (double)V[(long long)d * ld + i];
        int p = 0;
#pragma unroll
        for (int a = 0; a < NV; ++a)
#pragma unroll
            for (int b = a; b < NV; ++b) acc[p++] += v[a] * v[b];
    }
    __shared__ double bsum[NP];
    block_sum_many<NP, GR_THREADS>(acc, NP, bsum);
    for (int p = threadIdx.x; p < NP; p += blockDim.x)
        part[(long long)p * GR_MAX_BLOCKS + blockIdx.x] = bsum[p];
}

// One workgroup per pair p sums its partials (thread t adds workgroups t,
// t + 256, ... in order, then a fixed tree) into gsum[p]; the last workgroup
// to arrive (KState::counter) takes the serial part on its thread 0: it picks
// the number m of vectors and the coefficients y:
//   scale s_d = 1/sqrt(G_dd); Gs = S G S;
//   for m = 1..k: extend the Cholesky factor of Gs[1..m][1..m] by one row
//   (stop before a pivot <= SSTEP_MIN_PIVOT or a zero vector);
//   z = L^{-1} Gs[1..m][0];
//   res^2 = 1 - |z|^2; stop at the first m with res^2 <= rtol^2;
//   y_i = yhat_i s_{i+1} / s_0 with L^T yhat = z.
// The serial part is unrolled for the basis size NV so that G, the factor, z
// and y stay in registers (a dependent chain through memory would cost tens
// of microseconds).
template <int NV>
__global__ __launch_bounds__(GR_THREADS) void k_sstep_solve(const double* __restrict__ part,
                                                            int nb, double rtol, KState* ks,
                                                            double* gsum) {
    constexpr int NP = NV * (NV + 1) / 2, K = NV - 1;
    __shared__ double red[GR_THREADS / 64];
    __shared__ int amlast;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    {
        const int p = blockIdx.x;
        double v = 0.0;
#pragma unroll
        for (int q = 0; q < (int)(GR_MAX_BLOCKS / GR_THREADS); ++q) {
            const int b = threadIdx.x + GR_THREADS * q;
            if (b < nb) v += part[(long long)p * GR_MAX_BLOCKS + b];
        }
        v = gr_wave_sum(v);
        if (lane == 0) red[wv] = v;
        __syncthreads();
        if (threadIdx.x == 0) {
            double t = 0.0;
#pragma unroll
            for (int q = 0; q < GR_THREADS / 64; ++q) t += red[q];
            gsum[p] = t;
        }
    }
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned prev = atomicAdd(&ks->counter, 1u);
        amlast = (prev == gridDim.x - 1);
    }
    __syncthreads();
    if (!amlast || threadIdx.x != 0) return;
    __threadfence();
    ks->counter = 0u;
    double G[NP];
#pragma unroll
    for (int p = 0; p < NP; ++p) G[p] = gsum[p];
    auto gidx = [](int a, int b) { return a * NV - a * (a - 1) / 2 + (b - a); };   // a <= b
    const double g00 = G[0];
    int bad = !isfinite(g00);
    int m = 0;
    double res2 = 1.0;
    double y[K > 0 ? K : 1];
#pragma unroll
    for (int i = 0; i < K; ++i) y[i] = 0.0;
    if (g00 > 0.0 && !bad) {
        double sc[NV];
#pragma unroll
        for (int d = 0; d < NV; ++d) {
            const double gd = G[gidx(d, d)];
            if (!isfinite(gd)) bad = 1;
            sc[d] = gd > 0.0 ? 1.0 / sqrt(gd) : 0.0;
        }
        // Lf holds the factor, ri the reciprocals of its diagonal (one division
        // per column on the dependent chain instead of one per entry)
        double Lf[K > 0 ? K : 1][K > 0 ? K : 1], z[K > 0 ? K : 1], ri[K > 0 ? K : 1];
        bool stop = bad != 0;
        double zz = 0.0;
#pragma unroll
        for (int r = 0; r < K; ++r) {
            if (!stop) {
                if (sc[r + 1] == 0.0) {
                    stop = true;
                } else {
#pragma unroll
                    for (int c = 0; c < r; ++c) {
                        double v = G[gidx(c + 1, r + 1)] * sc[c + 1] * sc[r + 1];
#pragma unroll
                        for (int e = 0; e < c; ++e) v -= Lf[r][e] * Lf[c][e];
                        Lf[r][c] = v * ri[c];
                    }
                    double piv = 1.0;   // Gs[r][r] = 1 by the scaling
#pragma unroll
                    for (int e = 0; e < r; ++e) piv -= Lf[r][e] * Lf[r][e];
                    if (!(piv > SSTEP_MIN_PIVOT)) {
                        stop = true;
                    } else {
                        Lf[r][r] = sqrt(piv);
                        ri[r] = 1.0 / Lf[r][r];
                        double v = G[gidx(0, r + 1)] * sc[0] * sc[r + 1];
#pragma unroll
                        for (int e = 0; e < r; ++e) v -= Lf[r][e] * z[e];
                        z[r] = v * ri[r];
                        zz += z[r] * z[r];
                        m = r + 1;
                        res2 = fmax(1.0 - zz, 0.0);
                        if (res2 <= rtol * rtol) stop = true;
                    }
                }
            }
        }
        // back substitution L^T yhat = z over the first m rows, unscaled
#pragma unroll
        for (int i = K - 1; i >= 0; --i) {
            if (i < m) {
                double v = z[i];
#pragma unroll
                for (int c = i + 1; c < K; ++c)
                    if (c < m) v -= Lf[c][i] * y[c];
                y[i] = v * ri[i];
            }
        }
#pragma unroll
        for (int i = 0; i < K; ++i) {
            if (i < m) {
                y[i] *= sc[i + 1] / sc[0];
                if (!isfinite(y[i])) bad = 1;
            }
        }
    }
    if (bad) m = 0;
#pragma unroll
    for (int i = 0; i < K; ++i)
        if (i < m) ks->y[i] = y[i];
    ks->k = m;
    ks->beta = sqrt(g00);
    ks->est = sqrt(res2) * sqrt(g00);
    ks->bad = bad;
    ks->done = 1;
}

template <typename T>
static void gram_dispatch(hipStream_t s, unsigned nb, long long n, const T* V, long long ld,
                          int vec, int nv, double* part) {
#define ST_GRAM_CASE(NVV)                                                                      \
    case NVV:                                                                                  \
        hipLaunchKernelGGL((k_gram<T, NVV>), dim3(nb), dim3(GR_THREADS), 0, s, n, V, ld, vec,  \
                           part);                                                              \
        break;
    switch (nv) {
        ST_GRAM_CASE(2) ST_GRAM_CASE(3) ST_GRAM_CASE(4) ST_GRAM_CASE(5) ST_GRAM_CASE(6)
        ST_GRAM_CASE(7) ST_GRAM_CASE(8) ST_GRAM_CASE(9) ST_GRAM_CASE(10) ST_GRAM_CASE(11)
        ST_GRAM_CASE(12) ST_GRAM_CASE(13) ST_GRAM_CASE(14) ST_GRAM_CASE(15) ST_GRAM_CASE(16)
        default: break;
    }
#undef ST_GRAM_CASE
}

void launch_sstep_coefficients(hipStream_t s, long long n, int prec, const void* V, long long ld,
                               int nv, double rtol, double* part, KState* ks) {
    static_assert(GR_MAXNV >= 16, "basis size");
    const unsigned nb = gram_grid(n);
    const size_t esz = prec ? 4 : 8;
    const int vec = ld % 4 == 0 && ((uintptr_t)V % (4 * esz)) == 0;
    if (prec)
        gram_dispatch<float>(s, nb, n, (const float*)V, ld, vec, nv, part);
    else
        gram_dispatch<double>(s, nb, n, (const double*)V, ld, vec, nv, part);
#define ST_SOLVE_CASE(NVV)                                                                     \
    case NVV:                                                                                  \
        hipLaunchKernelGGL((k_sstep_solve<NVV>), dim3(NVV * (NVV + 1) / 2), dim3(GR_THREADS), 0, \
                           s, part, (int)nb, rtol, ks, part + GR_MAX_BLOCKS * GR_MAXP);       \
        break;
    switch (nv) {
        ST_SOLVE_CASE(2) ST_SOLVE_CASE(3) ST_SOLVE_CASE(4) ST_SOLVE_CASE(5) ST_SOLVE_CASE(6)
        ST_SOLVE_CASE(7) ST_SOLVE_CASE(8) ST_SOLVE_CASE(9) ST_SOLVE_CASE(10) ST_SOLVE_CASE(11)
        ST_SOLVE_CASE(12) ST_SOLVE_CASE(13) ST_SOLVE_CASE(14) ST_SOLVE_CASE(15) ST_SOLVE_CASE(16)
        default: break;
    }
#undef ST_SOLVE_CASE
}

}  // namespace st
