// Design-chain kernels of the topology optimisation formulation (§3.3):
// Heaviside projection and its chain rule, the p-norm objective of the
// element-averaged temperature and its gradient.
#include "st_internal.hpp"

namespace st {

// ---------------------------------------------------------------------------
// Heaviside projection of the filtered design (§3.3.2):
//   H(x) = (tanh(b e) + tanh(b (x - e))) / (tanh(b e) + tanh(b (1 - e))),
//   H'(x) = b (1 - tanh^2(b (x - e))) / (tanh(b e) + tanh(b (1 - e))).
__global__ void k_heaviside(long long n, const double* __restrict__ x, double beta, double eta,
                            double* __restrict__ out, double* __restrict__ dout) {
    const double den = tanh(beta * eta) + tanh(beta * (1.0 - eta));
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        const double t = tanh(beta * (x[i] - eta));
        if (out) out[i] = (tanh(beta * eta) + t) / den;
        if (dout) dout[i] = beta * (1.0 - t * t) / den;
    }
}

// g_out = H'(x) g_in (g_out may be g_in): the projection's chain rule.
__global__ void k_heaviside_chain(long long n, const double* __restrict__ x, double beta,
                                  double eta, const double* g_in, double* g_out) {
    const double den = tanh(beta * eta) + tanh(beta * (1.0 - eta));
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        const double t = tanh(beta * (x[i] - eta));
        g_out[i] = beta * (1.0 - t * t) / den * g_in[i];
    }
}

void launch_heaviside(hipStream_t s, long long n, const double* x, double beta, double eta,
                      double* out, double* dout) {
    long long nb = (n + 255) / 256;
    if (nb > 4096) nb = 4096;
    hipLaunchKernelGGL(k_heaviside, dim3((unsigned)nb), dim3(256), 0, s, n, x, beta, eta, out,
                       dout);
}

void launch_heaviside_chain(hipStream_t s, long long n, const double* x, double beta, double eta,
                            const double* g_in, double* g_out) {
    long long nb = (n + 255) / 256;
    if (nb > 4096) nb = 4096;
    hipLaunchKernelGGL(k_heaviside_chain, dim3((unsigned)nb), dim3(256), 0, s, n, x, beta, eta,
                       g_in, g_out);
}

// ---------------------------------------------------------------------------
// p-norm objective of the element-averaged temperature (§3.3.1):
// theta = sum_e T_avg,e^P over the space-time elements, in a fixed reduction
// order (per-workgroup partials, then one workgroup sums them in order).
constexpr int PN_THREADS = 256;
constexpr int PN_MAXB = 1024;

__device__ __forceinline__ double pn_tavg(const double* __restrict__ T, long long P_, int rowp,
                                          int n, int j, int i) {
    const long long b = (long long)n * P_ + (long long)j * rowp + i;
    return 0.125 * (((T[b] + T[b + 1]) + (T[b + rowp] + T[b + rowp + 1])) +
                    ((T[b + P_] + T[b + P_ + 1]) + (T[b + P_ + rowp] + T[b + P_ + rowp + 1])));
}

__global__ __launch_bounds__(PN_THREADS) void k_pnorm_partials(FineGeom g, const double* __restrict__ T,
                                                               double Pw, double* __restrict__ part) {
    const int nx = g.nx, ny = g.ny, nt = g.nt;
    const int rowp = nx + 1;
    const long long P_ = (long long)rowp * (ny + 1);
    const long long ne = (long long)nx * ny * nt;
    double acc = 0.0;
    for (long long e = blockIdx.x * (long long)PN_THREADS + threadIdx.x; e < ne;
         e += (long long)gridDim.x * PN_THREADS) {
        const int n = (int)(e / ((long long)nx * ny));
        const long long r = e - (long long)n * nx * ny;
        const int j = (int)(r / nx), i = (int)(r - (long long)j * nx);
        acc += pow(pn_tavg(T, P_, rowp, n, j, i), Pw);
    }
    __shared__ double red[PN_THREADS / 64];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double v = 0.0;
        for (int w = 0; w < PN_THREADS / 64; ++w) v += red[w];
        part[blockIdx.x] = v;
    }
}

__global__ void k_sum_in_order(const double* __restrict__ part, int nb, double* __restrict__ out) {
    if (threadIdx.x == 0) {
        double v = 0.0;
        for (int b = 0; b < nb; ++b) v += part[b];
        *out = v;
    }
}

void launch_pnorm_theta(hipStream_t s, const FineGeom& g, const double* T, double Pw,
                        double* partials, double* theta) {
    const long long ne = (long long)g.nx * g.ny * g.nt;
    long long nb = (ne + PN_THREADS - 1) / PN_THREADS;
    if (nb > PN_MAXB) nb = PN_MAXB;
    hipLaunchKernelGGL(k_pnorm_partials, dim3((unsigned)nb), dim3(PN_THREADS), 0, s, g, T, Pw,
                       partials);
    hipLaunchKernelGGL(k_sum_in_order, dim3(1), dim3(64), 0, s, partials, (int)nb, theta);
}

// dphi/dT at every node: sum over the (up to 8) elements around it of
// theta^((1-P)/P) T_avg,e^(P-1) / 8.
__global__ void k_pnorm_grad(FineGeom g, const double* __restrict__ T, double Pw,
                             const double* __restrict__ theta, double* __restrict__ out) {
    const int nx = g.nx, ny = g.ny, nt = g.nt;
    const int rowp = nx + 1;
    const long long P_ = (long long)rowp * (ny + 1);
    const long long N = P_ * (nt + 1);
    const double c = pow(*theta, (1.0 - Pw) / Pw) * 0.125;
    for (long long a = blockIdx.x * (long long)blockDim.x + threadIdx.x; a < N;
         a += (long long)gridDim.x * blockDim.x) {
        const int n = (int)(a / P_);
        const long long r = a - (long long)n * P_;
        const int j = (int)(r / rowp), i = (int)(r - (long long)j * rowp);
        double v = 0.0;
        for (int en = n - 1; en <= n; ++en) {
            if (en < 0 || en >= nt) continue;
            for (int ej = j - 1; ej <= j; ++ej) {
                if (ej < 0 || ej >= ny) continue;
                for (int ei = i - 1; ei <= i; ++ei) {
                    if (ei < 0 || ei >= nx) continue;
                    v += pow(pn_tavg(T, P_, rowp, en, ej, ei), Pw - 1.0);
                }
            }
        }
        out[a] = c * v;
    }
}

void launch_pnorm_grad(hipStream_t s, const FineGeom& g, const double* T, double Pw,
                       const double* theta, double* out) {
    const long long N = (long long)(g.nx + 1) * (g.ny + 1) * (g.nt + 1);
    long long nb = (N + 255) / 256;
    if (nb > 65535) nb = 65535;
    hipLaunchKernelGGL(k_pnorm_grad, dim3((unsigned)nb), dim3(256), 0, s, g, T, Pw, theta, out);
}

}  // namespace st
