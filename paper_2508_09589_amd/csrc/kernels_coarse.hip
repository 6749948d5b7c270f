// Exact solve on the coarsest level.
//
// The paper solves the coarsest system with Jacobi-preconditioned GMRES to a
// relative tolerance (§3.2); at the semi-coarsened hierarchies' coarsest grids
// that solve runs into its iteration cap on every call and dominates the
// V-cycle's latency on a GPU.  The coarse operator is block tridiagonal in
// time (a 27-point stencil couples time level s only to s - 1 and s + 1), with
// one P x P block per level, P = (nx + 1)(ny + 1), so it is factorised once per
// operator as
//     J = Lb Ub,  Lb: diagonal D'_s, sub-diagonal L_s;  Ub: unit diagonal,
//                 super-diagonal G_s = D'_s^{-1} U_s,
//     D'_0 = D_0,  D'_s = D_s - L_s G_{s-1},
// with D'_s^{-1} formed explicitly (Gauss-Jordan, partial pivoting).  A solve is
// then a forward and a backward sweep over the time levels with dense P x P
// matrix-vector products:
//     J x = b:    z_s = D'_s^{-1} (b_s - L_s z_{s-1}),  x_s = z_s - G_s x_{s+1}
//     J^T x = b:  w_s = b_s - G_{s-1}^T w_{s-1},
//                 x_s = D'_s^{-T} (w_s - L_{s+1}^T x_{s+1}).
// One workgroup does each; the factors (2 P^2 per time level, FP64) stay in L2.
//
// Small planes (P <= CD_FAST_P, whole vector in LDS) take a faster solve: the
// factorisation also forms H_s = D'_s^{-1} L_s and M_s = D'_s^{-T} L_{s+1}^T,
// so every step of a sweep is one dense product whose matrix rows are loaded
// into registers a step ahead and whose vector lives in LDS:
//     J x = b:    z_s = D'_s^{-1} b_s - H_s z_{s-1},  x_s = z_s - G_s x_{s+1}
//     J^T x = b:  w_s = b_s - G_{s-1}^T w_{s-1},
//                 x_s = D'_s^{-T} w_s - M_s x_{s+1}.
// (one barrier per time level instead of a chain of dependent global loads).
#include <algorithm>

#include "st_internal.hpp"

namespace st {

constexpr int CDT = 1024;   // threads of the coarse factor / solve workgroup
constexpr int CW_NB = CW_PANEL_NB;   // panel width of the wide Gauss-Jordan
constexpr int CD_SEG = 8;   // lanes that share one row of a dense product

// Stencil entry of row (plane n, in-plane index r) towards the neighbour at
// offset (dn, dj, di); the caller checks that the neighbour exists.
__device__ __forceinline__ double cd_entry(const double* st, const int* pmap, long long DS, int P,
                                           int n, int r, int dn, int dj, int di) {
    const int d = (dn + 1) * 9 + (dj + 1) * 3 + (di + 1);
    return st[(long long)d * DS + (long long)pmap[n] * P + r];
}

// Block-wide argmax of |A[i][k]| over rows i >= k (smallest index on ties).
__device__ int cd_pivot(const double* A, int P, int k, double* rv, int* ri) {
    double best = -1.0;
    int bi = k;
    for (int i = k + threadIdx.x; i < P; i += CDT) {
        const double v = fabs(A[(long long)i * P + k]);
        if (v > best) {
            best = v;
            bi = i;
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const double ov = __shfl_down(best, o, 64);
        const int oi = __shfl_down(bi, o, 64);
        if (ov > best || (ov == best && oi < bi)) {
            best = ov;
            bi = oi;
        }
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) {
        rv[wave] = best;
        ri[wave] = bi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double b = rv[0];
        int i0 = ri[0];
        for (int w = 1; w < CDT / 64; ++w)
            if (rv[w] > b || (rv[w] == b && ri[w] < i0)) {
                b = rv[w];
                i0 = ri[w];
            }
        ri[CDT / 64] = i0;
        rv[CDT / 64] = b;
    }
    __syncthreads();
    return ri[CDT / 64];
}

// Factorisation (one workgroup).  A: P x P working matrix (LDS when it fits,
// else global); Dinv: [nt + 1][P][P]; G: [nt][P][P]; H, M: [nt + 1][P][P] or
// null (H_0 and M_nt unused); colk: P doubles of scratch (global); status:
// set to 1 when a pivot is zero.
template <bool ALDS>
__global__ __launch_bounds__(CDT) void k_coarse_factor(int nx, int ny, int nt, int nplanes,
                                                       const double* __restrict__ st,
                                                       const int* __restrict__ pmap,
                                                       double* __restrict__ Ag,
                                                       double* __restrict__ Dinv,
                                                       double* __restrict__ G,
                                                       double* __restrict__ H,
                                                       double* __restrict__ M,
                                                       double* __restrict__ colk,
                                                       int* __restrict__ perm, int* status) {
    extern __shared__ double dyn[];
    double* A = ALDS ? dyn : Ag;
    __shared__ double rv[CDT / 64 + 1];
    __shared__ int ri[CDT / 64 + 1];
    const int row = nx + 1, P = row * (ny + 1);
    const long long PP = (long long)P * P;
    const long long DS = (long long)P * nplanes;
    const int tid = threadIdx.x;
    if (tid == 0) *status = 0;
    for (int s = 0; s <= nt; ++s) {
        // D'_s = D_s - L_s G_{s-1}, element (a, c) gathered from the stencils.
        for (long long e = tid; e < PP; e += CDT) {
            const int a = (int)(e / P), c = (int)(e - (long long)a * P);
            const int ja = a / row, ia = a - ja * row;
            const int jc = c / row, ic = c - jc * row;
            double v = 0.0;
            const int dj = jc - ja, di = ic - ia;
            if (dj >= -1 && dj <= 1 && di >= -1 && di <= 1)
                v = cd_entry(st, pmap, DS, P, s, a, 0, dj, di);
            if (s > 0) {
                const double* Gp = G + (long long)(s - 1) * PP;
                for (int qj = -1; qj <= 1; ++qj) {
                    const int jb = ja + qj;
                    if (jb < 0 || jb > ny) continue;
                    for (int qi = -1; qi <= 1; ++qi) {
                        const int ib = ia + qi;
                        if (ib < 0 || ib > nx) continue;
                        const double l = cd_entry(st, pmap, DS, P, s, a, -1, qj, qi);
                        if (l != 0.0) v -= l * Gp[(long long)(jb * row + ib) * P + c];
                    }
                }
            }
            A[e] = v;
        }
        __syncthreads();
        // In-place Gauss-Jordan inverse with partial pivoting (row interchanges
        // recorded, undone as column interchanges at the end).
        for (int k = 0; k < P; ++k) {
            const int p = cd_pivot(A, P, k, rv, ri);
            if (tid == 0) {
                perm[k] = p;
                if (rv[CDT / 64] == 0.0) *status = 1;
            }
            if (p != k)
                for (int c = tid; c < P; c += CDT) {
                    const double t = A[(long long)k * P + c];
                    A[(long long)k * P + c] = A[(long long)p * P + c];
                    A[(long long)p * P + c] = t;
                }
            __syncthreads();
            const double piv = A[(long long)k * P + k];
            const double ipiv = 1.0 / piv;
            for (int i = tid; i < P; i += CDT) colk[i] = A[(long long)i * P + k];
            __syncthreads();
            for (int c = tid; c < P; c += CDT)
                A[(long long)k * P + c] = (c == k ? 1.0 : A[(long long)k * P + c]) * ipiv;
            __syncthreads();
            for (long long e = tid; e < PP; e += CDT) {
                const int i = (int)(e / P), c = (int)(e - (long long)i * P);
                if (i == k) continue;
                const double f = colk[i];
                A[e] = (c == k ? 0.0 : A[e]) - f * A[(long long)k * P + c];
            }
            __syncthreads();
        }
        for (int k = P - 1; k >= 0; --k) {
            const int p = perm[k];
            if (p != k)
                for (int i = tid; i < P; i += CDT) {
                    const double t = A[(long long)i * P + k];
                    A[(long long)i * P + k] = A[(long long)i * P + p];
                    A[(long long)i * P + p] = t;
                }
            __syncthreads();
        }
        double* Di = Dinv + (long long)s * PP;
        for (long long e = tid; e < PP; e += CDT) Di[e] = A[e];
        // G_s = D'_s^{-1} U_s: U_s[b][c] is the (dn = +1) entry of row b towards
        // node c of level s + 1, non-zero only for in-plane neighbours b of c.
        if (s < nt) {
            double* Gs = G + (long long)s * PP;
            for (long long e = tid; e < PP; e += CDT) {
                const int a = (int)(e / P), c = (int)(e - (long long)a * P);
                const int jc = c / row, ic = c - jc * row;
                double v = 0.0;
                for (int qj = -1; qj <= 1; ++qj) {
                    const int jb = jc + qj;
                    if (jb < 0 || jb > ny) continue;
                    for (int qi = -1; qi <= 1; ++qi) {
                        const int ib = ic + qi;
                        if (ib < 0 || ib > nx) continue;
                        const int b = jb * row + ib;
                        const double u = cd_entry(st, pmap, DS, P, s, b, 1, -qj, -qi);
                        if (u != 0.0) v += A[(long long)a * P + b] * u;
                    }
                }
                Gs[e] = v;
            }
        }
        // H_s = D'_s^{-1} L_s: L_s[b][c] is the (dn = -1) entry of row b towards
        // node c of level s - 1.  M_s = (L_{s+1} D'_s^{-1})^T: L_{s+1}[c][b] is
        // the (dn = -1) entry of row c of level s + 1 towards node b of level s.
        if (H && s > 0) {
            double* Hs = H + (long long)s * PP;
            for (long long e = tid; e < PP; e += CDT) {
                const int a = (int)(e / P), c = (int)(e - (long long)a * P);
                const int jc = c / row, ic = c - jc * row;
                double v = 0.0;
                for (int qj = -1; qj <= 1; ++qj) {
                    const int jb = jc + qj;
                    if (jb < 0 || jb > ny) continue;
                    for (int qi = -1; qi <= 1; ++qi) {
                        const int ib = ic + qi;
                        if (ib < 0 || ib > nx) continue;
                        const int b = jb * row + ib;
                        const double l = cd_entry(st, pmap, DS, P, s, b, -1, -qj, -qi);
                        if (l != 0.0) v += A[(long long)a * P + b] * l;
                    }
                }
                Hs[e] = v;
            }
        }
        if (M && s < nt) {
            double* Ms = M + (long long)s * PP;
            for (long long e = tid; e < PP; e += CDT) {
                const int a = (int)(e / P), c = (int)(e - (long long)a * P);
                const int jc = c / row, ic = c - jc * row;
                double v = 0.0;
                for (int qj = -1; qj <= 1; ++qj) {
                    const int jb = jc + qj;
                    if (jb < 0 || jb > ny) continue;
                    for (int qi = -1; qi <= 1; ++qi) {
                        const int ib = ic + qi;
                        if (ib < 0 || ib > nx) continue;
                        const int b = jb * row + ib;
                        const double l = cd_entry(st, pmap, DS, P, s + 1, c, -1, qj, qi);
                        if (l != 0.0) v += l * A[(long long)b * P + a];
                    }
                }
                Ms[e] = v;
            }
        }
        __syncthreads();
    }
}

// Fast solve (P <= CD_FAST_P, 2 (nt + 1) P doubles of LDS).  Thread t owns row
// r = t / 8 of each product and its columns c = t % 8 + 8 k; the row slices of
// the next step's matrices are loaded while the current step reduces and
// waits at the barrier.  Bv holds b, Zv the sweeps' vectors.
constexpr int CD_NC = CD_FAST_P / CD_SEG;
template <typename TIO>
__global__ __launch_bounds__(CDT) void k_coarse_direct_fast(int P, int nt,
                                                            const double* __restrict__ Dinv,
                                                            const double* __restrict__ G,
                                                            const double* __restrict__ H,
                                                            const double* __restrict__ M,
                                                            const TIO* __restrict__ b,
                                                            TIO* __restrict__ x, int trans) {
    extern __shared__ double dyn[];
    const int n = (nt + 1) * P;
    double* Bv = dyn;
    double* Zv = dyn + n;
    const long long PP = (long long)P * P;
    const int tid = threadIdx.x, r = tid / CD_SEG, q = tid & (CD_SEG - 1);
    const bool own = r < P && q == 0;
    for (int i = tid; i < n; i += CDT) Bv[i] = (double)b[i];
    double m1[CD_NC], m2[CD_NC];
    // Row r (tr = 0) or column r (tr = 1) of Mx, this thread's columns.
    auto load = [&](double (&m)[CD_NC], const double* Mx, int tr) {
#pragma unroll
        for (int k = 0; k < CD_NC; ++k) {
            const int c = q + CD_SEG * k;
            m[k] = (r < P && c < P) ? (tr ? Mx[(long long)c * P + r] : Mx[(long long)r * P + c]) : 0.0;
        }
    };
    auto dot = [&](const double (&m)[CD_NC], const double* v) {
        double a = 0.0;
#pragma unroll
        for (int k = 0; k < CD_NC; ++k) {
            const int c = q + CD_SEG * k;
            if (c < P) a += m[k] * v[c];
        }
#pragma unroll
        for (int o = CD_SEG / 2; o > 0; o >>= 1) a += __shfl_xor(a, o, 64);
        return a;
    };
    if (!trans) {
        load(m1, Dinv, 0);
        __syncthreads();
        for (int s = 0; s <= nt; ++s) {   // z_s = D'^{-1}_s b_s - H_s z_{s-1}
            double a = dot(m1, Bv + (long long)s * P);
            if (s > 0) a -= dot(m2, Zv + (long long)(s - 1) * P);
            if (s < nt) {
                load(m1, Dinv + (long long)(s + 1) * PP, 0);
                load(m2, H + (long long)(s + 1) * PP, 0);
            } else if (nt > 0) {
                load(m1, G + (long long)(nt - 1) * PP, 0);
            }
            if (own) Zv[(long long)s * P + r] = a;
            __syncthreads();
        }
        for (int s = nt - 1; s >= 0; --s) {   // x_s = z_s - G_s x_{s+1}
            const double a = dot(m1, Zv + (long long)(s + 1) * P);
            if (s > 0) load(m1, G + (long long)(s - 1) * PP, 0);
            if (own) Zv[(long long)s * P + r] -= a;
            __syncthreads();
        }
        for (int i = tid; i < n; i += CDT) x[i] = (TIO)Zv[i];
    } else {
        if (nt > 0) load(m1, G, 1);
        __syncthreads();
        for (int i = tid; i < P; i += CDT) Zv[i] = Bv[i];
        __syncthreads();
        for (int s = 1; s <= nt; ++s) {   // w_s = b_s - G_{s-1}^T w_{s-1}
            const double a = dot(m1, Zv + (long long)(s - 1) * P);
            if (s < nt) load(m1, G + (long long)s * PP, 1);
            if (own) Zv[(long long)s * P + r] = Bv[(long long)s * P + r] - a;
            __syncthreads();
        }
        load(m1, Dinv + (long long)nt * PP, 1);
        for (int s = nt; s >= 0; --s) {   // x_s = D'^{-T}_s w_s - M_s x_{s+1}, into Bv
            double a = dot(m1, Zv + (long long)s * P);
            if (s < nt) a -= dot(m2, Bv + (long long)(s + 1) * P);
            if (s > 0) {
                load(m1, Dinv + (long long)(s - 1) * PP, 1);
                load(m2, M + (long long)(s - 1) * PP, 0);
            }
            // slot s of Bv (b_s) was last read in the first sweep
            if (own) Bv[(long long)s * P + r] = a;
            __syncthreads();
        }
        for (int i = tid; i < n; i += CDT) x[i] = (TIO)Bv[i];
    }
}

// ---------------------------------------------------------------------------
// Wide factorisation and solve (planes larger than CD_FAST_P): the same block
// LU, with every step spread over the whole GPU.
//
// D'_s^{-1} by blocked Gauss-Jordan with partial pivoting, in place on A:
// the steps of CW_NB consecutive columns (a panel) are carried out on the
// P x CW_NB panel alone by one workgroup (the row interchanges go to whole
// rows at once); their product is the identity except in the panel's
// columns, E = I + W B^T with W = (panel after the steps) - (identity
// columns), so every other column then takes the rank-CW_NB update
// A[:, c] += W A[B, c] (A[B, c]: the panel's pivot rows before the update).
// Columns done by earlier panels hold columns of the inverse under
// construction and are updated like the others.  At the end the row
// interchanges are undone as column interchanges (last first).

__global__ void k_cw_init_status(int* status) { *status = 0; }

// A = D_s - L_s G_{s-1} (no coupling term for s = 0).
__global__ void k_cw_schur(int nx, int ny, int nplanes, const double* __restrict__ st,
                           const int* __restrict__ pmap, int s, const double* __restrict__ Gp,
                           double* __restrict__ A) {
    const int row = nx + 1, P = row * (ny + 1);
    const long long PP = (long long)P * P;
    const long long DS = (long long)P * nplanes;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < PP;
         e += (long long)gridDim.x * blockDim.x) {
        const int a = (int)(e / P), c = (int)(e - (long long)a * P);
        const int ja = a / row, ia = a - ja * row;
        const int jc = c / row, ic = c - jc * row;
        double v = 0.0;
        const int dj = jc - ja, di = ic - ia;
        if (dj >= -1 && dj <= 1 && di >= -1 && di <= 1) v = cd_entry(st, pmap, DS, P, s, a, 0, dj, di);
        if (Gp) {
            for (int qj = -1; qj <= 1; ++qj) {
                const int jb = ja + qj;
                if (jb < 0 || jb > ny) continue;
                for (int qi = -1; qi <= 1; ++qi) {
                    const int ib = ia + qi;
                    if (ib < 0 || ib > nx) continue;
                    const double l = cd_entry(st, pmap, DS, P, s, a, -1, qj, qi);
                    if (l != 0.0) v -= l * Gp[(long long)(jb * row + ib) * P + c];
                }
            }
        }
        A[e] = v;
    }
}

// The Gauss-Jordan steps of panel columns k0 .. k0 + nb - 1 (one workgroup).
// pan: the P x CW_NB panel (LDS when it fits, else global scratch), colk: P
// doubles.  Writes the panel back into A, W = panel - identity columns, and
// R = the pivot rows' entries outside the panel (zero inside it).
template <bool LDSPAN>
__global__ __launch_bounds__(CDT) void k_cw_panel(int P, int k0, double* __restrict__ A,
                                                  double* __restrict__ panel_g,
                                                  double* __restrict__ colk_g,
                                                  double* __restrict__ W, double* __restrict__ R,
                                                  int* __restrict__ perm, int* __restrict__ status) {
    extern __shared__ double dyn[];
    double* pan = LDSPAN ? dyn : panel_g;
    double* colk = LDSPAN ? dyn + (long long)P * CW_NB : colk_g;
    __shared__ double rv[CDT / 64 + 1];
    __shared__ int ri[CDT / 64 + 1];
    const int tid = threadIdx.x;
    const int nb = min(CW_NB, P - k0);
    for (long long e = tid; e < (long long)P * CW_NB; e += CDT) {
        const int i = (int)(e / CW_NB), j = (int)(e - (long long)i * CW_NB);
        pan[e] = j < nb ? A[(long long)i * P + k0 + j] : 0.0;
    }
    __syncthreads();
    for (int j = 0; j < nb; ++j) {
        const int k = k0 + j;
        // pivot: largest |pan[i][j]| over rows i >= k (smallest index on ties)
        double best = -1.0;
        int bi = k;
        for (int i = k + tid; i < P; i += CDT) {
            const double v = fabs(pan[(long long)i * CW_NB + j]);
            if (v > best) {
                best = v;
                bi = i;
            }
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const double ov = __shfl_down(best, o, 64);
            const int oi = __shfl_down(bi, o, 64);
            if (ov > best || (ov == best && oi < bi)) {
                best = ov;
                bi = oi;
            }
        }
        if ((tid & 63) == 0) {
            rv[tid >> 6] = best;
            ri[tid >> 6] = bi;
        }
        __syncthreads();
        if (tid == 0) {
            double b = rv[0];
            int i0 = ri[0];
            for (int w = 1; w < CDT / 64; ++w)
                if (rv[w] > b || (rv[w] == b && ri[w] < i0)) {
                    b = rv[w];
                    i0 = ri[w];
                }
            ri[CDT / 64] = i0;
            perm[k] = i0;
            if (b == 0.0) *status = 1;
        }
        __syncthreads();
        const int p = ri[CDT / 64];
        if (p != k) {
            for (int c = tid; c < CW_NB; c += CDT) {
                const double t = pan[(long long)k * CW_NB + c];
                pan[(long long)k * CW_NB + c] = pan[(long long)p * CW_NB + c];
                pan[(long long)p * CW_NB + c] = t;
            }
            for (int c = tid; c < P; c += CDT) {
                if (c >= k0 && c < k0 + nb) continue;
                const double t = A[(long long)k * P + c];
                A[(long long)k * P + c] = A[(long long)p * P + c];
                A[(long long)p * P + c] = t;
            }
        }
        __syncthreads();
        const double ipiv = 1.0 / pan[(long long)k * CW_NB + j];
        for (int i = tid; i < P; i += CDT) colk[i] = pan[(long long)i * CW_NB + j];
        __syncthreads();
        for (int c = tid; c < nb; c += CDT)
            pan[(long long)k * CW_NB + c] = (c == j ? 1.0 : pan[(long long)k * CW_NB + c]) * ipiv;
        __syncthreads();
        for (long long e = tid; e < (long long)P * CW_NB; e += CDT) {
            const int i = (int)(e / CW_NB), c = (int)(e - (long long)i * CW_NB);
            if (i == k || c >= nb) continue;
            pan[e] = (c == j ? 0.0 : pan[e]) - colk[i] * pan[(long long)k * CW_NB + c];
        }
        __syncthreads();
    }
    for (long long e = tid; e < (long long)P * CW_NB; e += CDT) {
        const int i = (int)(e / CW_NB), j = (int)(e - (long long)i * CW_NB);
        const double v = pan[e];
        if (j < nb) A[(long long)i * P + k0 + j] = v;
        W[e] = j < nb ? v - (i == k0 + j ? 1.0 : 0.0) : 0.0;
    }
    for (long long e = tid; e < (long long)CW_NB * P; e += CDT) {
        const int j = (int)(e / P), c = (int)(e - (long long)j * P);
        R[e] = (j < nb && (c < k0 || c >= k0 + nb)) ? A[(long long)(k0 + j) * P + c] : 0.0;
    }
}

// A[i][c] += sum_j W[i][j] R[j][c] for the columns outside the panel
// (R is zero in the panel's columns); grid (columns / 256, P rows).
__global__ __launch_bounds__(256) void k_cw_update(int P, int k0, double* __restrict__ A,
                                                   const double* __restrict__ W,
                                                   const double* __restrict__ R) {
    const int i = blockIdx.y;
    const int c = blockIdx.x * 256 + threadIdx.x;
    if (c >= P || (c >= k0 && c < k0 + CW_NB)) return;
    double w[CW_NB];
#pragma unroll
    for (int j = 0; j < CW_NB; ++j) w[j] = W[(long long)i * CW_NB + j];
    double acc = 0.0;
#pragma unroll
    for (int j = 0; j < CW_NB; ++j) acc += w[j] * R[(long long)j * P + c];
    A[(long long)i * P + c] += acc;
}

// Undo the row interchanges as column interchanges (last first):
// Dinv[i][c] = A[i][idx[c]].  One thread forms idx.
__global__ void k_cw_colperm(int P, const int* __restrict__ perm, int* __restrict__ idx) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    for (int c = 0; c < P; ++c) idx[c] = c;
    for (int k = P - 1; k >= 0; --k) {
        const int p = perm[k];
        const int t = idx[k];
        idx[k] = idx[p];
        idx[p] = t;
    }
}
__global__ void k_cw_gather(int P, const double* __restrict__ A, const int* __restrict__ idx,
                            double* __restrict__ Dinv) {
    const long long PP = (long long)P * P;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < PP;
         e += (long long)gridDim.x * blockDim.x) {
        const int i = (int)(e / P), c = (int)(e - (long long)i * P);
        Dinv[e] = A[(long long)i * P + idx[c]];
    }
}

// G_s = D'_s^{-1} U_s (U_s: the dn = +1 entries; only in-plane neighbours
// b of c are non-zero).
__global__ void k_cw_gmat(int nx, int ny, int nplanes, const double* __restrict__ st,
                          const int* __restrict__ pmap, int s, const double* __restrict__ Di,
                          double* __restrict__ Gs) {
    const int row = nx + 1, P = row * (ny + 1);
    const long long PP = (long long)P * P;
    const long long DS = (long long)P * nplanes;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < PP;
         e += (long long)gridDim.x * blockDim.x) {
        const int a = (int)(e / P), c = (int)(e - (long long)a * P);
        const int jc = c / row, ic = c - jc * row;
        double v = 0.0;
        for (int qj = -1; qj <= 1; ++qj) {
            const int jb = jc + qj;
            if (jb < 0 || jb > ny) continue;
            for (int qi = -1; qi <= 1; ++qi) {
                const int ib = ic + qi;
                if (ib < 0 || ib > nx) continue;
                const int b = jb * row + ib;
                const double u = cd_entry(st, pmap, DS, P, s, b, 1, -qj, -qi);
                if (u != 0.0) v += Di[(long long)a * P + b] * u;
            }
        }
        Gs[e] = v;
    }
}

// H_t = D'_t^{-1} L_t (t >= 1; L_t: the dn = -1 entries of level t, towards
// level t - 1) and MT_t = L_{t+1} D'_t^{-1} (t < nt), so that every step of a
// sweep is a dense product alone:
//     z_t = D'^{-1}_t b_t - H_t z_{t-1},    x_t = D'^{-T}_t w_t - MT_t^T x_{t+1}.
__global__ void k_cw_hmat(int nx, int ny, int nplanes, const double* __restrict__ st,
                          const int* __restrict__ pmap, int t, const double* __restrict__ Di,
                          double* __restrict__ Hs) {
    const int row = nx + 1, P = row * (ny + 1);
    const long long PP = (long long)P * P;
    const long long DS = (long long)P * nplanes;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < PP;
         e += (long long)gridDim.x * blockDim.x) {
        const int a = (int)(e / P), c = (int)(e - (long long)a * P);
        const int jc = c / row, ic = c - jc * row;
        double v = 0.0;
        for (int qj = -1; qj <= 1; ++qj) {
            const int jb = jc + qj;
            if (jb < 0 || jb > ny) continue;
            for (int qi = -1; qi <= 1; ++qi) {
                const int ib = ic + qi;
                if (ib < 0 || ib > nx) continue;
                const int b = jb * row + ib;
                const double l = cd_entry(st, pmap, DS, P, t, b, -1, -qj, -qi);
                if (l != 0.0) v += Di[(long long)a * P + b] * l;
            }
        }
        Hs[e] = v;
    }
}
__global__ void k_cw_mtmat(int nx, int ny, int nplanes, const double* __restrict__ st,
                           const int* __restrict__ pmap, int t, const double* __restrict__ Di,
                           double* __restrict__ MTs) {
    const int row = nx + 1, P = row * (ny + 1);
    const long long PP = (long long)P * P;
    const long long DS = (long long)P * nplanes;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < PP;
         e += (long long)gridDim.x * blockDim.x) {
        const int a = (int)(e / P), c = (int)(e - (long long)a * P);
        const int ja = a / row, ia = a - ja * row;
        double v = 0.0;
        for (int qj = -1; qj <= 1; ++qj) {
            const int jb = ja + qj;
            if (jb < 0 || jb > ny) continue;
            for (int qi = -1; qi <= 1; ++qi) {
                const int ib = ia + qi;
                if (ib < 0 || ib > nx) continue;
                const int b = jb * row + ib;
                const double l = cd_entry(st, pmap, DS, P, t + 1, a, -1, qj, qi);
                if (l != 0.0) v += l * Di[(long long)b * P + c];
            }
        }
        MTs[e] = v;
    }
}

size_t cw_panel_lds(int P) { return (size_t)P * (CW_NB + 1) * sizeof(double); }

void launch_coarse_factor_wide(hipStream_t s, const Level& L, int lds_max, double* A,
                               double* Dinv, double* G, double* H, double* MT, double* panel,
                               double* colk, double* W, double* R, int* perm, int* idx,
                               int* status) {
    const int P = (L.nx + 1) * (L.ny + 1);
    const long long PP = (long long)P * P;
    const unsigned eb = (unsigned)std::min<long long>((PP + 255) / 256, 65535);
    const size_t lds = cw_panel_lds(P);
    const bool lds_panel = lds <= (size_t)lds_max;
    if (lds_panel && lds > 65536)
        (void)hipFuncSetAttribute((const void*)&k_cw_panel<true>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(k_cw_init_status, dim3(1), dim3(1), 0, s, status);
    for (int t = 0; t <= L.nt; ++t) {
        hipLaunchKernelGGL(k_cw_schur, dim3(eb), dim3(256), 0, s, L.nx, L.ny, L.nplanes, L.st64,
                           L.plane_map, t, t > 0 ? G + (long long)(t - 1) * PP : nullptr, A);
        for (int k0 = 0; k0 < P; k0 += CW_NB) {
            if (lds_panel)
                hipLaunchKernelGGL(k_cw_panel<true>, dim3(1), dim3(CDT), lds, s, P, k0, A, panel,
                                   colk, W, R, perm, status);
            else
                hipLaunchKernelGGL(k_cw_panel<false>, dim3(1), dim3(CDT), 0, s, P, k0, A, panel,
                                   colk, W, R, perm, status);
            hipLaunchKernelGGL(k_cw_update, dim3((P + 255) / 256, P), dim3(256), 0, s, P, k0, A, W,
                               R);
        }
        hipLaunchKernelGGL(k_cw_colperm, dim3(1), dim3(1), 0, s, P, perm, idx);
        double* Di = Dinv + (long long)t * PP;
        hipLaunchKernelGGL(k_cw_gather, dim3(eb), dim3(256), 0, s, P, A, idx, Di);
        if (t < L.nt) {
            hipLaunchKernelGGL(k_cw_gmat, dim3(eb), dim3(256), 0, s, L.nx, L.ny, L.nplanes, L.st64,
                               L.plane_map, t, Di, G + (long long)t * PP);
            hipLaunchKernelGGL(k_cw_mtmat, dim3(eb), dim3(256), 0, s, L.nx, L.ny, L.nplanes,
                               L.st64, L.plane_map, t, Di, MT + (long long)t * PP);
        }
        if (t > 0)
            hipLaunchKernelGGL(k_cw_hmat, dim3(eb), dim3(256), 0, s, L.nx, L.ny, L.nplanes, L.st64,
                               L.plane_map, t, Di, H + (long long)t * PP);
    }
}

// Wide solve.  z: forward-sweep vectors, xo: solution, both [nt + 1][P]
// FP64.  Every step is one launch of up to two dense products, in row form
// out[r] = base[r] + s1 (M1 v1)[r] + s2 (M2 v2)[r] (one wave per row, lanes
// across columns, four partial sums in flight) or column form with M1^T, M2^T
// (lanes across outputs, the workgroup's waves across segments of c).  The
// vectors are read from global memory (L2).
constexpr int CW_CSEG = 16;     // waves (column segments) per workgroup in the column form

template <typename TV1, typename TB>
__global__ __launch_bounds__(256) void k_cw_rows(int P, const double* __restrict__ M1,
                                                 const TV1* __restrict__ v1, double s1,
                                                 const double* __restrict__ M2,
                                                 const double* __restrict__ v2, double s2,
                                                 const TB* __restrict__ base,
                                                 double* __restrict__ out,
                                                 double* __restrict__ out2) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r = blockIdx.x * 4 + wave;
    if (r >= P) return;
    auto rowdot = [&](const double* Mr, auto v) -> double {
        double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
        int c = lane;
        for (; c + 192 < P; c += 256) {
            a0 += Mr[c] * (double)v[c];
            a1 += Mr[c + 64] * (double)v[c + 64];
            a2 += Mr[c + 128] * (double)v[c + 128];
            a3 += Mr[c + 192] * (double)v[c + 192];
        }
        for (; c < P; c += 64) a0 += Mr[c] * (double)v[c];
        return (a0 + a1) + (a2 + a3);
    };
    double acc = s1 * rowdot(M1 + (long long)r * P, v1);
    if (M2) acc += s2 * rowdot(M2 + (long long)r * P, v2);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if (lane == 0) {
        const double val = base ? (double)base[r] + acc : acc;
        out[r] = val;
        if (out2) out2[r] = val;
    }
}

template <typename TB>
__global__ __launch_bounds__(64 * CW_CSEG) void k_cw_cols(int P, const double* __restrict__ M1,
                                                          const double* __restrict__ v1, double s1,
                                                          const double* __restrict__ M2,
                                                          const double* __restrict__ v2, double s2,
                                                          const TB* __restrict__ base,
                                                          double* __restrict__ out) {
    __shared__ double part[CW_CSEG][64];
    const int lane = threadIdx.x & 63, seg = threadIdx.x >> 6;
    const int r = blockIdx.x * 64 + lane;
    const int cs = (P + CW_CSEG - 1) / CW_CSEG;
    const int c0 = seg * cs, c1 = min(P, c0 + cs);
    auto coldot = [&](const double* M, const double* v) -> double {
        double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
        int c = c0;
        for (; c + 3 < c1; c += 4) {
            a0 += M[(long long)c * P + r] * v[c];
            a1 += M[(long long)(c + 1) * P + r] * v[c + 1];
            a2 += M[(long long)(c + 2) * P + r] * v[c + 2];
            a3 += M[(long long)(c + 3) * P + r] * v[c + 3];
        }
        for (; c < c1; ++c) a0 += M[(long long)c * P + r] * v[c];
        return (a0 + a1) + (a2 + a3);
    };
    double acc = 0.0;
    if (r < P) {
        acc = s1 * coldot(M1, v1);
        if (M2) acc += s2 * coldot(M2, v2);
    }
    part[seg][lane] = acc;
    __syncthreads();
    if (seg == 0 && r < P) {
        double sum = 0.0;
        for (int q = 0; q < CW_CSEG; ++q) sum += part[q][lane];
        out[r] = base ? (double)base[r] + sum : sum;
    }
}

template <typename TIO>
__global__ void k_cw_in(long long n, const TIO* __restrict__ b, double* __restrict__ z) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        z[i] = (double)b[i];
}

template <typename TIO>
__global__ void k_cw_out(long long n, const double* __restrict__ xo, TIO* __restrict__ x) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        x[i] = (TIO)xo[i];
}

template <typename TIO>
static void cw_solve(hipStream_t s, const Level& L, int trans, const TIO* b, TIO* x,
                     const double* Dinv, const double* G, const double* H, const double* MT,
                     double* work) {
    const int P = (L.nx + 1) * (L.ny + 1), nt = L.nt;
    const long long PP = (long long)P * P, n = (long long)P * (nt + 1);
    double* z = work;
    double* xo = work + n;
    const dim3 grow((P + 3) / 4), gcol((P + 63) / 64);
    const double* nul = nullptr;
    if (!trans) {
        // z_t = D'^{-1}_t b_t - H_t z_{t-1};  x_nt = z_nt
        for (int t = 0; t <= nt; ++t)
            hipLaunchKernelGGL((k_cw_rows<TIO, double>), grow, dim3(256), 0, s, P,
                               Dinv + (long long)t * PP, b + (long long)t * P, 1.0,
                               t > 0 ? H + (long long)t * PP : nul,
                               t > 0 ? z + (long long)(t - 1) * P : nul, -1.0, nul,
                               z + (long long)t * P, t == nt ? xo + (long long)t * P : nullptr);
        // x_t = z_t - G_t x_{t+1}
        for (int t = nt - 1; t >= 0; --t)
            hipLaunchKernelGGL((k_cw_rows<double, double>), grow, dim3(256), 0, s, P,
                               G + (long long)t * PP, xo + (long long)(t + 1) * P, -1.0, nul, nul,
                               0.0, z + (long long)t * P, xo + (long long)t * P, nullptr);
    } else {
        // w_0 = b_0, w_t = b_t - G_{t-1}^T w_{t-1}
        hipLaunchKernelGGL(k_cw_in<TIO>, dim3((P + 255) / 256), dim3(256), 0, s, (long long)P, b, z);
        for (int t = 1; t <= nt; ++t)
            hipLaunchKernelGGL(k_cw_cols<TIO>, gcol, dim3(64 * CW_CSEG), 0, s, P,
                               G + (long long)(t - 1) * PP, z + (long long)(t - 1) * P, -1.0, nul,
                               nul, 0.0, b + (long long)t * P, z + (long long)t * P);
        // x_t = D'^{-T}_t w_t - MT_t^T x_{t+1}
        for (int t = nt; t >= 0; --t)
            hipLaunchKernelGGL(k_cw_cols<double>, gcol, dim3(64 * CW_CSEG), 0, s, P,
                               Dinv + (long long)t * PP, z + (long long)t * P, 1.0,
                               t < nt ? MT + (long long)t * PP : nul,
                               t < nt ? xo + (long long)(t + 1) * P : nul, -1.0, nul,
                               xo + (long long)t * P);
    }
    hipLaunchKernelGGL(k_cw_out<TIO>, dim3((unsigned)std::min<long long>((n + 255) / 256, 4096)),
                       dim3(256), 0, s, n, xo, x);
}

size_t coarse_direct_lds(int P) { return (size_t)P * P * sizeof(double); }
bool coarse_direct_fast(int P, int nt) {
    return P <= CD_FAST_P && (long long)(nt + 1) * P <= CD_FAST_NODES;
}
bool coarse_direct_fits(int P) { return P <= CD_MAX_PLANE; }

void launch_coarse_factor(hipStream_t s, const Level& L, double* Ag, double* Dinv, double* G,
                          double* H, double* M, double* colk, int* perm, int* status) {
    const int P = (L.nx + 1) * (L.ny + 1);
    const size_t lds = coarse_direct_lds(P);
    if (lds <= CD_LDS_MAX)
        hipLaunchKernelGGL(k_coarse_factor<true>, dim3(1), dim3(CDT), lds, s, L.nx, L.ny, L.nt,
                           L.nplanes, L.st64, L.plane_map, Ag, Dinv, G, H, M, colk, perm, status);
    else
        hipLaunchKernelGGL(k_coarse_factor<false>, dim3(1), dim3(CDT), 0, s, L.nx, L.ny, L.nt,
                           L.nplanes, L.st64, L.plane_map, Ag, Dinv, G, H, M, colk, perm, status);
}

void launch_coarse_direct(hipStream_t s, const Level& L, int prec_io, int trans, const void* b,
                          void* x, const double* Dinv, const double* G, const double* H,
                          const double* M, double* work, int wide) {
    const int P = (L.nx + 1) * (L.ny + 1);
    if (wide) {
        if (prec_io == 0)
            cw_solve<double>(s, L, trans, (const double*)b, (double*)x, Dinv, G, H, M, work);
        else
            cw_solve<float>(s, L, trans, (const float*)b, (float*)x, Dinv, G, H, M, work);
        return;
    }
    if (H && M) {
        const size_t lds = (size_t)2 * P * (L.nt + 1) * sizeof(double);
        if (prec_io == 0)
            hipLaunchKernelGGL(k_coarse_direct_fast<double>, dim3(1), dim3(CDT), lds, s, P, L.nt,
                               Dinv, G, H, M, (const double*)b, (double*)x, trans);
        else
            hipLaunchKernelGGL(k_coarse_direct_fast<float>, dim3(1), dim3(CDT), lds, s, P, L.nt,
                               Dinv, G, H, M, (const float*)b, (float*)x, trans);
        return;
    }
}

}  // namespace st
