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
#include "st_internal.hpp"

namespace st {

constexpr int CDT = 1024;   // threads of the coarse factor / solve workgroup
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

// out[r] = sum_c M[r][c] v[c] (trans = 0) or sum_c M[c][r] v[c] (trans = 1),
// r < P; CD_SEG lanes share one output.  v in LDS, M in global.
__device__ void cd_gemv(const double* __restrict__ M, const double* v, int P, int trans,
                        double* out, double sub_sign, const double* base) {
    const int q = threadIdx.x & (CD_SEG - 1);
    for (int r0 = 0; r0 < P; r0 += CDT / CD_SEG) {
        const int r = r0 + threadIdx.x / CD_SEG;
        double acc = 0.0;
        if (r < P) {
            if (!trans)
                for (int c = q; c < P; c += CD_SEG) acc += M[(long long)r * P + c] * v[c];
            else
                for (int c = q; c < P; c += CD_SEG) acc += M[(long long)c * P + r] * v[c];
        }
#pragma unroll
        for (int o = CD_SEG / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
        if (r < P && q == 0) out[r] = base ? base[r] + sub_sign * acc : acc;
    }
}

// Solve J x = b (trans = 0) or J^T x = b (trans = 1) with the factors; one
// workgroup.  t, u: 2 P doubles of LDS; work: (nt + 1) P doubles (global).
template <typename TIO>
__global__ __launch_bounds__(CDT) void k_coarse_direct(int nx, int ny, int nt, int nplanes,
                                                       const double* __restrict__ st,
                                                       const int* __restrict__ pmap,
                                                       const double* __restrict__ Dinv,
                                                       const double* __restrict__ G,
                                                       const TIO* __restrict__ b,
                                                       TIO* __restrict__ x,
                                                       double* __restrict__ work, int trans) {
    extern __shared__ double dyn[];
    const int row = nx + 1, P = row * (ny + 1);
    const long long PP = (long long)P * P;
    const long long DS = (long long)P * nplanes;
    double* t = dyn;
    double* u = dyn + P;
    const int tid = threadIdx.x;
    // Coupling of row a of level s to the level sn = s + dn vector y (global):
    // forward uses row a's own entries, the transpose the entries of the rows
    // of level sn that point at a.
    auto couple = [&](int s, int a, int dn, const double* y, int transposed) -> double {
        const int ja = a / row, ia = a - ja * row;
        const int sn = s + dn;
        double acc = 0.0;
        for (int qj = -1; qj <= 1; ++qj) {
            const int jb = ja + qj;
            if (jb < 0 || jb > ny) continue;
            for (int qi = -1; qi <= 1; ++qi) {
                const int ib = ia + qi;
                if (ib < 0 || ib > nx) continue;
                const int bb = jb * row + ib;
                const double c = transposed ? cd_entry(st, pmap, DS, P, sn, bb, -dn, -qj, -qi)
                                            : cd_entry(st, pmap, DS, P, s, a, dn, qj, qi);
                acc += c * y[(long long)sn * P + bb];
            }
        }
        return acc;
    };
    if (!trans) {
        for (int s = 0; s <= nt; ++s) {   // z_s = D'^{-1}_s (b_s - L_s z_{s-1})
            for (int a = tid; a < P; a += CDT) {
                double v = (double)b[(long long)s * P + a];
                if (s > 0) v -= couple(s, a, -1, work, 0);
                t[a] = v;
            }
            __syncthreads();
            cd_gemv(Dinv + (long long)s * PP, t, P, 0, work + (long long)s * P, 0.0, nullptr);
            __syncthreads();
        }
        for (int s = nt - 1; s >= 0; --s) {   // x_s = z_s - G_s x_{s+1}
            for (int a = tid; a < P; a += CDT) u[a] = work[(long long)(s + 1) * P + a];
            __syncthreads();
            cd_gemv(G + (long long)s * PP, u, P, 0, work + (long long)s * P, -1.0,
                    work + (long long)s * P);
            __syncthreads();
        }
    } else {
        for (int s = 0; s <= nt; ++s) {   // w_s = b_s - G_{s-1}^T w_{s-1}
            if (s == 0) {
                for (int a = tid; a < P; a += CDT) work[a] = (double)b[a];
            } else {
                for (int a = tid; a < P; a += CDT) {
                    u[a] = work[(long long)(s - 1) * P + a];
                    t[a] = (double)b[(long long)s * P + a];
                }
                __syncthreads();
                cd_gemv(G + (long long)(s - 1) * PP, u, P, 1, work + (long long)s * P, -1.0, t);
            }
            __syncthreads();
        }
        for (int s = nt; s >= 0; --s) {   // x_s = D'^{-T}_s (w_s - L_{s+1}^T x_{s+1})
            for (int a = tid; a < P; a += CDT) {
                double v = work[(long long)s * P + a];
                if (s < nt) v -= couple(s, a, 1, work, 1);
                t[a] = v;
            }
            __syncthreads();
            cd_gemv(Dinv + (long long)s * PP, t, P, 1, work + (long long)s * P, 0.0, nullptr);
            __syncthreads();
        }
    }
    const long long n = (long long)P * (nt + 1);
    for (long long i = tid; i < n; i += CDT) x[i] = (TIO)work[i];
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
                          const double* M, double* work) {
    const int P = (L.nx + 1) * (L.ny + 1);
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
    const size_t lds = (size_t)2 * P * sizeof(double);
    if (prec_io == 0)
        hipLaunchKernelGGL(k_coarse_direct<double>, dim3(1), dim3(CDT), lds, s, L.nx, L.ny, L.nt,
                           L.nplanes, L.st64, L.plane_map, Dinv, G, (const double*)b, (double*)x,
                           work, trans);
    else
        hipLaunchKernelGGL(k_coarse_direct<float>, dim3(1), dim3(CDT), lds, s, L.nx, L.ny, L.nt,
                           L.nplanes, L.st64, L.plane_map, Dinv, G, (const float*)b, (float*)x,
                           work, trans);
}

}  // namespace st
