/*
 * st_api.h -- C ABI of the MI355X space-time heat-conduction solver.
 *
 * Solves the all-at-once stabilised continuous-Galerkin space-time finite
 * element system J s = f for transient heat conduction with SIMP
 * density-dependent conductivity and capacity (Alexandersen & Appel, arXiv
 * 2508.09589: §2.1 governing equation, §2.2 SIMP interpolation, §3.1
 * discretisation), by FGMRES right-preconditioned with one space-time
 * multigrid V-cycle over a semi-coarsened Galerkin hierarchy (§3.2,
 * Algorithm 1), with Jacobi-GMRES smoothing and a Jacobi-GMRES coarsest-level
 * solve.  Adjoint solves and density sensitivities follow §3.3.3; the PDE
 * density filter follows §3.3.2.
 *
 * Conventions
 *  - Every pointer named *_dev is a device pointer on the GPU that is current
 *    when the handle is created; every *_host pointer is host memory.
 *  - Node arrays are float64 [nt+1][ny+1][nx+1] with x1 fastest; node
 *    (i, j, n) sits at x1 = i*dx, x2 = j*dx, t = n*dt (§3.1.2, square elements).
 *  - Element arrays are float64 [nt][ny][nx]; a time-constant design is
 *    [1][ny][nx] and is extruded over all slabs (§3.4.1).
 *  - Ownership: the caller owns every input, output and the workspace.  The
 *    library allocates no device memory: st_setup carves the caller's
 *    workspace (size from st_footprint_bytes) and copies what it keeps.
 *  - Streams: all work is enqueued on the HIP stream given to st_setup
 *    (NULL = the null stream).  Functions that return results or info
 *    synchronise that stream before returning.
 *  - Errors: negative status codes leave outputs undefined;
 *    ST_NOT_CONVERGED still writes the best iterate and fills st_info.
 *  - One thread at a time per handle; different handles may be used
 *    concurrently from different threads on different streams.
 */
#ifndef ST_API_H
#define ST_API_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    ST_OK = 0,
    ST_NOT_CONVERGED = 1,   /* warning: outputs valid, tolerance not met   */
    ST_ERR_ARG = -1,        /* invalid argument (host-side validation)     */
    ST_ERR_OOM = -2,        /* workspace smaller than st_footprint_bytes   */
    ST_ERR_HIP = -3,        /* a HIP runtime call failed                   */
    ST_ERR_BREAKDOWN = -4,  /* NaN/Inf or Krylov breakdown                 */
    ST_ERR_STATE = -5       /* call not valid in the handle's state        */
} st_status;

enum { ST_FP64 = 0, ST_MIXED = 1 };

/* Boundary lines of the spatial rectangle that can carry a T = 0 patch. */
enum { ST_EDGE_X1_LO = 0, ST_EDGE_X1_HI = 1, ST_EDGE_X2_LO = 2, ST_EDGE_X2_HI = 3 };

/* Option flags. */
enum {
    ST_FLAG_TIME_KERNELS = 1,   /* record per-kernel-class GPU times in st_info;
                                   bits 8.. of flags select classes (0 = all)     */
    ST_FLAG_NO_PLANE_DEDUP = 2, /* keep every time level of coarse stencils       */
    ST_FLAG_FULL_COARSENING = 8, /* full space-time coarsening on every level (the
                                   paper's comparison to Algorithm 1, §5.1.2);
                                   fixed at setup                                */
    ST_FLAG_SSTEP_SMOOTHER = 16, /* smoothing in s-step form: the same GMRES
                                   minimisation from a monomial Krylov basis and
                                   its Gram matrix (one pass for all inner
                                   products instead of Arnoldi's growing ones);
                                   smoothings of more than 10 iterations keep
                                   the Arnoldi form (the monomial basis is too
                                   ill-conditioned beyond that)                 */
    ST_FLAG_OUTER_CGS2 = 32,    /* outer FGMRES orthogonalised by classical CGS2
                                   (three passes per step) instead of delayed
                                   CGS2 (two passes; the same iterates in exact
                                   arithmetic)                                  */
    ST_FLAG_ROW_MARCH = 64,     /* coarse stencil applies by the row march (one
                                   thread per in-plane node) instead of the wave
                                   form (a wave per 62 consecutive nodes); the
                                   library takes the row march by itself for a
                                   level whose vectors pass 2 GiB.  Test access
                                   to that path; same results to rounding     */
    ST_FLAG_COARSE_GMRES = 4    /* coarsest level: Jacobi-GMRES (coarse_max_it,
                                   coarse_rtol, coarse_restart) as in §3.2, instead
                                   of the default exact solve by block-tridiagonal
                                   factorisation in time (used when
                                   (nx + 1)(ny + 1) <= 2048 on that level)        */
};

#define ST_MAX_LEVELS 32
#define ST_MAX_PATCHES 4
#define ST_MAX_HIST 1024
#define ST_NUM_KCLASS 12

/* Grid: nx x ny x nt elements of size dx x dx x dt (§3.1.2). */
typedef struct { int32_t nx, ny, nt; double dx, dt; } st_grid;

/* Modified SIMP endpoints and penalties (§2.2):
 *   k(rho) = k_ins + (k_con - k_ins) rho^p_k,  C(rho) = c_ins + (c_con - c_ins) rho^p_c */
typedef struct { double k_ins, k_con, p_k, c_ins, c_con, p_c; } st_material;

/* A T = 0 patch on one edge: nodes whose coordinate along the edge lies in
 * [centre - half_width, centre + half_width] (1e-12 slack), at every time level. */
typedef struct { int32_t edge; double centre, half_width; } st_patch;

typedef struct {
    int32_t precision;        /* ST_FP64: all FP64.  ST_MIXED: V-cycle in FP32
                                 (coarsest solve FP64) under FP64 FGMRES        */
    int32_t bf16_from_level;  /* ST_MIXED: store stencils of levels >= this in
                                 BF16 (0 = never)                                */
    int32_t restart;          /* FGMRES restart length m (<= 32), default 30    */
    double rtol;              /* ||f - J s||_2 <= rtol ||f||_2, default 1e-8    */
    int32_t max_it;           /* total FGMRES iterations, default 1000          */
    int32_t smooth_its;       /* GMRES smoothing iterations (<= 16), default 10 */
    double smooth_rtol;       /* default 1e-6                                   */
    int32_t coarse_max_it;    /* default 200                                    */
    double coarse_rtol;       /* default 1e-6                                   */
    int32_t coarse_restart;   /* default 30 (<= 32)                             */
    double lambda_crit;       /* Algorithm 1 threshold, default 0.5             */
    int32_t max_levels;       /* N_l, default 8 (the paper's space-time runs):
                                 at most this many levels unless the coarsest
                                 one is too large to factorise exactly (planes
                                 over 2048 nodes or factors over 16 GiB); 1 =
                                 one level (the coarsest solve alone)          */
    int64_t max_coarse_nodes; /* stop coarsening at <= this many nodes, 4096    */
    double filter_r;          /* PDE filter radius in elements (r_x = r dx,
                                 r_t = r dt); 0 = no filter                      */
    int32_t flags;            /* ST_FLAG_*                                      */
    double proj_beta;         /* Heaviside projection of the filtered design
                                 (§3.3.2): sharpness beta; 0 = no projection    */
    double proj_eta;          /* projection threshold eta, default 0.5          */
    int32_t filter_max_it;    /* PDE filter: CG iteration cap, default 2000;
                                 reaching it gives ST_NOT_CONVERGED             */
    double filter_rtol;       /* PDE filter: CG stops at ||r|| <= filter_rtol
                                 ||r_0||, default 1e-13                         */
} st_opts;

typedef struct {
    int32_t iterations;       /* outer FGMRES iterations                        */
    int32_t restarts;
    int32_t levels;
    int32_t level_dims[ST_MAX_LEVELS][3];   /* nx, ny, nt of every level        */
    int32_t level_planes[ST_MAX_LEVELS];    /* distinct stencil time levels     */
    double rel_res_est;       /* FGMRES residual estimate / ||f||               */
    double true_rel_res;      /* ||f - J s||_2 / ||f||_2 recomputed at the end  */
    double rhs_norm;
    double t_setup_s, t_solve_s;
    int32_t n_hist;
    double res_hist[ST_MAX_HIST];           /* residual estimate per iteration   */
    /* ST_FLAG_TIME_KERNELS: GPU milliseconds, launch counts and algorithmic
       bytes per class: 0 fine apply FP64, 1 fine apply in the V-cycle
       precision, 2 coarse stencil apply, 3 level-0 smoother multi-dot,
       4 level-0 smoother maxpy+norm, 5 restriction/prolongation, 6 coarsest
       solve, 7 casts, 8/9 multi-dot/maxpy on coarse levels, 10 FGMRES
       orthogonalisation, 11 solution updates                                 */
    double kclass_ms[ST_NUM_KCLASS];
    int64_t kclass_launches[ST_NUM_KCLASS];
    int64_t kclass_bytes[ST_NUM_KCLASS];    /* algorithmic bytes moved           */
} st_info;

typedef struct st_handle st_handle;

/* Fill *o with the defaults listed above (§3.2 solver parameters; rtol 1e-8). */
void st_opts_default(st_opts* o);

/* Human-readable name of a status code. */
const char* st_status_string(st_status s);

/* Bytes of device workspace st_setup needs for this grid, material, options
 * and design layout (rho_time_varying: 0 = [1][ny][nx], 1 = [nt][ny][nx]).
 * Pure host computation; ST_ERR_ARG on invalid sizes (a grid must have fewer
 * than 2^29 nodes, so that a node vector of FP64 values is below 4 GiB). */
st_status st_footprint_bytes(const st_grid* grid, const st_material* mat, const st_opts* opts,
                             int32_t rho_time_varying, size_t* bytes);

/* Build a problem: SIMP coefficients from rho (filtered first when
 * opts->filter_r > 0), Algorithm 1 hierarchy, Galerkin coarse operators
 * (§3.2), diagonals and the consistent load (§3.1.2).
 *   rho_dev    design, [1][ny][nx] or [nt][ny][nx] per rho_time_varying
 *   ic_dev     initial temperature on the t = 0 plane [ny+1][nx+1], or NULL (0)
 *   source_dev nodal heat source [nt+1][ny+1][nx+1] (trilinear interpolant),
 *              or NULL for a uniform q0
 *   patches    n_patches (<= ST_MAX_PATCHES) T = 0 patches
 *   workspace  >= st_footprint_bytes, 256-byte aligned, device memory
 * rho, ic and source are copied; no caller pointer is kept.
 * A density with a NaN or Inf entry gives ST_ERR_ARG.  When the density filter
 * reaches opts->filter_max_it, the handle is still created from the field it
 * reached and ST_NOT_CONVERGED is returned (the caller may st_destroy it). */
st_status st_setup(const st_grid* grid, const st_material* mat,
                   const double* rho_dev, int32_t rho_time_varying,
                   const double* ic_dev, const double* source_dev, double q0,
                   const st_patch* patches, int32_t n_patches,
                   const st_opts* opts, void* workspace_dev, size_t workspace_bytes,
                   void* hip_stream, st_handle** out);

/* Replace the design (same layout as at setup) and rebuild every
 * density-dependent quantity; allocations are reused.  Status as for
 * st_setup: ST_ERR_ARG for a non-finite density (the handle keeps no valid
 * operators until a finite one is loaded), ST_NOT_CONVERGED when the filter
 * reaches its cap. */
st_status st_update_density(st_handle* h, const double* rho_dev);

/* Forward solve J s = f.  T_dev: in = initial guess (warm start, §3.2),
 * out = solution.  info may be NULL. */
st_status st_solve(st_handle* h, double* T_dev, st_info* info);

/* Size in MiB of the static device scratch of st_solve_noalloc. */
#define ST_NOALLOC_SCRATCH_MIB 256

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): st_setup,
 * st_solve and st_destroy in one call, with the workspace in a static device
 * array of ST_NOALLOC_SCRATCH_MIB MiB that the library holds on every GPU it
 * runs on (resolved once per device).  No device or pinned host memory is
 * allocated.  Arguments as for st_setup (without the workspace) and st_solve;
 * T_dev: in = initial guess, out = solution.  ST_ERR_OOM (with a message on
 * stderr) when st_footprint_bytes exceeds the scratch; per-kernel timing is
 * not recorded.  Every call on one GPU uses the same array: calls that
 * overlap on one GPU (from several threads or streams) race. */
st_status st_solve_noalloc(const st_grid* grid, const st_material* mat, const double* rho_dev,
                           int32_t rho_time_varying, const double* ic_dev,
                           const double* source_dev, double q0, const st_patch* patches,
                           int32_t n_patches, const st_opts* opts, void* hip_stream,
                           double* T_dev, st_info* info);

/* Adjoint solve J^T lambda = N g (§3.3.3); lambda is zero on Dirichlet nodes.
 * g_dev: nodal dphi/ds.  lambda_dev: in = initial guess, out = solution. */
st_status st_adjoint_solve(st_handle* h, const double* g_dev, double* lambda_dev, st_info* info);

/* Density sensitivities (§3.3.3): g_e = -lambda_e^T (k'_e A + C'_e B) s_e per
 * element, summed over slabs for a time-constant design (§3.4.1), multiplied
 * by the projection's derivative at the filtered design when the problem
 * projects, then sent through the filter (F^T = F, §3.3.2) when it filters.
 * dJdrho_dev has the design's layout.  ST_NOT_CONVERGED (output written)
 * when that filter solve reaches opts->filter_max_it. */
st_status st_sensitivity(st_handle* h, const double* T_dev, const double* lambda_dev,
                         double* dJdrho_dev);

/* J = f^T T with the unmasked consistent load (int Q T dV). */
st_status st_objective(st_handle* h, const double* T_dev, double* J_host);

/* Copy the unmasked consistent load f (= dJ/dT of st_objective) to f_dev. */
st_status st_load_vector(st_handle* h, double* f_dev);

/* p-norm objective of §3.3.1: phi = (sum_e T_avg,e^P)^(1/P) over all
 * space-time elements, T_avg,e the mean of the element's 8 nodal values of
 * T_dev (the full state).  dphi_dT_dev (nullable, node layout) receives the
 * assembled dphi/dT (§3.3.3: theta^((1-P)/P) T_avg,e^(P-1) / 8 to each node
 * of e), the right-hand side of the p-norm adjoint solve.  P > 0; a
 * non-integer P needs T_avg >= 0. */
st_status st_pnorm(st_handle* h, const double* T_dev, double P, double* phi_host,
                   double* dphi_dT_dev);

/* Volume constraint of §3.3.1 on the physical design (filtered, projected,
 * extruded over time): chi = sum_e rho_e v_e / (vf |Pi|) - 1.  dchi_drho_dev
 * (nullable, design layout) receives dchi/d(design), the constant
 * v_e / (vf |Pi|) sent through the same chain rule as st_sensitivity.
 * 0 < vf. */
st_status st_volume(st_handle* h, double vf, double* chi_host, double* dchi_drho_dev);

/* Apply the density filter F (§3.3.2) to an element field of the design's
 * layout.  ST_ERR_STATE when the problem has no filter; ST_NOT_CONVERGED
 * (output written from the last CG iterate) when the filter's CG reaches
 * opts->filter_max_it before opts->filter_rtol. */
st_status st_filter(st_handle* h, const double* in_dev, double* out_dev);

/* Move a built problem to another HIP stream (e.g. a serving slot's); the
 * old stream is synchronised first. */
st_status st_set_stream(st_handle* h, void* hip_stream);

/* Replace the option flags (ST_FLAG_TIME_KERNELS and its class mask,
 * ST_FLAG_COARSE_GMRES, ST_FLAG_SSTEP_SMOOTHER, ST_FLAG_OUTER_CGS2, ST_FLAG_ROW_MARCH) of a built problem; ST_FLAG_NO_PLANE_DEDUP,
 * ST_FLAG_FULL_COARSENING and the other options are fixed at setup.  Switching to the exact coarse solve
 * factorises the coarsest operator on the next V-cycle. */
st_status st_set_flags(st_handle* h, int32_t flags);

/* Fill the hierarchy fields of *info (levels, dims, distinct planes). */
st_status st_hierarchy(st_handle* h, st_info* info);

/* Release host-side state (the workspace stays the caller's). */
void st_destroy(st_handle* h);

/* ---- test entry points: single pieces of the V-cycle, all in FP64 I/O ---- */

/* y = A_l x (transpose: A_l^T x) on level l in precision prec (ST_FP64 or
 * ST_MIXED = that level's V-cycle storage); x, y are FP64 level vectors. */
st_status st_debug_apply(st_handle* h, int32_t level, int32_t transpose, int32_t prec,
                         const double* x_dev, double* y_dev);
/* Level-l 27-point stencil, expanded to [27][nt+1][ny+1][nx+1] FP64; entry
 * d = (dn+1)*9 + (dj+1)*3 + (di+1) holds A(node, node + offset).  Level 0 is
 * materialised from the matrix-free operator by probing. */
st_status st_debug_stencil(st_handle* h, int32_t level, double* out_dev);
/* Inverse diagonal (FP64) and Dirichlet mask (uint8) of level l. */
st_status st_debug_diag(st_handle* h, int32_t level, double* invdiag_dev, uint8_t* mask_dev);
/* prolong = 0: out = P_m^T in (level l -> l+1); 1: out = P_m in (l+1 -> l). */
st_status st_debug_transfer(st_handle* h, int32_t level, int32_t prolong,
                            const double* in_dev, double* out_dev);
/* One Jacobi-GMRES smoothing on level l in FP64 (its iterations, rtol):
 * x = GMRES(A_l, b, x0) with x0 = 0 when zero_x0 else the content of x. */
st_status st_debug_smooth(st_handle* h, int32_t level, int32_t transpose, const double* b_dev,
                          double* x_dev, int32_t zero_x0, int32_t its, double rtol);
/* One application of the V-cycle preconditioner in the handle's precision,
 * FP64 input and output: x = M^-1 b. */
st_status st_debug_vcycle(st_handle* h, int32_t transpose, const double* b_dev, double* x_dev);
/* ABI layout check (no GPU needed): writes up to n of sizeof(st_grid),
 * sizeof(st_material), sizeof(st_patch), sizeof(st_opts), sizeof(st_info),
 * offsetof(st_opts, flags), offsetof(st_info, kclass_ms) into out. */
st_status st_abi_sizes(size_t* out, int32_t n);

#ifdef __cplusplus
}
#endif

#endif /* ST_API_H */
