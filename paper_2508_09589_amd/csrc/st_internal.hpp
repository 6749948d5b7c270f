// Internal declarations of the space-time solver library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>
#include <vector>
#include <string>

#include "st_api.h"

namespace st {

// ---------------------------------------------------------------------------
// Small fixed limits.
constexpr int KMAX = 32;          // largest Krylov basis (FGMRES / coarse restart)
constexpr int SMAX = 16;          // largest smoother basis
constexpr int RED_BLOCKS = 2048;  // most blocks of a grid-stride reduction kernel
constexpr int RED_WIDTH = 2 * 32 + 4;   // most accumulators per block (delayed CGS2: 2j + 3)
// Reduction scratch: [RED_BLOCKS][RED_WIDTH] block partials, then the arrival
// counter of reductions without a KState.
constexpr size_t PARTIALS_DOUBLES = (size_t)RED_BLOCKS * RED_WIDTH + 64;
constexpr size_t PARTIALS_COUNTER = (size_t)RED_BLOCKS * RED_WIDTH + 32;
constexpr int VEC_THREADS = 256;

// Device-resident state of one GMRES / FGMRES cycle.  Every small scalar step
// (projections, Givens rotations, the least-squares solve, convergence test)
// runs on the device so that a whole smoothing needs no host round trip.
struct KState {
    double H[KMAX + 1][KMAX];   // rotated Hessenberg (upper triangular part = R)
    double cs[KMAX], sn[KMAX];
    double g[KMAX + 1];         // rotated right-hand side beta e1
    double scale[KMAX + 1];     // 1 / ||w_d|| of the (unnormalised) basis vector d
    double hcol[KMAX + 1];      // projections of the current column (scaled)
    double coef[KMAX + 1];      // maxpy coefficients for the unnormalised basis
    double y[KMAX];             // update coefficients
    double ref;                 // reference norm of the relative tolerance
    double rtol;
    double est;                 // |g_k|: residual estimate after k steps
    double beta;                // initial residual norm of this cycle
    int k;                      // completed iterations this cycle
    int done;                   // 1 = converged / breakdown / maxit reached
    int maxit;                  // iterations allowed this cycle
    int bad;                    // NaN or Inf seen
    unsigned counter;           // arrival counter of the last-block reduction
    int scale_update;           // 1: y_d multiplied by scale_d (unnormalised basis)
    int pending;                // delayed CGS2: the cycle ends after this column
    int pad1;
    double gcarry[2];           // fused smoother: unrotated g of the next column,
                                // alternating by column parity
    // delayed CGS2 (outer FGMRES): re-orthogonalisation coefficients of the
    // current vector, its norm, and the scalars of the update pass
    double ds[KMAX];
    double d_nuinv, d_c, d_eta, d_etainv;
    int d_brk, d_pad;
};

// Finalisation modes of the fused reduction kernels.
enum FinMode {
    FIN_INIT_SELF = 0,   // beta = sqrt(sum); ref = beta
    FIN_INIT_REF = 1,    // beta = sqrt(sum); ref unchanged (set by host)
    FIN_PROJ1 = 2,       // first CGS projections h_d
    FIN_PROJ2 = 3,       // re-orthogonalisation projections (CGS2)
    FIN_GIVENS = 4,      // norm of the new vector, Givens update, convergence test
    FIN_SUM = 5,         // plain sums to out[]
    FIN_NONE = 6,        // maxpy only: subtract, no reduction
    FIN_DCGS2 = 7,       // delayed CGS2 step: [s, t, alpha, beta, gamma] -> column j-1 final,
                         // column j provisional, update coefficients
    FIN_DCGS2_LAST = 8   // last column of a cycle: [s', alpha'] -> final column, y
};

// T = 0 patches translated to index ranges.
struct PatchSet {
    int n;
    int edge[ST_MAX_PATCHES];
    int lo[ST_MAX_PATCHES];
    int hi[ST_MAX_PATCHES];
};

struct FineGeom {
    int nx, ny, nt;       // elements
    double dt6;           // dt / 6 times 1/6 of the 2-D stiffness (= dt / 36)
    double mw;            // dx^2 / 36
    int tconst;           // coefficient arrays have a single slab
    int cuniform;         // capacity uniform (value c0, no C array)
    double c0;
    int ic_dir;           // the t = 0 plane is Dirichlet
    PatchSet patches;
};

// Level of the multigrid hierarchy (host view of device buffers).
struct Level {
    int nx, ny, nt;
    long long nn;           // nodes
    long long ld;           // basis stride: nn rounded up to 64 elements
    double dx, dt;
    int how;                // 0 finest, 1 space-coarsened, 2 time-coarsened, 3 both
    int nplanes;            // distinct stencil time levels
    int vprec;              // 0 = FP64 vectors, 1 = FP32 vectors in the V-cycle
    int sprec;              // stencil storage: 0 FP64, 1 FP32, 2 BF16
    uint8_t* mask = nullptr;       // [nn] 1 = Dirichlet
    int* plane_map = nullptr;      // [nt+1] -> distinct plane
    double* st64 = nullptr;        // [27][nplanes][ny+1][nx+1]
    float* st32 = nullptr;
    uint16_t* st16 = nullptr;
    float* cen32 = nullptr;        // BF16 stencils: compensated centres [3][nplanes][ny+1][nx+1]
    double* invd64 = nullptr;
    float* invd32 = nullptr;
    void* x = nullptr;             // V-cycle vectors (vprec)
    void* b = nullptr;
    void* r = nullptr;
    void* V = nullptr;             // smoother basis [SMAX+1][nn]
    KState* ks = nullptr;
};

struct Workspace;  // memory carving

}  // namespace st

// Kernel launchers (defined in the .hip files).
namespace st {
struct Coef {
    const double* k64; const double* c64;   // element coefficients (FP64)
    const float* k32; const float* c32;     // FP32 copies
};
void launch_simp(hipStream_t s, long long ne, const double* rho, const st_material* m,
                 double* k, double* c, double* dk, double* dc, float* k32, float* c32, int cuniform);
void launch_fine_apply(hipStream_t s, const FineGeom& g, const Coef& cf, int prec_in, int prec_out,
                       int compute64, int trans, const void* x, void* y, const void* b,
                       int jacobi, const double* scale, const int* skip, int mask_in,
                       int dir_rows);
void launch_fine_invdiag(hipStream_t s, const FineGeom& g, const Coef& cf, double dx, double dt,
                         double* invd64, float* invd32, uint8_t* mask);
// row_march: the row-march kernel instead of the wave form (which it
// replaces by itself where a level's vectors pass 2 GiB)
void launch_stencil_apply(hipStream_t s, const Level& L, int prec, int trans, const void* x,
                          void* y, const void* b, const void* invd, const double* scale,
                          const int* skip, bool row_march);
void launch_restrict(hipStream_t s, const Level& F, const Level& C, int prec, const void* rf,
                     void* bc);
void launch_prolong(hipStream_t s, const Level& F, const Level& C, int prec, const void* ec,
                    void* xf, int accumulate);
void launch_coarse_mask(hipStream_t s, const Level& F, const Level& C);
void launch_probe_fill(hipStream_t s, const Level& C, int color, double* e);
void launch_probe_extract(hipStream_t s, const Level& C, int color, const double* yc, double* st);
void launch_identity_rows(hipStream_t s, const Level& C, double* st);
void launch_plane_equal(hipStream_t s, const Level& C, const double* st, int* neq);
void launch_plane_compact(hipStream_t s, const Level& C, double* st, const int* src_plane,
                          int ndistinct);
void launch_stencil_invdiag(hipStream_t s, const Level& L, double* invd64, float* invd32);
void launch_stencil_expand(hipStream_t s, const Level& L, double* out);
void launch_stencil_cast(hipStream_t s, const Level& L, float* st32, uint16_t* st16);
void launch_cast(hipStream_t s, long long n, int from, int to, const void* in, void* out,
                 const double* scale);
void launch_fill(hipStream_t s, long long n, int prec, void* p, double v);

// Krylov kernels.
void launch_scale(hipStream_t s, long long n, int prec, const void* b, const void* invd, void* w);
void launch_scale_norm(hipStream_t s, long long n, int prec, const void* b, const void* invd,
                       void* w, double* partials, KState* ks, int mode, int maxit, double rtol,
                       int scale_update);
void launch_mdot(hipStream_t s, long long n, int prec_w, int prec_v, const void* w,
                 const void* V, long long ldv, int nd, double* partials, KState* ks, int mode,
                 int j, int maxd);
void launch_maxpy(hipStream_t s, long long n, int prec_w, int prec_v, void* w, const void* V,
                  long long ldv, int nd, double* partials, KState* ks, int mode, int j, int maxd);
// Delayed CGS2 for the FP64 outer basis: one reduction pass (launch_dcgs2_dots)
// and one update pass (launch_dcgs2_update) per FGMRES step.
void launch_dcgs2_dots(hipStream_t s, long long n, const double* V, long long ldv, int j,
                       double* partials, KState* ks);
void launch_dcgs2_update(hipStream_t s, long long n, double* V, long long ldv, int j, KState* ks);
// Fused CGS2 middle passes (FP64): false when the layout does not allow it.
bool launch_maxpy_mdot(hipStream_t s, long long n, double* w, const double* V, long long ldv,
                       int nd, double* partials, KState* ks, int j);
void launch_update(hipStream_t s, long long n, int prec_x, int prec_v, void* x, const void* V,
                   long long ldv, KState* ks, int zero_x0, int maxd);
void launch_init_state(hipStream_t s, KState* ks, int maxit, double rtol, int scale_update,
                       const double* ref);
void launch_dot(hipStream_t s, long long n, const double* a, const double* b, double* partials,
                double* out);
void launch_coarse_solve(hipStream_t s, const Level& L, int prec_io, int trans, const void* b,
                         void* x, double* V, double* work, int maxit, int restart, double rtol,
                         int zero_x0);

// Fused smoother for small coarse levels (two kernels per GMRES iteration).
bool sm_fused_plan(const Level& L, int* nchunk, int* gx, int* gy);
size_t sm_partials_doubles();
void launch_sm_init(hipStream_t s, const Level& L, int prec, int trans, const void* b,
                    const void* x, int zero_x0, const void* invd, void* V0, KState* ks,
                    double* part, int maxit, double rtol, int* nbn);
void launch_sm_iteration(hipStream_t s, const Level& L, int prec, int trans, const void* invd,
                         void* V, int j, KState* ks, double* part, int* nbn);
void launch_sm_update(hipStream_t s, const Level& L, int prec, void* x, const void* V, KState* ks,
                      const double* part, int nbn, int its, int zero_x0);

// s-step Jacobi-GMRES smoother: Gram matrix of the basis V[0..nv-1] and the
// coefficients y, k of KState (nv <= SMAX), partials of gram_partials_doubles().
size_t gram_partials_doubles();
constexpr int SSTEP_MAX_ITS = 10;   // longer smoothings use the Arnoldi form
void launch_sstep_coefficients(hipStream_t s, long long n, int prec, const void* V, long long ld,
                               int nv, double rtol, double* part, KState* ks);

// Exact coarsest-level solve by block-tridiagonal factorisation in time.
constexpr int CD_MAX_PLANE = 2048;        // largest (nx + 1)(ny + 1) it is used for
constexpr double CD_MAX_FACTOR_BYTES = 16.0 * (1ull << 30);   // largest factor storage
constexpr size_t CD_LDS_MAX = 56 * 1024;  // Gauss-Jordan matrix in LDS up to this size
constexpr int CD_FAST_P = 128;            // fast solve: plane size bound (8 | CD_FAST_P)
constexpr int CD_FAST_NODES = 3072;       // fast solve: whole level in 2 x 24 KB of LDS
bool coarse_direct_fits(int P);
bool coarse_direct_fast(int P, int nt);
size_t coarse_direct_lds(int P);
// Wide factorisation (planes over CD_FAST_P or levels over CD_FAST_NODES):
// A: P^2 working matrix, panel: P x CW_PANEL_NB (used when the panel does not
// fit lds_max bytes of LDS), colk: P, W: P x CW_PANEL_NB, R: CW_PANEL_NB x P,
// perm, idx: P ints.
constexpr int CW_PANEL_NB = 16;
void launch_coarse_factor_wide(hipStream_t s, const Level& L, int lds_max, double* A,
                               double* Dinv, double* G, double* H, double* MT, double* panel,
                               double* colk, double* W, double* R, int* perm, int* idx,
                               int* status);
void launch_coarse_factor(hipStream_t s, const Level& L, double* Ag, double* Dinv, double* G,
                          double* H, double* M, double* colk, int* perm, int* status);
// wide: the wide solve (H = D'^{-1} L, M = L D'^{-1} per time level); else the
// one-workgroup fast solve (H = D'^{-1} L, M = D'^{-T} L^T).
void launch_coarse_direct(hipStream_t s, const Level& L, int prec_io, int trans, const void* b,
                          void* x, const double* Dinv, const double* G, const double* H,
                          const double* M, double* work, int wide);

// Right-hand side, objective, sensitivities, filter.
void launch_load_uniform(hipStream_t s, const FineGeom& g, double q0, double dx, double dt,
                         double* f);
void launch_tensor_op(hipStream_t s, int nx, int ny, int nt, double dx, double dt, double dxx,
                      double dtt, const double* x, double* y, const double* b, const double* invd,
                      const int* skip);
void launch_tensor_invdiag(hipStream_t s, int nx, int ny, int nt, double dx, double dt,
                           double dxx, double dtt, double* invd);
void launch_lift(hipStream_t s, long long n, const uint8_t* mask, const double* f,
                 const double* Jg, const double* g, double* fm);
void launch_mask_vec(hipStream_t s, long long n, const uint8_t* mask, const double* in,
                     double* out);
void launch_elem_to_node(hipStream_t s, int nx, int ny, int nt, double w, const double* e,
                         double* nodal);
void launch_node_to_elem(hipStream_t s, int nx, int ny, int nt, const double* nodal, double* e);
void launch_sensitivity(hipStream_t s, const FineGeom& g, double dx, double dt, const double* T,
                        const double* lam, const double* dk, const double* dc, double* out,
                        int sum_slabs);
void launch_ic_lift_vector(hipStream_t s, const FineGeom& g, const double* ic, double* gvec);
void launch_heaviside(hipStream_t s, long long n, const double* x, double beta, double eta,
                      double* out, double* dout);
void launch_heaviside_chain(hipStream_t s, long long n, const double* x, double beta, double eta,
                            const double* g_in, double* g_out);
void launch_pnorm_theta(hipStream_t s, const FineGeom& g, const double* T, double Pw,
                        double* partials, double* theta);
void launch_pnorm_grad(hipStream_t s, const FineGeom& g, const double* T, double Pw,
                       const double* theta, double* out);
void launch_cg_step(hipStream_t s, int step, long long n, double* x, double* r, double* z,
                    double* p, const double* q, const double* invd, double* partials,
                    double* scal, const int* skip);
}  // namespace st

// st_setup with a choice of host staging (solver.cpp): pinned_host = true is
// st_setup itself; false keeps the staging in the handle (no hipHostMalloc),
// for the entry point that allocates nothing.
st_status setup_impl(const st_grid* grid, const st_material* mat, const double* rho_dev,
                     int32_t rho_time_varying, const double* ic_dev, const double* source_dev,
                     double q0, const st_patch* patches, int32_t n_patches, const st_opts* opts,
                     void* workspace_dev, size_t workspace_bytes, void* hip_stream,
                     bool pinned_host, st_handle** out);
