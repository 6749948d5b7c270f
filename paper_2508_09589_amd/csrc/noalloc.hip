// The allocation-free solve: st_setup + st_solve + st_destroy with the
// workspace in a static device array instead of caller memory.
//
// The array below is a per-device object of the code object: each GPU the
// library runs on holds its own copy, at its own address, until the process
// ends.  Host code never passes the array's name to a kernel or a copy (on the
// host that name is only a stand-in symbol); it asks the runtime for the
// device address once per device, with that device current, and uses that.
#include <mutex>
#include <cstdio>

#include "st_internal.hpp"

namespace {

constexpr size_t NOALLOC_BYTES = (size_t)ST_NOALLOC_SCRATCH_MIB << 20;
constexpr int MAX_DEVICES = 64;

__device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

std::mutex g_mu;
void* g_scratch[MAX_DEVICES] = {};

// Device address of the current device's scratch array (resolved once per
// device), or nullptr with the HIP error printed.
void* scratch_address(int dev) {
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            fprintf(stderr, "st_solve_noalloc: hipGetSymbolAddress failed on device %d: %s\n", dev,
                    hipGetErrorString(e));
            return nullptr;
        }
        g_scratch[dev] = p;
    }
    return g_scratch[dev];
}

}  // namespace

extern "C" st_status st_solve_noalloc(const st_grid* grid, const st_material* mat,
                                      const double* rho_dev, int32_t rho_time_varying,
                                      const double* ic_dev, const double* source_dev, double q0,
                                      const st_patch* patches, int32_t n_patches,
                                      const st_opts* opts, void* hip_stream, double* T_dev,
                                      st_info* info) {
    if (!grid || !mat || !opts || !rho_dev || !T_dev) return ST_ERR_ARG;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) return ST_ERR_HIP;
    // per-kernel timing would create HIP events; this entry point creates nothing
    st_opts o = *opts;
    o.flags &= ~ST_FLAG_TIME_KERNELS;
    size_t need = 0;
    st_status rc = st_footprint_bytes(grid, mat, &o, rho_time_varying, &need);
    if (rc != ST_OK) return rc;
    if (need > NOALLOC_BYTES) {
        fprintf(stderr,
                "st_solve_noalloc: this problem needs %zu bytes of workspace; the static scratch "
                "holds %zu (use st_setup with a caller workspace)\n", need, NOALLOC_BYTES);
        return ST_ERR_OOM;
    }
    void* ws = scratch_address(dev);
    if (!ws) return ST_ERR_HIP;
    st_handle* h = nullptr;
    rc = setup_impl(grid, mat, rho_dev, rho_time_varying, ic_dev, source_dev, q0, patches,
                    n_patches, &o, ws, NOALLOC_BYTES, hip_stream, false, &h);
    if (rc != ST_OK && rc != ST_NOT_CONVERGED) return rc;
    const st_status rs = st_solve(h, T_dev, info);
    st_destroy(h);
    return rs != ST_OK ? rs : rc;
}
