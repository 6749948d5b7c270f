// Host-side checks of libst's C ABI, built with AddressSanitizer and
// UndefinedBehaviorSanitizer on the host code (tests/test_host_sanitizers.py):
// option defaults and validation, the Algorithm 1 hierarchy and the
// workspace sizing pass over many grid shapes and option sets, and the
// argument checks of st_setup.  Nothing here touches a GPU.
#include <cstdio>
#include <cstdlib>
#include <cmath>

#include "st_api.h"

static int failures = 0;

static void expect(bool ok, const char* what, int a = 0, int b = 0, int c = 0) {
    if (!ok) {
        std::fprintf(stderr, "FAIL %s (%d %d %d)\n", what, a, b, c);
        ++failures;
    }
}

static st_status footprint(int nx, int ny, int nt, const st_opts& o, int tv, size_t* bytes) {
    st_grid g{nx, ny, nt, 1.0 / (nx > ny ? nx : ny), 1.0 / nt};
    st_material m{1e-3, 1.0, 3.0, 1.0, 1.0, 1.0};
    return st_footprint_bytes(&g, &m, &o, tv, bytes);
}

int main() {
    st_opts o;
    st_opts_default(&o);
    expect(o.restart == 30 && o.smooth_its == 10 && o.filter_max_it == 2000, "defaults");
    for (int s = -6; s <= 2; ++s) expect(st_status_string((st_status)s) != nullptr, "status");

    // every grid shape up to 40 x 40 x 40 in steps, odd and even, both
    // precisions and design layouts, semi and full coarsening
    const int sizes[] = {1, 2, 3, 4, 5, 7, 8, 9, 15, 16, 17, 31, 32, 33, 40};
    for (int nx : sizes)
        for (int ny : sizes)
            for (int nt : sizes)
                for (int prec = 0; prec < 2; ++prec)
                    for (int tv = 0; tv < 2; ++tv) {
                        st_opts q = o;
                        q.precision = prec;
                        q.bf16_from_level = prec ? 1 : 0;
                        q.flags = ((nx + nt) & 1) ? ST_FLAG_FULL_COARSENING : 0;
                        q.max_coarse_nodes = (nx * ny) % 3 == 0 ? 64 : 4096;
                        size_t b = 0;
                        st_status rc = footprint(nx, ny, nt, q, tv, &b);
                        expect(rc == ST_OK && b > 0, "footprint", nx, ny, nt);
                    }
    // the large workloads
    {
        st_opts q = o;
        q.precision = ST_MIXED;
        q.restart = 20;
        q.bf16_from_level = 1;
        size_t b = 0, b64 = 0;
        expect(footprint(512, 512, 1024, q, 0, &b) == ST_OK, "large mixed");
        q.precision = ST_FP64;
        q.bf16_from_level = 0;
        expect(footprint(512, 512, 1024, q, 0, &b64) == ST_OK && b64 > b, "large fp64");
        q.max_levels = 3;
        expect(footprint(512, 512, 1024, q, 1, &b) == ST_OK, "large 3 levels");
    }
    // invalid options
    {
        size_t b = 0;
        st_opts q = o;
        q.restart = 2;
        expect(footprint(8, 8, 8, q, 0, &b) == ST_ERR_ARG, "restart");
        q = o;
        q.smooth_its = 99;
        expect(footprint(8, 8, 8, q, 0, &b) == ST_ERR_ARG, "smooth_its");
        q = o;
        q.filter_rtol = NAN;
        expect(footprint(8, 8, 8, q, 0, &b) == ST_ERR_ARG, "filter_rtol");
        q = o;
        q.rtol = -1;
        expect(footprint(8, 8, 8, q, 0, &b) == ST_ERR_ARG, "rtol");
        expect(footprint(0, 8, 8, o, 0, &b) == ST_ERR_ARG, "nx");
        expect(footprint(8, 8, -3, o, 0, &b) == ST_ERR_ARG, "nt");
        expect(footprint(1024, 1024, 512, o, 0, &b) == ST_ERR_ARG, "2^29 nodes");
        expect(footprint(1022, 1022, 510, o, 0, &b) == ST_OK, "under 2^29 nodes");
        st_grid g{8, 8, 8, 0.125, 0.125};
        st_material m{1e-3, 1.0, 3.0, 1.0, 1.0, 1.0};
        expect(st_footprint_bytes(nullptr, &m, &o, 0, &b) == ST_ERR_ARG, "null grid");
        expect(st_footprint_bytes(&g, &m, &o, 0, nullptr) == ST_ERR_ARG, "null out");
        st_material bad{0.0, 1.0, 3.0, 1.0, 1.0, 1.0};
        expect(st_footprint_bytes(&g, &bad, &o, 0, &b) == ST_ERR_ARG, "k_ins");
        st_handle* h = nullptr;
        expect(st_setup(&g, &m, nullptr, 0, nullptr, nullptr, 1.0, nullptr, 0, &o, nullptr, 0,
                        nullptr, &h) == ST_ERR_ARG && h == nullptr, "setup nulls");
        expect(st_solve(nullptr, nullptr, nullptr) == ST_ERR_ARG, "solve null");
        expect(st_adjoint_solve(nullptr, nullptr, nullptr, nullptr) == ST_ERR_ARG, "adjoint null");
        expect(st_sensitivity(nullptr, nullptr, nullptr, nullptr) == ST_ERR_ARG, "sens null");
        st_destroy(nullptr);
    }
    size_t sz[7];
    expect(st_abi_sizes(sz, 7) == ST_OK && sz[0] == sizeof(st_grid) && sz[3] == sizeof(st_opts),
           "abi sizes");
    if (failures) {
        std::fprintf(stderr, "%d failures\n", failures);
        return 1;
    }
    std::printf("host_check ok\n");
    return 0;
}
