// Drives the library's host code without a GPU -- the FP64 hierarchy build
// (grids, Shortley-Weller rows, injection, Galerkin products, polynomial
// coefficients, the coarsest inverse) and the host-only ABI calls (parameter
// validation, level plans, exact workspace sizes, batched sizes) -- on valid
// and invalid parameters, built with AddressSanitizer and
// UndefinedBehaviorSanitizer by tests/test_host_sanitize.py.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "csg.h"
#include "csg_internal.h"

namespace {

csg_params base(int dim)
{
    csg_params p;
    std::memset(&p, 0, sizeof p);
    p.dim = dim;
    for (int a = 0; a < dim; ++a) {
        p.n[a] = dim == 2 ? 37 + 4 * a : 13 + 2 * a;
        p.layer_lo[a] = 3 + a;
        p.layer_hi[a] = 4;
    }
    p.h = 1.0 / 40;
    p.gamma = 0.5235987755982988;
    p.beta = 0.3;
    p.s = 3;
    p.nu1 = p.nu2 = 1;
    p.max_rhs = 2;
    p.restart = 12;
    return p;
}

int check(const csg_params &p, bool valid)
{
    size_t bytes = 0;
    const int rc = csg_workspace_bytes(&p, &bytes);
    if ((rc == CSG_OK) != valid) {
        std::printf("workspace_bytes rc %d (%s), expected %s\n", rc, csg_last_error(), valid ? "ok" : "error");
        return 1;
    }
    if (!valid) return 0;
    int levels = 0, dims[CSG_MAX_LEVELS][3];
    if (csg_plan_levels(&p, &levels, dims) != CSG_OK) {
        std::printf("plan_levels: %s\n", csg_last_error());
        return 1;
    }
    size_t b2 = 0;
    // batched operators take the GMRES(s) smoother only
    if (p.smoother == 0 && (csg_batch_workspace_bytes(&p, 2, &b2) != CSG_OK || b2 <= bytes)) {
        std::printf("batch_workspace_bytes: %s (%zu vs %zu)\n", csg_last_error(), b2, bytes);
        return 1;
    }
    long N = 1;
    for (int a = 0; a < p.dim; ++a) N *= dims[0][a];
    std::vector<double> phi((size_t)N);
    for (long i = 0; i < N; ++i) phi[(size_t)i] = 900.0 * (1.0 + 0.25 * std::sin(0.03 * (double)i));
    csg::HostHier hh;
    std::string err;
    if (csg::build_hierarchy(p, phi.data(), hh, err) != CSG_OK) {
        std::printf("build_hierarchy: %s\n", err.c_str());
        return 1;
    }
    if (hh.L != levels || hh.nc <= 0) {
        std::printf("hierarchy: %d levels (plan %d), coarsest %d\n", hh.L, levels, hh.nc);
        return 1;
    }
    return 0;
}

}  // namespace

int main()
{
    int bad = 0;
    for (int dim = 2; dim <= 3; ++dim) {
        csg_params p = base(dim);
        bad |= check(p, true);
        p.smoother = 1;
        bad |= check(p, true);
        p = base(dim);
        p.coarse_op = 1;
        p.shift_re = 1.0;
        p.shift_im = 0.4;
        bad |= check(p, true);
        p = base(dim);
        p.levels = 2;
        p.s = 4;
        p.cycle_prec = 1;
        p.slab_blocks = 7;
        p.tile_mult = 4;
        p.slab_min = -1;
        bad |= check(p, true);
        p = base(dim);
        for (int a = 0; a < dim; ++a) p.layer_lo[a] = 0;
        bad |= check(p, true);
        // invalid parameters
        p = base(dim);
        p.beta = 0.7;
        bad |= check(p, false);
        p = base(dim);
        p.tile_mult = 3;
        bad |= check(p, false);
        p = base(dim);
        p.coarse_op = 1;
        p.smoother = 1;
        bad |= check(p, false);
        p = base(dim);
        p.max_rhs = 0;
        bad |= check(p, false);
        p = base(dim);
        p.shift_re = NAN;
        bad |= check(p, false);
    }
    size_t bytes = 0;
    bad |= csg_workspace_bytes(nullptr, &bytes) == CSG_OK;
    std::printf("library host driver: %s\n", bad ? "FAILED" : "ok");
    return bad;
}
