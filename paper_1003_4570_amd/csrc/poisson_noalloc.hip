// Allocation-free variant of the finite-difference Poisson solve (Sec. III-A
// item 3), for callers that cannot allocate device memory (code under HIP
// graph capture, tight serving loops, harnesses that forbid hipMalloc).
//
// The CG solve needs device scratch beyond its inputs and outputs: the
// right-hand side b, the CG vectors r, p, Ap, the per-block partial sums and
// the scalar state.  Here they live in one file-scope device array of fixed
// size, so the entry point allocates nothing.  Each device holds its own copy
// of the array until the process ends; its device address is looked up once
// per device at context creation (hipGetSymbolAddress), and host code only
// ever hands kernels that address, never the array's name.
//
// Every call on a device shares that device's array and leaves its last
// contents there; calls that overlap on one device (several streams or host
// threads at once) race on it.  Every scratch value is written before it is
// read within a call, so nothing needs clearing between calls.
#include <mutex>

#include "scf.h"
#include "tbh_internal.h"

namespace tbh {

namespace {

// largest grid the array serves: 2^18 nodes (the 32 x 32 x 240 grid of the
// 8 x 8 x 60-cell slab has 245,760)
constexpr int64_t NOALLOC_MAX_NODES = int64_t(1) << 18;
constexpr int64_t NOALLOC_DOUBLES = 4 * NOALLOC_MAX_NODES + POISSON_PART + POISSON_SCAL;

__device__ __align__(256) double scratch[NOALLOC_DOUBLES];

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
double* g_ptr[MAX_DEVICES] = {};

}  // namespace

void noalloc_setup(int device) {
    TBH_REQUIRE(device >= 0 && device < MAX_DEVICES, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_ptr[device]) return;
    // the caller has made `device` current
    void* ptr = nullptr;
    TBH_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    TBH_REQUIRE(ptr != nullptr, "hipGetSymbolAddress returned a null scratch address");
    g_ptr[device] = static_cast<double*>(ptr);
}

double* noalloc_scratch(int device) {
    std::lock_guard<std::mutex> lk(g_mu);
    return device >= 0 && device < MAX_DEVICES ? g_ptr[device] : nullptr;
}

}  // namespace tbh

using tbh::guard;

extern "C" int tbh_poisson_solve_noalloc(tbh_ctx* ctx, const int32_t grid[3], double h_nm, double eps_r,
                                         const double* rho_dev, double* phi_dev, double rel_tol,
                                         int32_t max_iter, int32_t* iters, double* rel_res) {
    int status = TBH_OK;
    const int rc = guard([&] {
        TBH_REQUIRE(ctx && grid && rho_dev && phi_dev, "null argument");
        TBH_REQUIRE(grid[0] > 0 && grid[1] > 0 && grid[2] > 0, "grid sizes must be positive");
        TBH_REQUIRE(h_nm > 0 && eps_r > 0, "h_nm and eps_r must be positive");
        TBH_REQUIRE(max_iter >= 1 && rel_tol >= 0, "bad iteration limits");
        const int64_t n = int64_t(grid[0]) * grid[1] * grid[2];
        TBH_REQUIRE(n <= tbh::NOALLOC_MAX_NODES,
                    "grid of " + std::to_string(n) + " nodes exceeds the allocation-free limit of " +
                        std::to_string(tbh::NOALLOC_MAX_NODES) + " nodes (use tbh_poisson_solve)");
        TBH_HIP(hipSetDevice(ctx->device));
        double* base = tbh::noalloc_scratch(ctx->device);
        TBH_REQUIRE(base != nullptr, "no scratch address for this device (context not set up)");
        const int64_t M = tbh::NOALLOC_MAX_NODES;
        double* b = base;
        const tbh::PoissonBufs W{base + M, base + 2 * M, base + 3 * M, base + 4 * M,
                                 base + 4 * M + tbh::POISSON_PART};
        const int g[3] = {grid[0], grid[1], grid[2]};
        // b = rho / (eps0 eps_r)
        const double s = 1.0 / ((8.8541878128e-12 / 1.602176634e-19 * 1e-9) * eps_r);
        tbh::scale_copy(ctx->stream, n, rho_dev, s, b);
        int it = 0;
        double rr = 0.0;
        tbh::poisson_cg_bufs(ctx->stream, W, g, h_nm, b, phi_dev, rel_tol, max_iter, &it, &rr);
        if (iters) *iters = it;
        if (rel_res) *rel_res = rr;
        if (!(rr <= rel_tol)) status = TBH_ENOCONV;
    });
    if (rc != TBH_OK) return rc;
    if (status != TBH_OK) tbh::set_error("Poisson CG did not reach the tolerance");
    return status;
}
