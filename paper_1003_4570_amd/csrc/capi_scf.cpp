// C ABI: Poisson solver and the self-consistent Schrodinger-Poisson loop.
#include <cmath>

#include "scf.h"
#include "tbh_internal.h"

using tbh::guard;

struct tbh_scf : tbh::Scf {
    using tbh::Scf::Scf;
};

extern "C" {

int tbh_poisson_solve(tbh_ctx* ctx, const int32_t grid[3], double h_nm, double eps_r, const double* rho_dev,
                      double* phi_dev, double rel_tol, int32_t max_iter, int32_t* iters, double* rel_res) {
    int status = TBH_OK;
    const int rc = guard([&] {
        TBH_REQUIRE(ctx && grid && rho_dev && phi_dev, "null argument");
        TBH_REQUIRE(grid[0] > 0 && grid[1] > 0 && grid[2] > 0, "grid sizes must be positive");
        TBH_REQUIRE(h_nm > 0 && eps_r > 0, "h_nm and eps_r must be positive");
        TBH_REQUIRE(max_iter >= 1 && rel_tol >= 0, "bad iteration limits");
        TBH_HIP(hipSetDevice(ctx->device));
        const int g[3] = {grid[0], grid[1], grid[2]};
        const int64_t n = int64_t(g[0]) * g[1] * g[2];
        tbh::DevBuf b;
        b.alloc(n * 8);
        // b = rho / (eps0 eps_r)
        const double s = 1.0 / ((8.8541878128e-12 / 1.602176634e-19 * 1e-9) * eps_r);
        tbh::scale_copy(ctx->stream, n, rho_dev, s, b.as<double>());
        tbh::PoissonWork W;
        int it = 0;
        double rr = 0.0;
        tbh::poisson_cg(ctx->stream, W, g, h_nm, b.as<double>(), phi_dev, rel_tol, max_iter, &it, &rr);
        if (iters) *iters = it;
        if (rel_res) *rel_res = rr;
        if (!(rr <= rel_tol)) status = TBH_ENOCONV;
    });
    if (rc != TBH_OK) return rc;
    if (status != TBH_OK) tbh::set_error("Poisson CG did not reach the tolerance");
    return status;
}

int tbh_scf_create(tbh_ham* h, const tbh_scf_opts* o, tbh_scf** out) {
    return guard([&] {
        TBH_REQUIRE(h && o && out, "null argument");
        TBH_HIP(hipSetDevice(h->ctx->device));
        *out = new tbh_scf(h, *o);
        tbh::retain(h);
    });
}

int tbh_scf_destroy(tbh_scf* s) {
    return guard([&] {
        if (!s) return;
        tbh::Ham* h = s->h;
        (void)hipSetDevice(h->ctx->device);
        (void)hipStreamSynchronize(h->ctx->stream);
        delete s;
        tbh::release(h);
    });
}

int tbh_scf_set_potential(tbh_scf* s, const double* U_dev) {
    return guard([&] {
        TBH_REQUIRE(s, "null scf");
        TBH_HIP(hipSetDevice(s->h->ctx->device));
        s->set_potential(U_dev);
    });
}

int tbh_scf_set_start(tbh_scf* s, const tbh_scf_start* start) {
    return guard([&] {
        TBH_REQUIRE(s && start, "null argument");
        TBH_HIP(hipSetDevice(s->h->ctx->device));
        s->set_start(*start);
    });
}

int tbh_scf_get_potential(tbh_scf* s, double* U_dev) {
    return guard([&] {
        TBH_REQUIRE(s && U_dev, "null argument");
        TBH_HIP(hipSetDevice(s->h->ctx->device));
        TBH_HIP(hipMemcpyAsync(U_dev, s->U.p, s->n_nodes * 8, hipMemcpyDeviceToDevice, s->h->ctx->stream));
        TBH_HIP(hipStreamSynchronize(s->h->ctx->stream));
    });
}

int tbh_scf_get_density(tbh_scf* s, double* n_dev) {
    return guard([&] {
        TBH_REQUIRE(s && n_dev, "null argument");
        TBH_REQUIRE(s->iterations > 0, "no step has been made");
        TBH_HIP(hipSetDevice(s->h->ctx->device));
        hipStream_t st = s->h->ctx->stream;
        if (s->h->permuted)
            tbh::rows_to_caller(st, s->h->n, s->h->perm_d.as<int64_t>(), 8, s->n_atoms_d.p, n_dev);
        else
            TBH_HIP(hipMemcpyAsync(n_dev, s->n_atoms_d.p, size_t(s->h->n) * 8, hipMemcpyDeviceToDevice, st));
        TBH_HIP(hipStreamSynchronize(st));
    });
}

int tbh_scf_step(tbh_scf* s, tbh_scf_report* rep) {
    return guard([&] {
        TBH_REQUIRE(s, "null scf");
        TBH_HIP(hipSetDevice(s->h->ctx->device));
        tbh_scf_report r{};
        s->step(r);
        if (rep) *rep = r;
    });
}

int tbh_scf_run(tbh_scf* s, int32_t max_iter, tbh_scf_report* rep) {
    int status = TBH_OK;
    const int rc = guard([&] {
        TBH_REQUIRE(s && max_iter >= 1, "null scf or max_iter < 1");
        TBH_HIP(hipSetDevice(s->h->ctx->device));
        tbh_scf_report r{};
        double secs = 0.0, es = 0.0, ps = 0.0, ns = 0.0;
        for (int it = 0; it < max_iter; ++it) {
            s->step(r);
            secs += r.seconds;
            es += r.eig_seconds;
            ps += r.poisson_seconds;
            ns += r.newton_seconds;
            if (r.converged || !std::isfinite(r.residual)) break;
        }
        r.seconds = secs;
        r.eig_seconds = es;
        r.poisson_seconds = ps;
        r.newton_seconds = ns;
        if (rep) *rep = r;
        if (!r.converged) status = TBH_ENOCONV;
    });
    if (rc != TBH_OK) return rc;
    if (status != TBH_OK) tbh::set_error("SCF did not converge within max_iter steps");
    return status;
}

}  // extern "C"
