// C ABI: block Lanczos eigensolver and the dense projected eigensolve.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <limits>
#include <numeric>
#include <vector>

#include "block_lanczos.h"
#include "lanczos.h"
#include "tbh_internal.h"

using tbh::guard;

namespace {

tbh::BlWork& bl_workspace(tbh::Ham& h) {
    if (!h.bl) h.bl = std::make_shared<tbh::BlWork>();
    return *h.bl;
}

}  // namespace

extern "C" {

int tbh_symm_eig_near(tbh_ctx* ctx, int32_t n, const double* A, double sigma, int32_t nc, double* theta,
                      double* vecs) {
    return guard([&] {
        TBH_REQUIRE(ctx && A && theta, "null argument");
        TBH_REQUIRE(n >= 1 && n <= 2048 && nc >= 1 && nc <= n, "need 1 <= nc <= n <= 2048");
        TBH_HIP(hipSetDevice(ctx->device));
        hipStream_t st = ctx->stream;
        tbh::DevBuf Ad, th, S;
        Ad.alloc(size_t(n) * n * 8);
        th.alloc(size_t(nc) * 8);
        S.alloc(size_t(nc) * n * 8);
        TBH_HIP(hipMemcpyAsync(Ad.p, A, size_t(n) * n * 8, hipMemcpyHostToDevice, st));
        tbh::EigWork w;
        tbh::symm_eig_near(st, n, Ad.as<double>(), sigma, nc, w, th.as<double>(), S.as<double>());
        TBH_HIP(hipMemcpyAsync(theta, th.p, size_t(nc) * 8, hipMemcpyDeviceToHost, st));
        if (vecs) TBH_HIP(hipMemcpyAsync(vecs, S.p, size_t(nc) * n * 8, hipMemcpyDeviceToHost, st));
        TBH_HIP(hipStreamSynchronize(st));
    });
}

int tbh_block_lanczos_eigs(tbh_ham* h, const tbh_block_lanczos_opts* o, double* evals, double* refined,
                           double* res, double* evecs_dev, tbh_block_lanczos_report* rep) {
    int status = TBH_OK;
    const int rc = guard([&] {
        TBH_REQUIRE(h && o, "null argument");
        const int b = o->block, m = o->steps, k = o->k;
        TBH_REQUIRE(b == 16 || b == 32 || b == 64, "block must be 16, 32 or 64");
        TBH_REQUIRE(m >= 1 && int64_t(m) * b <= 2048, "steps must satisfy 1 <= steps and steps * block <= 2048");
        TBH_REQUIRE(k >= 1 && k <= b, "k must satisfy 1 <= k <= block");
        TBH_REQUIRE(o->cycles >= 1, "cycles must be >= 1");
        TBH_REQUIRE(h->has_mv && h->has_f64,
                    "block Lanczos needs the multi-vector copy and an FP64 copy (build TBH_F32 with multi_vector=1, "
                    "keep_f64=1)");
        TBH_HIP(hipSetDevice(h->ctx->device));
        const auto t0 = std::chrono::steady_clock::now();
        hipStream_t st = h->ctx->stream;
        tbh::BlWork& W = bl_workspace(*h);
        W.ensure(*h, b, m, b);
        tbh::BlOpts bo;
        bo.b = b;
        bo.m = m;
        bo.nc = b;
        bo.sigma = o->sigma;
        bo.defl_tol = o->defl_tol > 0 ? o->defl_tol : 1e-6;
        bo.time_hx = true;
        bo.fold = o->fold != 0;
        const double res_tol = o->res_tol > 0 ? o->res_tol : 1e-4;
        tbh::DevBuf X0;
        X0.alloc(size_t(h->dim) * b * 4);
        if (o->x0_dev)
            tbh::block_from_states(st, h->dim, b, o->x0_dev, X0.as<float>());
        else
            tbh::block_random(st, h->dim, b, 0x5eedb10c4ull, X0.as<float>());
        std::vector<double> rr(size_t(b) * 4);
        int cyc = 0, defl = 0;
        double hx_ms = 0.0;
        std::vector<int> order;
        for (;;) {
            tbh::block_lanczos_run(*h, W, bo, X0.as<float>());
            ++cyc;
            defl += W.deflated;
            hx_ms += W.hx_ms;
            TBH_HIP(hipMemcpyAsync(rr.data(), W.res.p, rr.size() * 8, hipMemcpyDeviceToHost, st));
            TBH_HIP(hipStreamSynchronize(st));
            // the k candidates nearest sigma by Ritz value (ties: lower value)
            order.resize(size_t(b));
            std::iota(order.begin(), order.end(), 0);
            std::stable_sort(order.begin(), order.end(), [&](int a, int c) {
                const double da = std::fabs(rr[4 * a] - o->sigma), dc = std::fabs(rr[4 * c] - o->sigma);
                if (da != dc) return da < dc;
                return rr[4 * a] < rr[4 * c];
            });
            bool done = true;
            for (int t = 0; t < k; ++t)
                if (!(rr[4 * order[size_t(t)] + 1] <= res_tol)) done = false;
            if (done || cyc >= o->cycles) break;
            // restart from the b Ritz vectors nearest sigma
            tbh::block_from_states(st, h->dim, b, W.Y.as<double>(), X0.as<float>());
        }
        // report the k converged candidates nearest sigma, ascending
        std::vector<int> conv;
        for (int t = 0; t < b && int(conv.size()) < k; ++t)
            if (rr[4 * order[size_t(t)] + 1] <= res_tol) conv.push_back(order[size_t(t)]);
        std::stable_sort(conv.begin(), conv.end(), [&](int a, int c) { return rr[4 * a + 2] < rr[4 * c + 2]; });
        const int nf = int(conv.size());
        const double nan = std::numeric_limits<double>::quiet_NaN();
        double mres = 0.0;
        for (int t = 0; t < k; ++t) {
            if (t < nf) {
                const int c = conv[size_t(t)];
                if (evals) evals[t] = rr[4 * c];
                if (refined) refined[t] = rr[4 * c + 2];
                if (res) res[t] = rr[4 * c + 1];
                mres = std::max(mres, rr[4 * c + 1]);
                if (evecs_dev)
                    tbh::scale_copy(st, h->dim, W.Y.as<double>() + size_t(c) * h->dim, 1.0 / rr[4 * c + 3],
                                    evecs_dev + size_t(t) * h->dim);
            } else {
                if (evals) evals[t] = nan;
                if (refined) refined[t] = nan;
                if (res) res[t] = nan;
                if (evecs_dev)
                    TBH_HIP(hipMemsetAsync(evecs_dev + size_t(t) * h->dim, 0, size_t(h->dim) * 8, st));
            }
        }
        TBH_HIP(hipStreamSynchronize(st));
        if (rep) {
            rep->cycles = cyc;
            rep->n_found = nf;
            rep->deflated = defl;
            rep->max_res = mres;
            rep->hx_seconds = hx_ms * 1e-3;
            rep->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        }
        if (nf < k) status = TBH_ENOCONV;
    });
    if (rc != TBH_OK) return rc;
    if (status != TBH_OK) tbh::set_error("block Lanczos: fewer than k Ritz pairs converged");
    return status;
}

int tbh_filtered_eigs(tbh_ham* h, const tbh_filter_opts* o, double* evals, double* res, double* evecs_dev,
                      tbh_filter_report* rep) {
    int status = TBH_OK;
    const int rc = guard([&] {
        TBH_REQUIRE(h && o, "null argument");
        const int b = o->block;
        TBH_REQUIRE(b == 16 || b == 32 || b == 64, "block must be 16, 32 or 64");
        TBH_REQUIRE(o->k >= 1 && o->k <= b, "k must satisfy 1 <= k <= block");
        TBH_REQUIRE(o->degree >= 1 && o->degree_cold >= 1 && o->max_iter >= 0, "bad degree or iteration count");
        TBH_REQUIRE(h->has_mv && !h->cplx_h, "the filtered solver needs a real H built with multi_vector=1");
        TBH_HIP(hipSetDevice(h->ctx->device));
        const auto t0 = std::chrono::steady_clock::now();
        hipStream_t st = h->ctx->stream;
        tbh::BlWork& W = bl_workspace(*h);
        if (!h->fs) h->fs = std::make_shared<tbh::FsWork>();
        tbh::FsWork& F = *h->fs;
        F.ensure(h->dim, b);
        tbh::FsSolve so;
        so.s = o->sigma;
        so.degree = o->degree;
        so.degree_cold = o->degree_cold;
        so.max_iter = o->max_iter;
        so.k = o->k;
        so.res_tol = o->res_tol > 0 ? o->res_tol : 1e-4;
        tbh::spectral_bounds(*h, &so.emin, &so.emax);
        if (o->x0_dev) tbh::block_from_states(st, h->dim, b, o->x0_dev, F.Y.as<float>());
        std::vector<double> r4(size_t(b) * 4);
        const int it = tbh::filtered_solve(*h, W, F, so, o->x0_dev != nullptr, nullptr, r4.data());
        // the k converged pairs nearest sigma, ascending
        std::vector<int> order(static_cast<size_t>(b));
        std::iota(order.begin(), order.end(), 0);
        std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
            const double dx = std::fabs(r4[4 * x] - so.s), dy = std::fabs(r4[4 * y] - so.s);
            return dx != dy ? dx < dy : r4[4 * x] < r4[4 * y];
        });
        std::vector<int> conv;
        for (int t = 0; t < b && int(conv.size()) < o->k; ++t)
            if (r4[4 * order[size_t(t)] + 1] <= so.res_tol) conv.push_back(order[size_t(t)]);
        std::sort(conv.begin(), conv.end(), [&](int x, int y) { return r4[4 * x] < r4[4 * y]; });
        const int nf = int(conv.size());
        const double nan = std::numeric_limits<double>::quiet_NaN();
        double mres = 0.0;
        for (int t = 0; t < o->k; ++t) {
            if (t < nf) {
                const int c = conv[size_t(t)];
                if (evals) evals[t] = r4[4 * c];
                if (res) res[t] = r4[4 * c + 1];
                mres = std::max(mres, r4[4 * c + 1]);
                if (evecs_dev)
                    tbh::scale_copy(st, h->dim, F.states.as<double>() + size_t(c) * h->dim, 1.0 / r4[4 * c + 3],
                                    evecs_dev + size_t(t) * h->dim);
            } else {
                if (evals) evals[t] = nan;
                if (res) res[t] = nan;
                if (evecs_dev)
                    TBH_HIP(hipMemsetAsync(evecs_dev + size_t(t) * h->dim, 0, size_t(h->dim) * 8, st));
            }
        }
        TBH_HIP(hipStreamSynchronize(st));
        if (rep) {
            rep->iterations = it;
            rep->n_found = nf;
            rep->max_res = mres;
            rep->emin = so.emin;
            rep->emax = so.emax;
            rep->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        }
        if (nf < o->k) status = TBH_ENOCONV;
    });
    if (rc != TBH_OK) return rc;
    if (status != TBH_OK) tbh::set_error("filtered eigensolve: fewer than k Ritz pairs converged");
    return status;
}

}  // extern "C"
