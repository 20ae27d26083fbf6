// C ABI: Lanczos eigensolver entry points and the converged-set selection.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <cmath>
#include <limits>

#include "lanczos.h"
#include "tbh_internal.h"

using tbh::guard;

namespace {

struct Cand {
    double theta, res, refined, ynorm;
    int c;
};

// Distinct converged values nearest sigma (see tbh_lanczos_eigs).  A
// candidate's value is its FP64 Rayleigh quotient: for a converged pair it is
// within res^2 / gap of the eigenvalue, while the raw Ritz value of an FP32
// recurrence can be off by more than merge_tol, which would keep two copies
// of one eigenvalue apart.
std::vector<std::pair<int, int>> select_converged(const std::vector<Cand>& cs, double sigma, int k,
                                                  double res_tol, double merge_tol) {
    std::vector<int> conv;
    for (int i = 0; i < int(cs.size()); ++i)
        if (cs[i].res <= res_tol) conv.push_back(i);
    std::stable_sort(conv.begin(), conv.end(), [&](int a, int b) { return cs[a].refined < cs[b].refined; });
    std::vector<std::pair<int, int>> reps;  // (representative, copies)
    size_t s = 0;
    while (s < conv.size()) {
        size_t e = s + 1;
        while (e < conv.size() && cs[conv[e]].refined - cs[conv[e - 1]].refined <= merge_tol) ++e;
        int best = conv[s];
        for (size_t t = s; t < e; ++t) {
            const int i = conv[t];
            if (cs[i].res < cs[best].res || (cs[i].res == cs[best].res && i < best)) best = i;
        }
        reps.push_back({best, int(e - s)});
        s = e;
    }
    std::stable_sort(reps.begin(), reps.end(), [&](const auto& a, const auto& b) {
        const double da = std::fabs(cs[a.first].refined - sigma), db = std::fabs(cs[b.first].refined - sigma);
        if (da != db) return da < db;
        return cs[a.first].refined < cs[b.first].refined;
    });
    if (int(reps.size()) > k) reps.resize(k);
    std::stable_sort(reps.begin(), reps.end(),
                     [&](const auto& a, const auto& b) { return cs[a.first].refined < cs[b.first].refined; });
    return reps;
}

// device pointer of the FP64 start vector in stream order (uploaded into buf
// when given on the host, reordered into buf when the stream order is not the
// caller's)
const double* start_vector(tbh::Ham& h, const tbh_lanczos_opts* o, tbh::DevBuf& buf) {
    const size_t ns = size_t(h.dim) * (h.cplx_h ? 2 : 1);
    const size_t row = size_t(h.n_o) * (h.cplx_h ? 2 : 1) * sizeof(double);
    hipStream_t st = h.ctx->stream;
    if (!o->v0) {
        TBH_REQUIRE(o->v0_dev, "null start vector (v0 and v0_dev)");
        if (!h.permuted) return o->v0_dev;
        buf.alloc(ns * sizeof(double));
        tbh::rows_to_stream(st, h.n, h.perm_d.as<int64_t>(), row, o->v0_dev, buf.p);
        return buf.as<double>();
    }
    const double* v0 = o->v0;
    double nrm = 0.0;
    for (size_t i = 0; i < ns; ++i) nrm += v0[i] * v0[i];
    TBH_REQUIRE(nrm > 0.0 && std::isfinite(nrm), "start vector is zero or not finite");
    if (!h.permuted) {
        buf.alloc(ns * sizeof(double));
        TBH_HIP(hipMemcpyAsync(buf.p, v0, ns * sizeof(double), hipMemcpyHostToDevice, st));
        return buf.as<double>();
    }
    std::vector<double> v(ns);
    const size_t rd = row / sizeof(double);
    for (int64_t k = 0; k < h.n; ++k)
        std::memcpy(&v[size_t(k) * rd], v0 + size_t(h.perm_h[size_t(k)]) * rd, row);
    buf.alloc(ns * sizeof(double));
    TBH_HIP(hipMemcpyAsync(buf.p, v.data(), ns * sizeof(double), hipMemcpyHostToDevice, st));
    TBH_HIP(hipStreamSynchronize(st));   // v is a local
    return buf.as<double>();
}

tbh::LzWork& workspace(tbh::Ham& h) {
    if (!h.lz) h.lz = std::make_shared<tbh::LzWork>();
    return *h.lz;
}

}  // namespace

extern "C" {

int tbh_lanczos_run(tbh_ham* h, const tbh_lanczos_opts* o, double* alpha, double* beta, int32_t time_hx,
                    tbh_lanczos_report* rep) {
    return guard([&] {
        TBH_REQUIRE(h && o, "null argument");
        const int m = o->max_iter, reorth = o->reorth;
        TBH_REQUIRE(m >= 1 && m <= 100000, "max_iter must be in 1..100000");
        TBH_REQUIRE(reorth == 0 || reorth == 1, "reorth must be 0 or 1");
        TBH_HIP(hipSetDevice(h->ctx->device));
        const auto t0 = std::chrono::steady_clock::now();
        tbh::DevBuf v0d;
        const double* v0 = start_vector(*h, o, v0d);
        tbh::LzWork& W = workspace(*h);
        int steps = 0, brk = 0;
        double hx_ms = 0.0;
        tbh::lanczos_recurrence(*h, W, m, reorth != 0, v0, alpha, beta, &steps, &brk,
                                time_hx ? &hx_ms : nullptr);
        if (rep) {
            *rep = tbh_lanczos_report{};
            rep->steps = steps;
            rep->breakdown = brk;
            rep->hx_seconds = hx_ms * 1e-3;
            rep->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        }
    });
}

int tbh_lanczos_eigs(tbh_ham* h, const tbh_lanczos_opts* o, double* evals, double* refined, double* res,
                     int32_t* copies, double* evecs_dev, tbh_lanczos_report* rep) {
    int status = TBH_OK;
    const int rc = guard([&] {
        TBH_REQUIRE(h && o, "null argument");
        TBH_REQUIRE(o->k >= 1, "k must be >= 1");
        TBH_REQUIRE(o->max_iter >= 1 && o->max_iter <= 100000, "max_iter must be in 1..100000");
        TBH_REQUIRE(o->reorth == 0 || o->reorth == 1, "reorth must be 0 or 1");
        TBH_REQUIRE(h->has_f64, "refinement needs an FP64 copy of H (build with keep_f64=1)");
        TBH_HIP(hipSetDevice(h->ctx->device));
        const auto t0 = std::chrono::steady_clock::now();
        const double res_tol = o->res_tol > 0 ? o->res_tol : 1e-4;
        const double merge_tol = o->merge_tol > 0 ? o->merge_tol : 1e-6;
        tbh::DevBuf v0d;
        const double* v0 = start_vector(*h, o, v0d);
        tbh::LzWork& W = workspace(*h);
        int steps = 0, brk = 0;
        tbh::lanczos_recurrence(*h, W, o->max_iter, o->reorth != 0, v0, nullptr, nullptr, &steps, &brk,
                                nullptr, /*keep_basis=*/true);
        TBH_REQUIRE(steps >= 1, "Lanczos made no step");
        int ncand = o->n_cand > 0 ? o->n_cand : std::min(steps, std::max(4 * o->k, o->k + 16));
        ncand = std::min(ncand, steps);
        tbh::RitzOut R;
        tbh::ritz_pairs(*h, W, steps, o->sigma, ncand, R);
        std::vector<double> rr(4 * size_t(ncand));
        hipStream_t st = h->ctx->stream;
        TBH_HIP(hipMemcpyAsync(rr.data(), R.res.p, rr.size() * 8, hipMemcpyDeviceToHost, st));
        TBH_HIP(hipStreamSynchronize(st));
        std::vector<Cand> cs(ncand);
        for (int c = 0; c < ncand; ++c) cs[c] = Cand{rr[4 * c], rr[4 * c + 1], rr[4 * c + 2], rr[4 * c + 3], c};
        auto reps = select_converged(cs, o->sigma, o->k, res_tol, merge_tol);
        const int nf = int(reps.size());
        const double nan = std::numeric_limits<double>::quiet_NaN();
        double mres = 0.0;
        const size_t ns = size_t(h->dim) * (h->cplx_h ? 2 : 1);
        for (int t = 0; t < o->k; ++t) {
            if (t < nf) {
                const Cand& c = cs[reps[t].first];
                if (evals) evals[t] = c.theta;
                if (refined) refined[t] = c.refined;
                if (res) res[t] = c.res;
                if (copies) copies[t] = reps[t].second;
                mres = std::max(mres, c.res);
                if (evecs_dev) {
                    const double* y = R.Y.as<double>() + size_t(c.c) * ns;
                    if (h->permuted)
                        tbh::rows_to_caller_f64(st, h->n, h->perm_d.as<int64_t>(), h->n_o * (h->cplx_h ? 2 : 1),
                                                1.0 / c.ynorm, y, evecs_dev + size_t(t) * ns);
                    else
                        tbh::scale_copy(st, int64_t(ns), y, 1.0 / c.ynorm, evecs_dev + size_t(t) * ns);
                }
            } else {
                if (evals) evals[t] = nan;
                if (refined) refined[t] = nan;
                if (res) res[t] = nan;
                if (copies) copies[t] = 0;
                if (evecs_dev) TBH_HIP(hipMemsetAsync(evecs_dev + size_t(t) * ns, 0, ns * sizeof(double), st));
            }
        }
        TBH_HIP(hipStreamSynchronize(st));
        if (rep) {
            *rep = tbh_lanczos_report{};
            rep->steps = steps;
            rep->breakdown = brk;
            rep->n_found = nf;
            rep->n_cand = ncand;
            rep->max_res = mres;
            rep->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        }
        if (nf < o->k) status = TBH_ENOCONV;
    });
    if (rc != TBH_OK) return rc;
    if (status != TBH_OK) tbh::set_error("fewer than k eigenvalues converged");
    return status;
}

int tbh_tridiag_eig(tbh_ctx* ctx, int32_t m, const double* diag, const double* off, double* theta) {
    return guard([&] {
        TBH_REQUIRE(ctx && diag && theta, "null argument");
        TBH_REQUIRE(m >= 1 && m <= 1000000, "m out of range");
        TBH_REQUIRE(m == 1 || off, "null off-diagonal");
        TBH_HIP(hipSetDevice(ctx->device));
        tbh::DevBuf a, b, t;
        a.alloc(sizeof(double) * m);
        b.alloc(sizeof(double) * (m + 1));
        t.alloc(sizeof(double) * m);
        std::vector<double> bb(m + 1, 0.0);
        for (int i = 0; i + 1 < m; ++i) bb[i + 1] = off[i];
        TBH_HIP(hipMemcpyAsync(a.p, diag, sizeof(double) * m, hipMemcpyHostToDevice, ctx->stream));
        TBH_HIP(hipMemcpyAsync(b.p, bb.data(), sizeof(double) * (m + 1), hipMemcpyHostToDevice, ctx->stream));
        tbh::tridiag_gpu(ctx->stream, m, a.as<double>(), b.as<double>(), t.as<double>());
        TBH_HIP(hipMemcpyAsync(theta, t.p, sizeof(double) * m, hipMemcpyDeviceToHost, ctx->stream));
        TBH_HIP(hipStreamSynchronize(ctx->stream));
    });
}

}  // extern "C"
