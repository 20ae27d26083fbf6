// C ABI: the convolutional surrogate (inference, gradients, training step).
#include <cmath>
#include <vector>

#include "conv.h"
#include "tbh_internal.h"

using tbh::guard;

struct tbh_net : tbh::Net {
    using tbh::Net::Net;
};

namespace {

// canonical W[co][ci][t] (t = dz*9 + dy*3 + dx) <-> internal W[co][t][ci]
void to_internal(const tbh::Net& n, const float* in, std::vector<float>& out) {
    out.assign(n.n_params, 0.f);
    for (int l = 0; l < n.L; ++l) {
        const int ci_n = n.lin[l], co_n = n.lout[l];
        for (int co = 0; co < co_n; ++co)
            for (int ci = 0; ci < ci_n; ++ci)
                for (int t = 0; t < 27; ++t)
                    out[n.off_w[l] + (int64_t(co) * 27 + t) * ci_n + ci] =
                        in[n.off_w[l] + (int64_t(co) * ci_n + ci) * 27 + t];
        for (int co = 0; co < co_n; ++co) out[n.off_b[l] + co] = in[n.off_b[l] + co];
    }
}

void to_canonical(const tbh::Net& n, const float* in, float* out) {
    for (int l = 0; l < n.L; ++l) {
        const int ci_n = n.lin[l], co_n = n.lout[l];
        for (int co = 0; co < co_n; ++co)
            for (int ci = 0; ci < ci_n; ++ci)
                for (int t = 0; t < 27; ++t)
                    out[n.off_w[l] + (int64_t(co) * ci_n + ci) * 27 + t] =
                        in[n.off_w[l] + (int64_t(co) * 27 + t) * ci_n + ci];
        for (int co = 0; co < co_n; ++co) out[n.off_b[l] + co] = in[n.off_b[l] + co];
    }
}

}  // namespace

extern "C" {

int tbh_net_create(tbh_ctx* ctx, int32_t channels, int32_t in_channels, int32_t n_layers,
                   const int32_t* dilations, const int32_t grid[3], tbh_net** out) {
    return guard([&] {
        TBH_REQUIRE(ctx && grid && out, "null argument");
        TBH_REQUIRE(dilations || n_layers == 4, "dilations may be NULL only for 4 layers");
        TBH_REQUIRE(n_layers >= 2 && n_layers <= tbh::Net::MAX_LAYERS, "n_layers must be in 2..8");
        TBH_HIP(hipSetDevice(ctx->device));
        const int g[3] = {grid[0], grid[1], grid[2]};
        int d[tbh::Net::MAX_LAYERS] = {1, 2, 4, 1};
        if (dilations)
            for (int l = 0; l < n_layers; ++l) d[l] = dilations[l];
        auto n = std::make_unique<tbh_net>(ctx, channels, in_channels, n_layers, d, g);
        std::vector<float> z(n->n_params, 0.f);
        TBH_HIP(hipMemcpy(n->w32.p, z.data(), z.size() * 4, hipMemcpyHostToDevice));
        n->sync_half();
        tbh::retain(ctx);
        *out = n.release();
    });
}

int tbh_net_destroy(tbh_net* n) {
    return guard([&] {
        if (!n) return;
        tbh::Ctx* c = n->ctx;
        (void)hipSetDevice(c->device);
        (void)hipStreamSynchronize(c->stream);
        delete n;
        tbh::release(c);
    });
}

int tbh_net_num_params(const tbh_net* n, int64_t* count) {
    return guard([&] {
        TBH_REQUIRE(n && count, "null argument");
        *count = n->n_params;
    });
}

int tbh_net_set_params(tbh_net* n, const float* params) {
    return guard([&] {
        TBH_REQUIRE(n && params, "null argument");
        TBH_HIP(hipSetDevice(n->ctx->device));
        std::vector<float> w;
        to_internal(*n, params, w);
        TBH_HIP(hipMemcpyAsync(n->w32.p, w.data(), w.size() * 4, hipMemcpyHostToDevice, n->ctx->stream));
        n->sync_half();
        n->zero_moments();
        TBH_HIP(hipStreamSynchronize(n->ctx->stream));
    });
}

int tbh_net_get_params(tbh_net* n, float* params) {
    return guard([&] {
        TBH_REQUIRE(n && params, "null argument");
        TBH_HIP(hipSetDevice(n->ctx->device));
        std::vector<float> w(n->n_params);
        TBH_HIP(hipMemcpyAsync(w.data(), n->w32.p, w.size() * 4, hipMemcpyDeviceToHost, n->ctx->stream));
        TBH_HIP(hipStreamSynchronize(n->ctx->stream));
        to_canonical(*n, w.data(), params);
    });
}

int tbh_net_set_loss_weights(tbh_net* n, const float* w_dev) {
    return guard([&] {
        TBH_REQUIRE(n, "null argument");
        TBH_HIP(hipSetDevice(n->ctx->device));
        n->set_loss_weights(w_dev);
        TBH_HIP(hipStreamSynchronize(n->ctx->stream));
    });
}

int tbh_net_forward(tbh_net* n, const float* x_dev, float* y_dev) {
    return guard([&] {
        TBH_REQUIRE(n && x_dev && y_dev, "null argument");
        TBH_HIP(hipSetDevice(n->ctx->device));
        n->forward(x_dev, y_dev);
    });
}

int tbh_net_gradients(tbh_net* n, const float* x_dev, const float* t_dev, float* grad, double* loss) {
    return guard([&] {
        TBH_REQUIRE(n && x_dev && t_dev && grad, "null argument");
        TBH_HIP(hipSetDevice(n->ctx->device));
        n->zero_grad();
        const double l = n->accumulate_gradients(x_dev, t_dev);
        std::vector<float> g(n->n_params);
        TBH_HIP(hipMemcpyAsync(g.data(), n->grad.p, g.size() * 4, hipMemcpyDeviceToHost, n->ctx->stream));
        TBH_HIP(hipStreamSynchronize(n->ctx->stream));
        // the device accumulates the gradient of the sum of squares
        const float s = float(1.0 / double(n->nvox));
        for (auto& v : g) v *= s;
        to_canonical(*n, g.data(), grad);
        if (loss) *loss = l;
    });
}

int tbh_net_train_step(tbh_net* n, const float* const* x_dev, const float* const* t_dev, int32_t batch,
                       double lr, double* loss) {
    return guard([&] {
        TBH_REQUIRE(n && x_dev && t_dev && batch >= 1 && lr > 0, "bad arguments");
        TBH_HIP(hipSetDevice(n->ctx->device));
        n->zero_grad();
        double tot = 0.0;
        for (int b = 0; b < batch; ++b) {
            TBH_REQUIRE(x_dev[b] && t_dev[b], "null sample");
            tot += n->accumulate_gradients(x_dev[b], t_dev[b]);
        }
        // a non-finite loss or gradient (half-precision overflow) skips the update
        if (std::isfinite(tot)) (void)n->adam(lr, batch);
        if (loss) *loss = tot / batch;
    });
}

}  // extern "C"
