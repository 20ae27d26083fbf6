// C ABI: multi-vector H.X, the batched persistent launch, its HIP graph and
// the launch-configuration autotuner.
#include <chrono>
#include <cstdio>
#include <fstream>
#include <sstream>

#include "hx_multi.h"
#include "tbh_internal.h"

using tbh::guard;

struct tbh_batch {
    tbh::Ctx* ctx = nullptr;
    std::vector<tbh::Ham*> hams;   // referenced (retained) for the batch's lifetime
    int nrhs = 16, n_o = 0;
    bool cplx_h = false;
    std::vector<tbh::MvDesc> host;
    tbh::DevBuf desc;
    int64_t total = 0;
    int grid = 0, remap = 1;
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    ~tbh_batch() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (cap) (void)hipStreamDestroy(cap);
    }
    void launch(hipStream_t s) const {
        tbh::mv_launch(cplx_h, n_o, nrhs, desc.as<tbh::MvDesc>(), int(host.size()), total, grid, remap, s);
    }
    void capture() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        exec = nullptr;
        graph = nullptr;
        if (!cap) TBH_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
        TBH_HIP(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
        try {
            launch(cap);
        } catch (...) {
            hipGraph_t g = nullptr;
            (void)hipStreamEndCapture(cap, &g);
            if (g) (void)hipGraphDestroy(g);
            throw;
        }
        TBH_HIP(hipStreamEndCapture(cap, &graph));
        TBH_HIP(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
    }
    std::string key() const {
        std::ostringstream k;
        k << "mv n_o=" << n_o << " cplx=" << cplx_h << " nrhs=" << nrhs << " count=" << host.size()
          << " atoms=" << total;
        return k.str();
    }
};

namespace {

int default_grid(int device) {
    int cus = 256;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) cus = 256;
    return 8 * cus;
}

double time_ms(tbh_batch* b, int reps) {
    hipStream_t s = b->ctx->stream;
    hipEvent_t e0, e1;
    TBH_HIP(hipEventCreate(&e0));
    TBH_HIP(hipEventCreate(&e1));
    b->launch(s);  // warm
    TBH_HIP(hipEventRecord(e0, s));
    for (int r = 0; r < reps; ++r) b->launch(s);
    TBH_HIP(hipEventRecord(e1, s));
    TBH_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    TBH_HIP(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return double(ms) / reps;
}

}  // namespace

extern "C" {

int tbh_apply_h_multi(tbh_ham* h, const float* X, float* Y, int32_t nrhs) {
    return guard([&] {
        TBH_REQUIRE(h && X && Y, "null argument");
        TBH_REQUIRE(h->has_mv, "the ham has no multi-vector block copy (build with multi_vector=1)");
        TBH_REQUIRE(tbh::mv_supported(h->n_o, nrhs), "nrhs must be 16 or 32");
        TBH_REQUIRE(X != Y, "X and Y must not overlap");
        TBH_HIP(hipSetDevice(h->ctx->device));
        tbh::MvDesc d{h->mv_blocks.as<float>(), h->nbr_d.as<int32_t>(),
                      h->has_pot ? h->pot_d.as<double>() : nullptr, X, Y, 0, h->n};
        // one-entry table; rewriting it is ordered after the previous launch on the stream
        h->mv_desc.alloc(sizeof(tbh::MvDesc));
        TBH_HIP(hipMemcpyAsync(h->mv_desc.p, &d, sizeof(d), hipMemcpyHostToDevice, h->ctx->stream));
        const int grid = int(std::min<int64_t>(default_grid(h->ctx->device), h->n));
        tbh::mv_launch(h->cplx_h, h->n_o, nrhs, h->mv_desc.as<tbh::MvDesc>(), 1, h->n, grid, 1, h->ctx->stream);
    });
}

int tbh_batch_create(tbh_ctx* ctx, tbh_ham* const* hams, int32_t count, const float* const* X, float* const* Y,
                     int32_t nrhs, tbh_batch** out) {
    return guard([&] {
        TBH_REQUIRE(ctx && hams && X && Y && out, "null argument");
        TBH_REQUIRE(count >= 1, "count must be >= 1");
        TBH_HIP(hipSetDevice(ctx->device));
        auto b = std::make_unique<tbh_batch>();
        b->ctx = ctx;
        b->nrhs = nrhs;
        for (int i = 0; i < count; ++i) {
            const tbh_ham* h = hams[i];
            TBH_REQUIRE(h && X[i] && Y[i], "null ham or vector in the batch");
            TBH_REQUIRE(h->has_mv, "every ham needs the multi-vector block copy (multi_vector=1)");
            if (i == 0) {
                b->n_o = h->n_o;
                b->cplx_h = h->cplx_h;
            }
            TBH_REQUIRE(h->n_o == b->n_o && h->cplx_h == b->cplx_h,
                        "all hams of a batch need the same orbital count and complex-ness");
            b->host.push_back(tbh::MvDesc{h->mv_blocks.as<float>(), h->nbr_d.as<int32_t>(),
                                          h->has_pot ? h->pot_d.as<double>() : nullptr, X[i], Y[i], b->total,
                                          h->n});
            b->total += h->n;
        }
        TBH_REQUIRE(tbh::mv_supported(b->n_o, nrhs), "nrhs must be 16 or 32");
        b->desc.alloc(sizeof(tbh::MvDesc) * b->host.size());
        TBH_HIP(hipMemcpy(b->desc.p, b->host.data(), sizeof(tbh::MvDesc) * b->host.size(), hipMemcpyHostToDevice));
        b->grid = int(std::min<int64_t>(default_grid(ctx->device), b->total));
        b->remap = 1;
        b->capture();
        tbh::retain(ctx);
        for (int i = 0; i < count; ++i) {
            tbh::retain(hams[i]);
            b->hams.push_back(hams[i]);
        }
        *out = b.release();
    });
}

int tbh_batch_destroy(tbh_batch* b) {
    return guard([&] {
        if (!b) return;
        tbh::Ctx* c = b->ctx;
        std::vector<tbh::Ham*> hams = b->hams;
        (void)hipSetDevice(c->device);
        (void)hipStreamSynchronize(c->stream);
        delete b;
        for (tbh::Ham* h : hams) tbh::release(h);
        tbh::release(c);
    });
}

int tbh_batch_apply(tbh_batch* b) {
    return guard([&] {
        TBH_REQUIRE(b && b->exec, "null or unconfigured batch");
        TBH_HIP(hipSetDevice(b->ctx->device));
        TBH_HIP(hipGraphLaunch(b->exec, b->ctx->stream));
    });
}

int tbh_batch_apply_separate(tbh_batch* b) {
    return guard([&] {
        TBH_REQUIRE(b, "null batch");
        TBH_HIP(hipSetDevice(b->ctx->device));
        const int dg = default_grid(b->ctx->device);
        for (size_t i = 0; i < b->host.size(); ++i) {
            const int g = int(std::min<int64_t>(dg, b->host[i].n_atoms));
            tbh::mv_launch(b->cplx_h, b->n_o, b->nrhs, b->desc.as<tbh::MvDesc>() + i, 1, b->host[i].n_atoms, g, 1,
                           b->ctx->stream);
        }
    });
}

int tbh_batch_configure(tbh_batch* b, int32_t grid, int32_t remap) {
    return guard([&] {
        TBH_REQUIRE(b && grid >= 1 && remap >= 0 && remap <= 2, "bad configuration");
        TBH_HIP(hipSetDevice(b->ctx->device));
        b->grid = grid;
        b->remap = remap;
        b->capture();
    });
}

int tbh_batch_autotune(tbh_batch* b, const char* cache_path, int32_t* grid_out, int32_t* remap_out,
                       double* best_ms) {
    return guard([&] {
        TBH_REQUIRE(b, "null batch");
        TBH_HIP(hipSetDevice(b->ctx->device));
        const std::string key = b->key();
        // cache: one line per shape, "<key>|grid|remap|ms"
        std::vector<std::string> lines;
        bool found = false;
        int cg = 0, cr = 1;
        double cms = 0.0;
        if (cache_path) {
            std::ifstream in(cache_path);
            std::string line;
            while (std::getline(in, line)) {
                lines.push_back(line);
                const size_t p1 = line.find('|');
                if (p1 == std::string::npos || line.substr(0, p1) != key) continue;
                if (std::sscanf(line.c_str() + p1 + 1, "%d|%d|%lf", &cg, &cr, &cms) == 3 && cg >= 1) found = true;
            }
        }
        if (found) {
            b->grid = cg;
            b->remap = cr;
        } else {
            int cus = 256;
            (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, b->ctx->device);
            double best = 1e30;
            int bg = b->grid, br = b->remap;
            for (int per_cu : {2, 4, 8, 16, 32}) {
                for (int rm : {0, 1, 2}) {
                    b->grid = int(std::min<int64_t>(int64_t(per_cu) * cus, b->total));
                    b->remap = rm;
                    const double ms = time_ms(b, 3);
                    if (ms < best) {
                        best = ms;
                        bg = b->grid;
                        br = rm;
                    }
                }
            }
            b->grid = bg;
            b->remap = br;
            cms = best;
            if (cache_path) {
                std::ofstream o(cache_path);
                for (const auto& l : lines)
                    if (l.substr(0, l.find('|')) != key) o << l << "\n";
                o << key << "|" << bg << "|" << br << "|" << best << "\n";
            }
        }
        b->capture();
        if (grid_out) *grid_out = b->grid;
        if (remap_out) *remap_out = b->remap;
        if (best_ms) *best_ms = found ? cms : cms;
    });
}

}  // extern "C"
