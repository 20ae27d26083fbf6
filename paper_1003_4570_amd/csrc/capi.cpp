// C ABI: contexts, Hamiltonian build and H.x entry points.
#include <cstring>
#include <memory>

#include "hx_multi.h"
#include "tbh_internal.h"

namespace {
thread_local std::string g_err;
}  // namespace

namespace tbh {
void set_error(const std::string& msg) { g_err = msg; }
}  // namespace tbh

using tbh::guard;

namespace tbh {

int64_t Ham::hx_bytes() const {
    const int64_t vec = dim * (cplx_h ? 2 : 1) * (prec == TBH_F64 ? 8 : 4);
    return lay.bytes + n * 4 * 4 + 2 * vec + (has_pot ? n * 8 : 0);
}

namespace {

int choose_rows(int n_o, bool cplx_h, int prec, int64_t n_atoms, int lanes) {
    if (lanes > 0) {
        TBH_REQUIRE(lanes <= n_o && n_o % lanes == 0, "lanes_per_atom must divide the orbital count");
        const int R = n_o / lanes;
        TBH_REQUIRE(hx_shape_supported(n_o, cplx_h, R),
                    "no kernel for lanes_per_atom=" + std::to_string(lanes));
        return R;
    }
    // fewest lanes per atom (least gather redundancy) whose launch still has
    // enough wavefronts to fill 256 CUs many times over; otherwise the most
    // parallel shape available
    const int K = prec == TBH_F64 ? 2 : 4;
    int last = 0;
    for (int R : {20, 10, 5, 4, 2, 1}) {
        if (R > n_o || n_o % R || !hx_shape_supported(n_o, cplx_h, R)) continue;
        last = R;
        const int atoms_per_tile = 64 / (n_o / R);
        const int64_t tiles = (n_atoms + atoms_per_tile - 1) / atoms_per_tile;
        const bool aligned = (R * n_o * (cplx_h ? 2 : 1)) % K == 0;
        if (aligned && tiles >= 4096) return R;
    }
    TBH_REQUIRE(last > 0, "no H.x kernel shape for this orbital count");
    return last;
}

}  // namespace
}  // namespace tbh

namespace tbh {

void retain(Ctx* c) { c->refs.fetch_add(1); }

void release(Ctx* c) {
    if (c->refs.fetch_sub(1) != 1) return;
    (void)hipSetDevice(c->device);
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    delete static_cast<tbh_ctx*>(c);
}

void retain(Ham* h) { h->refs.fetch_add(1); }

void release(Ham* h) {
    if (h->refs.fetch_sub(1) != 1) return;
    Ctx* c = h->ctx;
    (void)hipSetDevice(c->device);
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    else (void)hipDeviceSynchronize();
    delete static_cast<tbh_ham*>(h);
    release(c);
}

}  // namespace tbh

namespace {

// y = H x with x, y in the caller's atom order: straight through when the
// stream order is the caller's, else through stream-order staging vectors
void apply_in_caller_order(tbh::Ham& h, const void* blocks, const tbh::Layout& lay, bool f64, const void* x,
                           void* y) {
    tbh::HxArgs a;
    a.blocks = blocks;
    a.nbr = h.nbr_d.as<int32_t>();
    a.keys = h.keys_d.as<uint8_t>();
    a.pot = h.has_pot ? h.pot_d.as<double>() : nullptr;
    a.n_atoms = h.n;
    hipStream_t st = h.ctx->stream;
    if (!h.permuted) {
        a.x = x;
        a.y = y;
        tbh::hx_launch(lay, f64, a, st);
        return;
    }
    const size_t row = size_t(h.n_o) * (h.cplx_h ? 2 : 1) * (f64 ? 8 : 4);
    h.xs.alloc(row * size_t(h.n));
    h.ys.alloc(row * size_t(h.n));
    tbh::rows_to_stream(st, h.n, h.perm_d.as<int64_t>(), row, x, h.xs.p);
    a.x = h.xs.p;
    a.y = h.ys.p;
    tbh::hx_launch(lay, f64, a, st);
    tbh::rows_to_caller(st, h.n, h.perm_d.as<int64_t>(), row, h.ys.p, y);
}

}  // namespace

extern "C" {

int tbh_version(void) { return 100; }

const char* tbh_last_error(void) { return g_err.c_str(); }

int tbh_ctx_create(int device, void* stream, tbh_ctx** out) {
    return guard([&] {
        TBH_REQUIRE(out, "null output pointer");
        int n = 0;
        TBH_HIP(hipGetDeviceCount(&n));
        TBH_REQUIRE(device >= 0 && device < n, "device index out of range");
        TBH_HIP(hipSetDevice(device));
        tbh::noalloc_setup(device);   // scratch address of the allocation-free entry point
        auto c = std::make_unique<tbh_ctx>();
        c->device = device;
        c->stream = static_cast<hipStream_t>(stream);
        *out = c.release();
    });
}

int tbh_ctx_destroy(tbh_ctx* c) {
    return guard([&] {
        if (!c) return;
        tbh::release(c);
    });
}

int tbh_ctx_set_stream(tbh_ctx* c, void* stream) {
    return guard([&] {
        TBH_REQUIRE(c, "null context");
        c->stream = static_cast<hipStream_t>(stream);
    });
}

int tbh_build_blocks_host(const tbh_geometry* g, const tbh_params* p, const tbh_build_opts* o,
                          int32_t* nbr, int8_t* wrap, double* onsite, double* bonds,
                          int32_t* is_complex) {
    return guard([&] {
        tbh::HostModel M;
        tbh::host_prepare(g, p, o, M);
        if (nbr) std::memcpy(nbr, M.nbr.data(), M.nbr.size() * 4);
        if (wrap) std::memcpy(wrap, M.wrap.data(), M.wrap.size());
        if (is_complex) *is_complex = M.cplx_h;
        if (!onsite && !bonds) return;
        const int no = M.n_o;
        std::vector<tbh::cplx> D(no * no), B(4 * no * no);
        const int cs = M.cplx_h ? 2 : 1;
        for (int64_t i = 0; i < M.n; ++i) {
            tbh::host_atom_blocks(M, i, D.data(), B.data());
            if (onsite)
                for (int k = 0; k < no * no; ++k) {
                    onsite[(i * no * no + k) * cs] = D[k].real();
                    if (cs == 2) onsite[(i * no * no + k) * cs + 1] = D[k].imag();
                }
            if (bonds)
                for (int k = 0; k < 4 * no * no; ++k) {
                    bonds[(i * 4 * no * no + k) * cs] = B[k].real();
                    if (cs == 2) bonds[(i * 4 * no * no + k) * cs + 1] = B[k].imag();
                }
        }
    });
}

int tbh_tabulate_host(const tbh_geometry* g, const tbh_params* p, const tbh_build_opts* o, double* table,
                      int64_t table_cap, int32_t* n_blocks, uint8_t* keys) {
    return guard([&] {
        TBH_REQUIRE(n_blocks, "null output pointer");
        tbh::HostModel M;
        tbh::host_prepare(g, p, o, M);
        std::vector<double> t;
        std::vector<uint8_t> k;
        int nu = 0;
        tbh::tabulate(M, nullptr, t, nu, k);
        *n_blocks = nu;
        if (table) {
            TBH_REQUIRE(table_cap >= int64_t(t.size()), "table capacity too small");
            std::memcpy(table, t.data(), t.size() * sizeof(double));
        }
        if (keys) std::memcpy(keys, k.data(), k.size());
    });
}

int tbh_build_hamiltonian(tbh_ctx* ctx, const tbh_geometry* g, const tbh_params* p,
                          const tbh_build_opts* o, tbh_ham** out) {
    return guard([&] {
        TBH_REQUIRE(ctx && out, "null context or output pointer");
        TBH_HIP(hipSetDevice(ctx->device));
        tbh::HostModel M;
        tbh::host_prepare(g, p, o, M);
        auto h = std::make_unique<tbh_ham>();
        h->ctx = ctx;
        h->n = M.n;
        h->n_o = M.n_o;
        h->n_base = M.n_base;
        h->dim = M.n * M.n_o;
        h->cplx_h = M.cplx_h;
        h->spin = M.spin;
        h->prec = o->prec;
        h->n_dangling = M.n_dangling;
        h->nbr_h = M.nbr;
        h->wrap_h = M.wrap;
        h->pos_h.assign(g->pos_q, g->pos_q + 3 * g->n_atoms);
        // stream order (the multi-vector copy, built for many small cells,
        // keeps the caller's order and so does every ham that has one)
        if (!o->multi_vector) h->perm_h = tbh::locality_order(g->pos_q, M.n);
        h->permuted = !h->perm_h.empty();
        const int64_t* perm = h->permuted ? h->perm_h.data() : nullptr;
        if (h->permuted) {
            h->perm_d.alloc(h->perm_h.size() * 8);
            TBH_HIP(hipMemcpy(h->perm_d.p, h->perm_h.data(), h->perm_h.size() * 8, hipMemcpyHostToDevice));
        }
        // diagonal on-site blocks need no spin-orbit, no passivation
        h->diag = !M.spin && !(M.par.passivation_eV != 0.0 && M.n_dangling > 0);
        // The build-time potential is the ham's per-atom potential in every
        // storage format: it stays out of the packed blocks and the kernels
        // add pot[i] x_i, so tbh_ham_set_potential replaces it (NULL = 0).
        std::vector<double> pot0;
        pot0.swap(M.pot);
        TBH_REQUIRE(!(o->tabulated && o->spin_diagonal), "tabulated and spin_diagonal exclude each other");
        if (o->tabulated) {
            TBH_REQUIRE(!o->multi_vector, "tabulated blocks do not combine with multi_vector");
            TBH_REQUIRE(o->lanes_per_atom == 0 || o->lanes_per_atom == 1, "tabulated blocks use one lane per atom");
            TBH_REQUIRE(M.n_o == 5 || M.n_o == 10, "tabulated blocks need 5 or 10 orbitals per atom");
            std::vector<double> table;
            std::vector<uint8_t> keys;
            int nu = 0;
            tbh::tabulate(M, perm, table, nu, keys);
            auto tab_layout = [&](int prec) {
                tbh::Layout L;
                L.tab = true;
                L.n_o = M.n_o;
                L.R = M.n_o;
                L.G = 1;
                L.A = 64;
                L.L = 64;
                L.cs = 1;
                L.esz = prec == TBH_F64 ? 8 : 4;
                L.K = 16 / L.esz;
                L.diag = true;
                L.n_tiles = (M.n + 63) / 64;
                L.nu = nu;
                L.ns = int(M.onsite_par.size() / 4);
                L.bytes = int64_t(table.size()) * L.esz + int64_t(keys.size());
                TBH_REQUIRE(int64_t(table.size()) * L.esz <= 49152, "block table larger than 48 KB");
                tbh::hx_tab_configure(L);
                return L;
            };
            auto upload = [&](tbh::DevBuf& dst, int prec) {
                if (prec == TBH_F64) {
                    dst.alloc(table.size() * 8);
                    TBH_HIP(hipMemcpy(dst.p, table.data(), table.size() * 8, hipMemcpyHostToDevice));
                } else {
                    std::vector<float> t32(table.begin(), table.end());
                    dst.alloc(t32.size() * 4);
                    TBH_HIP(hipMemcpy(dst.p, t32.data(), t32.size() * 4, hipMemcpyHostToDevice));
                }
            };
            h->lay = tab_layout(o->prec);
            upload(h->blocks, o->prec);
            h->keys_d.alloc(keys.size());
            TBH_HIP(hipMemcpy(h->keys_d.p, keys.data(), keys.size(), hipMemcpyHostToDevice));
            if (o->prec == TBH_F32 && o->keep_f64) {
                h->lay64 = tab_layout(TBH_F64);
                upload(h->blocks64, TBH_F64);
                h->has_f64 = true;
            } else if (o->prec == TBH_F64) {
                h->has_f64 = true;
            }
        } else if (o->spin_diagonal) {
            TBH_REQUIRE(M.spin, "spin_diagonal needs a model with spin");
            TBH_REQUIRE(!o->kfrac || (o->kfrac[0] == 0.0 && o->kfrac[1] == 0.0 && o->kfrac[2] == 0.0),
                        "spin_diagonal needs Gamma (a Bloch phase makes the bond blocks complex)");
            TBH_REQUIRE(o->lanes_per_atom == 0, "spin_diagonal chooses its own lanes per atom");
            // lanes own R orbitals in both spins: 2 of 10 (sp3d5s*) or 1 of 5 (sp3s*)
            const int R = M.n_o == 20 ? 2 : 1;
            h->lay = tbh::make_layout_sd(M.n, M.n_o, o->prec, R);
            {
                std::vector<char> host(size_t(h->lay.bytes));
                tbh::pack_layout(M, h->lay, false, host.data(), perm);
                h->blocks.alloc(host.size());
                TBH_HIP(hipMemcpy(h->blocks.p, host.data(), host.size(), hipMemcpyHostToDevice));
            }
            if (o->prec == TBH_F32 && o->keep_f64) {
                h->lay64 = tbh::make_layout_sd(M.n, M.n_o, TBH_F64, R);
                std::vector<char> host(size_t(h->lay64.bytes));
                tbh::pack_layout(M, h->lay64, false, host.data(), perm);
                h->blocks64.alloc(host.size());
                TBH_HIP(hipMemcpy(h->blocks64.p, host.data(), host.size(), hipMemcpyHostToDevice));
                h->has_f64 = true;
            } else if (o->prec == TBH_F64) {
                h->has_f64 = true;
            }
        } else {
            const int R = tbh::choose_rows(M.n_o, M.cplx_h, o->prec, M.n, o->lanes_per_atom);
            h->lay = tbh::make_layout(M.n, M.n_o, M.cplx_h, o->prec, R, h->diag);
            {
                std::vector<char> host(size_t(h->lay.bytes));
                tbh::pack_layout(M, h->lay, h->diag, host.data(), perm);
                h->blocks.alloc(host.size());
                TBH_HIP(hipMemcpy(h->blocks.p, host.data(), host.size(), hipMemcpyHostToDevice));
            }
            if (o->prec == TBH_F32 && o->keep_f64) {
                h->lay64 = tbh::make_layout(M.n, M.n_o, M.cplx_h, TBH_F64, R, h->diag);
                std::vector<char> host(size_t(h->lay64.bytes));
                tbh::pack_layout(M, h->lay64, h->diag, host.data(), perm);
                h->blocks64.alloc(host.size());
                TBH_HIP(hipMemcpy(h->blocks64.p, host.data(), host.size(), hipMemcpyHostToDevice));
                h->has_f64 = true;
            } else if (o->prec == TBH_F64) {
                h->has_f64 = true;
            }
        }
        if (o->multi_vector) {
            TBH_REQUIRE(o->prec == TBH_F32, "multi_vector needs TBH_F32");
            const int64_t stride = tbh::mv_block_floats(M.n_o, M.cplx_h);
            std::vector<float> host(size_t(stride) * M.n);
            tbh::pack_atom_major(M, stride, host.data());
            h->mv_blocks.alloc(host.size() * 4);
            TBH_HIP(hipMemcpy(h->mv_blocks.p, host.data(), host.size() * 4, hipMemcpyHostToDevice));
            h->has_mv = true;
        }
        if (!pot0.empty()) {
            std::vector<double> pot(size_t(M.n));
            for (int64_t k = 0; k < M.n; ++k) pot[size_t(k)] = pot0[size_t(perm ? perm[k] : k)];
            h->pot_d.alloc(pot.size() * 8);
            TBH_HIP(hipMemcpy(h->pot_d.p, pot.data(), pot.size() * 8, hipMemcpyHostToDevice));
            h->has_pot = true;
        }
        h->nbr_d.alloc(M.nbr.size() * 4);
        if (h->permuted) {
            // neighbour table in stream order: slot k's neighbours, renumbered
            std::vector<int64_t> inv(static_cast<size_t>(M.n));
            for (int64_t k = 0; k < M.n; ++k) inv[size_t(perm[k])] = k;
            std::vector<int32_t> nb(M.nbr.size());
            for (int64_t k = 0; k < M.n; ++k)
                for (int b = 0; b < 4; ++b) {
                    const int32_t j = M.nbr[size_t(perm[k]) * 4 + b];
                    nb[size_t(k) * 4 + b] = j >= 0 ? int32_t(inv[size_t(j)]) : -1;
                }
            TBH_HIP(hipMemcpy(h->nbr_d.p, nb.data(), nb.size() * 4, hipMemcpyHostToDevice));
        } else {
            TBH_HIP(hipMemcpy(h->nbr_d.p, M.nbr.data(), M.nbr.size() * 4, hipMemcpyHostToDevice));
        }
        tbh::retain(ctx);
        *out = h.release();
    });
}

int tbh_ham_destroy(tbh_ham* h) {
    return guard([&] {
        if (!h) return;
        tbh::release(h);
    });
}

int tbh_ham_info_get(const tbh_ham* h, tbh_ham_info* out) {
    return guard([&] {
        TBH_REQUIRE(h && out, "null argument");
        out->n_atoms = h->n;
        out->dim = h->dim;
        out->n_orb = h->n_o;
        out->is_complex = h->cplx_h;
        out->prec = h->prec;
        out->lanes_per_atom = h->lay.G;
        out->onsite_diagonal = h->diag;
        out->has_f64 = h->has_f64;
        out->n_dangling = h->n_dangling;
        out->stored_bytes = h->lay.bytes;
        out->hx_bytes = h->hx_bytes();
        out->tabulated = h->lay.tab;
        out->spin_diagonal = h->lay.sd;
    });
}

int tbh_ham_neighbours(const tbh_ham* h, int32_t* nbr, int8_t* wrap) {
    return guard([&] {
        TBH_REQUIRE(h, "null ham");
        if (nbr) std::memcpy(nbr, h->nbr_h.data(), h->nbr_h.size() * 4);
        if (wrap) std::memcpy(wrap, h->wrap_h.data(), h->wrap_h.size());
    });
}

int tbh_ham_set_potential(tbh_ham* h, const double* pot_dev) {
    return guard([&] {
        TBH_REQUIRE(h, "null ham");
        TBH_HIP(hipSetDevice(h->ctx->device));
        if (!pot_dev) {
            h->has_pot = false;
            return;
        }
        h->pot_d.alloc(size_t(h->n) * 8);
        if (h->permuted)
            tbh::rows_to_stream(h->ctx->stream, h->n, h->perm_d.as<int64_t>(), 8, pot_dev, h->pot_d.p);
        else
            TBH_HIP(hipMemcpyAsync(h->pot_d.p, pot_dev, size_t(h->n) * 8, hipMemcpyDeviceToDevice,
                                   h->ctx->stream));
        h->has_pot = true;
    });
}

int tbh_apply_h(tbh_ham* h, const void* x, void* y, int32_t nrhs) {
    return guard([&] {
        TBH_REQUIRE(h && x && y, "null argument");
        TBH_REQUIRE(nrhs == 1, "tbh_apply_h: nrhs must be 1 (multi-vector form: tbh_apply_h_multi)");
        TBH_REQUIRE(x != y, "x and y must not overlap");
        TBH_REQUIRE((reinterpret_cast<uintptr_t>(x) | reinterpret_cast<uintptr_t>(y)) % 16 == 0,
                    "x and y must be 16-byte aligned");
        TBH_HIP(hipSetDevice(h->ctx->device));
        apply_in_caller_order(*h, h->blocks.p, h->lay, h->prec == TBH_F64, x, y);
    });
}

int tbh_apply_h_f64(tbh_ham* h, const double* x, double* y) {
    return guard([&] {
        TBH_REQUIRE(h && x && y, "null argument");
        TBH_REQUIRE(h->has_f64, "no FP64 copy of H (build with keep_f64=1)");
        TBH_REQUIRE(x != y, "x and y must not overlap");
        TBH_REQUIRE((reinterpret_cast<uintptr_t>(x) | reinterpret_cast<uintptr_t>(y)) % 16 == 0,
                    "x and y must be 16-byte aligned");
        TBH_HIP(hipSetDevice(h->ctx->device));
        const bool main64 = h->prec == TBH_F64;
        apply_in_caller_order(*h, main64 ? h->blocks.p : h->blocks64.p, main64 ? h->lay : h->lay64, true, x, y);
    });
}

}  // extern "C"
