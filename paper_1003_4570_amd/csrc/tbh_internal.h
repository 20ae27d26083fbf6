// Internal declarations shared by the host builder, the kernels and the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <complex>
#include <memory>
#include <cstdint>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/tbh.h"

namespace tbh {

using cplx = std::complex<double>;

// An error that crosses back to the C ABI as a status code + message.
struct Error : std::runtime_error {
    int code;
    Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define TBH_HIP(call)                                                              \
    do {                                                                           \
        hipError_t e_ = (call);                                                    \
        if (e_ != hipSuccess)                                                      \
            throw ::tbh::Error(TBH_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

#define TBH_REQUIRE(cond, msg)                                                     \
    do {                                                                           \
        if (!(cond)) throw ::tbh::Error(TBH_EINVAL, msg);                         \
    } while (0)

// Device buffer owned by the library.
struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    ~DevBuf() { release(); }
    void alloc(size_t n) {
        if (n <= bytes && p) return;
        release();
        if (n == 0) return;
        if (hipMalloc(&p, n) != hipSuccess) {
            p = nullptr;
            (void)hipGetLastError();   // clear the error so later status checks do not see it
            throw Error(TBH_ENOMEM, "hipMalloc of " + std::to_string(n) + " bytes failed");
        }
        bytes = n;
    }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    template <typename T> T* as() const { return static_cast<T*>(p); }
};

// ---------------------------------------------------------------------------
// host model builder
// ---------------------------------------------------------------------------
struct HostModel {
    int64_t n = 0;
    int n_base = 0, n_o = 0;
    bool spin = false, cplx_h = false;
    std::vector<int32_t> nbr;     // [n][4]
    std::vector<int8_t> wrap;     // [n][4][3]
    std::vector<uint8_t> sub;     // 0 = A, 1 = B
    int64_t n_dangling = 0;
    // inputs kept for block assembly
    tbh_params par{};
    std::vector<double> onsite_par, sk_par, so_par;
    std::vector<uint8_t> species;
    std::vector<double> bond_scale;   // [n][4] or empty
    std::vector<double> pot;          // [n] or empty
    double kfrac[3] = {0, 0, 0};
};

// Validate inputs, find neighbours.  Throws Error on invalid geometry.
void host_prepare(const tbh_geometry* g, const tbh_params* p, const tbh_build_opts* o,
                  HostModel& m);
// Assemble the FP64 blocks of atom i: onsite [n_o*n_o], bonds [4][n_o*n_o].
void host_atom_blocks(const HostModel& m, int64_t i, cplx* onsite, cplx* bonds);
// Slater-Koster two-centre block (n_base x n_base, row-major) for the unit
// direction (l, m, n) with the 14 canonical integrals V.
void sk_block_closed_form(int model, const double* V, double l, double m, double n, double* out);

// ---------------------------------------------------------------------------
// packed layout streamed by the H.x kernels
//
// Each lane of a 64-wide wavefront owns R consecutive rows of one atom;
// G = n_o / R lanes share an atom and a tile holds A = 64 / G atoms
// (L = A * G active lanes).  A lane's private stream is: for each bond slot
// b, its R rows of B_ib (R * n_o elements, padded to whole 16-byte chunks),
// then its R rows of the on-site block (dense) or its R diagonal entries
// (diagonal).  Streams are interleaved chunk-major across the tile's lanes
// so that every chunk of a wavefront is one contiguous L*16-byte read:
//   byte offset of (tile t, chunk c, lane l) = ((t * C + c) * L + l) * 16.
// ---------------------------------------------------------------------------
struct Layout {
    int n_o = 0, R = 0, G = 0, A = 0, L = 0;
    int cs = 1;            // scalars per element (2 for complex)
    int esz = 4;           // bytes per scalar
    int K = 4;             // scalars per 16-byte chunk
    int bond_chunks = 0;   // chunks per bond segment
    int onsite_chunks = 0; // chunks of the on-site segment
    int C = 0;             // chunks per lane
    bool diag = false;
    int64_t n_tiles = 0;
    int64_t bytes = 0;
    // tabulated bond blocks: table of nu blocks [nu][n_o][n_o] followed by
    // the on-site diagonals [ns][n_o]; 8-byte key record per atom
    bool tab = false;
    int nu = 0, ns = 0;
    // blocks of the tabulated launch (at most those resident on the device;
    // hx_tab_configure)
    int64_t tab_grid = 0;
    // spin-diagonal bonds (tbh_build_opts.spin_diagonal): a lane owns R of the
    // n_o / 2 orbitals in both spins; its stream holds, per bond, its R rows
    // of the real n_o/2 x n_o/2 block, then its 2R complex rows of the
    // on-site block (spin up rows, then spin down)
    bool sd = false;
};
Layout make_layout(int64_t n_atoms, int n_o, bool cplx_h, int prec, int R, bool diag);
Layout make_layout_sd(int64_t n_atoms, int n_o, int prec, int R);
// Pack atoms into the layout (T = float or double); slot k of the stream
// holds caller atom perm[k] (perm null: k).
void pack_layout(const HostModel& m, const Layout& lay, bool diag, void* dst, const int64_t* perm = nullptr);
// Stream order of the atoms: by row of conventional cells (z, y), then
// diamond basis class (position mod 4), then x, stable.  Returns perm
// (stream slot -> caller atom), or an empty vector when the caller's order
// already is that order.
std::vector<int64_t> locality_order(const int32_t* pos_q, int64_t n);
// Tabulated bond blocks (see tbh_build_opts.tabulated): fills table
// [nu][n_o][n_o] + on-site diagonals [ns][n_o] (FP64) and the key records
// [n][8] in stream order (perm: stream slot -> caller atom, null = identity):
// bytes 0..3 the table index of bond slots 0..3 (255 = dangling), byte 4 the
// atom's species.  The atoms' on-site blocks are taken without M.pot.
// Throws TBH_EINVAL when the blocks are not determined by the key.
void tabulate(const HostModel& m, const int64_t* perm, std::vector<double>& table, int& nu,
              std::vector<uint8_t>& keys);
// Atom-major FP32 copy for the multi-vector kernels: per atom [5][n_o][n_o]
// (bond slots 0..3, on-site), complex interleaved, padded to stride floats.
void pack_atom_major(const HostModel& m, int64_t stride, float* dst);

// ---------------------------------------------------------------------------
// the Hamiltonian object
// ---------------------------------------------------------------------------
struct Ctx;
struct LzWork;
struct BlWork;
struct FsWork;
struct Ham {
    Ctx* ctx = nullptr;
    int64_t n = 0, dim = 0;
    int n_o = 0, n_base = 0;
    bool cplx_h = false, spin = false;
    int prec = TBH_F32;
    bool diag = false;
    int64_t n_dangling = 0;
    Layout lay, lay64;
    DevBuf blocks, blocks64, nbr_d, pot_d, mv_blocks, mv_desc, keys_d;
    bool has_f64 = false, has_pot = false, has_mv = false;
    std::vector<int32_t> nbr_h;
    std::vector<int8_t> wrap_h;
    std::vector<int32_t> pos_h;   // [n][3] positions (a/4 units)
    std::shared_ptr<LzWork> lz;   // Lanczos workspace kept between calls
    std::shared_ptr<BlWork> bl;   // block Lanczos workspace kept between calls
    std::shared_ptr<FsWork> fs;   // filtered-subspace block kept between calls (warm starts)
    // The packed stream, nbr_d, pot_d and every vector inside the library
    // (Lanczos basis, SCF states) use the stream order; the caller's atom
    // order is restored at the boundary (tbh_apply_h*, start vectors, Ritz
    // vectors, potentials).  perm_h: stream slot -> caller atom.
    bool permuted = false;
    std::vector<int64_t> perm_h;
    DevBuf perm_d, xs, ys;        // device perm; staging vectors of tbh_apply_h*
    int64_t caller(int64_t k) const { return permuted ? perm_h[size_t(k)] : k; }
    int64_t hx_bytes() const;
    std::atomic<int> refs{1};
};

// ---------------------------------------------------------------------------
// caller order <-> stream order (order.hip)
// ---------------------------------------------------------------------------
// dst[k] = src[perm[k]] for rows of row_bytes (a multiple of 4)
void rows_to_stream(hipStream_t st, int64_t n, const int64_t* perm_d, size_t row_bytes, const void* src,
                    void* dst);
// dst[perm[k]] = scale * src[k] for rows of row_doubles FP64 values
void rows_to_caller_f64(hipStream_t st, int64_t n, const int64_t* perm_d, int row_doubles, double scale,
                        const double* src, double* dst);
// dst[perm[k]] = src[k] for rows of row_bytes (a multiple of 4)
void rows_to_caller(hipStream_t st, int64_t n, const int64_t* perm_d, size_t row_bytes, const void* src,
                    void* dst);

struct Ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    DevBuf partial, scal;  // reduction scratch
    std::atomic<int> refs{1};   // the caller's handle plus one per object built on it
};

// Reference counts: a ham, net or batch keeps its context alive, and an SCF
// loop or batch keeps its hams alive, until it is destroyed itself, so the
// handles can be destroyed in any order.  release() frees the object (after
// synchronising its stream) when the last reference goes.
void retain(Ctx* c);
void release(Ctx* c);
void retain(Ham* h);
void release(Ham* h);

// ---------------------------------------------------------------------------
// kernel launchers (hx.hip)
// ---------------------------------------------------------------------------
struct HxArgs {
    const void* blocks = nullptr;
    const int32_t* nbr = nullptr;
    const void* x = nullptr;
    void* y = nullptr;
    const double* pot = nullptr;     // per-atom potential (FP64) or null
    int64_t n_atoms = 0;
    // Lanczos epilogue: y = H x - beta * xprev; partials of Re(x^H y), |y|^2
    const void* xprev = nullptr;
    const double* beta = nullptr;    // device scalar (null: 0)
    double* partial = nullptr;       // [n_blocks][2] or null
    const uint8_t* keys = nullptr;   // tabulated layout: key records [n][8]
};
// Partial-sum slots a fused launch of the layout writes (one per wavefront).
int64_t hx_num_blocks(const Layout& lay);
// Sizes the tabulated launch to the blocks resident on the current device.
void hx_tab_configure(Layout& lay);
bool hx_shape_supported(int n_o, bool cplx_h, int R);
void hx_launch(const Layout& lay, bool f64, const HxArgs& a, hipStream_t s);

// error slot shared by every C ABI translation unit (thread-local)
void set_error(const std::string& msg);
// allocation-free entry points: look up this device's scratch address once
// (the device must be current); the address, or null before set-up
void noalloc_setup(int device);
double* noalloc_scratch(int device);

// Run f, translating exceptions into a status code and the error message.
template <typename F>
int guard(F&& f) {
    try {
        f();
        set_error("");
        return TBH_OK;
    } catch (const Error& e) {
        set_error(e.what());
        return e.code;
    } catch (const std::bad_alloc&) {
        set_error("host allocation failed");
        return TBH_ENOMEM;
    } catch (const std::exception& e) {
        set_error(e.what());
        return TBH_EINVAL;
    }
}

}  // namespace tbh

struct tbh_ctx : tbh::Ctx {};
struct tbh_ham : tbh::Ham {};
