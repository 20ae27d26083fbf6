// Schrodinger-Poisson self-consistency on the GPU (Sec. III-A):
// eigenstates (Lanczos) -> charge from filling the states, with the Fermi
// level from charge neutrality or given -> finite-difference Poisson solved
// by FP64 conjugate gradients -> the potential updates the Hamiltonian ->
// repeat until self-consistent.
//
// Grid: the a/4 lattice nodes, [nz][ny][nx], periodic in x and y, phi = 0 on
// the ghost planes z = -1 and z = nz; atom (qx, qy, qz) sits on node
// (qx, qy, qz).  -eps0 eps_r Lap_h phi = rho; electron potential energy
// U = -phi (eV).  Donors are +e point charges on their atoms' nodes.
//
// The grid (a quarter of a million nodes for the 30,720-atom slab, 2 MB in
// FP64) lives in the L2/Infinity Cache, so CG is latency-bound: one stencil
// kernel with the fused p.Ap partial sums, one update kernel with the fused
// r.r partial sums, and single-block scalar kernels; no host round trip per
// iteration.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <limits>

#include "conv.h"
#include "lanczos.h"
#include "scf.h"

#include "tbh_internal.h"

namespace tbh {

namespace {

constexpr int TPB = 256;
constexpr double EPS0_E_PER_V_NM = 8.8541878128e-12 / 1.602176634e-19 * 1e-9;
constexpr double KB_EV = 8.617333262e-5;

__device__ __forceinline__ double warp_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// block sum of one double; valid in thread 0
__device__ double block_sum1(double v) {
    __shared__ double sh[4];
    v = warp_sum(v);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    double r = (sh[0] + sh[1]) + (sh[2] + sh[3]);
    __syncthreads();
    return r;
}

__device__ double block_max1(double v) {
    __shared__ double sh[4];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    double r = fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]));
    __syncthreads();
    return r;
}

__device__ double block_min1(double v) { return -block_max1(-v); }

__device__ double reduce_part(const double* part, int64_t n) {
    double v = 0.0;
    for (int64_t b = threadIdx.x; b < n; b += TPB) v += part[b];
    return block_sum1(v);
}

#define GRID_LOOP(i, n) \
    for (int64_t i = blockIdx.x * int64_t(TPB) + threadIdx.x; i < (n); i += int64_t(gridDim.x) * TPB)

// A p = -Lap_h p; partial sums of p . A p
__global__ void k_stencil(int nx, int ny, int nz, double inv_h2, const double* __restrict__ p,
                          double* __restrict__ Ap, double* part, const double* done) {
    if (done && *done != 0.0) return;
    const int64_t n = int64_t(nx) * ny * nz;
    double acc = 0.0;
    GRID_LOOP(i, n) {
        const int x = int(i % nx);
        const int y = int((i / nx) % ny);
        const int z = int(i / (int64_t(nx) * ny));
        const double c = p[i];
        const int64_t row = i - x, plane = i - x - int64_t(y) * nx;
        double s = p[row + (x + 1 == nx ? 0 : x + 1)] + p[row + (x == 0 ? nx - 1 : x - 1)];
        s += p[plane + int64_t(y + 1 == ny ? 0 : y + 1) * nx + x] + p[plane + int64_t(y == 0 ? ny - 1 : y - 1) * nx + x];
        if (z + 1 < nz) s += p[i + int64_t(nx) * ny];
        if (z > 0) s += p[i - int64_t(nx) * ny];
        const double a = (6.0 * c - s) * inv_h2;
        Ap[i] = a;
        acc += c * a;
    }
    if (part) {
        const double r = block_sum1(acc);
        if (threadIdx.x == 0) part[blockIdx.x] = r;
    }
}

// scalar slots of the CG state
enum { CG_RR = 0, CG_ALPHA = 1, CG_BETA = 2, CG_DONE = 3, CG_BB = 4, CG_ITERS = 5, CG_REL = 6, CG_NS = 8 };

__global__ void k_cg_alpha(const double* part, int64_t nb, double* s) {
    if (s[CG_DONE] != 0.0) return;
    const double pap = reduce_part(part, nb);
    if (threadIdx.x == 0) s[CG_ALPHA] = pap != 0.0 ? s[CG_RR] / pap : 0.0;
}

__global__ void k_cg_update(int64_t n, double* x, double* r, const double* p, const double* Ap, double* s,
                            double* part) {
    if (s[CG_DONE] != 0.0) return;
    const double a = s[CG_ALPHA];
    double acc = 0.0;
    GRID_LOOP(i, n) {
        x[i] += a * p[i];
        const double rv = r[i] - a * Ap[i];
        r[i] = rv;
        acc += rv * rv;
    }
    const double t = block_sum1(acc);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// beta, convergence; tol is relative to |b|
__global__ void k_cg_beta(const double* part, int64_t nb, double* s, double rel_tol, int max_iter) {
    if (s[CG_DONE] != 0.0) return;
    const double rr = reduce_part(part, nb);
    if (threadIdx.x != 0) return;
    s[CG_BETA] = s[CG_RR] != 0.0 ? rr / s[CG_RR] : 0.0;
    s[CG_RR] = rr;
    s[CG_ITERS] += 1.0;
    const double rel = s[CG_BB] > 0.0 ? sqrt(rr / s[CG_BB]) : 0.0;
    s[CG_REL] = rel;
    if (rel <= rel_tol || s[CG_ITERS] >= max_iter) s[CG_DONE] = 1.0;
}

__global__ void k_cg_p(int64_t n, const double* r, double* p, const double* s) {
    if (s[CG_DONE] != 0.0) return;
    const double b = s[CG_BETA];
    GRID_LOOP(i, n) p[i] = r[i] + b * p[i];
}

// r = b - A x (Ax in r on entry), p = r, partial r.r and b.b
__global__ void k_cg_init(int64_t n, const double* b, double* r, double* p, double* part) {
    double rr = 0.0, bb = 0.0;
    GRID_LOOP(i, n) {
        const double v = b[i] - r[i];
        r[i] = v;
        p[i] = v;
        rr += v * v;
        bb += b[i] * b[i];
    }
    const double t1 = block_sum1(rr);
    const double t2 = block_sum1(bb);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = t1;
        part[2 * blockIdx.x + 1] = t2;
    }
}

__global__ void k_cg_init_scalars(const double* part, int64_t nb, double* s, double rel_tol) {
    double rr = 0.0, bb = 0.0;
    for (int64_t b = threadIdx.x; b < nb; b += TPB) {
        rr += part[2 * b];
        bb += part[2 * b + 1];
    }
    rr = block_sum1(rr);
    bb = block_sum1(bb);
    if (threadIdx.x != 0) return;
    for (int k = 0; k < CG_NS; ++k) s[k] = 0.0;
    s[CG_RR] = rr;
    s[CG_BB] = bb;
    const double rel = bb > 0.0 ? sqrt(rr / bb) : 0.0;
    s[CG_REL] = rel;
    if (rel <= rel_tol) s[CG_DONE] = 1.0;
}

__global__ void k_scale(int64_t n, const double* a, double s, double* b) {
    GRID_LOOP(i, n) b[i] = s * a[i];
}

// ---------------------------------------------------------------------------
// charge
// ---------------------------------------------------------------------------

// partial <psi_c|U|psi_c> over atom blocks: part[c * nb + block]
__global__ void k_state_pot(const double* Y, int64_t ns, int n_o, int cs, int64_t n_atoms, const double* Ua,
                            double* part) {
    const int c = blockIdx.y;
    const double* y = Y + int64_t(c) * ns;
    double acc = 0.0;
    const int per = n_o * cs;
    GRID_LOOP(i, n_atoms) {
        double w = 0.0;
        for (int k = 0; k < per; ++k) {
            const double v = y[i * per + k];
            w += v * v;
        }
        acc += Ua[i] * w;
    }
    const double t = block_sum1(acc);
    if (threadIdx.x == 0) part[int64_t(c) * gridDim.x + blockIdx.x] = t;
}

__global__ void k_reduce_rows(const double* part, int64_t nb, double* out) {
    const int c = blockIdx.x;
    const double t = reduce_part(part + int64_t(c) * nb, nb);
    if (threadIdx.x == 0) out[c] = t;
}

__device__ double fermi(double E, double Ef, double kT) {
    if (kT <= 0.0) return E < Ef ? 1.0 : (E == Ef ? 0.5 : 0.0);
    const double t = (E - Ef) / kT;
    return t > 0 ? exp(-t) / (1.0 + exp(-t)) : 1.0 / (1.0 + exp(t));
}

// occupations (2 f for counted states, 0 otherwise), E_F, counts.
// res4 = [ncand][4] (theta, residual, refined, |y|); q = <y|U|y> (unnormalised)
// One wavefront: lane t owns candidates t, t + 64, ...; sums and extrema are
// reduced across the wavefront in a fixed order, so every lane holds the same
// totals and takes the same bisection steps.
__device__ __forceinline__ double wave_sum_all(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__global__ __launch_bounds__(64) void k_fermi(int ncand, const double* res4, const double* q, double res_tol,
                                              double sigma_mid, double n_elec, double kT, double ef_fixed,
                                              int use_fixed, double* occ, double* out) {
    const int t = threadIdx.x;
    double ncb = 0.0, nconv = 0.0;
    double emin = INFINITY, emax = -INFINITY;
    for (int c = t; c < ncand; c += 64) {
        const double r = res4[4 * c + 1], E = res4[4 * c + 2], yn = res4[4 * c + 3];
        const bool conv = r <= res_tol;
        const bool cb = conv && (E - q[c] / (yn * yn) > sigma_mid);
        nconv += conv;
        occ[c] = cb ? 1.0 : -1.0;
        if (cb) {
            ncb += 1.0;
            emin = fmin(emin, E);
            emax = fmax(emax, E);
        }
    }
    ncb = wave_sum_all(ncb);
    nconv = wave_sum_all(nconv);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        emin = fmin(emin, __shfl_xor(emin, off, 64));
        emax = fmax(emax, __shfl_xor(emax, off, 64));
    }
    double Ef = ef_fixed;
    if (!use_fixed && ncb > 0) {
        double lo = emin - 60 * kT - 1.0, hi = emax + 60 * kT + 1.0;
        for (int it = 0; it < 400; ++it) {
            const double mid = 0.5 * (lo + hi);
            double s = 0.0;
            for (int c = t; c < ncand; c += 64)
                if (occ[c] > 0) s += 2.0 * fermi(res4[4 * c + 2], mid, kT);
            s = wave_sum_all(s);
            if (s < n_elec) lo = mid; else hi = mid;
            if (hi - lo < 1e-13) break;
        }
        Ef = 0.5 * (lo + hi);
    }
    double tot = 0.0;
    for (int c = t; c < ncand; c += 64) {
        if (occ[c] > 0) {
            const double yn = res4[4 * c + 3];
            const double f2 = 2.0 * fermi(res4[4 * c + 2], Ef, kT);
            occ[c] = f2 / (yn * yn);
            tot += f2;
        } else {
            occ[c] = 0.0;
        }
    }
    tot = wave_sum_all(tot);
    if (t == 0) {
        out[0] = Ef;
        out[1] = ncb;
        out[2] = nconv;
        out[3] = tot;
        out[6] = ncb > 0 ? emin : 0.0;
    }
}

// electrons per atom n_i = sum_c occ_c sum_alpha |y_c(i, alpha)|^2, then
// b[node_i] -= n_i / (h^3 eps0 eps_r); b holds the donor term on entry
__global__ void k_density_rhs(const double* Y, int64_t ns, int ncand, int n_o, int cs, int64_t n_atoms,
                              const double* occ, const int64_t* node, double scale, double* b, double* n_out) {
    const int per = n_o * cs;
    GRID_LOOP(i, n_atoms) {
        double ni = 0.0;
        for (int c = 0; c < ncand; ++c) {
            const double o = occ[c];
            if (o == 0.0) continue;
            const double* y = Y + int64_t(c) * ns + i * per;
            double w = 0.0;
            for (int k = 0; k < per; ++k) w += y[k] * y[k];
            ni += o * w;
        }
        if (n_out) n_out[i] = ni;
        b[node[i]] -= ni * scale;
    }
}

// U_out = -phi; partial max |U_out - U|; U += alpha (U_out - U); partial min U
__global__ void k_mix(int64_t n, const double* phi, double* U, double alpha, double* part) {
    double mx = 0.0, mn = INFINITY;
    GRID_LOOP(i, n) {
        const double d = -phi[i] - U[i];
        mx = fmax(mx, fabs(d));
        const double u = U[i] + alpha * d;
        U[i] = u;
        mn = fmin(mn, u);
    }
    const double a = block_max1(mx);
    const double b = block_min1(mn);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = a;
        part[2 * blockIdx.x + 1] = b;
    }
}

__global__ void k_mix_reduce(const double* part, int64_t nb, double* out) {
    double mx = -INFINITY, mn = INFINITY;
    for (int64_t b = threadIdx.x; b < nb; b += TPB) {
        mx = fmax(mx, part[2 * b]);
        mn = fmin(mn, part[2 * b + 1]);
    }
    mx = block_max1(mx);
    mn = block_min1(mn);
    if (threadIdx.x == 0) {
        out[0] = mx;
        out[1] = mn;
    }
}

// partial max and min of U (reduced by k_mix_reduce into out[0], out[1])
__global__ void k_minmax(int64_t n, const double* U, double* part) {
    double mn = INFINITY, mx = -INFINITY;
    GRID_LOOP(i, n) {
        mn = fmin(mn, U[i]);
        mx = fmax(mx, U[i]);
    }
    const double a = block_max1(mx);
    const double b = block_min1(mn);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = a;
        part[2 * blockIdx.x + 1] = b;
    }
}

// partial max |U - U_ref| (reduced by k_mix_reduce into out[0])
__global__ void k_drift(int64_t n, const double* U, const double* Uref, double* part) {
    double mx = 0.0;
    GRID_LOOP(i, n) mx = fmax(mx, fabs(U[i] - Uref[i]));
    const double a = block_max1(mx);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = a;
        part[2 * blockIdx.x + 1] = 0.0;
    }
}

__global__ void k_gather_atoms(int64_t n_atoms, const int64_t* node, const double* U, double* Ua) {
    GRID_LOOP(i, n_atoms) Ua[i] = U[node[i]];
}

int64_t grid_for(int64_t n) {
    int64_t g = (n + TPB - 1) / TPB;
    return g < 1 ? 1 : (g > 4096 ? 4096 : g);
}

// the network's input maps: donor count, A mask, B mask, U_bare / feat_scale
__global__ void k_start_inputs(int64_t n, const float* dmap, const float* mask, const double* ubare,
                               double inv_fs, float* x) {
    GRID_LOOP(i, n) {
        x[i] = dmap[i];
        x[n + i] = mask[i];
        x[2 * n + i] = mask[n + i];
        x[3 * n + i] = float(ubare[i] * inv_fs);
    }
}

// out[c][z][y][x] = in[c][z][Y][X], (Y, X) the in-plane point operation op
// (0 identity, 1 (110) mirror, 2 two-fold rotation, 3 (1-10) mirror; each
// its own inverse); nx == ny for the mirrors
__global__ void k_point_op(int64_t n, int channels, int nx, int ny, int op, const float* in, float* out) {
    const int64_t total = n * channels;
    for (int64_t i = blockIdx.x * int64_t(TPB) + threadIdx.x; i < total; i += int64_t(gridDim.x) * TPB) {
        const int64_t c = i / n, v = i % n;
        const int x = int(v % nx), y = int((v / nx) % ny);
        const int64_t zb = v - (int64_t(y) * nx + x);
        int X = x, Y = y;
        if (op == 1) {
            X = y;
            Y = x;
        } else if (op == 2) {
            X = (nx - x) % nx;
            Y = (ny - y) % ny;
        } else if (op == 3) {
            X = (ny - y) % ny;
            Y = (nx - x) % nx;
        }
        out[i] = in[c * n + zb + int64_t(Y) * nx + X];
    }
}

// acc (+)= y
__global__ void k_accum(int64_t n, const float* y, float* acc, int first) {
    GRID_LOOP(i, n) acc[i] = first ? y[i] : acc[i] + y[i];
}

// U = U_bare + mean + scale * acc
__global__ void k_start_combine(int64_t n, const double* ubare, const float* mean, const float* acc, double scale,
                                double* U) {
    GRID_LOOP(i, n) {
        double u = ubare[i];
        if (mean) u += double(mean[i]);
        if (acc) u += scale * double(acc[i]);
        U[i] = u;
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// Poisson
// ---------------------------------------------------------------------------

void PoissonWork::ensure(int64_t nodes) {
    if (n == nodes && r.p) return;
    r.alloc(nodes * 8);
    p.alloc(nodes * 8);
    Ap.alloc(nodes * 8);
    part.alloc(2 * 4096 * 8);
    s.alloc(CG_NS * 8);
    n = nodes;
}

void poisson_cg_bufs(hipStream_t st, const PoissonBufs& W, const int grid[3], double h, const double* b,
                     double* x, double rel_tol, int max_iter, int* iters, double* rel_res) {
    const int nx = grid[0], ny = grid[1], nz = grid[2];
    const int64_t n = int64_t(nx) * ny * nz;
    const double inv_h2 = 1.0 / (h * h);
    const int64_t g = grid_for(n);
    double* part = W.part;
    double* s = W.s;
    // r = A x (into r), then r = b - r, p = r; every scratch value is written
    // before it is read, so nothing needs clearing between calls
    hipLaunchKernelGGL(k_stencil, dim3(g), dim3(TPB), 0, st, nx, ny, nz, inv_h2, x, W.r,
                       (double*)nullptr, (const double*)nullptr);
    hipLaunchKernelGGL(k_cg_init, dim3(g), dim3(TPB), 0, st, n, b, W.r, W.p, part);
    hipLaunchKernelGGL(k_cg_init_scalars, dim3(1), dim3(TPB), 0, st, part, g, s, rel_tol);
    double hs[CG_NS];
    const int chunk = 25;
    for (int it = 0; it < max_iter; it += chunk) {
        for (int k = 0; k < chunk; ++k) {
            hipLaunchKernelGGL(k_stencil, dim3(g), dim3(TPB), 0, st, nx, ny, nz, inv_h2, W.p, W.Ap, part,
                               s + CG_DONE);
            hipLaunchKernelGGL(k_cg_alpha, dim3(1), dim3(TPB), 0, st, part, g, s);
            hipLaunchKernelGGL(k_cg_update, dim3(g), dim3(TPB), 0, st, n, x, W.r, W.p, W.Ap, s, part);
            hipLaunchKernelGGL(k_cg_beta, dim3(1), dim3(TPB), 0, st, part, g, s, rel_tol, max_iter);
            hipLaunchKernelGGL(k_cg_p, dim3(g), dim3(TPB), 0, st, n, W.r, W.p, s);
        }
        TBH_HIP(hipMemcpyAsync(hs, s, sizeof(hs), hipMemcpyDeviceToHost, st));
        TBH_HIP(hipStreamSynchronize(st));
        if (hs[CG_DONE] != 0.0) break;
    }
    TBH_HIP(hipGetLastError());
    if (iters) *iters = int(hs[CG_ITERS]);
    if (rel_res) *rel_res = hs[CG_REL];
}

void poisson_cg(hipStream_t st, PoissonWork& W, const int grid[3], double h, const double* b, double* x,
                double rel_tol, int max_iter, int* iters, double* rel_res) {
    const int64_t n = int64_t(grid[0]) * grid[1] * grid[2];
    W.ensure(n);
    const PoissonBufs v{W.r.as<double>(), W.p.as<double>(), W.Ap.as<double>(), W.part.as<double>(),
                        W.s.as<double>()};
    poisson_cg_bufs(st, v, grid, h, b, x, rel_tol, max_iter, iters, rel_res);
}

// ---------------------------------------------------------------------------
// SCF driver
// ---------------------------------------------------------------------------

Scf::Scf(Ham* h_, const tbh_scf_opts& o) : h(h_), opt(o) {
    TBH_REQUIRE(h->has_f64, "the SCF loop needs an FP64 copy of H (build with keep_f64=1)");
    for (int a = 0; a < 3; ++a) {
        grid[a] = o.grid[a];
        TBH_REQUIRE(grid[a] > 0, "grid sizes must be positive");
    }
    TBH_REQUIRE(o.h_nm > 0 && o.eps_r > 0 && o.T_K >= 0, "h_nm, eps_r must be positive, T_K >= 0");
    TBH_REQUIRE(o.mix_alpha > 0 && o.mix_alpha <= 1, "mix_alpha must be in (0, 1]");
    TBH_REQUIRE(o.eig_mode == 0 || o.eig_mode == 1, "eig_mode must be 0 (Lanczos) or 1 (filtered block)");
    if (o.eig_mode == 0)
        TBH_REQUIRE(o.n_cand >= 1 && o.lanczos_iter >= o.n_cand, "need n_cand >= 1 and lanczos_iter >= n_cand");
    else
        TBH_REQUIRE((o.block == 16 || o.block == 32 || o.block == 64) && o.k_states >= 1 && o.k_states <= o.block &&
                        o.filter_degree >= 1 && o.filter_degree_cold >= 1 && o.filter_max_iter >= 1 &&
                        o.filter_max_iter_cold >= 0 &&
                        h->has_mv && !h->cplx_h,
                    "filtered eigen-solve: block 16/32/64, 1 <= k_states <= block, degrees and filter_max_iter >= 1, "
                    "filter_max_iter_cold >= 0, "
                    "and a real H built with multi_vector = 1");
    TBH_REQUIRE(o.update_mode == 0 || o.update_mode == 1, "update_mode must be 0 (linear mixing) or 1 (Newton)");
    if (o.update_mode == 1)
        TBH_REQUIRE(!h->cplx_h && o.newton_states >= 1 && o.newton_states <= 128 && o.newton_kT > 0 &&
                        o.anderson_depth >= 0 && o.anderson_depth <= 8 && o.newton_cg_tol > 0 &&
                        o.newton_cg_max_iter >= 1,
                    "Newton update: real H, 1 <= newton_states <= 128, newton_kT > 0, 0 <= anderson_depth <= 8, "
                    "newton_cg_tol > 0, newton_cg_max_iter >= 1");
    TBH_REQUIRE(o.n_donors >= 0 && (o.n_donors == 0 || o.donor_atoms), "bad donor list");
    TBH_REQUIRE(o.v0, "null start vector");
    n_nodes = int64_t(grid[0]) * grid[1] * grid[2];
    // atom -> node, for the atoms in the ham's stream order (per-atom data
    // inside the loop lives in that order)
    std::vector<int64_t> node(h->n);
    TBH_REQUIRE(!h->pos_h.empty(), "ham has no positions");
    std::vector<char> seen(n_nodes, 0);
    auto node_of = [&](int64_t caller_atom) {
        const int32_t* pq = &h->pos_h[3 * caller_atom];
        TBH_REQUIRE(pq[0] < grid[0] && pq[1] < grid[1] && pq[2] < grid[2], "atom outside the Poisson grid");
        return (int64_t(pq[2]) * grid[1] + pq[1]) * grid[0] + pq[0];
    };
    for (int64_t i = 0; i < h->n; ++i) {
        node[i] = node_of(h->caller(i));
        seen[node[i]] = 1;
    }
    node_d.alloc(h->n * 8);
    hipStream_t st = h->ctx->stream;
    TBH_HIP(hipMemcpy(node_d.p, node.data(), h->n * 8, hipMemcpyHostToDevice));
    // donor term of the right-hand side: +1/(h^3 eps0 eps_r) per donor at its node
    const double scale = 1.0 / (o.h_nm * o.h_nm * o.h_nm * EPS0_E_PER_V_NM * o.eps_r);
    std::vector<double> b0(n_nodes, 0.0);
    for (int d = 0; d < o.n_donors; ++d) {
        const int32_t a = o.donor_atoms[d];   // caller's atom index
        TBH_REQUIRE(a >= 0 && a < h->n, "donor atom index out of range");
        b0[node_of(a)] += scale;
    }
    b0_d.alloc(n_nodes * 8);
    TBH_HIP(hipMemcpy(b0_d.p, b0.data(), n_nodes * 8, hipMemcpyHostToDevice));
    // donor count and sublattice occupation per node (the learned start's inputs)
    {
        std::vector<float> dm(size_t(n_nodes), 0.f), mk(size_t(2 * n_nodes), 0.f);
        for (int d = 0; d < o.n_donors; ++d) dm[size_t(node_of(o.donor_atoms[d]))] += 1.f;
        for (int64_t a = 0; a < h->n; ++a) {
            const int32_t* pq = &h->pos_h[3 * a];
            const bool bsub = (pq[0] + pq[1] + pq[2]) % 4 == 3;
            mk[size_t((bsub ? n_nodes : 0) + node_of(a))] = 1.f;
        }
        dmap_d.alloc(size_t(n_nodes) * 4);
        mask_d.alloc(size_t(2 * n_nodes) * 4);
        TBH_HIP(hipMemcpy(dmap_d.p, dm.data(), dm.size() * 4, hipMemcpyHostToDevice));
        TBH_HIP(hipMemcpy(mask_d.p, mk.data(), mk.size() * 4, hipMemcpyHostToDevice));
    }
    U.alloc(n_nodes * 8);
    phi.alloc(n_nodes * 8);
    b.alloc(n_nodes * 8);
    std::vector<double> z(n_nodes, 0.0);
    TBH_HIP(hipMemcpy(U.p, z.data(), n_nodes * 8, hipMemcpyHostToDevice));
    TBH_HIP(hipMemcpy(phi.p, z.data(), n_nodes * 8, hipMemcpyHostToDevice));
    Ua.alloc(h->n * 8);
    const size_t ns = size_t(h->dim) * (h->cplx_h ? 2 : 1);
    v0.alloc(ns * 8);
    if (h->permuted) {
        const size_t rd = size_t(h->n_o) * (h->cplx_h ? 2 : 1);
        std::vector<double> v(ns);
        for (int64_t k = 0; k < h->n; ++k)
            std::memcpy(&v[size_t(k) * rd], o.v0 + size_t(h->perm_h[size_t(k)]) * rd, rd * sizeof(double));
        TBH_HIP(hipMemcpy(v0.p, v.data(), ns * 8, hipMemcpyHostToDevice));
    } else {
        TBH_HIP(hipMemcpy(v0.p, o.v0, ns * 8, hipMemcpyHostToDevice));
    }
    const int64_t nst = o.eig_mode == 1 ? o.block : o.n_cand;
    part.alloc(size_t(std::max<int64_t>(2 * 4096, nst * 4096)) * 8);
    occ.alloc(size_t(nst) * 8);
    q.alloc(size_t(nst) * 8);
    out.alloc(8 * 8);
    n_atoms_d.alloc(h->n * 8);
    (void)st;
}

void Scf::compute_ubare() {
    if (have_ubare) return;
    hipStream_t st = h->ctx->stream;
    ubare_d.alloc(size_t(n_nodes) * 8);
    DevBuf phib;
    phib.alloc(size_t(n_nodes) * 8);
    hipLaunchKernelGGL(k_scale, dim3(grid_for(n_nodes)), dim3(TPB), 0, st, n_nodes, b0_d.as<double>(), 0.0,
                       phib.as<double>());
    int it = 0;
    double rr = 0.0;
    poisson_cg(st, pw, grid, opt.h_nm, b0_d.as<double>(), phib.as<double>(), 1e-12, 100000, &it, &rr);
    TBH_REQUIRE(rr <= 1e-10, "bare-donor Poisson solve did not converge");
    hipLaunchKernelGGL(k_scale, dim3(grid_for(n_nodes)), dim3(TPB), 0, st, n_nodes, phib.as<double>(), -1.0,
                       ubare_d.as<double>());
    TBH_HIP(hipStreamSynchronize(st));
    have_ubare = true;
}

void Scf::set_start(const tbh_scf_start& sp) {
    hipStream_t st = h->ctx->stream;
    TBH_REQUIRE(sp.kind >= 0 && sp.kind <= 2, "start kind must be 0 (zero), 1 (mean) or 2 (learned)");
    TBH_REQUIRE(sp.first_res_limit >= 0, "first_res_limit must be >= 0");
    if (sp.kind == 0) {
        set_potential(nullptr);
    } else {
        TBH_REQUIRE(sp.mean_dev, "mean and learned starts need the mean map");
        compute_ubare();
        const int64_t gn = grid_for(n_nodes);
        if (sp.kind == 1) {
            hipLaunchKernelGGL(k_start_combine, dim3(gn), dim3(TPB), 0, st, n_nodes, ubare_d.as<double>(),
                               sp.mean_dev, (const float*)nullptr, 0.0, U.as<double>());
        } else {
            TBH_REQUIRE(sp.net, "the learned start needs a network");
            Net& net = *reinterpret_cast<Net*>(sp.net);
            TBH_REQUIRE(net.CI == 4 && net.g[0] == grid[0] && net.g[1] == grid[1] && net.g[2] == grid[2],
                        "the network needs 4 input channels on the loop's grid");
            TBH_REQUIRE(sp.feat_scale > 0, "feat_scale must be positive");
            TBH_REQUIRE(!sp.symmetrize || grid[0] == grid[1], "symmetrizing over the point operations needs nx = ny");
            xin_d.alloc(size_t(4 * n_nodes) * 4);
            xop_d.alloc(size_t(4 * n_nodes) * 4);
            yop_d.alloc(size_t(2 * n_nodes) * 4);
            acc_d.alloc(size_t(n_nodes) * 4);
            hipLaunchKernelGGL(k_start_inputs, dim3(gn), dim3(TPB), 0, st, n_nodes, dmap_d.as<float>(),
                               mask_d.as<float>(), ubare_d.as<double>(), 1.0 / sp.feat_scale, xin_d.as<float>());
            const int nops = sp.symmetrize ? 4 : 1;
            float* y = yop_d.as<float>();
            float* yb = y + n_nodes;
            for (int op = 0; op < nops; ++op) {
                hipLaunchKernelGGL(k_point_op, dim3(grid_for(4 * n_nodes)), dim3(TPB), 0, st, n_nodes, 4, grid[0],
                                   grid[1], op, xin_d.as<float>(), xop_d.as<float>());
                net.forward(xop_d.as<float>(), y);
                hipLaunchKernelGGL(k_point_op, dim3(gn), dim3(TPB), 0, st, n_nodes, 1, grid[0], grid[1], op, y, yb);
                hipLaunchKernelGGL(k_accum, dim3(gn), dim3(TPB), 0, st, n_nodes, yb, acc_d.as<float>(), op == 0 ? 1 : 0);
            }
            hipLaunchKernelGGL(k_start_combine, dim3(gn), dim3(TPB), 0, st, n_nodes, ubare_d.as<double>(),
                               sp.mean_dev, acc_d.as<float>(), sp.scale / nops, U.as<double>());
        }
        TBH_HIP(hipGetLastError());
        set_potential(U.as<double>());
    }
    start_kind = sp.kind;
    first_res_limit = sp.first_res_limit;
    since_start = 0;
    grow = 0;
}

void Scf::set_potential(const double* Ud) {
    hipStream_t st = h->ctx->stream;
    // null: the zero start; the loop's own buffer (a start built in place): kept as it is
    zero_start = Ud == nullptr;
    if (!Ud)
        hipLaunchKernelGGL(k_scale, dim3(grid_for(n_nodes)), dim3(TPB), 0, st, n_nodes, U.as<double>(), 0.0,
                           U.as<double>());
    else if (Ud != U.as<double>())
        TBH_HIP(hipMemcpyAsync(U.p, Ud, n_nodes * 8, hipMemcpyDeviceToDevice, st));
    // phi guess for the next Poisson solve: -U
    hipLaunchKernelGGL(k_scale, dim3(grid_for(n_nodes)), dim3(TPB), 0, st, n_nodes, U.as<double>(), -1.0,
                       phi.as<double>());
    TBH_HIP(hipGetLastError());
    // a new start: the previous step's filled states no longer locate the band
    // edge, and the Newton steps' history belongs to the old iterates
    have_prev = false;
    nw.reset();
    have_bounds = false;
    fs_reuse = false;
    last_res = 0.0;
    start_kind = 0;
    since_start = 0;
    grow = 0;
}

void Scf::step(tbh_scf_report& rep) {
    hipStream_t st = h->ctx->stream;
    const auto t0 = std::chrono::steady_clock::now();
    const int64_t ga = grid_for(h->n), gn = grid_for(n_nodes);
    double* pt = part.as<double>();
    // potential on the atoms -> H
    hipLaunchKernelGGL(k_gather_atoms, dim3(ga), dim3(TPB), 0, st, h->n, node_d.as<int64_t>(), U.as<double>(),
                       Ua.as<double>());
    h->pot_d.alloc(size_t(h->n) * 8);
    TBH_HIP(hipMemcpyAsync(h->pot_d.p, Ua.p, h->n * 8, hipMemcpyDeviceToDevice, st));
    h->has_pot = true;
    // band-edge estimates: bulk edges shifted by the extreme potential
    hipLaunchKernelGGL(k_minmax, dim3(gn), dim3(TPB), 0, st, n_nodes, U.as<double>(), pt);
    hipLaunchKernelGGL(k_mix_reduce, dim3(1), dim3(TPB), 0, st, pt, gn, out.as<double>() + 4);
    double mm[2];
    TBH_HIP(hipMemcpyAsync(mm, out.as<double>() + 4, 16, hipMemcpyDeviceToHost, st));
    TBH_HIP(hipStreamSynchronize(st));
    const double u_max = mm[0];
    // without a previous step's states, the conduction-band edge is estimated
    // as the bulk edge shifted by a low quantile of the potential over the
    // atoms (the 1st percentile): the single-node wells a start potential
    // carries at donor sites are too narrow to bind a state that deep, and the
    // plain minimum would put the eigen-solve's window far below the states
    double u_low = mm[1];
    if (!have_prev) {
        std::vector<double> ua(static_cast<size_t>(h->n));
        TBH_HIP(hipMemcpyAsync(ua.data(), Ua.p, ua.size() * 8, hipMemcpyDeviceToHost, st));
        TBH_HIP(hipStreamSynchronize(st));
        const size_t iq = size_t(0.01 * double(ua.size()));
        std::nth_element(ua.begin(), ua.begin() + iq, ua.end());
        u_low = ua[iq];
    }
    int steps = 0, ncand = 0;
    const double* Ys = nullptr;
    const double* res4 = nullptr;
    double res_tol_fill = opt.res_tol;
    double sigma = 0.0;
    if (opt.eig_mode == 0) {
        // target: just below the lowest filled state of the previous step; on
        // the first step (or if none was filled) the bulk CBM shifted by min U
        sigma = have_prev ? prev_emin - 0.05 : opt.e_cbm + u_low;
        if (!lz) lz = std::make_shared<LzWork>();
        int brk = 0;
        lanczos_recurrence(*h, *lz, opt.lanczos_iter, true, v0.as<double>(), nullptr, nullptr, &steps, &brk,
                           nullptr);
        ncand = std::min(opt.n_cand, steps);
        ritz_pairs(*h, *lz, steps, sigma, ncand, ritz);
        Ys = ritz.Y.as<double>();
        res4 = ritz.res.as<double>();
    } else {
        if (!fs) {
            fs = std::make_shared<FsWork>();
            blw = std::make_shared<BlWork>();
        }
        fs->ensure(h->dim, opt.block);
        // the bounds hold while no potential value has moved by more than their
        // 2 eV margin since they were taken (a diagonal change shifts every
        // eigenvalue by at most its largest magnitude)
        if (have_bounds) {
            hipLaunchKernelGGL(k_drift, dim3(gn), dim3(TPB), 0, st, n_nodes, U.as<double>(), U_bounds.as<double>(), pt);
            hipLaunchKernelGGL(k_mix_reduce, dim3(1), dim3(TPB), 0, st, pt, gn, out.as<double>() + 4);
            double dr[2];
            TBH_HIP(hipMemcpyAsync(dr, out.as<double>() + 4, 16, hipMemcpyDeviceToHost, st));
            TBH_HIP(hipStreamSynchronize(st));
            if (!(dr[0] <= 1.5)) have_bounds = false;
        }
        if (!have_bounds) {
            U_bounds.alloc(size_t(n_nodes) * 8);
            TBH_HIP(hipMemcpyAsync(U_bounds.p, U.p, size_t(n_nodes) * 8, hipMemcpyDeviceToDevice, st));
            spectral_bounds(*h, &emin_b, &emax_b);
            // room for the potential to change over the loop
            emin_b -= 2.0;
            emax_b += 2.0;
            have_bounds = true;
        }
        const double e_cb = have_prev ? prev_emin : opt.e_cbm + u_low;
        const double e_vb = opt.e_vbm + u_max;
        FsSolve so;
        so.s = e_vb + 0.75 * (e_cb - e_vb);
        so.emin = emin_b;
        so.emax = emax_b;
        so.degree = opt.filter_degree;
        so.degree_cold = opt.filter_degree_cold;
        so.min_iter = 1;
        // the first solve of a zero start under linear mixing needs little
        // accuracy (the next steps' tolerance follows its large residual)
        so.max_iter = (!fs_warm && zero_start && opt.update_mode == 0 && opt.filter_max_iter_cold > 0)
                          ? opt.filter_max_iter_cold
                          : opt.filter_max_iter;
        so.k = opt.k_states;
        // linear mixing moves U by a small fraction of the residual per step, so
        // early states need not be sharper than a tenth of it; a Newton step can
        // move U by the whole residual, so its states are held to a hundredth.
        // The first (cold) solve of a start stops at 0.01 eV: the next step's
        // tolerance follows from the residual it produces
        so.res_tol = fs_warm ? std::max(opt.res_tol, (opt.update_mode == 0 ? 0.1 : 0.01) * last_res)
                             : std::max(opt.res_tol, 1e-2);
        // a linear-mixing step moves U by a small fraction of the residual, so
        // the Ritz values the last solve ended with still bound the block's
        // spectrum for the filter: the Rayleigh-Ritz pass of the start block
        // is skipped
        so.reuse_ritz = fs_warm && fs_reuse && opt.update_mode == 0;
        sigma = so.s;
        steps = filtered_solve(*h, *blw, *fs, so, fs_warm, nullptr, nullptr);
        fs_warm = true;
        fs_reuse = true;
        ncand = opt.block;
        Ys = fs->states.as<double>();
        res4 = fs->res4.as<double>();
        res_tol_fill = INFINITY;   // every state of the block takes part in the filling
    }
    const auto t1 = std::chrono::steady_clock::now();
    // charge
    const size_t ns = size_t(h->dim) * (h->cplx_h ? 2 : 1);
    const int cs = h->cplx_h ? 2 : 1;
    dim3 g2(ga, ncand);
    hipLaunchKernelGGL(k_state_pot, g2, dim3(TPB), 0, st, Ys, int64_t(ns), h->n_o, cs, h->n, Ua.as<double>(), pt);
    hipLaunchKernelGGL(k_reduce_rows, dim3(ncand), dim3(TPB), 0, st, pt, ga, q.as<double>());
    const double kT = KB_EV * opt.T_K;
    const int use_fixed = std::isnan(opt.fermi_fixed) ? 0 : 1;
    hipLaunchKernelGGL(k_fermi, dim3(1), dim3(64), 0, st, ncand, res4, q.as<double>(), res_tol_fill,
                       opt.sigma_mid, double(opt.n_donors), kT, use_fixed ? opt.fermi_fixed : 0.0, use_fixed,
                       occ.as<double>(), out.as<double>());
    const double scale = 1.0 / (opt.h_nm * opt.h_nm * opt.h_nm * EPS0_E_PER_V_NM * opt.eps_r);
    TBH_HIP(hipMemcpyAsync(b.p, b0_d.p, n_nodes * 8, hipMemcpyDeviceToDevice, st));
    hipLaunchKernelGGL(k_density_rhs, dim3(ga), dim3(TPB), 0, st, Ys, int64_t(ns), ncand,
                       h->n_o, cs, h->n, occ.as<double>(), node_d.as<int64_t>(), scale, b.as<double>(),
                       n_atoms_d.as<double>());
    // Poisson: the direct solve, then conjugate gradients from it, which stop
    // at once when its residual already meets the tolerance
    int cg_it = 0;
    double cg_rel = 0.0;
    fp.setup(grid, opt.h_nm);
    fp.solve(st, b.as<double>(), phi.as<double>());
    poisson_cg(st, pw, grid, opt.h_nm, b.as<double>(), phi.as<double>(), opt.cg_tol, opt.cg_max_iter, &cg_it,
               &cg_rel);
    const auto t2 = std::chrono::steady_clock::now();
    // linear mixing (update_mode 0); the Newton update leaves U to newton_update
    hipLaunchKernelGGL(k_mix, dim3(gn), dim3(TPB), 0, st, n_nodes, phi.as<double>(), U.as<double>(),
                       opt.update_mode == 0 ? opt.mix_alpha : 0.0, pt);
    hipLaunchKernelGGL(k_mix_reduce, dim3(1), dim3(TPB), 0, st, pt, gn, out.as<double>() + 4);
    double o[8];
    TBH_HIP(hipMemcpyAsync(o, out.p, sizeof(o), hipMemcpyDeviceToHost, st));
    TBH_HIP(hipStreamSynchronize(st));
    TBH_HIP(hipGetLastError());
    // a step whose filling could not place every electron (too few states in
    // the eigen-solve's window) is not a solution, whatever its residual
    const bool neutral_ok =
        use_fixed || std::fabs(o[3] - double(opt.n_donors)) <= 1e-6 * std::max(1.0, double(opt.n_donors));
    rep.newton_cg_iters = 0;
    rep.newton_pairs = 0;
    rep.newton_seconds = 0.0;
    if (opt.update_mode == 1 && !(o[4] < opt.tol_eV && neutral_ok)) {
        const auto tn = std::chrono::steady_clock::now();
        // the filled-class states of the step (the same test as k_fermi), lowest first
        std::vector<double> r4(static_cast<size_t>(ncand) * 4), qh(static_cast<size_t>(ncand));
        TBH_HIP(hipMemcpyAsync(r4.data(), res4, r4.size() * 8, hipMemcpyDeviceToHost, st));
        TBH_HIP(hipMemcpyAsync(qh.data(), q.p, qh.size() * 8, hipMemcpyDeviceToHost, st));
        TBH_HIP(hipStreamSynchronize(st));
        std::vector<int> cb;
        for (int c = 0; c < ncand; ++c) {
            const double r = r4[size_t(4 * c + 1)], E = r4[size_t(4 * c + 2)], yn = r4[size_t(4 * c + 3)];
            if (r <= res_tol_fill && E - qh[size_t(c)] / (yn * yn) > opt.sigma_mid) cb.push_back(c);
        }
        std::stable_sort(cb.begin(), cb.end(),
                         [&](int x, int y) { return r4[size_t(4 * x + 2)] < r4[size_t(4 * y + 2)]; });
        if (int(cb.size()) > opt.newton_states) cb.resize(size_t(opt.newton_states));
        NewtonIn ni;
        ni.Y = Ys;
        ni.ns = int64_t(ns);
        ni.n_o = h->n_o;
        ni.n_atoms = h->n;
        ni.node = node_d.as<int64_t>();
        for (int a = 0; a < 3; ++a) ni.grid[a] = grid[a];
        ni.h = opt.h_nm;
        ni.kappa = scale;
        ni.b = b.as<double>();
        ni.sel = cb;
        for (int c : cb) {
            ni.E.push_back(r4[size_t(4 * c + 2)]);
            ni.inv_norm.push_back(1.0 / r4[size_t(4 * c + 3)]);
        }
        ni.Ef = o[0];
        ni.kT = opt.newton_kT;
        ni.fixed = use_fixed != 0;
        ni.cg_tol = opt.newton_cg_tol;
        ni.cg_max_iter = opt.newton_cg_max_iter;
        ni.depth = opt.anderson_depth;
        ni.pre = &fp;
        NewtonOut no;
        newton_update(st, nw, ni, U.as<double>(), &no);
        rep.newton_cg_iters = no.cg_iters;
        rep.newton_pairs = no.npairs;
        rep.newton_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - tn).count();
        // phi guess for the next Poisson solve: -U
        hipLaunchKernelGGL(k_scale, dim3(gn), dim3(TPB), 0, st, n_nodes, U.as<double>(), -1.0, phi.as<double>());
        TBH_HIP(hipGetLastError());
    }
    ++iterations;
    have_prev = o[1] > 0;
    prev_emin = o[6];
    last_res = o[4];
    // fallback: a start that is not the zero start is abandoned when the loop
    // diverges from it (non-finite residual, three rises in a row) or its first
    // residual exceeds the limit
    rep.fell_back = 0;
    ++since_start;
    if (start_kind != 0 && !(o[4] < opt.tol_eV)) {
        grow = (since_start > 1 && o[4] > prev_res) ? grow + 1 : 0;
        const bool bad = !std::isfinite(o[4]) || grow >= 3 ||
                         (since_start == 1 && first_res_limit > 0 && o[4] > first_res_limit);
        if (bad) {
            set_potential(nullptr);
            rep.fell_back = 1;
        }
    }
    prev_res = o[4];
    rep.iterations = iterations;
    rep.residual = o[4];
    rep.converged = o[4] < opt.tol_eV && neutral_ok;
    rep.fermi = o[0];
    rep.n_cb = int(o[1]);
    rep.n_conv = int(o[2]);
    rep.electrons = o[3];
    rep.cg_iters = cg_it;
    rep.cg_rel_res = cg_rel;
    rep.lanczos_steps = steps;
    rep.u_min = o[5];
    rep.sigma = sigma;
    rep.eig_seconds = std::chrono::duration<double>(t1 - t0).count();
    rep.poisson_seconds = std::chrono::duration<double>(t2 - t1).count();
    rep.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace tbh
